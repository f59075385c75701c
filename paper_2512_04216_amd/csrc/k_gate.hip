// k_gate.hip -- per-gate state-vector update kernels for gfx950.
//
// Every gate of the state-vector method (Sec. II) multiplies groups of
// amplitudes by a small matrix. These kernels stream the state through HBM once
// per gate and read/write only the amplitudes the gate changes.
//
// Work layout. A wavefront owns "segments": 64 lanes x 16 bytes = 1 KiB of
// contiguous amplitudes (index bits below LB = 6 for complex128, 7 for
// complex64). Gate bits at or above LB select which segments a wavefront
// loads together (pure coalesced streaming); gate bits below LB are resolved
// inside the wavefront: a lane gets its partners' values from other lanes with
// ds_bpermute (and from the other half of its own 16-byte slice for complex64).
// Fixed (control / pattern) bits above LB are skipped by index deposit, so
// e.g. a controlled gate whose control is a high qubit reads only half the state.
// Below LB, lanes outside the gate's amplitudes stay idle, except where a
// member shares a 64-byte run with non-members (a fixed bit that selects runs
// of 16 or 32 bytes): there the whole run is read and written back, unchanged
// where not a member, since scattered 16- and 32-byte writes into every line
// cost more than rewriting it (CX(0,1) at 28 qubits, complex128: 2.09 ms with
// member-only stores, a full-state sweep takes 1.35 ms).
#include "sv_device.h"
#include "sv_kernels.h"

#include <algorithm>
#include <vector>
#include <cstring>

using namespace svd;

namespace {

constexpr int kBlock = 256;   // 4 wavefronts per workgroup
constexpr int kSlots = 2;     // outer indices per wavefront (loads in flight)

// Outer indices per wavefront of a group kernel: gates whose members lie in
// different segments (high flip bits) already load two or four segments per
// index and stream best with one index per wavefront; the others take two.
// (28 qubits, complex128: one U3 on qubit 10 at 6.32 vs 6.00 TB/s with one vs
// two; on qubit 3 at 6.33 vs 6.39 TB/s.)
template <int KH>
constexpr int group_slots() { return KH > 0 ? 1 : 2; }

// Index bits (amplitude units) inside one 64-byte run.
template <typename T>
constexpr uint32_t run_bits() { return 64 / (2 * sizeof(T)) - 1; }

template <typename T>
struct GArgs {
    uint64_t n_outer;    // number of outer indices (segment groups)
    uint64_t fv_high;    // fixed-bit values above LB
    uint64_t soff[4];    // segment offset of each high-member combination
    uint32_t fm_low, fv_low;
    uint32_t lF[2];      // low flip vectors
    uint32_t mixlow;     // low part of a flip vector that also has high bits
    uint32_t nlow_valid; // min(2^n, amplitudes per segment)
    int nhb;
    int hb[40];          // fixed-bit positions >= LB, ascending
    T tab[2 * 16];       // tab[m][d] = U[m][m ^ d], complex, row-major
};

template <typename T, int KL>
__device__ inline uint32_t low_off(const GArgs<T> &a, int v) {
    uint32_t x = 0;
    if (KL >= 1 && (v & 1)) x ^= a.lF[0];
    if (KL >= 2 && (v & 2)) x ^= a.lF[1];
    return x;
}

// K = KH + KL flip vectors: the first KH only have bits >= LB (each selects
// a segment), the next KL only bits < LB (each selects a lane / register).
// MIX (K = 1 only): the single flip vector has high bits and the low part
// `mixlow` as well (e.g. a SWAP of a low and a high qubit).
template <typename T, int KH, int KL, bool MIX>
__global__ __launch_bounds__(kBlock) void k_group(GArgs<T> a, u4 *__restrict__ psi) {
    using A = Amp<T>;
    constexpr int E = A::E, LGE = A::LGE, LB = 6 + LGE;
    constexpr int NS = 1 << KH, NL = 1 << KL, M = 1 << (KH + KL);
    constexpr int SL = group_slots<KH>();
    const int lane = threadIdx.x & 63;
    const uint64_t wave = wave_id_xcd();

    // Which member (if any) each of this lane's amplitudes is, per segment, and
    // whether the lane moves its 16 bytes of segment s at all (`part`: it holds
    // a member, or shares a 64-byte run with one).
    constexpr uint32_t RUN = run_bits<T>();
    int ml[E];
    bool mem[NS][E];
    bool part[NS];
    bool lane_valid = (uint32_t)(lane * E) < a.nlow_valid;
#pragma unroll
    for (int s = 0; s < NS; ++s) part[s] = false;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t j = lane * E + r;
        const bool valid = j < a.nlow_valid;
        const uint32_t x = (j & a.fm_low) ^ a.fv_low;
        ml[r] = -1;
        if (KL == 0) {
            ml[r] = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const uint32_t want = (MIX && s) ? a.mixlow : 0u;
                mem[s][r] = valid && x == want;
                part[s] = part[s] || (valid && ((x ^ want) & ~RUN) == 0);
            }
        } else {
            bool near = false;
#pragma unroll
            for (int v = 0; v < NL; ++v) {
                if (x == low_off<T, KL>(a, v)) ml[r] = v;
                near = near || ((x ^ low_off<T, KL>(a, v)) & ~RUN) == 0;
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                mem[s][r] = valid && ml[r] >= 0;
                part[s] = part[s] || (valid && near);
            }
        }
    }

    // Matrix rows of this lane's members: tab[m][.], m = s | ml << KH.
    Cx<T> row[NS][E][M];
    if (KL > 0) {
        __shared__ T stab[2 * 16];
        if (threadIdx.x < 2 * M * M) stab[threadIdx.x] = a.tab[threadIdx.x];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int m = s | (max(ml[r], 0) << KH);
#pragma unroll
                for (int d = 0; d < M; ++d)
                    row[s][r][d] = Cx<T>{stab[2 * (m * M + d)], stab[2 * (m * M + d) + 1]};
            }
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int r = 0; r < E; ++r)
#pragma unroll
                for (int d = 0; d < M; ++d)
                    row[s][r][d] = Cx<T>{a.tab[2 * (s * M + d)], a.tab[2 * (s * M + d) + 1]};
    }

    // Issue every load of this wavefront's slots before any arithmetic. Lanes
    // that do not take part skip their loads (their amplitudes are neither
    // changed nor needed as partners).
    Q v[SL][NS];
    uint64_t vidx[SL][NS];
    bool act[SL];
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
        const uint64_t outer = wave * SL + sl;
        act[sl] = outer < a.n_outer;
        const uint64_t base = deposit(act[sl] ? outer : 0, a.hb, a.nhb, LB) | a.fv_high;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            vidx[sl][s] = ((base ^ a.soff[s]) >> LGE) + lane;
            v[sl][s].v = u4{0, 0, 0, 0};
            if (act[sl] && lane_valid && part[s]) v[sl][s].v = ld_nt(psi + vidx[sl][s]);
        }
    }

#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
        if (!act[sl]) continue;   // wavefront-uniform
        // Partner values from other lanes (all lanes execute the permutes).
        Q sh[NS][NL];
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2)
#pragma unroll
            for (int vl = 0; vl < NL; ++vl) {
                const uint32_t X = MIX ? a.mixlow : low_off<T, KL>(a, vl);
                const int lx = (int)(X >> LGE);
                sh[s2][vl] = (lx != 0 && (MIX || vl != 0)) ? lane_xor(v[sl][s2], lane, lx) : v[sl][s2];
            }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            Q out = v[sl][s];
#pragma unroll
            for (int r = 0; r < E; ++r) {
                if (!mem[s][r]) continue;
                Cx<T> acc{0, 0};
#pragma unroll
                for (int dh = 0; dh < NS; ++dh)
#pragma unroll
                    for (int dl = 0; dl < NL; ++dl) {
                        const int d = dh | (dl << KH);
                        uint32_t X;
                        Q src;
                        if (MIX) {
                            X = dh ? a.mixlow : 0u;
                            src = dh ? sh[s ^ 1][0] : v[sl][s];
                        } else {
                            X = low_off<T, KL>(a, dl);
                            src = sh[s ^ dh][dl];
                        }
                        const int rr = r ^ (int)(X & (E - 1));
                        acc = cfma(acc, row[s][r][d], A::get(src, rr));
                    }
                A::set(out, r, acc);
            }
            if (part[s]) st_nt(psi + vidx[sl][s], out.v);
        }
    }
}

template <typename T>
struct DArgs {
    uint64_t n_outer;
    uint64_t fv_high;
    uint32_t fm_low, fv_low;
    uint32_t nlow_valid;
    int nhb;
    int hb[40];
    int k;
    int targets[8];
    T d[2 * 32];
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag(DArgs<T> a, u4 *__restrict__ psi) {
    using A = Amp<T>;
    constexpr int E = A::E, LGE = A::LGE, LB = 6 + LGE;
    __shared__ T sd[2 * 32];
    if (threadIdx.x < (2u << a.k)) sd[threadIdx.x] = a.d[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint64_t wave = wave_id_xcd();
    // The lane moves its 16 bytes if they hold a controlled amplitude or share
    // a 64-byte run with one.
    constexpr uint32_t RUN = run_bits<T>();
    bool lane_valid = false;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t j = lane * E + r;
        lane_valid = lane_valid || (j < a.nlow_valid && (((j & a.fm_low) ^ a.fv_low) & ~RUN) == 0);
    }
    Q v[kSlots];
    uint64_t vidx[kSlots], base[kSlots];
    bool act[kSlots];
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
        const uint64_t outer = wave * kSlots + sl;
        act[sl] = outer < a.n_outer;
        base[sl] = deposit(act[sl] ? outer : 0, a.hb, a.nhb, LB) | a.fv_high;
        vidx[sl] = (base[sl] >> LGE) + lane;
        v[sl].v = u4{0, 0, 0, 0};
        if (act[sl] && lane_valid) v[sl].v = ld_nt(psi + vidx[sl]);
    }
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
        if (!act[sl] || !lane_valid) continue;
        Q out = v[sl];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t j = lane * E + r;
            if (j >= a.nlow_valid || ((j & a.fm_low) != a.fv_low)) continue;
            const uint64_t i = base[sl] | j;
            int m = 0;
            for (int t = 0; t < a.k; ++t) m |= (int)((i >> a.targets[t]) & 1u) << t;
            const Cx<T> dm{sd[2 * m], sd[2 * m + 1]};
            Cx<T> acc{0, 0};
            A::set(out, r, cfma(acc, dm, A::get(v[sl], r)));
        }
        st_nt(psi + vidx[sl], out.v);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(u4 *__restrict__ psi, uint64_t nvec, uint64_t basis) {
    using A = Amp<T>;
    const uint64_t bvec = basis >> A::LGE;
    const uint64_t i0 = xcd_block() * (kBlock * kSlots) + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
        const uint64_t i = i0 + u * kBlock;
        if (i >= nvec) continue;
        Q q;
        q.v = u4{0, 0, 0, 0};
        if (i == bvec) A::set(q, (int)(basis & (A::E - 1)), Cx<T>{T(1), T(0)});
        st_nt(psi + i, q.v);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale(u4 *__restrict__ psi, uint64_t nvec,
                                                  const double *__restrict__ norm2) {
    const double sc = 1.0 / sqrt(*norm2);
    const uint64_t i0 = xcd_block() * (kBlock * kSlots) + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
        const uint64_t i = i0 + u * kBlock;
        if (i >= nvec) continue;
        Q q;
        q.v = ld_nt(psi + i);
        if (sizeof(T) == 8) {
            q.d[0] *= sc;
            q.d[1] *= sc;
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) q.f[c] = (float)((double)q.f[c] * sc);
        }
        st_nt(psi + i, q.v);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(const Cx<T> *__restrict__ psi, const uint64_t *__restrict__ idx,
                                                   int64_t count, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    const Cx<T> a = psi[idx[i]];
    out[2 * i] = (double)a.re;
    out[2 * i + 1] = (double)a.im;
}

inline int popc64(uint64_t x) { return __builtin_popcountll(x); }

uint64_t oneshot_blocks(uint64_t nvec) {
    return std::max<uint64_t>(1, (nvec + kBlock * kSlots - 1) / (kBlock * kSlots));
}

// Common planning of the outer enumeration: high fixed bits, counts.
template <typename T>
void plan_outer(uint64_t fm, uint64_t fv, int n, int LB, uint64_t &n_outer, uint64_t &fv_high,
                uint32_t &fm_low, uint32_t &fv_low, uint32_t &nlow_valid, int &nhb, int *hb) {
    const uint64_t lowmask = (1ull << LB) - 1;
    const uint64_t fmh = fm & ~lowmask;
    nhb = 0;
    for (int p = LB; p < 64; ++p)
        if ((fmh >> p) & 1) hb[nhb++] = p;
    const int high_bits = n > LB ? n - LB : 0;
    n_outer = 1ull << (high_bits - nhb);
    fv_high = fv & ~lowmask;
    fm_low = (uint32_t)(fm & lowmask);
    fv_low = (uint32_t)(fv & lowmask);
    nlow_valid = (uint32_t)std::min<uint64_t>(1ull << n, 1ull << LB);
}

template <typename T, int KH, int KL, bool MIX>
hipError_t go_group(const GArgs<T> &a, void *psi, hipStream_t s) {
    constexpr int SL = group_slots<KH>();
    const uint64_t waves = (a.n_outer + SL - 1) / SL;
    const uint64_t blocks = (waves + (kBlock / 64) - 1) / (kBlock / 64);
    hipLaunchKernelGGL((k_group<T, KH, KL, MIX>), svk::grid_for(blocks), dim3(kBlock), 0, s, a, (u4 *)psi);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_group_t(const svk::GroupGate &g, void *psi, int n, hipStream_t s) {
    constexpr int LB = 6 + Amp<T>::LGE;
    const uint64_t lowmask = (1ull << LB) - 1;
    GArgs<T> a;
    memset(&a, 0, sizeof(a));
    plan_outer<T>(g.fm, g.fv, n, LB, a.n_outer, a.fv_high, a.fm_low, a.fv_low, a.nlow_valid, a.nhb,
                  a.hb);
    // kernel member bit order: high flip vectors first, then low ones
    int order[2] = {0, 1};
    int KH = 0, KL = 0;
    bool mix = false;
    if (g.K == 1) {
        const uint64_t h = g.F[0] & ~lowmask, l = g.F[0] & lowmask;
        if (h && l) {
            mix = true;
            KH = 1;
            a.soff[1] = h;
            a.mixlow = (uint32_t)l;
        } else if (h) {
            KH = 1;
            a.soff[1] = h;
        } else {
            KL = 1;
            a.lF[0] = (uint32_t)l;
        }
    } else if (g.K == 2) {
        const bool h0 = (g.F[0] & ~lowmask) != 0, h1 = (g.F[1] & ~lowmask) != 0;
        if (((g.F[0] & ~lowmask) && (g.F[0] & lowmask)) || ((g.F[1] & ~lowmask) && (g.F[1] & lowmask)))
            return hipErrorInvalidValue;   // caller routes such gates elsewhere
        if (h0 && h1) {
            KH = 2;
        } else if (!h0 && !h1) {
            KL = 2;
        } else {
            KH = 1;
            KL = 1;
            if (!h0) std::swap(order[0], order[1]);
        }
        int nh = 0, nl = 0;
        uint64_t hv[2] = {0, 0};
        for (int b = 0; b < 2; ++b) {
            const uint64_t f = g.F[order[b]];
            if (f & ~lowmask) hv[nh++] = f;
            else a.lF[nl++] = (uint32_t)f;
        }
        for (int sidx = 0; sidx < (1 << KH); ++sidx) {
            uint64_t o = 0;
            for (int b = 0; b < KH; ++b)
                if ((sidx >> b) & 1) o ^= hv[b];
            a.soff[sidx] = o;
        }
    }
    const int K = g.K, Mm = 1 << K;
    // permuted matrix: kernel member m <-> original member orig(m)
    auto orig = [&](int m) {
        int o = 0;
        for (int b = 0; b < K; ++b)
            if ((m >> b) & 1) o |= 1 << order[b];
        return o;
    };
    for (int m = 0; m < Mm; ++m)
        for (int d = 0; d < Mm; ++d) {
            const int r = orig(m), c = orig(m ^ d);
            a.tab[2 * (m * Mm + d)] = (T)g.U[2 * (r * Mm + c)];
            a.tab[2 * (m * Mm + d) + 1] = (T)g.U[2 * (r * Mm + c) + 1];
        }
    if (K == 0) return go_group<T, 0, 0, false>(a, psi, s);
    if (K == 1) {
        if (mix) return go_group<T, 1, 0, true>(a, psi, s);
        if (KH == 1) return go_group<T, 1, 0, false>(a, psi, s);
        return go_group<T, 0, 1, false>(a, psi, s);
    }
    if (KH == 2) return go_group<T, 2, 0, false>(a, psi, s);
    if (KH == 1) return go_group<T, 1, 1, false>(a, psi, s);
    return go_group<T, 0, 2, false>(a, psi, s);
}

template <typename T>
hipError_t launch_diag_t(const svk::DiagGate &g, void *psi, int n, hipStream_t s) {
    constexpr int LB = 6 + Amp<T>::LGE;
    DArgs<T> a;
    memset(&a, 0, sizeof(a));
    plan_outer<T>(g.cmask, g.cmask, n, LB, a.n_outer, a.fv_high, a.fm_low, a.fv_low, a.nlow_valid,
                  a.nhb, a.hb);
    a.k = g.k;
    for (int t = 0; t < g.k; ++t) a.targets[t] = g.targets[t];
    for (int m = 0; m < (2 << g.k); ++m) a.d[m] = (T)g.d[m];
    const uint64_t waves = (a.n_outer + kSlots - 1) / kSlots;
    const uint64_t blocks = (waves + 3) / 4;
    hipLaunchKernelGGL((k_diag<T>), svk::grid_for(blocks), dim3(kBlock), 0, s, a, (u4 *)psi);
    return hipGetLastError();
}

}  // namespace

namespace svk {

hipError_t launch_init(void *psi, int n, int is_c64, uint64_t basis, hipStream_t s) {
    const uint64_t nvec = is_c64 ? ((1ull << n) + 1) / 2 : (1ull << n);
    const uint64_t blocks = oneshot_blocks(nvec);
    if (is_c64)
        hipLaunchKernelGGL(k_init<float>, grid_for(blocks), dim3(kBlock), 0, s, (u4 *)psi, nvec, basis);
    else
        hipLaunchKernelGGL(k_init<double>, grid_for(blocks), dim3(kBlock), 0, s, (u4 *)psi, nvec, basis);
    return hipGetLastError();
}

hipError_t launch_group(const GroupGate &g, void *psi, int n, int is_c64, hipStream_t s) {
    return is_c64 ? launch_group_t<float>(g, psi, n, s) : launch_group_t<double>(g, psi, n, s);
}

hipError_t launch_diag(const DiagGate &g, void *psi, int n, int is_c64, hipStream_t s) {
    return is_c64 ? launch_diag_t<float>(g, psi, n, s) : launch_diag_t<double>(g, psi, n, s);
}

hipError_t launch_gather(const void *psi, int is_c64, const uint64_t *idx_dev, int64_t count, double *out_dev,
                         hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
    if (is_c64)
        hipLaunchKernelGGL(k_gather<float>, dim3(blocks), dim3(kBlock), 0, s, (const Cx<float> *)psi, idx_dev, count,
                           out_dev);
    else
        hipLaunchKernelGGL(k_gather<double>, dim3(blocks), dim3(kBlock), 0, s, (const Cx<double> *)psi, idx_dev, count,
                           out_dev);
    return hipGetLastError();
}

hipError_t launch_scale_by_norm(void *psi, int n, int is_c64, const double *norm2_dev, hipStream_t s) {
    const uint64_t nvec = is_c64 ? ((1ull << n) + 1) / 2 : (1ull << n);
    const uint64_t blocks = oneshot_blocks(nvec);
    if (is_c64)
        hipLaunchKernelGGL(k_scale<float>, grid_for(blocks), dim3(kBlock), 0, s, (u4 *)psi, nvec, norm2_dev);
    else
        hipLaunchKernelGGL(k_scale<double>, grid_for(blocks), dim3(kBlock), 0, s, (u4 *)psi, nvec, norm2_dev);
    return hipGetLastError();
}

}  // namespace svk
