// k_tiled.hip -- multi-gate passes over LDS-resident tiles for gfx950.
//
// The state-vector method applies each gate as one pass over 2^n amplitudes
// (Sec. II); a gate that only mixes amplitudes inside a group of qubits can be
// applied to any sub-block spanning those qubits on its own. A pass here takes
// a tile of 2^mb amplitudes spanning a chosen qubit set (the lb lowest qubits,
// so that loads and stores are contiguous 1 KiB runs, plus mb - lb higher
// ones), keeps it in LDS, applies every gate of the pass to it in circuit
// order, and writes it back: one HBM read and write of the state per pass.
//
// One workgroup owns one tile. Gates are enumerated per tile over their base
// members (the local indices whose fixed bits hold the gate's pattern), with
// the workgroup's threads striding over them, and a barrier between gates.
// Bits outside the tile that a gate fixes (controls, pattern bits) are the
// same for the whole tile, so such a gate either applies to the whole tile's
// member set or skips the tile.
#include "sv_device.h"
#include "sv_kernels.h"

#include <atomic>

using namespace svd;

namespace {

constexpr int kTT = 1024;   // threads per tile workgroup (16 wavefronts)
constexpr int kTableBytes = 4096;   // phase table of a parity run: at most 2*127+1 complex128

// Local index of base member e: zeros inserted at the gate's fixed local bits
// (ascending), then their values.
__device__ inline uint32_t base_member(uint32_t e, const svk::TileGate &g) {
    uint32_t j = e;
    for (int t = 0; t < g.nins; ++t) {
        const int p = g.ins[t];
        j = ((j >> p) << (p + 1)) | (j & ((1u << p) - 1u));
    }
    return j | g.lv;
}

template <typename T>
__device__ inline Cx<T> uent(const svk::TileGate &g, int i) {
    return Cx<T>{(T)g.u[2 * i], (T)g.u[2 * i + 1]};
}

template <typename T>
__device__ inline Cx<T> cmul(Cx<T> a, Cx<T> b) {
    return cfma(Cx<T>{0, 0}, a, b);
}

template <typename T, int MB>
__global__ __launch_bounds__(kTT) void k_tiled(svk::TileArgs a, const svk::TileGate *__restrict__ gates,
                                               u4 *__restrict__ psi) {
    using A = Amp<T>;
    constexpr int LGE = A::LGE;
    extern __shared__ __align__(16) unsigned char smem[];
    Cx<T> *lds = reinterpret_cast<Cx<T> *>(smem);
    u4 *ldsv = reinterpret_cast<u4 *>(smem);
    // LDS: the tile, the phase table of parity runs, the high-bit offsets
    Cx<T> *ptab = reinterpret_cast<Cx<T> *>(smem + (sizeof(Cx<T>) << MB));
    uint64_t *hoff = reinterpret_cast<uint64_t *>(smem + (sizeof(Cx<T>) << MB) + kTableBytes);
    const uint64_t tile = xcd_block();
    if (tile >= a.ntiles) return;   // the whole workgroup leaves together
    const int tid = threadIdx.x;
    const int mb = a.mb, lb = a.lb, hb = mb - lb;
    const uint64_t base = deposit(tile, a.qh, hb, lb);

    // Global offset of each value of the high local bits.
    for (int i = tid; i < (1 << hb); i += kTT) {
        uint64_t o = 0;
        for (int j = 0; j < hb; ++j)
            if ((i >> j) & 1) o |= 1ull << a.qh[j];
        hoff[i] = o;
    }
    __syncthreads();

    // Load: local vector s holds local amplitudes s << LGE ...; its low lb - LGE
    // bits run over a contiguous stretch of the state.
    const int lv = lb - LGE;
    const uint32_t nvec = 1u << (mb - LGE);
    for (uint32_t s = tid; s < nvec; s += kTT) {
        const uint64_t g = base + ((uint64_t)(s & ((1u << lv) - 1u)) << LGE) + hoff[s >> lv];
        ldsv[s] = ld_nt(psi + (g >> LGE));
    }
    __syncthreads();

    for (int gi = 0; gi < a.ngates; ++gi) {
        const svk::TileGate &g = gates[a.gate0 + gi];
        if ((base & g.gm) != g.gv) continue;   // uniform: the tile holds no member
        const uint32_t count = 1u << (mb - g.nins);
        if (g.kind == 0) {
            if (g.K == 0) {
                const Cx<T> ph = uent<T>(g, 0);
                for (uint32_t e = tid; e < count; e += kTT) {
                    const uint32_t j = base_member(e, g);
                    lds[j] = cmul(ph, lds[j]);
                }
            } else if (g.K == 1) {
                const Cx<T> u00 = uent<T>(g, 0), u01 = uent<T>(g, 1), u10 = uent<T>(g, 2), u11 = uent<T>(g, 3);
                const uint32_t F0 = g.F[0];
                for (uint32_t e = tid; e < count; e += kTT) {
                    const uint32_t j = base_member(e, g);
                    const Cx<T> x0 = lds[j], x1 = lds[j ^ F0];
                    lds[j] = cfma(cmul(u00, x0), u01, x1);
                    lds[j ^ F0] = cfma(cmul(u10, x0), u11, x1);
                }
            } else {
                const uint32_t F0 = g.F[0], F1 = g.F[1];
                for (uint32_t e = tid; e < count; e += kTT) {
                    const uint32_t j = base_member(e, g);
                    const uint32_t jm[4] = {j, j ^ F0, j ^ F1, j ^ F0 ^ F1};
                    Cx<T> x[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) x[m] = lds[jm[m]];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        Cx<T> acc{0, 0};
#pragma unroll
                        for (int m = 0; m < 4; ++m) acc = cfma(acc, uent<T>(g, 4 * r + m), x[m]);
                        lds[jm[r]] = acc;
                    }
                }
            }
        } else if (g.kind == 2) {
            // Phase run: angle sums, one sincos per amplitude. Terms entirely
            // outside the tile give one angle for the tile, terms on thread-index
            // bits one per thread, the others one per amplitude.
            constexpr int APT = (1 << MB) / kTT;   // amplitudes per thread: j = tid + q * kTT
            const uint32_t size = 1u << mb;
            double at = 0.0, aq[APT];
#pragma unroll
            for (int q = 0; q < APT; ++q) aq[q] = 0.0;
            const int nt = g.K;
            for (int t = 0; t < nt; ++t) {
                const svk::TileGate &h = gates[a.gate0 + gi + 1 + t];
                if ((base & h.gm) != h.gv) continue;   // uniform
                uint32_t mfix = 0, lmask = h.pm;
                int t0 = -1, t1 = -1;
                for (int i = 0; i < h.K; ++i) {
                    if (h.tl[i] < 0) mfix |= (uint32_t)((base >> h.tg[i]) & 1u) << i;
                    else lmask |= 1u << h.tl[i];
                }
                if (h.K > 0) t0 = h.tl[0];
                if (h.K > 1) t1 = h.tl[1];
                const double a0 = h.u[0], a1 = h.u[1], a2 = h.u[2], a3 = h.u[3];
                auto ang = [&](uint32_t j) {
                    uint32_t m = mfix;
                    if (t0 >= 0) m |= (j >> t0) & 1u;
                    if (t1 >= 0) m |= ((j >> t1) & 1u) << 1;
                    const double lo = (m & 1u) ? a1 : a0, hi = (m & 1u) ? a3 : a2;
                    return ((j & h.pm) == h.pv) ? ((m & 2u) ? hi : lo) : 0.0;
                };
                if (lmask < (uint32_t)kTT) {
                    at += ang((uint32_t)tid);
                } else {
#pragma unroll
                    for (int q = 0; q < APT; ++q) aq[q] += ang((uint32_t)tid + q * kTT);
                }
            }
#pragma unroll
            for (int q = 0; q < APT; ++q) {
                const uint32_t j = tid + q * kTT;
                if (j >= size) continue;
                double sn, cs;
                sincos(at + aq[q], &sn, &cs);
                lds[j] = cmul(Cx<T>{(T)cs, (T)sn}, lds[j]);
            }
            gi += nt;
        } else if (g.kind == 4) {
            // Parity run: angle(j) = c + sum_t w_t parity(j & mask_t) over the
            // global index. A term's bits outside the tile give it a fixed parity
            // f for the whole tile, and w (f xor p) = w f + (1 - 2f) w p: the
            // constant goes into c, the sign into the term.
            const int P = g.K;
            const svk::TileGate *terms = gates + a.gate0 + gi + 1;
            double c = g.u[0];
            for (int t = 0; t < P; ++t)
                if (__builtin_popcountll(base & terms[t].gm) & 1) c += terms[t].u[0];
            constexpr int APT = (1 << MB) / kTT;
            const uint32_t size = 1u << mb;
            if (g.pm) {
                // one common weight w: count the signed parities k in [-P, P] and
                // take exp(i (c + w k)) from a table filled once per tile
                const double w = g.u[1];
                if (tid <= 2 * P) {
                    double sn, cs;
                    sincos(c + w * (double)(tid - P), &sn, &cs);
                    ptab[tid] = Cx<T>{(T)cs, (T)sn};
                }
                __syncthreads();
                // terms outer, this thread's amplitudes inner: each term's mask and
                // sign are read once per thread
                int kq[APT];
#pragma unroll
                for (int q = 0; q < APT; ++q) kq[q] = P;
                for (int t = 0; t < P; ++t) {
                    const uint32_t lm = terms[t].pm;
                    if (lm == 0) continue;
                    const bool neg = __builtin_popcountll(base & terms[t].gm) & 1;
#pragma unroll
                    for (int q = 0; q < APT; ++q) {
                        const int par = __builtin_popcount((uint32_t)(tid + q * kTT) & lm) & 1;
                        kq[q] += neg ? -par : par;
                    }
                }
#pragma unroll
                for (int q = 0; q < APT; ++q) {
                    const uint32_t j = tid + q * kTT;
                    if (j < size) lds[j] = cmul(ptab[kq[q]], lds[j]);
                }
            } else if (sizeof(T) == 8) {
                // several weights, complex128: terms outer as above, one FP64
                // angle per amplitude (8 of them per thread)
                double aq[APT];
#pragma unroll
                for (int q = 0; q < APT; ++q) aq[q] = c;
                for (int t = 0; t < P; ++t) {
                    const uint32_t lm = terms[t].pm;
                    if (lm == 0) continue;
                    const double wt = (__builtin_popcountll(base & terms[t].gm) & 1) ? -terms[t].u[0] : terms[t].u[0];
#pragma unroll
                    for (int q = 0; q < APT; ++q)
                        if (__builtin_popcount((uint32_t)(tid + q * kTT) & lm) & 1) aq[q] += wt;
                }
#pragma unroll
                for (int q = 0; q < APT; ++q) {
                    const uint32_t j = tid + q * kTT;
                    if (j >= size) continue;
                    double sn, cs;
                    sincos(aq[q], &sn, &cs);
                    lds[j] = cmul(Cx<T>{(T)cs, (T)sn}, lds[j]);
                }
            } else {
                // complex64 (16 amplitudes per thread): amplitudes outer, no
                // per-amplitude accumulators
#pragma unroll 1
                for (int q = 0; q < APT; ++q) {
                    const uint32_t j = tid + q * kTT;
                    if (j >= size) break;
                    double ang = c;
                    for (int t = 0; t < P; ++t) {
                        const double wt = (__builtin_popcountll(base & terms[t].gm) & 1) ? -terms[t].u[0]
                                                                                       : terms[t].u[0];
                        if (__builtin_popcount(j & terms[t].pm) & 1) ang += wt;
                    }
                    double sn, cs;
                    sincos(ang, &sn, &cs);
                    lds[j] = cmul(Cx<T>{(T)cs, (T)sn}, lds[j]);
                }
            }
            gi += P;
        } else {
            // diagonal: factor index from the target bits, the ones outside the tile fixed
            uint32_t mfix = 0;
            for (int i = 0; i < g.K; ++i)
                if (g.tl[i] < 0) mfix |= (uint32_t)((base >> g.tg[i]) & 1u) << i;
            for (uint32_t e = tid; e < count; e += kTT) {
                const uint32_t j = base_member(e, g);
                uint32_t m = mfix;
                for (int i = 0; i < g.K; ++i)
                    if (g.tl[i] >= 0) m |= ((j >> g.tl[i]) & 1u) << i;
                lds[j] = cmul(uent<T>(g, (int)m), lds[j]);
            }
        }
        __syncthreads();
    }

    for (uint32_t s = tid; s < nvec; s += kTT) {
        const uint64_t g = base + ((uint64_t)(s & ((1u << lv) - 1u)) << LGE) + hoff[s >> lv];
        st_nt(psi + (g >> LGE), ldsv[s]);
    }
}

template <typename T, int MB>
constexpr size_t tile_lds_bytes(int lb_full) {
    return (sizeof(Cx<T>) << MB) + kTableBytes + (sizeof(uint64_t) << (MB - lb_full));
}

template <typename T, int MB>
hipError_t go_tiled(const svk::TileArgs &a, const svk::TileGate *gates, void *psi, hipStream_t s, int lb_full) {
    static std::atomic<bool> attr_set{false};
    const size_t lds = tile_lds_bytes<T, MB>(lb_full);
    if (!attr_set.load(std::memory_order_acquire)) {
        hipError_t e = hipFuncSetAttribute((const void *)k_tiled<T, MB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        attr_set.store(true, std::memory_order_release);
    }
    hipLaunchKernelGGL((k_tiled<T, MB>), svk::grid_for(a.ntiles), dim3(kTT), lds, s, a, gates, (u4 *)psi);
    return hipGetLastError();
}

}  // namespace

namespace svk {

hipError_t launch_tiled(const TileArgs &a, const TileGate *gates_dev, void *psi, int is_c64, hipStream_t s) {
    const int lb_full = low_bits(is_c64);
    if (a.mb > tile_bits(is_c64) || a.lb > a.mb || a.mb - a.lb > tile_bits(is_c64) - lb_full || a.lb < 1)
        return hipErrorInvalidValue;
    if (is_c64) return go_tiled<float, 14>(a, gates_dev, psi, s, lb_full);
    return go_tiled<double, 13>(a, gates_dev, psi, s, lb_full);
}

}  // namespace svk
