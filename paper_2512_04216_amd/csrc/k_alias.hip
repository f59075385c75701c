// k_alias.hip -- Walker alias tables of |psi|^2, built in parallel, and O(1)
// draws from them (Sec. III-C item 1: the paper samples shots by the alias
// method).
//
// With N = 2^n and s_i = N p_i / W, entries with s_i < 1 are light (deficit
// 1 - s_i), the others heavy (excess s_i - 1). The table is the one of the
// sweep construction in index order -- light entries take the current heavy
// entry as alias, a heavy entry whose excess runs out becomes light and takes
// the next heavy entry -- written through prefix sums instead of a sweep.
// With D_k the inclusive prefix of the light deficits (k-th light in index
// order) and E_j that of the heavy excesses:
//   light k:  alias = heavy j, the first with E_j >= D_{k-1} (D_{-1} = 0);
//   heavy j:  exhausted by the first light k with D_k > E_j; then
//             prob = 1 - (D_k - E_j) and alias = heavy j + 1;
//             never exhausted (or the last heavy entry): prob = 1.
// Both prefixes are compensated (value + error term), so prob keeps FP64
// accuracy however large the prefixes grow.
//
// Passes: per-tile counts and sums (k_alias_tiles), one workgroup scanning
// the tiles (k_alias_scan), per-tile prefixes written with the light and
// heavy entries compacted in index order (k_alias_write), then the pairing by
// binary search over the sorted prefixes (k_alias_pair). Draws: k_alias_draw.
#include "sv_device.h"
#include "sv_kernels.h"

using namespace svd;

namespace {

constexpr int kTile = 4096;       // amplitudes per workgroup in the tile passes
constexpr int kT = 256;           // threads per tile workgroup
constexpr int kPer = kTile / kT;  // contiguous amplitudes per thread
constexpr int kScanT = 1024;      // threads of the tile scan

struct Acc {
    uint64_t nl;   // light entries
    DD d, e;       // deficits of light entries, excesses of heavy ones
};

__device__ inline Acc acc_zero() { return {0, dd_zero(), dd_zero()}; }
__device__ inline Acc acc_cat(const Acc &a, const Acc &b) {   // a precedes b
    return {a.nl + b.nl, dd_add(a.d, b.d), dd_add(a.e, b.e)};
}

// x - y of two compensated values, in FP64
__device__ inline double dd_diff(DD x, DD y) { return (x.s - y.s) + (x.c - y.c); }

__device__ inline uint64_t smix(uint64_t seed, uint64_t s) {
    uint64_t z = seed + (s + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ inline double u01(uint64_t seed, uint64_t s) { return (double)(smix(seed, s) >> 11) * 0x1.0p-53; }

template <typename T>
__device__ inline double prob_of(const Q &q, int r) {
    const Cx<T> a = Amp<T>::get(q, r);
    const double re = (double)a.re, im = (double)a.im;
    return fma(re, re, im * im);
}

// s values of tile `tile` into LDS, index order; returns the tile's length.
template <typename T>
__device__ inline int load_tile(const u4 *__restrict__ psi, int n, uint64_t tile, double scale, double *s_lds) {
    constexpr int E = Amp<T>::E;
    const uint64_t N = 1ull << n;
    const uint64_t a0 = tile * kTile;
    const int cnt = (int)((N - a0) < (uint64_t)kTile ? (N - a0) : (uint64_t)kTile);
    const int nvec = (cnt + E - 1) / E;
    for (int v = threadIdx.x; v < nvec; v += kT) {
        Q q;
        q.v = psi[a0 / E + (uint64_t)v];
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (v * E + e < cnt) s_lds[v * E + e] = prob_of<T>(q, e) * scale;
    }
    __syncthreads();
    return cnt;
}

// Inclusive scan of per-thread accumulators over the workgroup (Hillis-Steele,
// earlier threads first in every combination).
template <int NT>
__device__ inline Acc block_incl_scan(Acc v, Acc *buf) {
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        Acc o = acc_zero();
        const bool has = t >= off;
        if (has) o = buf[t - off];
        __syncthreads();
        if (has) v = acc_cat(o, v);
        buf[t] = v;
        __syncthreads();
    }
    return v;
}

// thread-local accumulation over this thread's contiguous amplitudes
__device__ inline Acc thread_acc(const double *s_lds, int cnt) {
    Acc a = acc_zero();
    const int b = threadIdx.x * kPer;
    for (int k = 0; k < kPer && b + k < cnt; ++k) {
        const double s = s_lds[b + k];
        if (s < 1.0) {
            a.nl++;
            neum_add(a.d, 1.0 - s);
        } else {
            neum_add(a.e, s - 1.0);
        }
    }
    return a;
}

template <typename T>
__global__ __launch_bounds__(kT) void k_alias_tiles(const u4 *__restrict__ psi, int n,
                                                    const double *__restrict__ norm2, Acc *__restrict__ rec) {
    __shared__ double s_lds[kTile];
    __shared__ Acc buf[kT];
    const double scale = (double)(1ull << n) / norm2[0];
    const int cnt = load_tile<T>(psi, n, blockIdx.x, scale, s_lds);
    const Acc tot = block_incl_scan<kT>(thread_acc(s_lds, cnt), buf);
    if (threadIdx.x == kT - 1) rec[blockIdx.x] = tot;
}

// Exclusive scan of the tile records in place; meta[0] = number of light entries.
__global__ __launch_bounds__(kScanT) void k_alias_scan(Acc *__restrict__ rec, uint64_t ntiles,
                                                       uint64_t *__restrict__ meta) {
    __shared__ Acc buf[kScanT];
    const uint64_t per = (ntiles + kScanT - 1) / kScanT;
    const uint64_t b = threadIdx.x * per, e = (b + per < ntiles) ? b + per : ntiles;
    Acc run = acc_zero();
    for (uint64_t i = b; i < e; ++i) run = acc_cat(run, rec[i]);
    const Acc incl = block_incl_scan<kScanT>(run, buf);
    // exclusive offset of this thread = inclusive of the previous one
    Acc off = threadIdx.x ? buf[threadIdx.x - 1] : acc_zero();
    __syncthreads();
    for (uint64_t i = b; i < e; ++i) {
        const Acc v = rec[i];
        rec[i] = off;
        off = acc_cat(off, v);
    }
    if (threadIdx.x == kScanT - 1) meta[0] = incl.nl;
}

template <typename T>
__global__ __launch_bounds__(kT) void k_alias_write(const u4 *__restrict__ psi, int n,
                                                    const double *__restrict__ norm2, const Acc *__restrict__ rec,
                                                    const uint64_t *__restrict__ meta, double *__restrict__ prob,
                                                    uint64_t *__restrict__ alias, uint64_t *__restrict__ idx,
                                                    DD *__restrict__ pre) {
    __shared__ double s_lds[kTile];
    __shared__ Acc buf[kT];
    const double scale = (double)(1ull << n) / norm2[0];
    const int cnt = load_tile<T>(psi, n, blockIdx.x, scale, s_lds);
    const Acc mine = thread_acc(s_lds, cnt);
    const Acc incl = block_incl_scan<kT>(mine, buf);
    Acc before = threadIdx.x ? buf[threadIdx.x - 1] : acc_zero();
    before = acc_cat(rec[blockIdx.x], before);
    const uint64_t nl = meta[0];
    const uint64_t a0 = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kPer;
    const int b = threadIdx.x * kPer;
    // running prefixes of this thread's own values, joined to `before`
    DD dl = dd_zero(), el = dd_zero();
    uint64_t lights = 0;
    for (int k = 0; k < kPer && b + k < cnt; ++k) {
        const double s = s_lds[b + k];
        const uint64_t gi = a0 + (uint64_t)k;
        if (s < 1.0) {
            neum_add(dl, 1.0 - s);
            const uint64_t r = before.nl + lights;
            idx[r] = gi;
            pre[r] = dd_add(before.d, dl);
            ++lights;
        } else {
            neum_add(el, s - 1.0);
            const uint64_t r = nl + (gi - (before.nl + lights));   // heavies before gi
            idx[r] = gi;
            pre[r] = dd_add(before.e, el);
            s_lds[b + k] = 1.0;   // heavy entries start with prob 1
        }
    }
    (void)incl;
    __syncthreads();
    // prob and the identity alias in index order, coalesced (the walk above
    // gives each thread a contiguous stretch, so its own stores would stride)
    const uint64_t t0 = (uint64_t)blockIdx.x * kTile;
    for (int v = threadIdx.x; v < cnt; v += kT) {
        prob[t0 + v] = s_lds[v];
        alias[t0 + v] = t0 + v;
    }
}

__global__ __launch_bounds__(kT) void k_alias_pair(uint64_t N, const uint64_t *__restrict__ meta,
                                                   const uint64_t *__restrict__ idx, const DD *__restrict__ pre,
                                                   double *__restrict__ prob, uint64_t *__restrict__ alias) {
    const uint64_t nl = meta[0], nh = N - nl;
    const uint64_t stride = grid_blocks() * kT;
    for (uint64_t g = block_linear() * kT + threadIdx.x; g < N; g += stride) {
        if (nh == 0) {   // uniform up to rounding: every slot keeps its outcome
            prob[g] = 1.0;
            continue;
        }
        if (g < nl) {
            const DD key = g ? pre[g - 1] : dd_zero();
            uint64_t lo = 0, hi = nh;   // first heavy with E_j >= key
            while (lo < hi) {
                const uint64_t mid = lo + (hi - lo) / 2;
                if (dd_diff(pre[nl + mid], key) < 0.0) lo = mid + 1;
                else hi = mid;
            }
            alias[idx[g]] = idx[nl + (lo < nh ? lo : nh - 1)];
        } else {
            const uint64_t j = g - nl;
            if (j + 1 == nh) continue;
            const DD e = pre[g];
            uint64_t lo = 0, hi = nl;   // first light with D_k > E_j
            while (lo < hi) {
                const uint64_t mid = lo + (hi - lo) / 2;
                if (dd_diff(e, pre[mid]) < 0.0) hi = mid;
                else lo = mid + 1;
            }
            if (lo == nl) continue;
            const double p = 1.0 - dd_diff(pre[lo], e);
            prob[idx[g]] = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
            alias[idx[g]] = idx[g + 1];
        }
    }
}

__global__ __launch_bounds__(kT) void k_alias_draw(const double *__restrict__ prob, const uint64_t *__restrict__ alias,
                                                   int n, int64_t shots, uint64_t seed, uint64_t s0,
                                                   uint64_t *__restrict__ out) {
    const double N = (double)(1ull << n);
    const uint64_t stride = grid_blocks() * kT;
    for (uint64_t s = block_linear() * kT + threadIdx.x; s < (uint64_t)shots; s += stride) {
        const uint64_t c = s0 + s;
        const uint64_t slot = (uint64_t)(u01(seed, 2 * c) * N);
        out[s] = (u01(seed, 2 * c + 1) < prob[slot]) ? slot : alias[slot];
    }
}

dim3 capped(uint64_t items) {
    const uint64_t nb = (items + kT - 1) / kT;
    return dim3((unsigned)(nb < (1ull << 16) ? nb : (1ull << 16)));
}

struct AliasLayout {
    uint64_t prob, alias, idx, pre, rec, meta, total;
};

AliasLayout layout(int n) {
    const uint64_t N = 1ull << n, ntiles = (N + kTile - 1) / kTile;
    AliasLayout L;
    L.prob = 0;
    L.alias = L.prob + 8 * N;
    L.idx = L.alias + 8 * N;
    L.pre = L.idx + 8 * N;
    L.rec = L.pre + 16 * N;
    L.meta = L.rec + ((sizeof(Acc) * ntiles + 255) & ~255ull);
    L.total = L.meta + 256;
    return L;
}

}  // namespace

namespace svk {

uint64_t alias_workspace_bytes(int n) { return layout(n).total; }

const double *alias_prob(const void *aws) { return (const double *)aws; }
const uint64_t *alias_alias(const void *aws, int n) {
    return (const uint64_t *)((const char *)aws + layout(n).alias);
}

hipError_t launch_alias_build(const void *psi, int n, int is_c64, void *ws, void *aws, hipStream_t s) {
    const AliasLayout L = layout(n);
    char *w = (char *)aws;
    const uint64_t N = 1ull << n, ntiles = (N + kTile - 1) / kTile;
    hipError_t e = launch_norm(psi, n, is_c64, ws, s);
    if (e != hipSuccess) return e;
    const double *norm2 = norm2_dev_ptr(ws, n);
    Acc *rec = (Acc *)(w + L.rec);
    uint64_t *meta = (uint64_t *)(w + L.meta);
    if (is_c64)
        hipLaunchKernelGGL(k_alias_tiles<float>, dim3((unsigned)ntiles), dim3(kT), 0, s, (const u4 *)psi, n, norm2,
                           rec);
    else
        hipLaunchKernelGGL(k_alias_tiles<double>, dim3((unsigned)ntiles), dim3(kT), 0, s, (const u4 *)psi, n, norm2,
                           rec);
    hipLaunchKernelGGL(k_alias_scan, dim3(1), dim3(kScanT), 0, s, rec, ntiles, meta);
    double *prob = (double *)(w + L.prob);
    uint64_t *alias = (uint64_t *)(w + L.alias), *idx = (uint64_t *)(w + L.idx);
    DD *pre = (DD *)(w + L.pre);
    if (is_c64)
        hipLaunchKernelGGL(k_alias_write<float>, dim3((unsigned)ntiles), dim3(kT), 0, s, (const u4 *)psi, n, norm2,
                           rec, meta, prob, alias, idx, pre);
    else
        hipLaunchKernelGGL(k_alias_write<double>, dim3((unsigned)ntiles), dim3(kT), 0, s, (const u4 *)psi, n, norm2,
                           rec, meta, prob, alias, idx, pre);
    hipLaunchKernelGGL(k_alias_pair, capped(N), dim3(kT), 0, s, N, meta, idx, pre, prob, alias);
    return hipGetLastError();
}

hipError_t launch_alias_draw(const void *aws, int n, int64_t shots, uint64_t seed, uint64_t s0, uint64_t *out_dev,
                             hipStream_t s) {
    if (shots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_alias_draw, capped((uint64_t)shots), dim3(kT), 0, s, alias_prob(aws), alias_alias(aws, n), n,
                       shots, seed, s0, out_dev);
    return hipGetLastError();
}

}  // namespace svk
