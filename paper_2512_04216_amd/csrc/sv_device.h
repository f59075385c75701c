// sv_device.h -- device-side helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svd {

typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// One lane's 16-byte slice of a segment: one complex128 or two complex64.
union Q {
    u4 v;
    uint32_t w[4];
    double d[2];
    float f[4];
};

template <typename T>
struct Cx {
    T re, im;
};

template <typename T>
struct Amp;

template <>
struct Amp<double> {
    static constexpr int E = 1;    // amplitudes per 16-byte lane slice
    static constexpr int LGE = 0;
    static __device__ inline Cx<double> get(const Q &q, int) { return {q.d[0], q.d[1]}; }
    static __device__ inline void set(Q &q, int, Cx<double> c) {
        q.d[0] = c.re;
        q.d[1] = c.im;
    }
};

template <>
struct Amp<float> {
    static constexpr int E = 2;
    static constexpr int LGE = 1;
    static __device__ inline Cx<float> get(const Q &q, int r) {
        return r ? Cx<float>{q.f[2], q.f[3]} : Cx<float>{q.f[0], q.f[1]};
    }
    static __device__ inline void set(Q &q, int r, Cx<float> c) {
        if (r) {
            q.f[2] = c.re;
            q.f[3] = c.im;
        } else {
            q.f[0] = c.re;
            q.f[1] = c.im;
        }
    }
};

template <typename T>
__device__ inline Cx<T> cfma(Cx<T> acc, Cx<T> a, Cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
    return acc;
}

// Value of `q` held by lane (lane ^ x) of the wavefront (ds_bpermute; every
// lane of the wavefront must execute this together).
__device__ inline Q lane_xor(const Q &q, int lane, int x) {
    Q r;
    const int addr = (lane ^ x) << 2;
#pragma unroll
    for (int c = 0; c < 4; ++c) r.w[c] = __builtin_amdgcn_ds_bpermute(addr, (int)q.w[c]);
    return r;
}

// Inserts a zero bit at each position of hb (ascending, final coordinates)
// into c << lb: enumerates the indices whose bits at hb are zero.
__device__ inline uint64_t deposit(uint64_t c, const int *hb, int nhb, int lb) {
    uint64_t i = c << lb;
    for (int t = 0; t < nhb; ++t) {
        const int p = hb[t];
        const uint64_t lo = i & ((1ull << p) - 1ull);
        i = ((i >> p) << (p + 1)) | lo;
    }
    return i;
}

__device__ inline uint64_t wave_id_global() {
    return (uint64_t)blockIdx.x * (blockDim.x >> 6) +
           (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// XCD-aware block order. Workgroups are dealt round-robin to the 8 XCDs of
// the MI355X (block b runs on XCD b % 8); renumbering them so that XCD x works
// through one contiguous eighth of the grid keeps each XCD's L2 and its stream
// of HBM pages local. Measured on a 4 GiB in-place sweep: 6.1 -> 6.5 TB/s.
// Grids of more than 2^22 workgroups are launched two-dimensional (a grid
// dimension may not exceed 2^32 work-items); blocks are numbered x-fastest.
__device__ inline uint64_t block_linear() { return (uint64_t)blockIdx.y * gridDim.x + blockIdx.x; }
__device__ inline uint64_t grid_blocks() { return (uint64_t)gridDim.x * gridDim.y; }

__device__ inline uint64_t xcd_block() {
    const uint64_t nb = grid_blocks(), b = block_linear();
    const uint64_t per = nb >> 3;
    return (b < (per << 3)) ? ((b & 7) * per + (b >> 3)) : b;
}

__device__ inline uint64_t wave_id_xcd() {
    return xcd_block() * (blockDim.x >> 6) + (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Streaming accesses: the state is touched once per kernel, so loads and stores
// carry the non-temporal hint.
__device__ inline u4 ld_nt(const u4 *p) { return __builtin_nontemporal_load(p); }
__device__ inline void st_nt(u4 *p, u4 v) { __builtin_nontemporal_store(v, p); }

// ---- compensated FP64 arithmetic (Knuth TwoSum, Neumaier) ----------------
struct DD {
    double s, c;   // value = s + c, c collects rounding errors
};

__device__ inline DD dd_zero() { return {0.0, 0.0}; }

// Neumaier step: add x to (s, c)
__device__ inline void neum_add(DD &a, double x) {
    const double t = a.s + x;
    a.c += (fabs(a.s) >= fabs(x)) ? ((a.s - t) + x) : ((x - t) + a.s);
    a.s = t;
}

// Combine two compensated sums with TwoSum on the leading parts.
__device__ inline DD dd_add(DD a, DD b) {
    const double s = a.s + b.s;
    const double bp = s - a.s;
    const double e = (a.s - (s - bp)) + (b.s - bp);
    return {s, a.c + b.c + e};
}

__device__ inline double dd_value(DD a) { return a.s + a.c; }

__device__ inline double shfl_xor_d(double v, int lane, int x) {
    const int addr = (lane ^ x) << 2;
    union {
        double d;
        int w[2];
    } u;
    u.d = v;
    u.w[0] = __builtin_amdgcn_ds_bpermute(addr, u.w[0]);
    u.w[1] = __builtin_amdgcn_ds_bpermute(addr, u.w[1]);
    return u.d;
}

// Deterministic wavefront reduction of a compensated sum (fixed xor tree).
__device__ inline DD wave_reduce_dd(DD a, int lane) {
#pragma unroll
    for (int x = 32; x >= 1; x >>= 1) {
        DD b{shfl_xor_d(a.s, lane, x), shfl_xor_d(a.c, lane, x)};
        // combine in a lane-order-independent way: lower lane's value first
        a = ((lane & x) == 0) ? dd_add(a, b) : dd_add(b, a);
    }
    return a;
}

}  // namespace svd
