// k_fused.hip -- dense k-qubit blocks (k <= 5) for gfx950.
//
// A fused block multiplies every "column" (the 2^k amplitudes that differ only
// in the k target bits) by one 2^k x 2^k complex matrix: a complex GEMM of
// U (2^k x 2^k) with the state viewed as 2^k x (2^n / 2^k) columns.
//
// k_fused_mfma: the complex product is done as a real GEMM on the matrix cores
// with the real embedding
//     [Re y]   [Ur  -Ui] [Re x]
//     [Im y] = [Ui   Ur] [Im x]
// of size D = 2^(k+1). One wavefront owns a tile of 16 columns; its lanes load
// amplitudes straight into the B-operand layout of V_MFMA_*_16X16X4 (lane l
// holds B[l/16][l%16]) and store straight from the D layout (lane l holds four
// rows of column l%16, see drow). The embedded matrix sits in LDS; each
// instruction reads one A element per lane (A[l%16][l/16]). Double precision
// uses V_MFMA_F64_16X16X4_F64, single precision V_MFMA_F32_16X16X4_F32.
//
// k_dense_generic: one thread per column (gather, 2^k x 2^k product, scatter);
// used for states too small for 16-column tiles.
#include "sv_device.h"
#include "sv_kernels.h"

#include <algorithm>
#include <cstring>
#include <type_traits>

using namespace svd;

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct CT;
template <>
struct CT<double> {
    typedef d4 acc;
    typedef double2 amp;
};
template <>
struct CT<float> {
    typedef f4 acc;
    typedef float2 amp;
};

__device__ inline d4 mfma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// Output row held in accumulator register v by lane group g = lane / 16.
// V_MFMA_F64_16X16X4_F64 interleaves the groups (row g + 4v); the FP32
// instruction gives each group four consecutive rows (row 4g + v).
__device__ constexpr int drow(double *, int g, int v) { return g + 4 * v; }
__device__ constexpr int drow(float *, int g, int v) { return 4 * g + v; }

template <typename T>
struct FArgs {
    uint64_t n_tiles;      // 16-column tiles
    int nhb;               // positions excluded from the tile enumeration (targets + column bits), ascending
    int hb[12];
    int k;
    int targets[5];
    int colbits[4];        // the 4 lowest non-target positions: column index bits
    T ar[64 * 64];         // real embedding, row-major D x D (only D*D used)
};

// Bit deposit of the low bits of v into the positions pos[0..cnt).
__device__ inline uint64_t dep_bits(uint32_t v, const int *pos, int cnt) {
    uint64_t o = 0;
    for (int j = 0; j < cnt; ++j) o |= (uint64_t)((v >> j) & 1u) << pos[j];
    return o;
}

template <typename T, int KK>
__global__ __launch_bounds__(256) void k_fused_mfma(const FArgs<T> *__restrict__ args, typename CT<T>::amp *__restrict__ psi) {
    constexpr int R = 1 << KK;        // complex rows
    constexpr int D = 2 * R;          // real rows
    constexpr int RT = D / 16;        // row tiles
    constexpr int KS = D / 4;         // k-steps
    constexpr int KSR = KS / 2;       // k-steps over the real half (amplitude loads per lane)
    typedef typename CT<T>::acc ACC;
    typedef typename CT<T>::amp AMP;
    __shared__ T sA[D * D];
    const FArgs<T> &a = *args;
    for (int i = threadIdx.x; i < D * D; i += blockDim.x) sA[i] = a.ar[i];
    __shared__ int s_hb[12], s_t[5], s_c[4];
    if (threadIdx.x < 12) s_hb[threadIdx.x] = a.hb[threadIdx.x];
    if (threadIdx.x < 5) s_t[threadIdx.x] = a.targets[threadIdx.x];
    if (threadIdx.x < 4) s_c[threadIdx.x] = a.colbits[threadIdx.x];
    __syncthreads();
    const int nhb = a.nhb;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;
    const uint64_t coff = dep_bits(col, s_c, 4);
    // input rows of this lane: m = 4*ks + g, ks < KSR
    uint64_t roff_in[KSR];
#pragma unroll
    for (int ks = 0; ks < KSR; ++ks) roff_in[ks] = dep_bits(4 * ks + g, s_t, KK);
    // output rows of this lane: real row 16*rt + drow(g, v); complex row = that mod R
    uint64_t roff_out[RT / 2][4];
#pragma unroll
    for (int rt = 0; rt < RT / 2; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) roff_out[rt][v] = dep_bits(16 * rt + drow((T *)nullptr, g, v), s_t, KK);

    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t tile = wave_id_global(); tile < a.n_tiles; tile += nw) {
        const uint64_t base = deposit(tile, s_hb, nhb, 0) | coff;
        AMP x[KSR];
#pragma unroll
        for (int ks = 0; ks < KSR; ++ks) x[ks] = psi[base | roff_in[ks]];
        ACC acc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = ACC{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const T b = ks < KSR ? x[ks].x : x[ks - KSR].y;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const T av = sA[(16 * rt + col) * D + 4 * ks + g];
                acc[rt] = mfma(av, b, acc[rt]);
            }
        }
#pragma unroll
        for (int rt = 0; rt < RT / 2; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                AMP y;
                y.x = acc[rt][v];
                y.y = acc[rt + RT / 2][v];
                psi[base | roff_out[rt][v]] = y;
            }
    }
}

template <typename T>
struct GDArgs {
    uint64_t ncols;
    int k;
    int nhb;
    int hb[5];         // targets ascending
    int targets[5];
    T u[2 * 32 * 32];
};

template <typename T>
__global__ __launch_bounds__(256) void k_dense_generic(const GDArgs<T> *__restrict__ args,
                                                        typename CT<T>::amp *__restrict__ psi) {
    typedef typename CT<T>::amp AMP;
    const GDArgs<T> &a = *args;
    const int K = 1 << a.k;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.ncols; c += stride) {
        const uint64_t base = deposit(c, a.hb, a.nhb, 0);
        AMP v[32];
        for (int m = 0; m < K; ++m) v[m] = psi[base | dep_bits(m, a.targets, a.k)];
        for (int r = 0; r < K; ++r) {
            Cx<T> acc{0, 0};
            for (int m = 0; m < K; ++m)
                acc = cfma(acc, Cx<T>{a.u[2 * (r * K + m)], a.u[2 * (r * K + m) + 1]}, Cx<T>{v[m].x, v[m].y});
            AMP o;
            o.x = acc.re;
            o.y = acc.im;
            psi[base | dep_bits(r, a.targets, a.k)] = o;
        }
    }
}

}  // namespace

namespace svk {

// Kernel argument blocks for the fused kernels are too large for the kernarg
// segment (up to 32 KiB), so they are staged in a small device buffer owned by
// the caller's workspace (see fused_args_bytes).
uint64_t fused_args_bytes() { return std::max(sizeof(FArgs<double>), sizeof(GDArgs<double>)); }

hipError_t launch_fused_staged(const double *U, int k, const int *targets, void *psi, int n, int is_c64,
                               hipStream_t s, int use_mfma, void *args_dev, void *args_host) {
    // column-major choice: MFMA tiles need n >= k + 4
    int kk = k;
    int tg[5];
    for (int j = 0; j < k; ++j) tg[j] = targets[j];
    double Ue[2 * 32 * 32];
    const int K0 = 1 << k;
    for (int i = 0; i < 2 * K0 * K0; ++i) Ue[i] = U[i];
    const bool mfma_ok = use_mfma && n >= 4 + std::max(k, 4);
    if (mfma_ok && k < 4) {
        // pad to 4 targets with the lowest free qubits: U' = I (x) U
        uint64_t used = 0;
        for (int j = 0; j < k; ++j) used |= 1ull << tg[j];
        int p = 0;
        while (kk < 4) {
            while ((used >> p) & 1) ++p;
            tg[kk++] = p;
            used |= 1ull << p;
        }
        const int K1 = 1 << kk;
        for (int r = 0; r < K1; ++r)
            for (int c = 0; c < K1; ++c) {
                const bool same_hi = (r >> k) == (c >> k);
                const int rl = r & (K0 - 1), cl = c & (K0 - 1);
                Ue[2 * (r * K1 + c)] = same_hi ? U[2 * (rl * K0 + cl)] : 0.0;
                Ue[2 * (r * K1 + c) + 1] = same_hi ? U[2 * (rl * K0 + cl) + 1] : 0.0;
            }
    }
    const int K = 1 << kk;
    if (mfma_ok) {
        const int D = 2 * K;
        uint64_t tmask = 0;
        for (int j = 0; j < kk; ++j) tmask |= 1ull << tg[j];
        int colbits[4], nc = 0;
        for (int p = 0; p < n && nc < 4; ++p)
            if (!((tmask >> p) & 1)) colbits[nc++] = p;
        uint64_t excl = tmask;
        for (int j = 0; j < 4; ++j) excl |= 1ull << colbits[j];
        auto fill = [&](auto *fa) {
            using TT = std::remove_reference_t<decltype(fa->ar[0])>;
            memset(fa, 0, sizeof(*fa));
            fa->n_tiles = 1ull << (n - kk - 4);
            fa->nhb = 0;
            for (int p = 0; p < 64; ++p)
                if ((excl >> p) & 1) fa->hb[fa->nhb++] = p;
            fa->k = kk;
            for (int j = 0; j < kk; ++j) fa->targets[j] = tg[j];
            for (int j = 0; j < 4; ++j) fa->colbits[j] = colbits[j];
            for (int r = 0; r < K; ++r)
                for (int c = 0; c < K; ++c) {
                    const double ur = Ue[2 * (r * K + c)], ui = Ue[2 * (r * K + c) + 1];
                    fa->ar[r * D + c] = (TT)ur;
                    fa->ar[r * D + K + c] = (TT)(-ui);
                    fa->ar[(K + r) * D + c] = (TT)ui;
                    fa->ar[(K + r) * D + K + c] = (TT)ur;
                }
            return fa->n_tiles;
        };
        uint64_t tiles;
        size_t bytes;
        if (is_c64) {
            tiles = fill((FArgs<float> *)args_host);
            bytes = sizeof(FArgs<float>);
        } else {
            tiles = fill((FArgs<double> *)args_host);
            bytes = sizeof(FArgs<double>);
        }
        hipError_t e = hipMemcpyAsync(args_dev, args_host, bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        const uint64_t waves = tiles;
        const uint64_t blocks = std::min<uint64_t>((waves + 3) / 4, 256ull * 8);
        if (is_c64) {
            if (kk == 4)
                hipLaunchKernelGGL((k_fused_mfma<float, 4>), dim3((unsigned)blocks), dim3(256), 0, s,
                                   (const FArgs<float> *)args_dev, (float2 *)psi);
            else
                hipLaunchKernelGGL((k_fused_mfma<float, 5>), dim3((unsigned)blocks), dim3(256), 0, s,
                                   (const FArgs<float> *)args_dev, (float2 *)psi);
        } else {
            if (kk == 4)
                hipLaunchKernelGGL((k_fused_mfma<double, 4>), dim3((unsigned)blocks), dim3(256), 0, s,
                                   (const FArgs<double> *)args_dev, (double2 *)psi);
            else
                hipLaunchKernelGGL((k_fused_mfma<double, 5>), dim3((unsigned)blocks), dim3(256), 0, s,
                                   (const FArgs<double> *)args_dev, (double2 *)psi);
        }
        return hipGetLastError();
    }
    // generic path
    auto fillg = [&](auto *ga) {
        using TT = std::remove_reference_t<decltype(ga->u[0])>;
        memset(ga, 0, sizeof(*ga));
        ga->ncols = 1ull << (n - kk);
        ga->k = kk;
        int srt[5];
        for (int j = 0; j < kk; ++j) srt[j] = tg[j];
        std::sort(srt, srt + kk);
        ga->nhb = kk;
        for (int j = 0; j < kk; ++j) {
            ga->hb[j] = srt[j];
            ga->targets[j] = tg[j];
        }
        for (int i = 0; i < 2 * K * K; ++i) ga->u[i] = (TT)Ue[i];
        return ga->ncols;
    };
    uint64_t cols;
    size_t bytes;
    if (is_c64) {
        cols = fillg((GDArgs<float> *)args_host);
        bytes = sizeof(GDArgs<float>);
    } else {
        cols = fillg((GDArgs<double> *)args_host);
        bytes = sizeof(GDArgs<double>);
    }
    hipError_t e = hipMemcpyAsync(args_dev, args_host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    const uint64_t blocks = std::min<uint64_t>((cols + 255) / 256, 256ull * 16);
    if (is_c64)
        hipLaunchKernelGGL(k_dense_generic<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const GDArgs<float> *)args_dev, (float2 *)psi);
    else
        hipLaunchKernelGGL(k_dense_generic<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const GDArgs<double> *)args_dev, (double2 *)psi);
    return hipGetLastError();
}

}  // namespace svk
