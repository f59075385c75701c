// k_pblock.hip -- kernels of partitioned-block (p-block) states for gfx950.
//
// A p-block state keeps one state vector per group of qubits that have
// interacted (Sec. II, p-block simulation): a gate across groups merges their
// states into their tensor product, and a measured qubit leaves its group.
//   k_kron:       out[i] = A[A's bits of i] * B[B's bits of i] (merge of two groups)
//   k_kron_top:   the same with A's qubits above B's, writing into B's grown buffer
//   k_split_move: psi[i'] = c * psi[i' with bit j set to m], in place (a measured
//                 qubit leaves; the upper half of the buffer is given back)
#include "sv_device.h"
#include "sv_kernels.h"

using namespace svd;
using svk::BlockMap;
using svk::KronPos;

namespace {

constexpr int kB = 256;

template <typename T>
__device__ inline Cx<T> mul(Cx<T> x, Cx<T> y) {
    return Cx<T>{x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re};
}

// Output bit pos.p[k] (ascending k) is bit k of A's index (A: the smaller
// block); the other bits, in order, form B's index. Each work item reads one
// amplitude of B once and writes the 2^cl outputs that pair it with 2^cl
// consecutive amplitudes of A (A stays in cache), so B streams through
// exactly once however A's bits interleave with B's.
constexpr int kMaxCl = 4;   // at most 16 outputs per item

template <typename T>
__global__ __launch_bounds__(kB) void k_kron(const Cx<T> *__restrict__ A, KronPos pos, const Cx<T> *__restrict__ B,
                                             int b, int cl, uint64_t nitems, Cx<T> *__restrict__ out) {
    const uint64_t stride = grid_blocks() * kB;
    const uint64_t bmask = (1ull << b) - 1ull;
    for (uint64_t t = block_linear() * kB + threadIdx.x; t < nitems; t += stride) {
        const uint64_t ib = t & bmask, c = t >> b;
        const Cx<T> v = B[ib];
        // B's index bits spread over the positions A does not take
        uint64_t base = ib;
        for (int k = 0; k < pos.a; ++k) {
            const int p = pos.p[k];
            base = ((base >> p) << (p + 1)) | (base & ((1ull << p) - 1ull));
        }
        for (int kk = 0; kk < (1 << cl); ++kk) {
            const uint64_t ka = (c << cl) | (uint64_t)kk;
            uint64_t off = 0;
            for (int k = 0; k < pos.a; ++k) off |= ((ka >> k) & 1ull) << pos.p[k];
            out[base | off] = mul(A[ka], v);
        }
    }
}

// Merge with all of A's qubits above B's: out[ib + (ka << b)] = A[ka] B[ib].
// One item per amplitude of B writes all 2^a outputs after reading it, and B
// may be copy k of out itself (B's buffer grown around it): then the only
// output inside B's range that item ib writes is out[ib + (k << b)], the value
// it has just read.
template <typename T>
__global__ __launch_bounds__(kB) void k_kron_top(const Cx<T> *__restrict__ A, int a, const Cx<T> *B, int b,
                                                 Cx<T> *out) {
    const uint64_t stride = grid_blocks() * kB;
    const uint64_t nb = 1ull << b;
    for (uint64_t ib = block_linear() * kB + threadIdx.x; ib < nb; ib += stride) {
        const Cx<T> v = B[ib];
        for (int ka = 0; ka < (1 << a); ++ka) out[ib + ((uint64_t)ka << b)] = mul(A[ka], v);
    }
}

// In-place split, one batch: out block k (2^j amplitudes) <- c * in block
// 2k + m, for the blocks [k0, k1) of the batch. Batches run in the order
// {0}, {1}, [2, 4), [4, 8), ...: a batch reads only blocks at or above 2 k0 + m
// and writes below 2 k0, so no block is overwritten before it has been read.
template <typename T>
__global__ __launch_bounds__(kB) void k_split_move(Cx<T> *psi, int j, int m, double c, uint64_t k0, uint64_t k1) {
    const uint64_t stride = grid_blocks() * kB;
    const uint64_t lo = (1ull << j) - 1ull;
    const uint64_t i0 = k0 << j, i1 = k1 << j;
    for (uint64_t i = i0 + block_linear() * kB + threadIdx.x; i < i1; i += stride) {
        const uint64_t src = ((((i >> j) << 1) | (uint64_t)m) << j) | (i & lo);
        const Cx<T> v = psi[src];
        psi[i] = Cx<T>{(T)(v.re * c), (T)(v.im * c)};
    }
}

// Amplitude of a global index in one block: the block's bits of the index
// (local bit j = global qubit m.gq[j]) select the block amplitude, which
// multiplies the running product in FP64 (or starts it).
template <typename T>
__global__ __launch_bounds__(kB) void k_gather_mul(const Cx<T> *__restrict__ psi, BlockMap m,
                                                   const uint64_t *__restrict__ gidx, int64_t count,
                                                   double *__restrict__ acc, int first) {
    const int64_t i = (int64_t)block_linear() * kB + threadIdx.x;
    if (i >= count) return;
    const uint64_t *g = gidx + (uint64_t)i * m.W;
    uint64_t loc = 0;
    for (int j = 0; j < m.nq; ++j) loc |= ((g[m.gq[j] >> 6] >> (m.gq[j] & 63)) & 1ull) << j;
    const Cx<T> v = psi[loc];
    const double vr = (double)v.re, vi = (double)v.im;
    if (first) {
        acc[2 * i] = vr;
        acc[2 * i + 1] = vi;
    } else {
        const double ar = acc[2 * i], ai = acc[2 * i + 1];
        acc[2 * i] = ar * vr - ai * vi;
        acc[2 * i + 1] = ar * vi + ai * vr;
    }
}

// Scatter one block's sampled bits (bit j of local[s]) to their global
// positions in shot s's W words; `first` clears the words beforehand.
__global__ __launch_bounds__(kB) void k_place_bits(const uint64_t *__restrict__ local, int64_t cnt, BlockMap m,
                                                   uint64_t *__restrict__ out, int first) {
    const int64_t s = (int64_t)block_linear() * kB + threadIdx.x;
    if (s >= cnt) return;
    const uint64_t b = local[s];
    uint64_t *o = out + (uint64_t)s * m.W;
    for (int w = 0; w < m.W; ++w) {
        uint64_t v = first ? 0ull : o[w];
        for (int j = 0; j < m.nq; ++j)
            if ((m.gq[j] >> 6) == w) v |= ((b >> j) & 1ull) << (m.gq[j] & 63);
        o[w] = v;
    }
}

uint64_t blocks_for(uint64_t n) { return std::min<uint64_t>((n + kB - 1) / kB, 1ull << 16); }

dim3 grid_for(int64_t count) {
    const uint64_t nb = ((uint64_t)count + kB - 1) / kB;
    return nb <= (1ull << 22) ? dim3((unsigned)nb) : dim3(1u << 22, (unsigned)((nb + (1ull << 22) - 1) >> 22));
}

}  // namespace

namespace svk {

hipError_t launch_kron(const void *A, const KronPos &pos, const void *B, int b, void *out, int is_c64,
                       hipStream_t s) {
    const int cl = std::min(pos.a, kMaxCl);
    const uint64_t nitems = 1ull << (pos.a - cl + b);
    const dim3 g((unsigned)blocks_for(nitems));
    if (is_c64)
        hipLaunchKernelGGL(k_kron<float>, g, dim3(kB), 0, s, (const Cx<float> *)A, pos, (const Cx<float> *)B, b, cl,
                           nitems, (Cx<float> *)out);
    else
        hipLaunchKernelGGL(k_kron<double>, g, dim3(kB), 0, s, (const Cx<double> *)A, pos, (const Cx<double> *)B, b,
                           cl, nitems, (Cx<double> *)out);
    return hipGetLastError();
}

hipError_t launch_kron_top(const void *A, int a, const void *B, int b, void *out, int is_c64, hipStream_t s) {
    const dim3 g((unsigned)blocks_for(1ull << b));
    if (is_c64)
        hipLaunchKernelGGL(k_kron_top<float>, g, dim3(kB), 0, s, (const Cx<float> *)A, a, (const Cx<float> *)B, b,
                           (Cx<float> *)out);
    else
        hipLaunchKernelGGL(k_kron_top<double>, g, dim3(kB), 0, s, (const Cx<double> *)A, a, (const Cx<double> *)B, b,
                           (Cx<double> *)out);
    return hipGetLastError();
}

hipError_t launch_split_inplace(void *psi, int n, int j, int m, double c, int is_c64, hipStream_t s) {
    const uint64_t nblk = 1ull << (n - 1 - j);   // blocks of 2^j amplitudes in the result
    for (uint64_t k0 = 0, k1 = 1; k0 < nblk; k0 = k1, k1 = std::min<uint64_t>(nblk, k1 ? 2 * k1 : 1)) {
        const dim3 g((unsigned)blocks_for((k1 - k0) << j));
        if (is_c64)
            hipLaunchKernelGGL(k_split_move<float>, g, dim3(kB), 0, s, (Cx<float> *)psi, j, m, c, k0, k1);
        else
            hipLaunchKernelGGL(k_split_move<double>, g, dim3(kB), 0, s, (Cx<double> *)psi, j, m, c, k0, k1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (k1 == nblk) break;
    }
    return hipSuccess;
}

hipError_t launch_gather_mul(const void *psi, int is_c64, const BlockMap &m, const uint64_t *gidx_dev, int64_t count,
                             double *acc_dev, int first, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (is_c64)
        hipLaunchKernelGGL(k_gather_mul<float>, grid_for(count), dim3(kB), 0, s, (const Cx<float> *)psi, m, gidx_dev,
                           count, acc_dev, first);
    else
        hipLaunchKernelGGL(k_gather_mul<double>, grid_for(count), dim3(kB), 0, s, (const Cx<double> *)psi, m, gidx_dev,
                           count, acc_dev, first);
    return hipGetLastError();
}

hipError_t launch_place_bits(const uint64_t *local_dev, int64_t cnt, const BlockMap &m, uint64_t *out_dev, int first,
                             hipStream_t s) {
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_place_bits, grid_for(cnt), dim3(kB), 0, s, local_dev, cnt, m, out_dev, first);
    return hipGetLastError();
}

}  // namespace svk
