// k_pblock.hip -- kernels of partitioned-block (p-block) states for gfx950.
//
// A p-block state keeps one state vector per group of qubits that have
// interacted (Sec. II, p-block simulation): a gate across groups merges their
// states into their tensor product, and a measured qubit leaves its group.
//   k_kron:  out[i] = A[A's bits of i] * B[B's bits of i] (merge of two groups)
//   k_split: out[i'] = c * psi[i' with bit j set to m] (a measured qubit leaves)
// Both stream their output once; every thread writes whole 16-byte slices.
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

template <typename T>
__global__ __launch_bounds__(kB) void k_split(const Cx<T> *__restrict__ psi, int j, int m, double c, uint64_t nout,
                                              Cx<T> *__restrict__ out) {
    const uint64_t stride = grid_blocks() * kB;
    const uint64_t lo = (1ull << j) - 1ull;
    for (uint64_t i = block_linear() * kB + threadIdx.x; i < nout; i += stride) {
        const uint64_t src = ((i & ~lo) << 1) | ((uint64_t)m << j) | (i & lo);
        const Cx<T> v = psi[src];
        out[i] = Cx<T>{(T)(v.re * c), (T)(v.im * c)};
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

hipError_t launch_split(const void *psi, int n, int j, int m, double c, void *out, int is_c64, hipStream_t s) {
    const uint64_t nout = 1ull << (n - 1);
    const dim3 g((unsigned)blocks_for(nout));
    if (is_c64)
        hipLaunchKernelGGL(k_split<float>, g, dim3(kB), 0, s, (const Cx<float> *)psi, j, m, c, nout, (Cx<float> *)out);
    else
        hipLaunchKernelGGL(k_split<double>, g, dim3(kB), 0, s, (const Cx<double> *)psi, j, m, c, nout,
                           (Cx<double> *)out);
    return hipGetLastError();
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
