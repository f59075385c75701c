// pblock.cpp -- partitioned-block (p-block) states (Sec. II, p-block
// simulation; Sec. III-E, distributed circuits).
//
// The state of n qubits is a tensor product of blocks; each block is an
// ordinary device state (sv_state) of the qubits that have interacted. A gate
// spanning several blocks merges them (k_kron; when the smaller block's
// qubits all lie above the larger one's, the larger block's buffer grows in
// place and k_kron_top writes the product into it); a measured or reset
// qubit leaves its block (k_split_move projects, rescales and drops its bit in
// place, and the upper half of the buffer goes back to the arena), so
// communication qubits return to blocks of their own as soon as a protocol
// measures them, without a second copy of the block. A block's index bits
// hold its qubits in ascending order, so its amplitudes, CDF and draws do not
// depend on the order of the merges. Small blocks live at the top of the
// arena, leaving the bottom for large blocks to grow. Gates on one block queue
// up and run as one sv_run call (per gate, fused or tiled) when the block is
// next merged, measured or read.
#include "sv_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>

using namespace svh;

namespace {

constexpr int kSmallBlock = 16;   // qubits of the blocks placed at the top of the arena

struct PBlk {
    sv_state st = nullptr;
    std::vector<int> q;          // global qubit of local index bit j
    std::vector<sv_op> pending;  // queued gates on local qubit indices
};

}  // namespace

struct sv_pblock_s {
    sv_ctx ctx = nullptr;
    sv_dtype dt = SV_C128;
    int n = 0, W = 1;
    std::vector<PBlk *> blocks;   // storage order (unordered)
    std::vector<PBlk *> of;       // of[q]: block holding qubit q
    std::vector<int> pos;         // pos[q]: local bit of q in its block
    ShotScratch w;
    char *pin = nullptr, *dev = nullptr;
    int last_fuse = 0;            // fuse_k of the queued gates
    uint64_t cur = 0, peak = 0;   // bytes of the block states held now / at most
};

namespace {

sv_status flush(sv_pblock p, PBlk *b) {
    if (b->pending.empty()) return SV_OK;
    sv_status r = sv_run(b->st, b->pending.data(), (int)b->pending.size(), p->last_fuse);
    b->pending.clear();
    return r;
}

sv_status flush_all(sv_pblock p) {
    for (PBlk *b : p->blocks) {
        sv_status r = flush(p, b);
        if (r) return r;
    }
    return SV_OK;
}

void reindex(sv_pblock p, PBlk *b) {
    for (size_t j = 0; j < b->q.size(); ++j) {
        p->of[b->q[j]] = b;
        p->pos[b->q[j]] = (int)j;
    }
}

void hold(sv_pblock p, sv_state st) {
    p->cur += st->bytes;
    p->peak = std::max(p->peak, p->cur);
}

void remove_block(sv_pblock p, PBlk *b) {
    p->blocks.erase(std::find(p->blocks.begin(), p->blocks.end(), b));
    if (b->st) {
        p->cur -= b->st->bytes;
        state_release(b->st);
    }
    delete b;
}

// B grows in place into A (x) B: A's qubits all lie above B's, A is small
// (its 2^a amplitudes per item), and the free arena extents just below and
// above B's amplitudes hold the other 2^a - 1 copies of B's size between them
// (B's old amplitudes then sit at copy k of the product, which is where
// k_kron_top reads them). Returns 0 when not applicable (nothing changed),
// 1 when done, -1 when the launch failed (the state is then unusable).
int merge_in_place(sv_pblock p, PBlk *A, PBlk *B) {
    const int a = (int)A->q.size(), b = (int)B->q.size();
    if (a > 4 || A->q.front() < B->q.back()) return 0;
    sv_ctx c = p->ctx;
    sv_state st = B->st;
    if (st->bytes % 256 != 0) return 0;   // the arena holds B in whole 256-byte units
    void *ws = c->arena.alloc_high(svk::measure_workspace_bytes(a + b));
    if (!ws) return 0;
    const uint64_t nbytes = state_bytes(a + b, p->dt);
    uint64_t k = 0;
    char *base = (char *)c->arena.grow_around(st->psi, 1ull << a, st->bytes, 1ull << 16, &k);
    if (!base) {
        c->arena.free(ws);
        return 0;
    }
    hipError_t e;
    {
        TraceScope ts(&c->tracer, st->stream, "kron", (double)nbytes + A->st->bytes + st->bytes);
        e = svk::launch_kron_top(A->st->psi, a, base + k * st->bytes, b, base, st->is_c64(), st->stream);
    }
    st->psi = base;   // the grown extent, whatever happened
    if (e != hipSuccess) {
        c->arena.free(ws);
        hip_fail(e, "block merge");
        return -1;
    }
    p->cur += nbytes - st->bytes;
    p->peak = std::max(p->peak, p->cur);
    c->arena.free(st->ws);
    st->ws = ws;
    st->ws_bytes = svk::measure_workspace_bytes(a + b);
    st->n = a + b;
    st->bytes = nbytes;
    st->sweeps_since_renorm = 0;
    B->q.insert(B->q.end(), A->q.begin(), A->q.end());
    return 1;
}

// Tensor product of two blocks (both flushed); A and B are freed (or B grows
// into the product).
sv_status merge(sv_pblock p, PBlk *A, PBlk *B, PBlk **out) {
    sv_status r = flush(p, A);
    if (!r) r = flush(p, B);
    if (r) return r;
    if (A->q.size() > B->q.size()) std::swap(A, B);   // the kernel walks the smaller block's bits
    const int a = (int)A->q.size(), b = (int)B->q.size();
    const int nmax = p->dt == SV_C64 ? SV_MAX_QUBITS_C64 : SV_MAX_QUBITS_C128;
    if (a + b > nmax)
        return fail(SV_E_INVALID, "entangled block of " + std::to_string(a + b) + " qubits exceeds " +
                                      std::to_string(nmax));
    const int ip = merge_in_place(p, A, B);
    if (ip < 0) return SV_E_DEVICE;
    if (ip > 0) {
        remove_block(p, A);
        reindex(p, B);
        *out = B;
        return SV_OK;
    }
    // small blocks come from the top of the arena, so that the bottom keeps
    // room for large blocks to grow into
    sv_state st = nullptr;
    r = state_alloc(p->ctx, a + b, p->dt, p->ctx->stream, &st, a + b <= kSmallBlock);
    if (r) return r;
    // block qubits stay in ascending order: A's qubits take their places among B's
    std::vector<int> mq(A->q);
    mq.insert(mq.end(), B->q.begin(), B->q.end());
    std::sort(mq.begin(), mq.end());
    svk::KronPos pos;
    pos.a = a;
    for (int k = 0; k < a; ++k) pos.p[k] = (int)(std::lower_bound(mq.begin(), mq.end(), A->q[k]) - mq.begin());
    {
        TraceScope ts(&p->ctx->tracer, st->stream, "kron", (double)st->bytes + A->st->bytes + B->st->bytes);
        hipError_t e = svk::launch_kron(A->st->psi, pos, B->st->psi, b, st->psi, st->is_c64(), st->stream);
        if (e != hipSuccess) {
            hipStreamSynchronize(st->stream);
            state_release(st);
            return hip_fail(e, "block merge");
        }
    }
    hold(p, st);
    PBlk *M = new PBlk();
    M->st = st;
    M->q = mq;
    // the sources' memory goes back to the arena; later users run on the same
    // stream, after the merge
    remove_block(p, A);
    remove_block(p, B);
    p->blocks.push_back(M);
    reindex(p, M);
    *out = M;
    return SV_OK;
}

// Measure (or reset) qubit q with draw u; returns the outcome.
sv_status measure(sv_pblock p, int q, bool reset, double u, int *m_out) {
    PBlk *B = p->of[q];
    sv_status r = flush(p, B);
    if (r) return r;
    const int j = p->pos[q];
    double p0, p1;
    r = qubit_probs(B->st, j, p->w, &p0, &p1);
    if (r) return r;
    const double tot = p0 + p1;
    if (!(tot > 0.0)) return fail(SV_E_NUMERIC, "block has zero norm at a measurement");
    const int m = u * tot >= p0 ? 1 : 0;
    const double pm = m ? p1 : p0;
    *m_out = m;
    if (B->q.size() == 1) return collapse(B->st, 0, m, pm, reset);
    // the projected state is |m>_q (x) rest: the rest keeps the amplitudes
    // with bit j = m, scaled by 1/sqrt(pm), compacted in place into the lower
    // half of the block, whose upper half goes back to the arena; q gets a
    // block of its own
    const int nb = (int)B->q.size();
    sv_state one = nullptr;
    r = state_create(p->ctx, 1, p->dt, p->ctx->stream, &one, true);
    if (r) return r;
    sv_state st = B->st;
    hipError_t e;
    {
        TraceScope ts(&p->ctx->tracer, st->stream, "split", (double)st->bytes);
        e = svk::launch_split_inplace(st->psi, nb, j, m, 1.0 / std::sqrt(pm), st->is_c64(), st->stream);
    }
    if (e == hipSuccess && !reset && m) e = svk::launch_init(one->psi, 1, one->is_c64(), 1, one->stream);
    if (e != hipSuccess) {
        hipStreamSynchronize(st->stream);
        state_release(one);
        return hip_fail(e, "block split");
    }
    const uint64_t half = state_bytes(nb - 1, p->dt);
    p->ctx->arena.shrink(st->psi, half);   // later users of the tail run on the same stream
    p->cur -= st->bytes - half;
    st->n = nb - 1;
    st->bytes = half;
    B->q.erase(B->q.begin() + j);
    hold(p, one);
    PBlk *Q = new PBlk();
    Q->st = one;
    Q->q = {q};
    p->blocks.push_back(Q);
    reindex(p, B);
    reindex(p, Q);
    return SV_OK;
}

// blocks in partition order (by smallest qubit)
std::vector<PBlk *> ordered(sv_pblock p) {
    std::vector<std::pair<int, PBlk *>> v;
    for (PBlk *b : p->blocks) v.push_back({*std::min_element(b->q.begin(), b->q.end()), b});
    std::sort(v.begin(), v.end(), [](const std::pair<int, PBlk *> &x, const std::pair<int, PBlk *> &y) {
        return x.first < y.first;
    });
    std::vector<PBlk *> out;
    for (auto &x : v) out.push_back(x.second);
    return out;
}

svk::BlockMap block_map(sv_pblock p, const PBlk *b) {
    svk::BlockMap m;
    m.nq = (int)b->q.size();
    m.W = p->W;
    for (int j = 0; j < m.nq; ++j) m.gq[j] = b->q[j];
    return m;
}

bool word_bit(const uint64_t *w, int q) { return (w[q >> 6] >> (q & 63)) & 1ull; }

// bits of a W-word mask beyond n qubits
bool beyond_n(const uint64_t *w, int n, int W) {
    for (int k = 0; k < W; ++k) {
        const int lo = 64 * k;
        const uint64_t valid = n - lo >= 64 ? ~0ull : ((1ull << (n - lo)) - 1ull);
        if (w[k] & ~valid) return true;
    }
    return false;
}

}  // namespace

extern "C" {

sv_status sv_pblock_create(sv_ctx c, int n, sv_dtype dt, sv_pblock *out) {
    if (!c || !out) return fail(SV_E_INVALID, "null argument");
    if (dt != SV_C64 && dt != SV_C128) return fail(SV_E_INVALID, "dtype must be SV_C64 or SV_C128");
    if (n < 1 || n > SV_PBLOCK_MAX_QUBITS) return fail(SV_E_INVALID, "n out of range [1, 1024]");
    sv_pblock p = new sv_pblock_s();
    p->ctx = c;
    p->dt = dt;
    p->n = n;
    p->W = (n + 63) / 64;
    p->of.assign(n, nullptr);
    p->pos.assign(n, 0);
    sv_status r = SV_OK;
    if (hipHostMalloc((void **)&p->pin, 64, hipHostMallocDefault) != hipSuccess) {
        p->pin = nullptr;
        r = fail(SV_E_OOM, "pinned scratch");
    }
    if (!r && !(p->dev = (char *)c->arena.alloc(64))) r = fail(SV_E_OOM, "arena cannot hold the scratch");
    if (!r) {
        p->w.hmask = (uint64_t *)p->pin;
        p->w.hres = (double *)(p->pin + 16);
        p->w.dmask = (uint64_t *)p->dev;
        p->w.dres = (double *)(p->dev + 16);
    }
    for (int q = 0; q < n && !r; ++q) {
        PBlk *b = new PBlk();
        r = state_create(c, 1, dt, c->stream, &b->st, true);
        if (r) {
            delete b;
            break;
        }
        b->q = {q};
        p->blocks.push_back(b);
        reindex(p, b);
        hold(p, b->st);
    }
    if (r) {
        sv_pblock_destroy(p);
        return r;
    }
    *out = p;
    return SV_OK;
}

sv_status sv_pblock_destroy(sv_pblock p) {
    if (!p) return fail(SV_E_INVALID, "null p-block state");
    hipStreamSynchronize(p->ctx->stream);
    for (PBlk *b : p->blocks) {
        if (b->st) state_release(b->st);
        delete b;
    }
    if (p->dev) p->ctx->arena.free(p->dev);
    if (p->pin) hipHostFree(p->pin);
    delete p;
    return SV_OK;
}

sv_status sv_pblock_run(sv_pblock p, const sv_op *ops, int nops, int fuse_k, uint64_t seed, uint64_t *clbits) {
    if (!p || (!ops && nops) || nops < 0 || !clbits) return fail(SV_E_INVALID, "bad argument");
    if (fuse_k != 0 && fuse_k != SV_FUSE_TILED && fuse_k != SV_FUSE_AUTO && (fuse_k < 2 || fuse_k > SV_MAX_FUSED))
        return fail(SV_E_INVALID, "fuse_k must be 0, 2..5, SV_FUSE_TILED or SV_FUSE_AUTO");
    for (int i = 0; i < nops; ++i) {
        const sv_op &o = ops[i];
        const std::string at = "op " + std::to_string(i) + ": ";
        if (o.kind == SV_OP_MEASURE || o.kind == SV_OP_RESET) {
            if (o.q[0] < 0 || o.q[0] >= p->n) return fail(SV_E_INVALID, at + "qubit out of range");
            if (o.kind == SV_OP_MEASURE && (o.q[1] < 0 || o.q[1] > 63))
                return fail(SV_E_INVALID, at + "classical bit out of range 0..63");
            if (o.cond != 0) return fail(SV_E_INVALID, at + "measurements cannot be conditional");
            continue;
        }
        const int nq = gate_nqubits(o.kind);
        if (nq < 0) return fail(SV_E_INVALID, at + "unknown gate kind");
        if (!cond_valid(o.cond)) return fail(SV_E_INVALID, at + "bad cond");
        for (int j = 0; j < nq; ++j) {
            if (o.q[j] < 0 || o.q[j] >= p->n) return fail(SV_E_INVALID, at + "qubit out of range");
            for (int k = 0; k < j; ++k)
                if (o.q[k] == o.q[j]) return fail(SV_E_INVALID, at + "duplicate qubit");
        }
        for (int j = 0; j < 3; ++j)
            if (!std::isfinite(o.p[j])) return fail(SV_E_NUMERIC, at + "non-finite angle");
    }
    sv_status r = SV_OK;
    if (fuse_k != p->last_fuse) r = flush_all(p);
    p->last_fuse = fuse_k;
    uint64_t k = 0;
    for (int i = 0; i < nops && !r; ++i) {
        const sv_op &o = ops[i];
        if (o.kind == SV_OP_MEASURE || o.kind == SV_OP_RESET) {
            int m = 0;
            r = measure(p, o.q[0], o.kind == SV_OP_RESET, host_u01(seed, k++), &m);
            if (!r && o.kind == SV_OP_MEASURE) {
                const uint64_t bit = 1ull << o.q[1];
                *clbits = m ? (*clbits | bit) : (*clbits & ~bit);
            }
            continue;
        }
        if (!cond_met(o.cond, *clbits)) continue;
        const int nq = gate_nqubits(o.kind);
        std::vector<PBlk *> bs;
        for (int j = 0; j < nq; ++j)
            if (std::find(bs.begin(), bs.end(), p->of[o.q[j]]) == bs.end()) bs.push_back(p->of[o.q[j]]);
        // merge the smallest first: every merge streams its larger input once
        std::sort(bs.begin(), bs.end(), [](const PBlk *x, const PBlk *y) { return x->q.size() < y->q.size(); });
        PBlk *B = bs[0];
        for (size_t t = 1; t < bs.size() && !r; ++t) r = merge(p, B, bs[t], &B);
        if (r) break;
        sv_op l = o;
        l.cond = 0;
        for (int j = 0; j < nq; ++j) l.q[j] = p->pos[o.q[j]];
        B->pending.push_back(l);
    }
    if (!r) r = flush_all(p);
    if (r)   // gates queued before the failing op are dropped, not run by a later call
        for (PBlk *b : p->blocks) b->pending.clear();
    hipError_t e = hipStreamSynchronize(p->ctx->stream);
    if (!r && e != hipSuccess) r = hip_fail(e, "p-block run");
    return r;
}

sv_status sv_pblock_info(sv_pblock p, int *nblocks, int *largest, uint64_t *state_bytes, uint64_t *peak_bytes) {
    if (!p) return fail(SV_E_INVALID, "null p-block state");
    int big = 0;
    uint64_t bytes = 0;
    for (PBlk *b : p->blocks) {
        big = std::max(big, (int)b->q.size());
        bytes += b->st->bytes;
    }
    if (nblocks) *nblocks = (int)p->blocks.size();
    if (largest) *largest = big;
    if (state_bytes) *state_bytes = bytes;
    if (peak_bytes) *peak_bytes = p->peak;
    return SV_OK;
}

sv_status sv_pblock_partition(sv_pblock p, int *block_of) {
    if (!p || !block_of) return fail(SV_E_INVALID, "null argument");
    const auto bs = ordered(p);
    for (size_t i = 0; i < bs.size(); ++i)
        for (int q : bs[i]->q) block_of[q] = (int)i;
    return SV_OK;
}

sv_status sv_pblock_block(sv_pblock p, int b, int *qubits_out, int *nq_out, sv_state *state_out) {
    if (!p) return fail(SV_E_INVALID, "null p-block state");
    if (b < 0 || b >= (int)p->blocks.size()) return fail(SV_E_INVALID, "block index out of range");
    PBlk *B = ordered(p)[b];
    sv_status r = flush(p, B);
    if (r) return r;
    if (qubits_out) std::copy(B->q.begin(), B->q.end(), qubits_out);
    if (nq_out) *nq_out = (int)B->q.size();
    if (state_out) *state_out = B->st;
    return SV_OK;
}

sv_status sv_pblock_get_amplitudes(sv_pblock p, const uint64_t *idx, int64_t count, double *out) {
    if (!p || count < 0 || (count > 0 && (!idx || !out))) return fail(SV_E_INVALID, "bad argument");
    if (count == 0) return SV_OK;
    for (int64_t i = 0; i < count; ++i)
        if (beyond_n(idx + (uint64_t)i * p->W, p->n, p->W)) return fail(SV_E_INVALID, "index >= 2^n");
    sv_status r = flush_all(p);
    if (r) return r;
    const uint64_t ib = 8ull * count * p->W, ob = 16ull * count;
    char *buf = (char *)p->ctx->arena.alloc(ib + ob);
    if (!buf) return fail(SV_E_OOM, "arena cannot hold the amplitude buffers");
    hipStream_t s = p->ctx->stream;
    hipError_t e = hipMemcpyAsync(buf, idx, ib, hipMemcpyHostToDevice, s);
    const auto bs = ordered(p);
    for (size_t b = 0; b < bs.size() && e == hipSuccess; ++b)
        e = svk::launch_gather_mul(bs[b]->st->psi, bs[b]->st->is_c64(), block_map(p, bs[b]), (const uint64_t *)buf,
                                   count, (double *)(buf + ib), b == 0 ? 1 : 0, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, buf + ib, ob, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) hipStreamSynchronize(s);
    p->ctx->arena.free(buf);
    if (e != hipSuccess) return hip_fail(e, "p-block amplitudes");
    return SV_OK;
}

sv_status sv_pblock_sample(sv_pblock p, int64_t shots, uint64_t seed, uint64_t *out) {
    if (!p || shots < 0) return fail(SV_E_INVALID, "bad argument");
    if (shots == 0) return SV_OK;
    if (!out) return fail(SV_E_INVALID, "null output");
    sv_status r = flush_all(p);
    if (r) return r;
    hipStream_t s = p->ctx->stream;
    const auto bs = ordered(p);
    // every block's CDF, then the shots in chunks: each block draws and places its bits
    std::vector<double> tot(bs.size(), 0.0);
    for (size_t b = 0; b < bs.size(); ++b) {
        sv_state st = bs[b]->st;
        TraceScope ts(&p->ctx->tracer, s, "cdf", (double)st->bytes);
        SV_HIP(svk::launch_cdf(st->psi, st->n, st->is_c64(), st->ws, s));
        SV_HIP(hipMemcpyAsync(&tot[b], svk::norm2_dev_ptr(st->ws, st->n), 8, hipMemcpyDeviceToHost, s));
    }
    int64_t chunk = std::min<int64_t>(shots, 1 << 20);
    char *buf = nullptr;
    while (!(buf = (char *)p->ctx->arena.alloc(8ull * chunk * (1 + p->W)))) {
        if (chunk <= 1024) return fail(SV_E_OOM, "arena cannot hold the shot buffers");
        chunk /= 2;
    }
    uint64_t *loc = (uint64_t *)buf, *glob = loc + chunk;
    hipError_t e = hipSuccess;
    for (int64_t s0 = 0; s0 < shots && e == hipSuccess; s0 += chunk) {
        const int64_t cnt = std::min(chunk, shots - s0);
        for (size_t b = 0; b < bs.size() && e == hipSuccess; ++b) {
            sv_state st = bs[b]->st;
            e = svk::launch_sample(st->psi, st->n, st->is_c64(), st->ws, cnt, seed, (uint64_t)b * shots + s0, loc, s);
            if (e == hipSuccess) e = svk::launch_place_bits(loc, cnt, block_map(p, bs[b]), glob, b == 0 ? 1 : 0, s);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(out + (uint64_t)s0 * p->W, glob, 8ull * cnt * p->W, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) hipStreamSynchronize(s);
    p->ctx->arena.free(buf);
    if (e != hipSuccess) return hip_fail(e, "p-block sampling");
    for (double t : tot)
        if (!(t > 0.0)) return fail(SV_E_NUMERIC, "a block has zero norm");
    return SV_OK;
}

sv_status sv_pblock_expect(sv_pblock p, const uint64_t *xmask, const uint64_t *zmask, const double *coeff,
                           int nterms, double *out_each, double *out_weighted) {
    if (!p || nterms < 0 || (nterms > 0 && (!xmask || !zmask))) return fail(SV_E_INVALID, "bad argument");
    const int W = p->W;
    for (int t = 0; t < nterms; ++t)
        if (beyond_n(xmask + (uint64_t)t * W, p->n, W) || beyond_n(zmask + (uint64_t)t * W, p->n, W))
            return fail(SV_E_INVALID, "Pauli mask beyond n qubits");
    sv_status r = flush_all(p);
    if (r) return r;
    std::vector<double> val(nterms, 1.0);
    std::vector<sv_pauli> lt;
    std::vector<int> owner;
    std::vector<double> got;
    for (PBlk *b : p->blocks) {
        lt.clear();
        owner.clear();
        for (int t = 0; t < nterms; ++t) {
            uint64_t xl = 0, zl = 0;
            for (size_t j = 0; j < b->q.size(); ++j) {
                xl |= (uint64_t)word_bit(xmask + (uint64_t)t * W, b->q[j]) << j;
                zl |= (uint64_t)word_bit(zmask + (uint64_t)t * W, b->q[j]) << j;
            }
            if (xl | zl) {
                lt.push_back(sv_pauli{xl, zl, 1.0});
                owner.push_back(t);
            }
        }
        if (lt.empty()) continue;
        got.assign(lt.size(), 0.0);
        r = sv_expect(b->st, lt.data(), (int)lt.size(), got.data(), nullptr);
        if (r) return r;
        for (size_t i = 0; i < lt.size(); ++i) val[owner[i]] *= got[i];
    }
    double wsum = 0.0;
    for (int t = 0; t < nterms; ++t) {
        if (out_each) out_each[t] = val[t];
        wsum += (coeff ? coeff[t] : 1.0) * val[t];
    }
    if (out_weighted) *out_weighted = wsum;
    return SV_OK;
}

}  // extern "C"
