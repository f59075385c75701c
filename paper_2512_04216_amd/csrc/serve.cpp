// serve.cpp -- continuous-batching request server over one GPU.
//
// The paper runs GPU backends from a single host thread (Sec. III-B) and sends
// heterogeneous batches of circuits through one interface (Sec. IV-B). Here one
// driver thread:
//   * admits queued circuits in arrival order while their footprint fits: the
//     2^n-amplitude state plus its measurement workspace and result buffers for
//     a large circuit, a slot in the next packed launch for a small one. A
//     request at the head that does not fit may be overtaken by later ones that
//     do, but at most kMaxBypass times; after that admission waits for it;
//   * launches all admitted small circuits (n <= small_qubits) together in one
//     persistent packed kernel (state in LDS, one workgroup per circuit);
//   * keeps the states of larger circuits resident and enqueues their gates in
//     chunks of kChunk gates per request per iteration, each request on one of
//     the server's streams, so new requests start while older ones still run
//     and their kernels overlap on the device;
//   * after a circuit's last gate enqueues its CDF, shots and expectations and
//     copies the results to pinned host memory; an event marks completion.
// Every request is validated and deep-copied at submission; results are
// returned through sv_poll / sv_wait.
#include "serve_policy.h"
#include "sv_host.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

namespace {

using namespace svh;

constexpr int kChunk = 48;            // gates (or fused blocks) per request per driver iteration
constexpr int kMaxBypass = 32;        // times a blocked head may be overtaken
constexpr int kMaxBatch = 2048;       // circuits per packed launch
constexpr int kMaxBatchGates = 1 << 19;
constexpr int kMaxBatchesInFlight = 2;
constexpr int kTB = 16;               // Z terms per expectation pass (matches the kernels)
constexpr int64_t kMaxShots = 1 << 24; // shots per request (results go through pinned memory)
constexpr int64_t kSmallMaxShots = 1 << 16;

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Req {
    uint64_t id = 0;
    int n = 0;
    sv_dtype dt = SV_C64;
    int fuse_k = 0;
    int64_t shots = 0;
    uint64_t seed = 0;
    std::vector<sv_op> ops;
    std::vector<sv_pauli> terms;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    int status = SV_OK;
    bool small = false;
    int bypassed = 0;
    uint64_t footprint = 0;
    // large path
    sv_state st = nullptr;
    int stream_idx = 0;
    std::vector<Block> blocks;
    // Blocks are prepared once, on the request's first pass: a kind per block
    // (0 one op, 1 matrix on <= 2 qubits, 2 fused kernel), the kind-1
    // matrices, and the kind-2 kernel argument blocks, copied to the device in
    // one transfer.
    bool prepared = false;
    std::vector<uint8_t> bkind;
    std::vector<uint32_t> bref;              // index into smallU (x16) or fl
    std::vector<cd> smallU;
    std::vector<svk::FusedLaunch> fl;
    std::vector<svk::TileArgs> targs;        // tiled passes (fuse_k = SV_FUSE_TILED)
    char *ahost = nullptr, *adev = nullptr;  // argument blocks or pass records (pinned / device)
    uint64_t astride = 0;
    size_t next = 0, total = 0;
    bool measuring = false;
    hipEvent_t ev = nullptr;
    char *dbuf = nullptr, *hbuf = nullptr;
    uint64_t dbytes = 0;
    int nzb = 0;
    std::vector<int> zi, xi;
    // results
    std::vector<uint64_t> samples;
    std::vector<double> expect;
    double weighted = 0, norm = 0;
};

struct Batch {
    std::vector<Req *> reqs;
    sv_dtype dt = SV_C64;
    hipEvent_t ev = nullptr;
    char *dbuf = nullptr, *hin = nullptr, *hout = nullptr;
    uint64_t in_bytes = 0, out_bytes = 0, samples_total = 0, res_total = 0;
    std::vector<uint64_t> sample_off, res_off;
};

// Bytes of the device result area of a large request: shots, then per Z
// batch (kTB + 1) doubles, two per X/Y term, then the Z masks.
uint64_t result_bytes(int64_t shots, int nzb, int nxz) {
    const uint64_t nres = (uint64_t)std::max(1, nzb) * (kTB + 1) + 2ull * nxz + 1;
    const uint64_t nmask = (uint64_t)std::max(1, nzb) * kTB;
    return 8ull * ((uint64_t)shots + nres + nmask);
}

}  // namespace

struct sv_server_s {
    sv_ctx ctx = nullptr;
    sv_server_opts o{};
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> queue;                     // submitted, not admitted
    std::unordered_map<uint64_t, Req *> live;    // every request not yet polled
    std::unordered_map<uint64_t, Req *> done;    // finished, not yet polled
    std::vector<Req *> large;                    // admitted large requests (driver)
    std::vector<Req *> pending_small;            // admitted small requests awaiting a launch (driver)
    std::vector<Batch *> batches;                // packed launches in flight (driver)
    std::vector<hipStream_t> streams;
    hipStream_t small_stream = nullptr;
    Arena pinned;
    char *pinned_base = nullptr;
    uint64_t next_id = 1;
    uint64_t held = 0, cap = 0;
    int active = 0;
    int rr = 0;
    int small_c64 = svk::packed_max_qubits(1), small_c128 = svk::packed_max_qubits(0);
    std::atomic<bool> stop{false};
    std::thread driver;
    sv_server_stats stats{};
};

namespace {

void finish(sv_server s, Req *r, int status) {
    r->status = status;
    r->t_done = now_ns();
    std::lock_guard<std::mutex> g(s->mu);
    s->done[r->id] = r;
    s->active--;
    s->stats.completed++;
    s->cv.notify_all();
}

void release_large(sv_server s, Req *r) {
    if (r->ev) hipEventDestroy(r->ev);
    r->ev = nullptr;
    if (r->st) state_release(r->st);   // its completion event has fired
    r->st = nullptr;
    if (r->dbuf) s->ctx->arena.free(r->dbuf);
    r->dbuf = nullptr;
    if (r->hbuf) s->pinned.free(r->hbuf);
    r->hbuf = nullptr;
    if (r->adev) s->ctx->arena.free(r->adev);
    if (r->ahost) s->pinned.free(r->ahost);
    r->adev = r->ahost = nullptr;
    s->held -= r->footprint;
}

// Allocate everything a large request needs; false if it does not fit now.
bool try_admit_large(sv_server s, Req *r) {
    if (s->held + r->footprint > s->cap) return false;
    r->zi.clear();
    r->xi.clear();
    for (int t = 0; t < (int)r->terms.size(); ++t) (r->terms[t].xmask ? r->xi : r->zi).push_back(t);
    r->nzb = (int)((r->zi.size() + kTB - 1) / kTB);
    r->dbytes = result_bytes(r->shots, r->nzb, (int)r->xi.size());
    r->hbuf = (char *)s->pinned.alloc(r->dbytes);
    if (!r->hbuf) return false;
    r->dbuf = (char *)s->ctx->arena.alloc(r->dbytes);
    if (!r->dbuf) {
        s->pinned.free(r->hbuf);
        r->hbuf = nullptr;
        return false;
    }
    r->stream_idx = s->rr++ % (int)s->streams.size();
    if (svh::state_create(s->ctx, r->n, r->dt, s->streams[r->stream_idx], &r->st) != SV_OK) {
        s->ctx->arena.free(r->dbuf);
        s->pinned.free(r->hbuf);
        r->dbuf = r->hbuf = nullptr;
        return false;
    }
    hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
    s->held += r->footprint;
    if (r->fuse_k >= 2) {
        r->blocks = plan_fusion(r->ops.data(), (int)r->ops.size(), std::min(r->fuse_k, r->n));
        r->total = r->blocks.size();
    } else {
        r->total = r->ops.size();
    }
    r->next = 0;
    r->measuring = false;
    r->prepared = r->fuse_k == 0;
    return true;
}

// Tiled passes of a request: plan, records staged in one transfer.
bool prepare_passes(sv_server s, Req *r) {
    std::vector<TiledOp> tops;
    tiled_ops(r->ops.data(), (int)r->ops.size(), tops);   // ops were validated at submission
    const int is_c64 = r->st->is_c64() ? 1 : 0;
    const int mbmax = svk::tile_bits(is_c64), lbf = svk::low_bits(is_c64);
    const auto passes = tops.empty() ? std::vector<Pass>() : plan_passes(tops, r->n, mbmax, lbf);
    std::vector<svk::TileGate> recs;
    r->targs.assign(passes.size(), svk::TileArgs{});
    for (size_t p = 0; p < passes.size(); ++p) {
        r->targs[p].gate0 = (int)recs.size();
        pass_records(r->ops.data(), tops, passes[p], r->n, mbmax, lbf, recs, r->targs[p]);
        r->targs[p].ngates = (int)recs.size() - r->targs[p].gate0;
    }
    const uint64_t bytes = recs.size() * sizeof(svk::TileGate);
    if (bytes > 0) {
        r->ahost = (char *)s->pinned.alloc(bytes);
        r->adev = r->ahost ? (char *)s->ctx->arena.alloc(bytes) : nullptr;
        if (!r->ahost || !r->adev) {
            if (r->ahost) s->pinned.free(r->ahost);
            r->ahost = nullptr;
            return false;
        }
        memcpy(r->ahost, recs.data(), bytes);
        if (hipMemcpyAsync(r->adev, r->ahost, bytes, hipMemcpyHostToDevice, r->st->stream) != hipSuccess) {
            s->ctx->arena.free(r->adev);
            s->pinned.free(r->ahost);
            r->adev = r->ahost = nullptr;
            return false;
        }
    }
    r->total = passes.size();
    r->prepared = true;
    return true;
}

// Block kinds, small matrices and fused argument blocks of a fused request
// (driver thread, outside the server lock). false: no memory for the argument
// blocks right now; the request stays admitted and is prepared later.
bool prepare_blocks(sv_server s, Req *r) {
    const int nb = (int)r->blocks.size();
    const int is_c64 = r->st->is_c64() ? 1 : 0;
    int nf = 0;
    for (const Block &b : r->blocks)
        if (b.ops.size() > 1 && b.qubits.size() > 2) ++nf;
    r->astride = (svk::fused_args_bytes_dt(is_c64) + 255) & ~255ull;
    if (nf > 0) {
        r->ahost = (char *)s->pinned.alloc(nf * r->astride);
        r->adev = r->ahost ? (char *)s->ctx->arena.alloc(nf * r->astride) : nullptr;
        if (!r->ahost || !r->adev) {
            if (r->ahost) s->pinned.free(r->ahost);
            r->ahost = nullptr;
            return false;
        }
    }
    r->bkind.assign(nb, 0);
    r->bref.assign(nb, 0);
    r->smallU.clear();
    r->fl.assign(nf, svk::FusedLaunch{});
    std::vector<cd> U;
    int f = 0;
    for (int j = 0; j < nb; ++j) {
        const Block &b = r->blocks[j];
        if (b.ops.size() == 1) continue;
        block_matrix(r->ops.data(), b, U);
        const int k = (int)b.qubits.size();
        if (k <= 2) {
            r->bkind[j] = 1;
            r->bref[j] = (uint32_t)(r->smallU.size() / 16);
            U.resize(16);
            r->smallU.insert(r->smallU.end(), U.begin(), U.end());
        } else {
            r->bkind[j] = 2;
            r->bref[j] = (uint32_t)f;
            svk::fused_prepare(reinterpret_cast<const double *>(U.data()), k, b.qubits.data(), r->n, is_c64,
                               fused_use_mfma(r->n, k) ? 1 : 0, r->ahost + f * r->astride, &r->fl[f]);
            ++f;
        }
    }
    if (nf > 0 &&
        hipMemcpyAsync(r->adev, r->ahost, nf * r->astride, hipMemcpyHostToDevice, r->st->stream) != hipSuccess) {
        s->ctx->arena.free(r->adev);
        s->pinned.free(r->ahost);
        r->adev = r->ahost = nullptr;
        return false;
    }
    r->prepared = true;
    return true;
}

// Admission under the server lock (policy in serve_policy.h).
bool admit_locked(sv_server s) {
    if (s->queue.empty()) return false;
    svp::Limits lim;
    lim.budget = s->cap;
    lim.max_large = s->o.max_active;
    lim.max_small = 4 * kMaxBatch;
    lim.max_bypass = kMaxBypass;
    lim.lookahead = 256;
    const size_t n = std::min<size_t>(s->queue.size(), (size_t)lim.lookahead);
    std::vector<svp::Candidate> cand(n);
    for (size_t i = 0; i < n; ++i) {
        cand[i].small = s->queue[i]->small;
        cand[i].footprint = s->queue[i]->footprint;
        cand[i].bypassed = s->queue[i]->bypassed;
    }
    auto plan = svp::plan_admission(cand, lim, s->held, (int)s->large.size(), (int)s->pending_small.size(),
                                    [&](size_t i) { return try_admit_large(s, s->queue[i]); });
    s->queue[0]->bypassed = cand[0].bypassed;
    if (plan.empty()) return false;
    std::vector<char> taken(n, 0);
    const uint64_t t = now_ns();
    for (auto &pa : plan) {
        Req *r = s->queue[pa.first];
        taken[pa.first] = 1;
        r->t_admit = t;
        s->active++;
        if (pa.second == svp::Action::AdmitSmall) {
            s->pending_small.push_back(r);
            s->stats.admitted++;
        } else if (pa.second == svp::Action::AdmitLarge) {
            s->large.push_back(r);
            s->stats.admitted++;
            s->stats.peak_bytes = std::max<uint64_t>(s->stats.peak_bytes, s->held);
        } else {
            // can never fit this server's memory
            s->stats.rejected++;
            r->status = SV_E_OOM;
            r->t_done = t;
            s->done[r->id] = r;
            s->active--;
            s->stats.completed++;
            s->cv.notify_all();
        }
    }
    for (size_t i = n; i-- > 0;)
        if (taken[i]) s->queue.erase(s->queue.begin() + i);
    return true;
}

// ---- packed launches ---------------------------------------------------------------
bool build_gate_records(const Req *r, std::vector<svk::PGate> &gates, std::vector<double> &pool) {
    for (const sv_op &o : r->ops) {
        cd U[16];
        int k, nc;
        if (!gate_matrix(o.kind, o.p, (o.flags & SV_OP_ADJOINT) != 0, U, &k, &nc)) return false;
        const GateDesc d = classify(U, k, o.q + nc, o.q, nc);
        svk::PGate g{};
        g.uoff = (uint32_t)(pool.size() / 2);
        if (d.kind == GateDesc::NOOP) continue;
        if (d.kind == GateDesc::GROUP) {
            const svk::GroupGate &G = d.group;
            g.fm = (uint32_t)G.fm;
            g.fv = (uint32_t)G.fv;
            g.f0 = (uint32_t)G.F[0];
            g.f1 = (uint32_t)G.F[1];
            g.type = G.K == 0 ? svk::PGate::PHASE : (G.K == 1 ? svk::PGate::PAIR : svk::PGate::QUAD);
            const int cnt = G.K == 0 ? 1 : (G.K == 1 ? 4 : 16);
            for (int i = 0; i < 2 * cnt; ++i) pool.push_back(G.U[i]);
        } else if (d.kind == GateDesc::DIAG) {
            const svk::DiagGate &D = d.diag;
            if (D.k > 4) return false;
            g.type = svk::PGate::DIAG;
            g.k = (uint16_t)D.k;
            g.fm = g.fv = (uint32_t)D.cmask;
            for (int t = 0; t < D.k; ++t) g.f0 |= (uint32_t)D.targets[t] << (8 * t);
            for (int i = 0; i < (2 << D.k); ++i) pool.push_back(D.d[i]);
        } else {
            return false;
        }
        gates.push_back(g);
    }
    return true;
}

bool launch_small(sv_server s) {
    if (s->pending_small.empty() || (int)s->batches.size() >= kMaxBatchesInFlight) return false;
    Batch *b = new Batch();
    b->dt = s->pending_small.front()->dt;
    std::vector<svk::PGate> gates;
    std::vector<double> pool;
    std::vector<svk::PCirc> circ;
    std::vector<uint64_t> tx, tz;
    int maxq = 1;
    std::vector<Req *> rest;
    for (Req *r : s->pending_small) {
        if (r->dt != b->dt || (int)b->reqs.size() >= kMaxBatch || (int)gates.size() >= kMaxBatchGates) {
            rest.push_back(r);
            continue;
        }
        svk::PCirc c{};
        c.n = r->n;
        c.gate_begin = (int)gates.size();
        build_gate_records(r, gates, pool);
        c.gate_end = (int)gates.size();
        c.term_begin = (int)tx.size();
        for (auto &t : r->terms) {
            tx.push_back(t.xmask);
            tz.push_back(t.zmask);
        }
        c.term_end = (int)tx.size();
        c.shots = r->shots;
        c.seed = r->seed;
        c.sample_off = b->samples_total;
        c.res_off = b->res_total;
        b->sample_off.push_back(b->samples_total);
        b->res_off.push_back(b->res_total);
        b->samples_total += (uint64_t)r->shots;
        b->res_total += 1 + r->terms.size();
        maxq = std::max(maxq, r->n);
        circ.push_back(c);
        b->reqs.push_back(r);
    }
    s->pending_small = rest;
    // input layout: circ | gates | pool | tx | tz ; output: samples | res
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    const uint64_t o_circ = 0, o_gates = al(o_circ + circ.size() * sizeof(svk::PCirc));
    const uint64_t o_pool = al(o_gates + gates.size() * sizeof(svk::PGate));
    const uint64_t o_tx = al(o_pool + pool.size() * sizeof(double));
    const uint64_t o_tz = al(o_tx + tx.size() * 8);
    b->in_bytes = al(o_tz + tz.size() * 8);
    const uint64_t o_samp = 0, o_res = al(b->samples_total * 8);
    b->out_bytes = al(o_res + b->res_total * 8);
    b->hin = (char *)s->pinned.alloc(b->in_bytes);
    b->hout = (char *)s->pinned.alloc(b->out_bytes);
    b->dbuf = (char *)s->ctx->arena.alloc(b->in_bytes + b->out_bytes);
    if (!b->hin || !b->hout || !b->dbuf) {
        // not now: put the circuits back and retry next iteration
        if (b->hin) s->pinned.free(b->hin);
        if (b->hout) s->pinned.free(b->hout);
        if (b->dbuf) s->ctx->arena.free(b->dbuf);
        s->pending_small.insert(s->pending_small.begin(), b->reqs.begin(), b->reqs.end());
        delete b;
        return false;
    }
    memcpy(b->hin + o_circ, circ.data(), circ.size() * sizeof(svk::PCirc));
    memcpy(b->hin + o_gates, gates.data(), gates.size() * sizeof(svk::PGate));
    memcpy(b->hin + o_pool, pool.data(), pool.size() * sizeof(double));
    memcpy(b->hin + o_tx, tx.data(), tx.size() * 8);
    memcpy(b->hin + o_tz, tz.data(), tz.size() * 8);
    char *din = b->dbuf, *dout = b->dbuf + b->in_bytes;
    svk::PackedBatch pb{};
    pb.circ = (const svk::PCirc *)(din + o_circ);
    pb.gates = (const svk::PGate *)(din + o_gates);
    pb.pool = (const double *)(din + o_pool);
    pb.tx = (const uint64_t *)(din + o_tx);
    pb.tz = (const uint64_t *)(din + o_tz);
    pb.samples = (uint64_t *)(dout + o_samp);
    pb.res = (double *)(dout + o_res);
    pb.ncirc = (int)circ.size();
    pb.max_amps = 1 << maxq;
    pb.max_leaves = maxq > 6 ? (1 << (maxq - 6)) : 1;
    hipStream_t st = s->small_stream;
    hipError_t e = hipMemcpyAsync(din, b->hin, b->in_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        TraceScope ts(&s->ctx->tracer, st, "packed", 0.0);
        e = svk::launch_packed(pb, b->dt == SV_C64, maxq, 256 * 4, st);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(b->hout, dout, b->out_bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(b->ev, st);
    if (e != hipSuccess) {
        fail(SV_E_DEVICE, std::string("packed launch: ") + hipGetErrorString(e));
        hipStreamSynchronize(st);
        for (Req *r : b->reqs) finish(s, r, SV_E_DEVICE);
        s->pinned.free(b->hin);
        s->pinned.free(b->hout);
        s->ctx->arena.free(b->dbuf);
        if (b->ev) hipEventDestroy(b->ev);
        delete b;
        return true;
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stats.packed_launches++;
        s->stats.packed_circuits += b->reqs.size();
    }
    s->batches.push_back(b);
    return true;
}

// ---- large requests -----------------------------------------------------------------
sv_status enqueue_measure(sv_server s, Req *r) {
    sv_state st = r->st;
    const hipStream_t str = st->stream;
    // No final rescale: the sampler draws against the FP64 total of the CDF
    // and every expectation is divided by the FP64 norm, and the state is
    // dropped after measuring.
    uint64_t *dsamp = (uint64_t *)r->dbuf;
    double *dres = (double *)(r->dbuf + 8 * r->shots);
    const uint64_t nres = (uint64_t)std::max(1, r->nzb) * (kTB + 1) + 2ull * r->xi.size() + 1;
    uint64_t *dmask = (uint64_t *)((char *)dres + 8 * nres);
    uint64_t *hmask = (uint64_t *)(r->hbuf + ((char *)dmask - r->dbuf));
    const uint64_t nmask = (uint64_t)std::max(1, r->nzb) * kTB;
    for (uint64_t i = 0; i < nmask; ++i) hmask[i] = i < r->zi.size() ? r->terms[r->zi[i]].zmask : 0;
    SV_HIP(hipMemcpyAsync(dmask, hmask, 8 * nmask, hipMemcpyHostToDevice, str));
    if (r->shots > 0) {
        SV_HIP(svk::launch_cdf(st->psi, st->n, st->is_c64(), st->ws, str));
        SV_HIP(svk::launch_sample(st->psi, st->n, st->is_c64(), st->ws, r->shots, r->seed, 0, dsamp, str));
    }
    for (int bz = 0; bz < std::max(1, r->nzb); ++bz) {
        const int cnt = std::min<int>(kTB, (int)r->zi.size() - bz * kTB);
        SV_HIP(svk::launch_expect_z(st->psi, st->n, st->is_c64(), dmask + bz * kTB, std::max(cnt, 0), st->ws,
                                    dres + bz * (kTB + 1), str));
    }
    for (size_t i = 0; i < r->xi.size(); ++i)
        SV_HIP(svk::launch_expect_xz(st->psi, st->n, st->is_c64(), r->terms[r->xi[i]].xmask, r->terms[r->xi[i]].zmask,
                                     st->ws, dres + std::max(1, r->nzb) * (kTB + 1) + 2 * i, str));
    SV_HIP(hipMemcpyAsync(r->hbuf, r->dbuf, 8 * (r->shots + nres), hipMemcpyDeviceToHost, str));
    SV_HIP(hipEventRecord(r->ev, str));
    return SV_OK;
}

void collect_large(Req *r) {
    const uint64_t *hs = (const uint64_t *)r->hbuf;
    const double *hr = (const double *)(r->hbuf + 8 * r->shots);
    r->samples.assign(hs, hs + r->shots);
    const int cnt0 = std::min<int>(kTB, (int)r->zi.size());
    r->norm = hr[std::max(cnt0, 0)];
    r->expect.assign(r->terms.size(), 0.0);
    const double nrm = r->norm > 0 ? r->norm : 1.0;
    for (size_t i = 0; i < r->zi.size(); ++i)
        r->expect[r->zi[i]] = hr[(i / kTB) * (kTB + 1) + (i % kTB)] / nrm;
    for (size_t i = 0; i < r->xi.size(); ++i) r->expect[r->xi[i]] = hr[std::max(1, r->nzb) * (kTB + 1) + 2 * i] / nrm;
    r->weighted = 0;
    for (size_t t = 0; t < r->terms.size(); ++t) r->weighted += r->terms[t].coeff * r->expect[t];
}

bool advance_large(sv_server s) {
    bool progress = false;
    for (Req *r : s->large) {
        if (r->measuring) continue;
        const int R = r->st->is_c64() ? s->ctx->renorm_period : 0;
        if (!r->prepared && r->fuse_k == SV_FUSE_AUTO) {
            // the mode the cost model predicts fastest, chosen outside the server lock
            r->fuse_k = choose_mode(s->ctx, r->ops.data(), (int)r->ops.size(), r->n, r->shots);
            if (r->fuse_k >= 2) {
                r->blocks = plan_fusion(r->ops.data(), (int)r->ops.size(), std::min(r->fuse_k, r->n));
                r->total = r->blocks.size();
            } else if (r->fuse_k == 0) {
                r->total = r->ops.size();
                r->prepared = true;
            }
        }
        if (!r->prepared && !(r->fuse_k == SV_FUSE_TILED ? prepare_passes(s, r) : prepare_blocks(s, r))) continue;
        int budget = kChunk;
        sv_status q = SV_OK;
        while (budget > 0 && r->next < r->total && q == SV_OK) {
            if (r->fuse_k == SV_FUSE_TILED) {
                TraceScope ts(&s->ctx->tracer, r->st->stream, "tiled_pass", 2.0 * (double)r->st->bytes);
                const hipError_t e = svk::launch_tiled(r->targs[r->next], (const svk::TileGate *)r->adev, r->st->psi,
                                                       r->st->is_c64() ? 1 : 0, r->st->stream);
                if (e != hipSuccess) q = hip_fail(e, "tiled pass launch");
            } else if (r->fuse_k >= 2) {
                const size_t j = r->next;
                const Block &b = r->blocks[j];
                if (r->bkind[j] == 0) {
                    q = apply_op(r->st, r->ops[b.ops[0]]);
                } else if (r->bkind[j] == 1) {
                    q = apply_matrix(r->st, r->smallU.data() + 16 * r->bref[j], (int)b.qubits.size(),
                                     b.qubits.data(), nullptr, 0);
                } else {
                    const svk::FusedLaunch &f = r->fl[r->bref[j]];
                    TraceScope ts(&s->ctx->tracer, r->st->stream, f.kind == 0 ? "fused_mfma" : "fused_generic",
                                  2.0 * (double)r->st->bytes);
                    const hipError_t e =
                        svk::fused_launch(f, r->adev + r->bref[j] * r->astride, r->st->psi, r->st->stream);
                    if (e != hipSuccess) q = hip_fail(e, "fused block launch");
                }
            } else {
                q = apply_op(r->st, r->ops[r->next]);
            }
            r->next++;
            --budget;
            if (q == SV_OK && R > 0 && ++r->st->sweeps_since_renorm >= R) q = renorm(r->st);
        }
        if (q == SV_OK && r->next == r->total) {
            q = enqueue_measure(s, r);
            if (q == SV_OK) r->measuring = true;
        }
        if (q != SV_OK) {
            // the request failed: wait for its stream, free it, report
            hipStreamSynchronize(r->st->stream);
            r->measuring = true;
            r->status = q;
            hipEventRecord(r->ev, r->st->stream);
        }
        progress = true;
    }
    return progress;
}

bool poll_done(sv_server s) {
    bool progress = false;
    for (size_t i = 0; i < s->batches.size();) {
        Batch *b = s->batches[i];
        if (hipEventQuery(b->ev) != hipSuccess) {
            ++i;
            continue;
        }
        const uint64_t *hs = (const uint64_t *)b->hout;
        const double *hr = (const double *)(b->hout + ((b->samples_total * 8 + 255) & ~255ull));
        for (size_t k = 0; k < b->reqs.size(); ++k) {
            Req *r = b->reqs[k];
            r->samples.assign(hs + b->sample_off[k], hs + b->sample_off[k] + r->shots);
            r->norm = hr[b->res_off[k]];
            r->expect.assign(hr + b->res_off[k] + 1, hr + b->res_off[k] + 1 + r->terms.size());
            r->weighted = 0;
            for (size_t t = 0; t < r->terms.size(); ++t) r->weighted += r->terms[t].coeff * r->expect[t];
            finish(s, r, SV_OK);
        }
        hipEventDestroy(b->ev);
        s->pinned.free(b->hin);
        s->pinned.free(b->hout);
        s->ctx->arena.free(b->dbuf);
        delete b;
        s->batches.erase(s->batches.begin() + i);
        progress = true;
    }
    for (size_t i = 0; i < s->large.size();) {
        Req *r = s->large[i];
        if (!r->measuring || hipEventQuery(r->ev) != hipSuccess) {
            ++i;
            continue;
        }
        const int st = r->status;
        if (st == SV_OK) collect_large(r);
        release_large(s, r);
        s->large.erase(s->large.begin() + i);
        finish(s, r, st);
        progress = true;
    }
    return progress;
}

void drive(sv_server s) {
    hipSetDevice(s->ctx->device);
    for (;;) {
        bool progress = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->stop && s->queue.empty() && s->active == 0) break;
            progress |= admit_locked(s);
        }
        progress |= launch_small(s);
        progress |= advance_large(s);
        progress |= poll_done(s);
        if (!progress) {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->stop && s->queue.empty() && s->active == 0) break;
            s->cv.wait_for(lk, std::chrono::microseconds(s->batches.empty() && s->large.empty() ? 2000 : 20));
        }
    }
}

sv_status validate(sv_server s, const sv_circuit *c) {
    if (!c) return fail(SV_E_INVALID, "null circuit");
    if (c->dtype != SV_C64 && c->dtype != SV_C128) return fail(SV_E_INVALID, "bad dtype");
    const int nmax = c->dtype == SV_C64 ? SV_MAX_QUBITS_C64 : SV_MAX_QUBITS_C128;
    if (c->n < 1 || c->n > nmax) return fail(SV_E_INVALID, "n out of range");
    if (c->nops < 0 || (c->nops > 0 && !c->ops)) return fail(SV_E_INVALID, "bad op list");
    if (c->nterms < 0 || (c->nterms > 0 && !c->terms)) return fail(SV_E_INVALID, "bad term list");
    if (c->shots < 0 || c->shots > kMaxShots) return fail(SV_E_INVALID, "shots out of range [0, 2^24]");
    if (c->fuse_k != 0 && c->fuse_k != SV_FUSE_TILED && c->fuse_k != SV_FUSE_AUTO &&
        (c->fuse_k < 2 || c->fuse_k > SV_MAX_FUSED))
        return fail(SV_E_INVALID, "fuse_k must be 0, 2..5, SV_FUSE_TILED or SV_FUSE_AUTO");
    for (int i = 0; i < c->nops; ++i) {
        const sv_op &o = c->ops[i];
        const int nq = gate_nqubits(o.kind);
        if (nq < 0) return fail(SV_E_INVALID, "unknown gate kind at op " + std::to_string(i));
        if (o.cond != 0) return fail(SV_E_INVALID, "conditional op " + std::to_string(i) + " needs classical bits");
        uint64_t m = 0;
        for (int j = 0; j < nq; ++j) {
            if (o.q[j] < 0 || o.q[j] >= c->n) return fail(SV_E_INVALID, "qubit out of range at op " + std::to_string(i));
            if ((m >> o.q[j]) & 1) return fail(SV_E_INVALID, "duplicate qubit at op " + std::to_string(i));
            m |= 1ull << o.q[j];
        }
        for (int j = 0; j < 3; ++j)
            if (!std::isfinite(o.p[j])) return fail(SV_E_NUMERIC, "non-finite angle at op " + std::to_string(i));
    }
    const uint64_t full = (1ull << c->n) - 1;
    for (int t = 0; t < c->nterms; ++t)
        if ((c->terms[t].xmask | c->terms[t].zmask) & ~full) return fail(SV_E_INVALID, "Pauli mask beyond n qubits");
    (void)s;
    return SV_OK;
}

}  // namespace

extern "C" {

sv_status sv_server_create(sv_ctx ctx, const sv_server_opts *opts, sv_server *out) {
    if (!ctx || !out) return fail(SV_E_INVALID, "null argument");
    sv_server s = new sv_server_s();
    s->ctx = ctx;
    if (opts) s->o = *opts;
    if (s->o.max_active <= 0) s->o.max_active = 256;
    if (s->o.max_queue <= 0) s->o.max_queue = 1 << 20;
    if (s->o.nstreams <= 0) s->o.nstreams = 3;
    if (s->o.small_qubits > 0) {
        s->small_c64 = std::min(s->o.small_qubits, svk::packed_max_qubits(1));
        s->small_c128 = std::min(s->o.small_qubits, svk::packed_max_qubits(0));
    }
    s->cap = s->o.arena_bytes ? std::min<uint64_t>(s->o.arena_bytes, ctx->arena.size()) : ctx->arena.size();
    const uint64_t pinned_bytes = 256ull << 20;
    if (hipHostMalloc((void **)&s->pinned_base, pinned_bytes, hipHostMallocDefault) != hipSuccess) {
        delete s;
        return fail(SV_E_OOM, "pinned host buffer");
    }
    s->pinned.init(s->pinned_base, pinned_bytes);
    for (int i = 0; i < s->o.nstreams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) hipStreamDestroy(x);
            hipHostFree(s->pinned_base);
            delete s;
            return fail(SV_E_DEVICE, "stream creation");
        }
        s->streams.push_back(st);
    }
    hipStreamCreateWithFlags(&s->small_stream, hipStreamNonBlocking);
    s->driver = std::thread(drive, s);
    *out = s;
    return SV_OK;
}

sv_status sv_server_destroy(sv_server s) {
    if (!s) return fail(SV_E_INVALID, "null server");
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    s->driver.join();
    for (auto &kv : s->live) delete kv.second;
    for (auto x : s->streams) hipStreamDestroy(x);
    hipStreamDestroy(s->small_stream);
    hipHostFree(s->pinned_base);
    delete s;
    return SV_OK;
}

sv_status sv_submit(sv_server s, const sv_circuit *c, uint64_t *req_id) {
    if (!s || !req_id) return fail(SV_E_INVALID, "null argument");
    sv_status v = validate(s, c);
    if (v) return v;
    Req *r = new Req();
    r->n = c->n;
    r->dt = (sv_dtype)c->dtype;
    r->fuse_k = c->fuse_k;
    r->shots = c->shots;
    r->seed = c->seed;
    r->ops.assign(c->ops, c->ops + c->nops);
    if (c->nterms > 0) r->terms.assign(c->terms, c->terms + c->nterms);
    r->small = r->n <= (r->dt == SV_C64 ? s->small_c64 : s->small_c128) && r->shots <= kSmallMaxShots;
    if (r->small) {
        std::vector<svk::PGate> g;
        std::vector<double> p;
        r->small = build_gate_records(r, g, p);
    }
    if (!r->small) {
        const int nzb = 0;
        int nz = 0, nx = 0;
        for (auto &t : r->terms) (t.xmask ? nx : nz)++;
        r->footprint = state_bytes(r->n, r->dt) + svk::measure_workspace_bytes(r->n) +
                       result_bytes(r->shots, (nz + kTB - 1) / kTB, nx) + 3 * 256;
        (void)nzb;
    }
    std::lock_guard<std::mutex> g(s->mu);
    if ((int)s->queue.size() >= s->o.max_queue) {
        delete r;
        return fail(SV_E_BUSY, "server queue is full");
    }
    r->id = s->next_id++;
    r->t_submit = now_ns();
    s->queue.push_back(r);
    s->live[r->id] = r;
    s->stats.submitted++;
    *req_id = r->id;
    s->cv.notify_all();
    return SV_OK;
}

static void copy_result(Req *r, sv_result *out) {
    if (!out) return;
    if (out->samples && !r->samples.empty()) memcpy(out->samples, r->samples.data(), 8 * r->samples.size());
    if (out->expect && !r->expect.empty()) memcpy(out->expect, r->expect.data(), 8 * r->expect.size());
    out->weighted = r->weighted;
    out->norm = r->norm;
    out->status = r->status;
    out->t_submit_ns = r->t_submit;
    out->t_admit_ns = r->t_admit;
    out->t_done_ns = r->t_done;
}

sv_status sv_poll(sv_server s, uint64_t id, sv_result *out) {
    if (!s) return fail(SV_E_INVALID, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->done.find(id);
    if (it != s->done.end()) {
        Req *r = it->second;
        copy_result(r, out);
        s->done.erase(it);
        s->live.erase(id);
        delete r;
        return SV_OK;
    }
    if (s->live.count(id)) return SV_PENDING;
    return fail(SV_E_NOTFOUND, "unknown request id");
}

sv_status sv_wait(sv_server s, uint64_t id, sv_result *out, int64_t timeout_ms) {
    if (!s) return fail(SV_E_INVALID, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
    for (;;) {
        auto it = s->done.find(id);
        if (it != s->done.end()) {
            Req *r = it->second;
            copy_result(r, out);
            s->done.erase(it);
            s->live.erase(id);
            delete r;
            return SV_OK;
        }
        if (!s->live.count(id)) return fail(SV_E_NOTFOUND, "unknown request id");
        if (timeout_ms < 0) {
            s->cv.wait(lk);
        } else if (s->cv.wait_until(lk, deadline) == std::cv_status::timeout) {
            if (!s->done.count(id)) return SV_PENDING;
        }
    }
}

sv_status sv_cancel(sv_server s, uint64_t id) {
    if (!s) return fail(SV_E_INVALID, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
        if ((*it)->id == id) {
            Req *r = *it;
            s->queue.erase(it);
            s->live.erase(id);
            delete r;
            s->stats.cancelled++;
            return SV_OK;
        }
    }
    if (s->live.count(id)) return fail(SV_E_BUSY, "request already admitted");
    return fail(SV_E_NOTFOUND, "unknown request id");
}

sv_status sv_server_stats_get(sv_server s, sv_server_stats *out) {
    if (!s || !out) return fail(SV_E_INVALID, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->queued = s->queue.size();
    out->active = (uint64_t)std::max(0, s->active);
    return SV_OK;
}

}  // extern "C"
