// gates.cpp -- gate matrices, gate classification and the fusion planner
// (host side of the state-vector library).
//
// Gate matrices follow Qiskit's definitions (the paper takes Qiskit and
// OpenQASM2 circuits as input, Sec. III-A), global phase included. A gate is
// classified by exact comparisons on its matrix so that each launch reads and
// writes only the amplitudes the gate changes: a single phase on a subspace
// (S, T, P, Z, CZ, CP), a general diagonal (RZ, RZZ), a two-level unitary (any
// one-qubit gate, CX, CY, SWAP, CCX) or a dense two-qubit matrix.
#include "sv_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace svh {

static const cd I1(0.0, 1.0);

int gate_nqubits(int kind) {
    switch (kind) {
    case SV_GATE_CX: case SV_GATE_CY: case SV_GATE_CZ: case SV_GATE_CP:
    case SV_GATE_SWAP: case SV_GATE_RZZ:
        return 2;
    case SV_GATE_CCX:
        return 3;
    default:
        return (kind >= 0 && kind < SV_GATE_COUNT) ? 1 : -1;
    }
}

bool gate_matrix(int kind, const double *p, bool adjoint, cd *U, int *k, int *nc) {
    for (int i = 0; i < 16; ++i) U[i] = 0.0;
    *nc = 0;
    *k = 1;
    const double r2 = 1.0 / std::sqrt(2.0);
    auto set2 = [&](cd a, cd b, cd c, cd d) {
        U[0] = a; U[1] = b; U[2] = c; U[3] = d;
    };
    auto half = [&](double t, double &c, double &s) {
        c = std::cos(0.5 * t);
        s = std::sin(0.5 * t);
    };
    double c, s;
    switch (kind) {
    case SV_GATE_H: set2(r2, r2, r2, -r2); break;
    case SV_GATE_X: set2(0.0, 1.0, 1.0, 0.0); break;
    case SV_GATE_Y: set2(0.0, -I1, I1, 0.0); break;
    case SV_GATE_Z: set2(1.0, 0.0, 0.0, -1.0); break;
    case SV_GATE_S: set2(1.0, 0.0, 0.0, I1); break;
    case SV_GATE_SDG: set2(1.0, 0.0, 0.0, -I1); break;
    case SV_GATE_T: set2(1.0, 0.0, 0.0, std::polar(1.0, M_PI / 4)); break;
    case SV_GATE_TDG: set2(1.0, 0.0, 0.0, std::polar(1.0, -M_PI / 4)); break;
    case SV_GATE_SX: set2(cd(0.5, 0.5), cd(0.5, -0.5), cd(0.5, -0.5), cd(0.5, 0.5)); break;
    case SV_GATE_RX: half(p[0], c, s); set2(c, -I1 * s, -I1 * s, c); break;
    case SV_GATE_RY: half(p[0], c, s); set2(c, -s, s, c); break;
    case SV_GATE_RZ: set2(std::polar(1.0, -0.5 * p[0]), 0.0, 0.0, std::polar(1.0, 0.5 * p[0])); break;
    case SV_GATE_P: set2(1.0, 0.0, 0.0, std::polar(1.0, p[0])); break;
    case SV_GATE_U3:
        half(p[0], c, s);
        set2(c, -std::polar(1.0, p[2]) * s, std::polar(1.0, p[1]) * s, std::polar(1.0, p[1] + p[2]) * c);
        break;
    case SV_GATE_CX: *nc = 1; set2(0.0, 1.0, 1.0, 0.0); break;
    case SV_GATE_CY: *nc = 1; set2(0.0, -I1, I1, 0.0); break;
    case SV_GATE_CZ: *nc = 1; set2(1.0, 0.0, 0.0, -1.0); break;
    case SV_GATE_CP: *nc = 1; set2(1.0, 0.0, 0.0, std::polar(1.0, p[0])); break;
    case SV_GATE_CCX: *nc = 2; set2(0.0, 1.0, 1.0, 0.0); break;
    case SV_GATE_SWAP:
        *k = 2;
        U[0] = 1.0; U[1 * 4 + 2] = 1.0; U[2 * 4 + 1] = 1.0; U[15] = 1.0;
        break;
    case SV_GATE_RZZ: {
        *k = 2;
        const cd a = std::polar(1.0, -0.5 * p[0]), b = std::polar(1.0, 0.5 * p[0]);
        U[0] = a; U[5] = b; U[10] = b; U[15] = a;
        break;
    }
    default:
        return false;
    }
    if (adjoint) {
        const int K = 1 << *k;
        cd A[16];
        for (int r = 0; r < K; ++r)
            for (int q = 0; q < K; ++q) A[r * K + q] = std::conj(U[q * K + r]);
        for (int i = 0; i < K * K; ++i) U[i] = A[i];
    }
    return true;
}

// ---- classification -------------------------------------------------------------

static uint64_t qubit_bits(int pattern, const int *targets, int k) {
    uint64_t m = 0;
    for (int j = 0; j < k; ++j)
        if ((pattern >> j) & 1) m |= 1ull << targets[j];
    return m;
}

static double group_bytes(int n, int s, int K, uint64_t fm) {
    return 2.0 * s * std::ldexp(1.0, n + K - __builtin_popcountll(fm));
}

static const char *group_name(int K, uint64_t F0, uint64_t F1, int lb) {
    const uint64_t low = (1ull << lb) - 1;
    if (K == 0) return "group_phase";
    if (K == 1) {
        const bool h = F0 & ~low, l = F0 & low;
        return (h && l) ? "group_mix" : (h ? "group_h1" : "group_l1");
    }
    const int nh = ((F0 & ~low) != 0) + ((F1 & ~low) != 0);
    return nh == 2 ? "group_h2" : (nh == 1 ? "group_h1l1" : "group_l2");
}

GateDesc classify(const cd *U, int k, const int *targets, const int *controls, int nc) {
    const int K = 1 << k;
    GateDesc d;
    uint64_t cmask = 0, tmask = 0;
    for (int j = 0; j < nc; ++j) cmask |= 1ull << controls[j];
    for (int j = 0; j < k; ++j) tmask |= 1ull << targets[j];
    bool diag = true;
    for (int r = 0; r < K && diag; ++r)
        for (int q = 0; q < K; ++q)
            if (r != q && U[r * K + q] != 0.0) {
                diag = false;
                break;
            }
    if (diag) {
        int nonunit = 0, which = -1;
        for (int m = 0; m < K; ++m)
            if (U[m * K + m] != 1.0) {
                ++nonunit;
                which = m;
            }
        if (nonunit == 0) {
            d.kind = GateDesc::NOOP;
            return d;
        }
        if (nonunit == 1) {
            d.kind = GateDesc::GROUP;
            d.group.fm = cmask | tmask;
            d.group.fv = cmask | qubit_bits(which, targets, k);
            d.group.K = 0;
            d.group.U[0] = U[which * K + which].real();
            d.group.U[1] = U[which * K + which].imag();
            return d;
        }
        d.kind = GateDesc::DIAG;
        d.diag.cmask = cmask;
        d.diag.k = k;
        for (int j = 0; j < k; ++j) d.diag.targets[j] = targets[j];
        for (int m = 0; m < K; ++m) {
            d.diag.d[2 * m] = U[m * K + m].real();
            d.diag.d[2 * m + 1] = U[m * K + m].imag();
        }
        return d;
    }
    // two-level: identity outside two basis states
    int active[32], na = 0;
    for (int m = 0; m < K; ++m) {
        bool ident = true;
        for (int q = 0; q < K; ++q) {
            const cd want = (m == q) ? cd(1.0) : cd(0.0);
            if (U[m * K + q] != want || U[q * K + m] != want) {
                ident = false;
                break;
            }
        }
        if (!ident) active[na++] = m;
    }
    if (na == 2) {
        const int p0 = active[0], p1 = active[1];
        d.kind = GateDesc::GROUP;
        d.group.fm = cmask | tmask;
        d.group.fv = cmask | qubit_bits(p0, targets, k);
        d.group.K = 1;
        d.group.F[0] = qubit_bits(p0 ^ p1, targets, k);
        const cd u2[4] = {U[p0 * K + p0], U[p0 * K + p1], U[p1 * K + p0], U[p1 * K + p1]};
        for (int i = 0; i < 4; ++i) {
            d.group.U[2 * i] = u2[i].real();
            d.group.U[2 * i + 1] = u2[i].imag();
        }
        return d;
    }
    if (k == 2) {
        d.kind = GateDesc::GROUP;
        d.group.fm = cmask | tmask;
        d.group.fv = cmask;
        d.group.K = 2;
        d.group.F[0] = 1ull << targets[0];
        d.group.F[1] = 1ull << targets[1];
        for (int i = 0; i < 16; ++i) {
            d.group.U[2 * i] = U[i].real();
            d.group.U[2 * i + 1] = U[i].imag();
        }
        return d;
    }
    d.kind = GateDesc::DENSE;
    return d;
}

double desc_bytes(const GateDesc &d, int n, int s) {
    if (d.kind == GateDesc::GROUP) return group_bytes(n, s, d.group.K, d.group.fm);
    if (d.kind == GateDesc::DIAG) return 2.0 * s * std::ldexp(1.0, n - __builtin_popcountll(d.diag.cmask));
    return 0.0;
}

sv_status apply_matrix(sv_state st, const cd *U, int k, const int *targets, const int *controls, int nc) {
    const int K = 1 << k;
    const int s = st->is_c64() ? 8 : 16;
    const int lb = svk::low_bits(st->is_c64());
    Tracer *tr = &st->ctx->tracer;
    const GateDesc d = classify(U, k, targets, controls, nc);
    if (d.kind == GateDesc::NOOP) return SV_OK;
    if (d.kind == GateDesc::GROUP) {
        const svk::GroupGate &g = d.group;
        TraceScope ts(tr, st->stream, group_name(g.K, g.F[0], g.F[1], lb), desc_bytes(d, st->n, s));
        SV_HIP(svk::launch_group(g, st->psi, st->n, st->is_c64(), st->stream));
        return SV_OK;
    }
    if (d.kind == GateDesc::DIAG) {
        TraceScope ts(tr, st->stream, "diag", desc_bytes(d, st->n, s));
        SV_HIP(svk::launch_diag(d.diag, st->psi, st->n, st->is_c64(), st->stream));
        return SV_OK;
    }
    // dense k >= 3 (a dense 1-qubit gate is always two-level)
    if (nc == 0) return apply_fused(st, U, k, targets);
    // controlled dense block: embed the controls as extra targets
    const int kk = k + nc;
    if (kk > SV_MAX_FUSED) return fail(SV_E_UNSUPPORTED, "controlled dense gate wider than 5 qubits");
    const int KK = 1 << kk;
    std::vector<cd> W(KK * KK, 0.0);
    for (int m = 0; m < KK; ++m) W[m * KK + m] = 1.0;
    const int off = KK - K;   // all control bits (the high bits) set
    for (int r = 0; r < K; ++r)
        for (int q = 0; q < K; ++q) W[(off + r) * KK + off + q] = U[r * K + q];
    int tg[SV_MAX_FUSED];
    for (int j = 0; j < k; ++j) tg[j] = targets[j];
    for (int j = 0; j < nc; ++j) tg[k + j] = controls[j];
    return apply_fused(st, W.data(), kk, tg);
}

// ---- fusion planner --------------------------------------------------------------
// DAG-aware greedy grouping: open blocks hold disjoint qubit sets. A gate joins
// the open block(s) its qubits meet if the union stays within fuse_k qubits
// (open blocks it meets are merged; gates of disjoint blocks commute, so the
// merged order is still valid); otherwise those blocks are closed and emitted
// and the gate opens a new block. Every gate is placed after all earlier gates
// that share a qubit with it, so the emitted order is a valid schedule.
std::vector<Block> plan_fusion(const sv_op *ops, int nops, int fuse_k) {
    struct Open {
        uint64_t q;
        std::vector<int> ops;
        int order;
    };
    std::vector<Open> open;
    std::vector<Block> out;
    int counter = 0;
    auto emit = [&](Open &o) {
        Block b;
        b.ops = o.ops;
        std::sort(b.ops.begin(), b.ops.end());
        for (int p = 0; p < 64; ++p)
            if ((o.q >> p) & 1) b.qubits.push_back(p);
        out.push_back(std::move(b));
    };
    for (int i = 0; i < nops; ++i) {
        uint64_t g = 0;
        const int nq = gate_nqubits(ops[i].kind);
        for (int j = 0; j < nq; ++j) g |= 1ull << ops[i].q[j];
        uint64_t uni = g;
        std::vector<int> hit;
        for (int b = 0; b < (int)open.size(); ++b)
            if (open[b].q & g) {
                hit.push_back(b);
                uni |= open[b].q;
            }
        if (__builtin_popcountll(uni) <= fuse_k) {
            Open merged{uni, {}, counter++};
            for (int b : hit) merged.ops.insert(merged.ops.end(), open[b].ops.begin(), open[b].ops.end());
            merged.ops.push_back(i);
            for (int h = (int)hit.size() - 1; h >= 0; --h) open.erase(open.begin() + hit[h]);
            open.push_back(std::move(merged));
        } else {
            // close the blocks the gate meets, oldest first
            std::sort(hit.begin(), hit.end(), [&](int a, int b) { return open[a].order < open[b].order; });
            for (int b : hit) emit(open[b]);
            std::vector<int> idx = hit;
            std::sort(idx.begin(), idx.end());
            for (int h = (int)idx.size() - 1; h >= 0; --h) open.erase(open.begin() + idx[h]);
            open.push_back(Open{g, {i}, counter++});
        }
    }
    std::sort(open.begin(), open.end(), [](const Open &a, const Open &b) { return a.order < b.order; });
    for (auto &o : open) emit(o);
    return out;
}

// ---- tiled passes ----------------------------------------------------------------
bool tiled_ops(const sv_op *ops, int nops, std::vector<TiledOp> &out) {
    out.clear();
    out.reserve(nops);
    for (int i = 0; i < nops; ++i) {
        const sv_op &o = ops[i];
        cd U[16];
        int k, nc;
        if (!gate_matrix(o.kind, o.p, (o.flags & SV_OP_ADJOINT) != 0, U, &k, &nc)) return false;
        TiledOp t;
        t.op = i;
        t.d = classify(U, k, o.q + nc, o.q, nc);
        for (int j = 0; j < k + nc; ++j) t.all |= 1ull << o.q[j];
        if (t.d.kind == GateDesc::NOOP) continue;
        if (t.d.kind == GateDesc::GROUP) t.mix = t.d.group.F[0] | t.d.group.F[1];
        else if (t.d.kind != GateDesc::DIAG) return false;   // wider than a named op can be
        out.push_back(t);
    }
    return true;
}

std::vector<Pass> plan_passes(const std::vector<TiledOp> &ops, int n, int mb_max, int lb_full) {
    const int lb = std::min(lb_full, n);
    const int hmax = std::min(mb_max, n) - lb;
    const uint64_t low = (1ull << lb) - 1ull;
    std::vector<Pass> out;
    std::vector<char> done(ops.size(), 0);
    size_t left = ops.size(), first = 0;
    // One scan over the unplaced ops: take, in order, every op whose mixed
    // qubits are (or, with `grow`, can still be added to) the tile qubits Q and
    // that shares no qubit with an op left for later.
    auto scan = [&](uint64_t Q, bool grow, std::vector<int> *take, uint64_t *Qout) {
        uint64_t blocked = 0;
        int h = __builtin_popcountll(Q & ~low), cnt = 0;
        for (size_t i = first; i < ops.size(); ++i) {
            if (done[i]) continue;
            const TiledOp &t = ops[i];
            if (t.all & blocked) {
                blocked |= t.all;
                continue;
            }
            const uint64_t need = t.mix & ~Q;
            const int c = __builtin_popcountll(need);
            if (c == 0 || (grow && h + c <= hmax)) {
                Q |= need;
                h += c;
                ++cnt;
                if (take) take->push_back((int)i);
            } else {
                blocked |= t.all;
            }
        }
        if (Qout) *Qout = Q;
        return cnt;
    };
    while (left > 0) {
        while (done[first]) ++first;
        // candidate tile sets: the greedy growing one, every window of hmax
        // consecutive qubits above the low ones, and the qubits the next
        // unplaced ops use most; the one that takes the most ops wins
        uint64_t bestQ = low;
        bool best_grow = true;
        int best = scan(low, true, nullptr, &bestQ);
        auto consider = [&](uint64_t Q) {
            const int c = scan(Q, false, nullptr, nullptr);
            if (c > best) {
                best = c;
                bestQ = Q;
                best_grow = false;
            }
        };
        if (hmax > 0) {
            for (int s0 = lb; s0 + hmax <= n; ++s0) consider(low | (((1ull << hmax) - 1ull) << s0));
            int score[64] = {0};
            int seen = 0;
            for (size_t i = first; i < ops.size() && seen < 256; ++i) {
                if (done[i]) continue;
                ++seen;
                for (int q = lb; q < n; ++q) score[q] += (int)(((ops[i].mix >> q) & 1) * 2 + ((ops[i].all >> q) & 1));
            }
            uint64_t Q = low;
            for (int k = 0; k < hmax; ++k) {
                int bq = -1;
                for (int q = lb; q < n; ++q)
                    if (!((Q >> q) & 1) && (bq < 0 || score[q] > score[bq])) bq = q;
                if (bq < 0) break;
                Q |= 1ull << bq;
            }
            consider(Q);
        }
        Pass p;
        uint64_t Q = bestQ;
        scan(bestQ, best_grow, &p.ops, &Q);
        for (int i : p.ops) done[i] = 1;
        left -= p.ops.size();
        // fill the tile with the lowest unused qubits: longer contiguous runs
        int h = __builtin_popcountll(Q & ~low);
        for (int q = lb; q < n && h < hmax; ++q)
            if (!((Q >> q) & 1)) {
                Q |= 1ull << q;
                ++h;
            }
        for (int q = lb; q < n; ++q)
            if ((Q >> q) & 1) p.qh.push_back(q);
        out.push_back(std::move(p));
    }
    return out;
}

void pass_records(const sv_op *sops, const std::vector<TiledOp> &ops, const Pass &p, int n, int mb_max,
                  int lb_full, std::vector<svk::TileGate> &recs, svk::TileArgs &args) {
    const int lb = std::min(lb_full, n);
    int local[64];
    uint64_t Q = (1ull << lb) - 1ull;
    for (int q = 0; q < 64; ++q) local[q] = q < lb ? q : -1;
    for (size_t j = 0; j < p.qh.size(); ++j) {
        local[p.qh[j]] = lb + (int)j;
        Q |= 1ull << p.qh[j];
    }
    auto compress = [&](uint64_t m) {
        uint32_t r = 0;
        for (int q = 0; q < 64; ++q)
            if (((m >> q) & 1) && local[q] >= 0) r |= 1u << local[q];
        return r;
    };
    auto fixed = [&](svk::TileGate &g, uint64_t fm, uint64_t fv) {
        // local positions of the fixed bits are ascending because local[] is monotone
        for (int q = 0; q < 64; ++q)
            if (((fm >> q) & 1) && local[q] >= 0) g.ins[g.nins++] = local[q];
        g.lv = compress(fv & fm & Q);
        g.gm = fm & ~Q;
        g.gv = fv & fm & ~Q;
    };
    auto targets = [&](svk::TileGate &g, int k, const int *tg) {
        for (int i = 0; i < k; ++i) {
            g.tl[i] = local[tg[i]];
            g.tg[i] = tg[i];
        }
    };
    // one gate description as a record
    auto emit_desc = [&](const GateDesc &d) {
        if (d.kind == GateDesc::NOOP) return;
        svk::TileGate g;
        if (d.kind == GateDesc::GROUP) {
            const svk::GroupGate &gg = d.group;
            g.kind = 0;
            g.K = gg.K;
            fixed(g, gg.fm, gg.fv);
            g.F[0] = compress(gg.F[0]);
            g.F[1] = compress(gg.F[1]);
            for (int i = 0; i < 2 << (2 * gg.K); ++i) g.u[i] = gg.U[i];
        } else {
            const svk::DiagGate &dg = d.diag;
            g.kind = 1;
            g.K = dg.k;
            fixed(g, dg.cmask, dg.cmask);
            targets(g, dg.k, dg.targets);
            for (int i = 0; i < 2 << dg.k; ++i) g.u[i] = dg.d[i];
        }
        recs.push_back(g);
    };
    // a run of diagonal ops as one phase run
    auto emit_run = [&](const int *idx, int cnt) {
        svk::TileGate h;
        h.kind = 2;
        h.K = cnt;
        recs.push_back(h);
        for (int r = 0; r < cnt; ++r) {
            const GateDesc &d = ops[idx[r]].d;
            svk::TileGate g;
            g.kind = 3;
            uint64_t fm, fv;
            {
                fm = fv = d.diag.cmask;
                g.K = d.diag.k;
                targets(g, d.diag.k, d.diag.targets);
                // the run adds the factors' angles and takes one sincos per amplitude
                for (int m = 0; m < 1 << d.diag.k; ++m) g.u[m] = std::atan2(d.diag.d[2 * m + 1], d.diag.d[2 * m]);
            }
            g.pm = compress(fm & Q);
            g.pv = compress(fv & fm & Q);
            g.gm = fm & ~Q;
            g.gv = fv & fm & ~Q;
            recs.push_back(g);
        }
    };
    // A run of uncontrolled diagonal ops as one parity run: every diagonal
    // factor on <= 2 qubits is exp(i a(m)) with a(m) = c + w0 b0 + w1 b1 +
    // w01 (b0 xor b1) (four values, four coefficients), so the run's angle is
    // a constant plus a weighted sum of parities of bit masks (RZZ(g): one mask
    // of weight g; RZ(t): one of weight t). Equal masks are merged; when every
    // weight is the same (a QAOA cost layer) the kernel counts parities and
    // looks the phase up in a per-tile table instead of one sincos per
    // amplitude.
    constexpr int kMaxParityTable = 127;
    auto emit_parity_run = [&](const int *idx, int cnt) {
        std::map<uint64_t, double> wsum;
        double c = 0.0;
        for (int r = 0; r < cnt; ++r) {
            const GateDesc &d = ops[idx[r]].d;
            double a[4];
            const int k = d.diag.k;
            for (int m = 0; m < 1 << k; ++m) a[m] = std::atan2(d.diag.d[2 * m + 1], d.diag.d[2 * m]);
            const uint64_t b0 = 1ull << d.diag.targets[0];
            if (k == 1) {
                c += a[0];
                wsum[b0] += a[1] - a[0];
            } else {
                const uint64_t b1 = 1ull << d.diag.targets[1];
                const double w01 = 0.5 * (a[1] + a[2] - a[3] - a[0]);
                c += a[0];
                wsum[b0] += a[1] - a[0] - w01;
                wsum[b1] += a[2] - a[0] - w01;
                wsum[b0 | b1] += w01;
            }
        }
        std::vector<std::pair<uint64_t, double>> terms;
        for (auto &kv : wsum)
            if (kv.second != 0.0) terms.push_back(kv);
        svk::TileGate h;
        h.kind = 4;
        h.K = (int)terms.size();
        h.u[0] = c;
        bool same = !terms.empty() && (int)terms.size() <= kMaxParityTable;
        for (auto &t : terms) same = same && t.second == terms[0].second;
        h.pm = same ? 1u : 0u;
        h.u[1] = terms.empty() ? 0.0 : terms[0].second;
        recs.push_back(h);
        for (auto &t : terms) {
            svk::TileGate g;
            g.kind = 5;
            g.pm = compress(t.first & Q);
            g.gm = t.first & ~Q;
            g.u[0] = t.second;
            recs.push_back(g);
        }
    };
    auto uncontrolled = [&](const int *idx, int cnt) {
        for (int r = 0; r < cnt; ++r)
            if (ops[idx[r]].d.diag.cmask != 0) return false;
        return true;
    };
    // Phase runs take general diagonal gates (every amplitude gets a factor, as
    // RZ and RZZ) with unit-modulus factors; a phase on one pattern (CP, CZ, S,
    // T) touches only its members and stays a gate of its own.
    auto is_diag = [&](int i) {
        const GateDesc &d = ops[i].d;
        if (d.kind != GateDesc::DIAG || d.diag.k > 2) return false;
        for (int m = 0; m < 1 << d.diag.k; ++m)
            if (std::fabs(std::hypot(d.diag.d[2 * m], d.diag.d[2 * m + 1]) - 1.0) > 1e-14) return false;
        return true;
    };
    // Greedy blocks of <= 2 tile qubits over a stretch of ops (the fusion rule
    // of plan_fusion: open blocks hold disjoint qubit sets; an op joins the
    // blocks it meets while their union has <= 2 qubits, otherwise they are
    // emitted, oldest first, before it).
    struct Open {
        uint64_t q;
        std::vector<int> ops;   // indices into `ops`
        int order;
    };
    std::vector<cd> U;
    auto emit_block = [&](Open &o) {
        if (o.ops.size() == 1) {
            emit_desc(ops[o.ops[0]].d);
            return;
        }
        std::sort(o.ops.begin(), o.ops.end());
        Block b;
        for (int i : o.ops) b.ops.push_back(ops[i].op);
        for (int q = 0; q < 64; ++q)
            if ((o.q >> q) & 1) b.qubits.push_back(q);
        block_matrix(sops, b, U);
        emit_desc(classify(U.data(), (int)b.qubits.size(), b.qubits.data(), nullptr, 0));
    };
    auto fuse_stretch = [&](const int *idx, int cnt) {
        std::vector<Open> open;
        int counter = 0;
        for (int r = 0; r < cnt; ++r) {
            const int i = idx[r];
            const uint64_t g = ops[i].all;
            const bool fusable = (g & ~Q) == 0 && __builtin_popcountll(g) <= 2;
            uint64_t uni = g;
            std::vector<int> hit;
            for (int b = 0; b < (int)open.size(); ++b)
                if (open[b].q & g) {
                    hit.push_back(b);
                    uni |= open[b].q;
                }
            if (fusable && __builtin_popcountll(uni) <= 2) {
                Open merged{uni, {}, counter++};
                for (int b : hit) merged.ops.insert(merged.ops.end(), open[b].ops.begin(), open[b].ops.end());
                merged.ops.push_back(i);
                for (int h = (int)hit.size() - 1; h >= 0; --h) open.erase(open.begin() + hit[h]);
                open.push_back(std::move(merged));
                continue;
            }
            std::sort(hit.begin(), hit.end(), [&](int x, int y) { return open[x].order < open[y].order; });
            for (int b : hit) emit_block(open[b]);
            std::sort(hit.begin(), hit.end());
            for (int h = (int)hit.size() - 1; h >= 0; --h) open.erase(open.begin() + hit[h]);
            if (fusable) open.push_back(Open{g, {i}, counter++});
            else emit_desc(ops[i].d);
        }
        std::sort(open.begin(), open.end(), [](const Open &x, const Open &y) { return x.order < y.order; });
        for (auto &o : open) emit_block(o);
    };
    constexpr int kMinRun = 3;
    const std::vector<int> &L = p.ops;
    const int nl = (int)L.size();
    auto run_len = [&](int i) {
        int j = i;
        while (j < nl && is_diag(L[j])) ++j;
        return j - i;
    };
    for (int i = 0; i < nl;) {
        const int rl = run_len(i);
        if (rl >= kMinRun) {
            if (uncontrolled(&L[i], rl)) emit_parity_run(&L[i], rl);
            else emit_run(&L[i], rl);
            i += rl;
            continue;
        }
        int e = i + std::max(rl, 1);
        while (e < nl) {
            const int r2 = run_len(e);
            if (r2 >= kMinRun) break;
            e += std::max(r2, 1);
        }
        fuse_stretch(&L[i], e - i);
        i = e;
    }
    args.lb = lb;
    args.mb = lb + (int)p.qh.size();
    for (size_t j = 0; j < p.qh.size(); ++j) args.qh[j] = p.qh[j];
    args.ntiles = 1ull << (n - args.mb);
    (void)mb_max;
}

// Block matrix: U = G_last ... G_first on the block's qubits, built by applying
// each gate to the rows of a K x K matrix that starts as the identity
// (complex128, real and imaginary parts in separate row-major arrays so the
// row updates vectorise). Every gate's matrix is built once. Diagonal gates
// scale rows and 0/1 permutations move them; other gates mix their rows.
void block_matrix(const sv_op *ops, const Block &b, std::vector<cd> &U) {
    const int k = (int)b.qubits.size();
    const int K = 1 << k;
    int pos[64];
    for (int j = 0; j < k; ++j) pos[b.qubits[j]] = j;
    std::vector<double> re((size_t)K * K, 0.0), im((size_t)K * K, 0.0), tr(4 * K), ti(4 * K);
    for (int r = 0; r < K; ++r) re[(size_t)r * K + r] = 1.0;
    for (int oi : b.ops) {
        const sv_op &o = ops[oi];
        cd G[16];
        int gk, nc;
        gate_matrix(o.kind, o.p, o.flags & SV_OP_ADJOINT, G, &gk, &nc);
        const int GK = 1 << gk;
        int tg[3];
        uint64_t tm = 0, cm = 0;
        for (int j = 0; j < nc; ++j) cm |= 1ull << pos[o.q[j]];
        for (int j = 0; j < gk; ++j) {
            tg[j] = pos[o.q[nc + j]];
            tm |= 1ull << tg[j];
        }
        bool diag = true, perm = true;
        for (int r = 0; r < GK; ++r)
            for (int m = 0; m < GK; ++m) {
                const cd g = G[r * GK + m];
                if (r != m && g != 0.0) diag = false;
                if (g != 0.0 && g != 1.0) perm = false;
            }
        for (int i = 0; i < K; ++i) {
            if ((i & tm) || (i & cm) != cm) continue;
            int idx[4];
            for (int m = 0; m < GK; ++m) {
                int a = i;
                for (int j = 0; j < gk; ++j)
                    if ((m >> j) & 1) a |= 1 << tg[j];
                idx[m] = a;
            }
            if (diag) {
                for (int r = 0; r < GK; ++r) {
                    const double gr = G[r * GK + r].real(), gi = G[r * GK + r].imag();
                    if (gr == 1.0 && gi == 0.0) continue;
                    double *xr = &re[(size_t)idx[r] * K], *xi = &im[(size_t)idx[r] * K];
                    for (int c = 0; c < K; ++c) {
                        const double a = xr[c], bb = xi[c];
                        xr[c] = gr * a - gi * bb;
                        xi[c] = gr * bb + gi * a;
                    }
                }
                continue;
            }
            // keep the gate's input rows, then write its output rows
            for (int m = 0; m < GK; ++m) {
                std::copy_n(&re[(size_t)idx[m] * K], K, &tr[(size_t)m * K]);
                std::copy_n(&im[(size_t)idx[m] * K], K, &ti[(size_t)m * K]);
            }
            for (int r = 0; r < GK; ++r) {
                double *yr = &re[(size_t)idx[r] * K], *yi = &im[(size_t)idx[r] * K];
                if (perm) {
                    int m = 0;
                    while (G[r * GK + m] == 0.0) ++m;
                    std::copy_n(&tr[(size_t)m * K], K, yr);
                    std::copy_n(&ti[(size_t)m * K], K, yi);
                    continue;
                }
                std::fill_n(yr, K, 0.0);
                std::fill_n(yi, K, 0.0);
                for (int m = 0; m < GK; ++m) {
                    const double gr = G[r * GK + m].real(), gi = G[r * GK + m].imag();
                    if (gr == 0.0 && gi == 0.0) continue;
                    const double *xr = &tr[(size_t)m * K], *xi = &ti[(size_t)m * K];
                    for (int c = 0; c < K; ++c) {
                        yr[c] += gr * xr[c] - gi * xi[c];
                        yi[c] += gr * xi[c] + gi * xr[c];
                    }
                }
            }
        }
    }
    U.resize((size_t)K * K);
    for (size_t e = 0; e < (size_t)K * K; ++e) U[e] = cd(re[e], im[e]);
}

}  // namespace svh
