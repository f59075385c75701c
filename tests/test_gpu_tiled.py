"""GPU parity of the multi-gate tiled passes (sv_run with SV_FUSE_TILED)
against the complex128 oracle, through the C ABI: every gate kind at sampled
placements inside one tile and across tiles (controls, pattern bits and
diagonal factors outside the tile), random circuits over several passes, the
single-tile edge sizes, QFT closed form, and a mirror against the per-gate
kernels."""
import math

import numpy as np
import pytest

import workloads as W
from conftest import infidelity
from test_gpu_gates import _check, _start, placements

pytestmark = pytest.mark.gpu

C128_TOL = 1e-12
TILED = -1


def _nq(g):
    return 1 if g in W.GATES_1Q else 2 if g in W.GATES_2Q else 3


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 3, 7, 12, 15, 17])
def test_every_gate_tiled(ctx, S, O, n, dtype):
    rng = np.random.default_rng(100 + n)
    with S.State(ctx, n, dtype) as st:
        for g in [g for g in W.GATES_1Q + W.GATES_2Q + W.GATES_3Q if _nq(g) <= n]:
            for qs in placements(n, _nq(g), 12, rng):
                params = tuple(rng.uniform(0, 2 * math.pi, W.circuits.N_PARAMS.get(g, 0)))
                for adj in (False, True):
                    psi0 = _start(n, int(rng.integers(1 << 30)), dtype)
                    want = O.apply_op(psi0.copy(), (g, qs, params), adjoint=adj)
                    st.copy_in(psi0)
                    st.run([(g, qs, params, adj)], fuse_k=TILED)
                    _check(st.copy_out(), want, dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,ngates", [(3, 150), (8, 300), (13, 300), (14, 300), (16, 400), (19, 400)])
def test_random_circuits_tiled(ctx, S, O, n, ngates, dtype):
    ops = W.random_circuit(n, ngates, seed=7 * n + ngates)
    psi0 = _start(n, n + 5, dtype)
    want = O.run(ops, n, psi=psi0.copy())
    with S.State(ctx, n, dtype) as st:
        st.copy_in(psi0)
        st.run(ops, fuse_k=TILED)
        got = st.copy_out()
    if dtype == "c128":
        assert np.max(np.abs(got - want)) <= C128_TOL
    else:
        assert infidelity(got, want) <= 1e-5


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [16, 20])
def test_qft_tiled_closed_form(ctx, S, O, n, dtype):
    x = W.random_basis_state(n, 20251205)
    with S.State(ctx, n, dtype) as st:
        st.reset(x)
        st.run(W.qft(n), fuse_k=TILED)
        got = st.copy_out()
    y = np.arange(1 << n, dtype=np.uint64)
    ph = ((np.uint64(x) * y) & np.uint64((1 << n) - 1)).astype(np.float64) / float(1 << n)
    closed = np.exp(2j * np.pi * ph) / math.sqrt(1 << n)
    if dtype == "c128":
        assert np.max(np.abs(got - closed)) <= C128_TOL
    else:
        assert infidelity(got, closed) <= 1e-5


def test_brickwork_tiled_matches_oracle(ctx, S, O):
    ops = W.brickwork(16, 20, seed=20251204)
    want = O.run(ops, 16)
    with S.State(ctx, 16, "c128") as st:
        st.run(ops, fuse_k=TILED)
        got = st.copy_out()
    assert np.max(np.abs(got - want)) <= C128_TOL


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("same", [False, True])
@pytest.mark.parametrize("n", [5, 13, 19])
def test_parity_runs_tiled(ctx, S, O, n, dtype, same):
    # runs of RZ / RZZ only (parity-form runs): random angles (one FP64 sum per
    # amplitude) or one angle for the whole run (the phase-table path), on qubits
    # inside and outside the tiles (one partial tile at n = 5, one full tile at
    # n = 13), between Hadamard layers
    rng = np.random.default_rng(11 + same + n)
    ops = []
    for layer in range(3):
        ops += [("h", (q,), ()) for q in range(n)]
        g = float(rng.uniform(0, 2 * np.pi))
        for _ in range(50):
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            ang = g if same else float(rng.uniform(0, 2 * np.pi))
            ops.append(("rzz", (a, b), (ang,)) if rng.random() < 0.7 else ("rz", (a,), (ang,)))
    psi0 = _start(n, 78, dtype)
    want = O.run(ops, n, psi=psi0.copy())
    with S.State(ctx, n, dtype) as st:
        st.copy_in(psi0)
        st.run(ops, fuse_k=TILED)
        got = st.copy_out()
    if dtype == "c128":
        assert np.max(np.abs(got - want)) <= C128_TOL
    else:
        assert infidelity(got, want) <= 1e-5


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tiled_forward_per_gate_inverse(ctx, S, dtype):
    n = 22
    ops = W.random_circuit(n, 500, seed=4242)
    inv = [(o[0], o[1], o[2], True) for o in reversed(ops)]
    with S.State(ctx, n, dtype) as st:
        st.run(ops, fuse_k=TILED)
        st.run(inv)
        amp = st.amplitudes([0])[0]
    err = 1.0 - abs(amp) ** 2
    assert err <= (1e-12 if dtype == "c128" else 1e-5)


def test_tiled_runs_back_to_back(ctx, S, O):
    # the staged pass records of one run must not be overwritten by the next
    n = 15
    a = W.random_circuit(n, 200, seed=1)
    b = W.random_circuit(n, 200, seed=2)
    want = O.run(a + b + a, n)
    with S.State(ctx, n, "c128") as st:
        st.run(a, fuse_k=TILED)
        st.run(b, fuse_k=TILED)
        st.run(a, fuse_k=TILED)
        got = st.copy_out()
    assert np.max(np.abs(got - want)) <= C128_TOL


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_diagonal_runs_tiled(ctx, S, O, dtype):
    # long runs of diagonal gates (one phase-run record per run) between
    # layers of Hadamards, with targets and controls inside and outside tiles
    n = 18
    diag = ["z", "s", "sdg", "t", "tdg", "rz", "p", "cz", "cp", "rzz"]
    ops = []
    for layer in range(4):
        ops += [("h", (q,), ()) for q in range(n)]
        ops += W.random_circuit(n, 60, seed=50 + layer, names=diag)
    ops += [("ccx", (17, 16, 2), ()), ("cx", (15, 1), ())] + W.random_circuit(n, 10, seed=99, names=diag)
    psi0 = _start(n, 77, dtype)
    want = O.run(ops, n, psi=psi0.copy())
    with S.State(ctx, n, dtype) as st:
        st.copy_in(psi0)
        st.run(ops, fuse_k=TILED)
        got = st.copy_out()
    if dtype == "c128":
        assert np.max(np.abs(got - want)) <= C128_TOL
    else:
        assert infidelity(got, want) <= 1e-5


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qaoa_tiled(ctx, S, O, dtype):
    n = 18
    ops, _edges, terms = W.qaoa_maxcut(n, 3, seed=31)
    want = O.run(ops, n)
    with S.State(ctx, n, dtype) as st:
        st.run(ops, fuse_k=TILED)
        got = st.copy_out()
        vals, _ = st.expect(terms)
    want_e = np.array([O.expect(want, x, z).real for x, z, _ in terms])
    if dtype == "c128":
        assert np.max(np.abs(got - want)) <= C128_TOL
        assert np.max(np.abs(vals - want_e)) <= 1e-12
    else:
        assert infidelity(got, want) <= 1e-5
        assert np.max(np.abs(vals - want_e)) <= 2 * math.sqrt(1e-5)
