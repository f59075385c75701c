"""GPU parity of the per-gate kernels against the complex128 oracle, through the
C ABI. Every gate kind at every target placement, explicit matrices of every
classification branch, and random circuits; complex128 and complex64."""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from conftest import infidelity

pytestmark = pytest.mark.gpu

C128_TOL = 1e-12


def _start(n, seed, dtype):
    psi = W.random_state(n, seed)
    if dtype == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)   # same input on both sides
    return psi


def _check(got, want, dtype, tol128=C128_TOL):
    if dtype == "c128":
        assert np.max(np.abs(got - want)) <= tol128
    else:
        assert infidelity(got, want) <= 1e-10
        assert np.max(np.abs(got - want)) <= 2e-6 * max(1.0, np.max(np.abs(want)))


def placements(n, nq, limit, rng):
    allp = list(itertools.permutations(range(n), nq))
    if len(allp) <= limit:
        return allp
    idx = rng.choice(len(allp), size=limit, replace=False)
    return [allp[i] for i in sorted(idx)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7, 8, 9, 12])
def test_every_gate_every_placement(ctx, S, O, n, dtype):
    rng = np.random.default_rng(n)
    st = S.State(ctx, n, dtype)
    try:
        names = [g for g in W.GATES_1Q + W.GATES_2Q + W.GATES_3Q
                 if (1 if g in W.GATES_1Q else 2 if g in W.GATES_2Q else 3) <= n]
        for g in names:
            nq = 1 if g in W.GATES_1Q else 2 if g in W.GATES_2Q else 3
            for qs in placements(n, nq, 40, rng):
                params = tuple(rng.uniform(0, 2 * math.pi, W.circuits.N_PARAMS.get(g, 0)))
                op = (g, qs, params)
                psi0 = _start(n, int(rng.integers(1 << 30)), dtype)
                want = O.apply_op(psi0.copy(), op)
                st.copy_in(psi0)
                st.run([op])
                _check(st.copy_out(), want, dtype)
                # adjoint flag
                st.copy_in(psi0)
                st.run([(g, qs, params, True)])
                _check(st.copy_out(), O.apply_op(psi0.copy(), op, adjoint=True), dtype)
    finally:
        st.close()


def special_matrices(rng):
    th = rng.uniform(0, 2 * math.pi, 4)
    out = [np.diag([np.exp(1j * th[0]), 1.0]),                          # single phase on |0>
           np.diag([np.exp(1j * th[0]), np.exp(1j * th[1])]),           # general diagonal
           np.eye(2),                                                     # identity: no-op
           W.random_unitary(1, int(rng.integers(1 << 30))),
           np.diag(np.exp(1j * th)),                                      # 2q general diagonal
           np.diag([1, 1, np.exp(1j * th[2]), 1]),                       # 2q single phase on |10>
           W.random_unitary(2, int(rng.integers(1 << 30)))]
    two_level = np.eye(4, dtype=np.complex128)                          # acts on |00>, |11> only
    u = W.random_unitary(1, int(rng.integers(1 << 30)))
    two_level[np.ix_([0, 3], [0, 3])] = u
    out.append(two_level)
    two_level2 = np.eye(4, dtype=np.complex128)                         # acts on |01>, |10>
    two_level2[np.ix_([1, 2], [1, 2])] = u
    out.append(two_level2)
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [4, 8, 11])
def test_explicit_matrices_with_controls(ctx, S, O, n, dtype):
    rng = np.random.default_rng(100 + n)
    st = S.State(ctx, n, dtype)
    try:
        for trial in range(60):
            for U in special_matrices(rng):
                k = int(round(math.log2(U.shape[0])))
                nc = int(rng.integers(0, min(3, n - k) + 1))
                qs = rng.choice(n, size=k + nc, replace=False)
                t, c = list(qs[:k]), list(qs[k:])
                psi0 = _start(n, int(rng.integers(1 << 30)), dtype)
                want = O.apply_matrix(psi0.copy(), U, t, c)
                st.copy_in(psi0)
                st.apply_gate(U, t, c)
                _check(st.copy_out(), want, dtype)
    finally:
        st.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,ngates", [(3, 200), (6, 300), (10, 300), (14, 250)])
def test_random_circuits(ctx, S, O, n, ngates, dtype):
    ops = W.random_circuit(n, ngates, seed=n * 31 + ngates)
    want = O.run(ops, n)
    with S.State(ctx, n, dtype) as st:
        st.run(ops)
        got = st.copy_out()
    if dtype == "c128":
        assert np.max(np.abs(got - want)) <= C128_TOL
    else:
        assert infidelity(got, want) <= 1e-5


def test_brickwork_12q_state(ctx, S, O):
    ops = W.brickwork(12, 20, seed=20251204)
    want = O.run(ops, 12)
    with S.State(ctx, 12, "c128") as st:
        st.run(ops)
        got = st.copy_out()
    assert np.max(np.abs(got - want)) <= C128_TOL


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [5, 16, 20])
def test_qft_matches_oracle_and_closed_form(ctx, S, O, n, dtype):
    x = W.random_basis_state(n, 20251205)
    with S.State(ctx, n, dtype) as st:
        st.reset(x)
        st.run(W.qft(n))
        got = st.copy_out()
    y = np.arange(1 << n, dtype=np.uint64)
    ph = ((np.uint64(x) * y) & np.uint64((1 << n) - 1)).astype(np.float64) / float(1 << n)
    closed = np.exp(2j * np.pi * ph) / math.sqrt(1 << n)
    if n <= 16:
        want = O.run(W.qft(n), n, basis=x)
        assert np.max(np.abs(want - closed)) <= 1e-12
    if dtype == "c128":
        assert np.max(np.abs(got - closed)) <= C128_TOL
    else:
        assert infidelity(got, closed) <= 1e-5


def test_reset_and_copy_roundtrip(ctx, S):
    with S.State(ctx, 7, "c128") as st:
        st.reset(77)
        got = st.copy_out()
        want = np.zeros(128, dtype=np.complex128)
        want[77] = 1
        assert np.array_equal(got, want)
    with S.State(ctx, 1, "c64") as st:
        st.reset(1)
        assert np.array_equal(st.copy_out(), np.array([0, 1], dtype=np.complex64))


def test_invalid_arguments_are_rejected(ctx, S):
    with S.State(ctx, 5, "c128") as st:
        with pytest.raises(S.SvError) as e:
            st.run([("h", (5,), ())])
        assert e.value.status == S._abi.SV_E_INVALID
        with pytest.raises(S.SvError):
            st.run([("cx", (2, 2), ())])
        with pytest.raises(S.SvError):
            st.apply_gate(np.eye(2), [1], [1])
        with pytest.raises(S.SvError) as e:
            st.apply_gate(np.array([[np.nan, 0], [0, 1]]), [0])
        assert e.value.status == S._abi.SV_E_NUMERIC
        with pytest.raises(S.SvError):
            st.reset(32)
    with pytest.raises(S.SvError) as e:
        S.State(ctx, 34, "c128")
    assert e.value.status == S._abi.SV_E_INVALID
    with pytest.raises(S.SvError) as e:
        S.State(ctx, 33, "c128")    # 128 GiB does not fit the 64 GiB test arena
    assert e.value.status == S._abi.SV_E_OOM
