"""GPU parity of the alias sampler (sv_sample_alias) against the oracle's
sequential sweep: the same table (prob within FP64 rounding, aliases equal
except where a comparison lands within rounding), the alias-table mass
identity on the device table, the same draws, and the degenerate states
(point mass, uniform, sparse), up to a 26-qubit state; on inputs where FP64
arithmetic is exact, the same table bit for bit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _masses(prob, alias):
    m = prob.astype(np.float64).copy()
    other = alias != np.arange(alias.size, dtype=np.uint64)
    np.add.at(m, alias[other].astype(np.int64), 1.0 - prob[other])
    return m


def _state(n, seed, dtype):
    psi = W.random_state(n, seed)
    rng = np.random.default_rng(seed)
    psi[rng.random(psi.size) < 0.2] = 0          # zeros: entries that must never be drawn
    psi[int(rng.integers(0, psi.size))] *= 4      # one heavy outlier
    psi = psi / np.linalg.norm(psi)
    if dtype == "c64":   # the same input on both sides
        psi = psi.astype(np.complex64).astype(np.complex128)
    return psi


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 3, 11, 12, 13, 16, 20, 24])
def test_table_and_draws_match_oracle(ctx, S, O, n, dtype):
    psi = _state(n, 1000 + n, dtype)
    N = 1 << n
    shots = 20000
    with S.State(ctx, n, dtype) as st:
        st.copy_in(psi)
        out, prob, alias = st.sample_alias(shots, 77, table=True)
    wp, wa = O.alias_build(psi)
    assert np.max(np.abs(prob - wp)) <= 1e-9
    diff = int(np.count_nonzero(alias != wa))
    assert diff <= 2 + N // 10**6, diff
    p = np.abs(psi) ** 2
    s = N * p / p.sum()
    tol = (1e-12 if dtype == "c128" else 1e-6) * max(1, N) ** 0.5 + 1e-12 * N
    assert np.max(np.abs(_masses(prob, alias) - s)) <= tol
    assert np.all(prob[p == 0] == 0) and np.all(out < N)
    ref = O.alias_sample(wp, wa, shots, 77)
    assert int(np.count_nonzero(out != ref)) <= 2
    assert np.all(p[out.astype(np.int64)] > 0)


def test_point_mass_and_ghz(ctx, S):
    with S.State(ctx, 14, "c128") as st:
        st.reset(12345)
        out, prob, alias = st.sample_alias(3000, 5, table=True)
        assert np.all(out == 12345) and np.all(alias == 12345) and prob[12345] == 1.0
        st.reset(0)
        st.run(W.ghz(14))
        out = st.sample_alias(20000, 6)
    assert set(np.unique(out).tolist()) == {0, (1 << 14) - 1}
    frac = float(np.mean(out == 0))
    assert abs(frac - 0.5) <= 5 * np.sqrt(0.25 / 20000)


def test_uniform_state(ctx, S):
    # every s_i is 1 up to rounding: whichever side of 1 an entry lands, the
    # masses stay 1 and the draws are uniform
    n = 12
    with S.State(ctx, n, "c128") as st:
        st.run([("h", (q,), ()) for q in range(n)])
        out, prob, alias = st.sample_alias(200000, 8, table=True)
    assert np.max(np.abs(_masses(prob, alias) - 1.0)) <= 1e-12
    hist = np.bincount(out.astype(np.int64), minlength=1 << n)
    exp = 200000 / (1 << n)
    chi2 = float(np.sum((hist - exp) ** 2 / exp))
    assert chi2 < (1 << n) + 6 * np.sqrt(2 * (1 << n))


def test_circuit_state_at_26_qubits(ctx, S, O):
    n = 26
    ops = W.brickwork(n, 6, seed=26)
    with S.State(ctx, n, "c128") as st:
        st.run(ops)
        out = st.sample_alias(100000, 99)
        psi = st.copy_out()
    wp, wa = O.alias_build(psi)
    ref = O.alias_sample(wp, wa, 100000, 99)
    assert int(np.count_nonzero(out != ref)) <= 2


def test_errors(ctx, S):
    with S.State(ctx, 4, "c128") as st:
        with pytest.raises(S.SvError):
            st.sample_alias(-1, 0)
        assert st.sample_alias(0, 0).size == 0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_one_qubit_states(ctx, S, O, dtype):
    # |1>, |+> and an unbalanced superposition: the smallest tables
    with S.State(ctx, 1, dtype) as st:
        st.reset(1)
        out, prob, alias = st.sample_alias(500, 3, table=True)
        assert np.all(out == 1) and prob.tolist() == [0.0, 1.0] and alias.tolist() == [1, 1]
        st.reset(0)
        st.run([("ry", (0,), (0.6,))])
        psi = st.copy_out().astype(np.complex128)
        out, prob, alias = st.sample_alias(4000, 4, table=True)
    wp, wa = O.alias_build(psi / np.linalg.norm(psi))
    assert np.max(np.abs(prob - wp)) <= (1e-12 if dtype == "c128" else 1e-6) and alias.tolist() == wa.tolist()
    assert abs(float(np.mean(out == 1)) - float(np.sin(0.3) ** 2)) <= 5 * np.sqrt(0.25 / 4000)



@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [2, 5, 11, 12, 14, 16])
def test_dyadic_states_bit_exact(ctx, S, O, n, dtype):
    # amplitudes whose squared norms, norm, s values and prefix sums are all
    # exact in FP64 (and whose amplitudes are exact in FP32): the device's
    # table must equal the oracle's sweep bit for bit, the order of equal
    # prefixes included, across several tiles and merge parts
    from test_oracle_alias import _dyadic_state
    rng = np.random.default_rng(500 + n)
    for mode in ("random", "sparse", "outlier"):
        psi = _dyadic_state(n, rng, mode)
        with S.State(ctx, n, dtype) as st:
            st.copy_in(psi)
            out, prob, alias = st.sample_alias(5000, 13, table=True)
        wp, wa = O.alias_build(psi)
        assert prob.tolist() == wp.tolist()
        assert alias.tolist() == wa.tolist()
        assert out.tolist() == O.alias_sample(wp, wa, 5000, 13).tolist()
