"""Parity at the full sizes of the measured workloads, through properties that
hold at any size and outputs computable one by one: 28-qubit brickwork mirror
and norm, 28-qubit QFT against its closed form on sampled outputs, 30-qubit
QAOA p=1 against the closed form, the 33-qubit complex128 / 34-qubit
complex64 fused and tiled paths by cross-mirror (fused blocks or tiled passes
forward, per-gate inverse), and both samplers at 28 qubits against the oracle
on the state read back. Per-gate, fused and tiled runs are all checked."""
import math

import numpy as np
import pytest

import workloads as W
from test_oracle_pins import qaoa_p1_edge_zz

pytestmark = pytest.mark.gpu

SEED = 20251205


@pytest.mark.parametrize("dtype,fuse_k", [("c128", 0), ("c64", 0), ("c128", 5), ("c128", -1), ("c64", -1)])
def test_brickwork_28q_mirror_and_norm(ctx, S, dtype, fuse_k):
    n = 28
    ops = W.brickwork(n, 20, seed=SEED)
    with S.State(ctx, n, dtype) as st:
        st.run(ops, fuse_k=fuse_k)
        nrm = st.norm2()
        st.run(S.inverse_ops(ops), fuse_k=fuse_k)
        a0 = st.amplitudes([0])[0]
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert abs(nrm - 1.0) <= tol
    assert 1.0 - abs(a0) ** 2 <= tol


@pytest.mark.parametrize("fuse_k", [0, -1])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qft_28q_closed_form_on_sampled_outputs(ctx, S, dtype, fuse_k):
    n = 28
    x = W.random_basis_state(n, SEED)
    rng = np.random.default_rng(1)
    y = np.concatenate([rng.integers(0, 1 << n, 1 << 16, dtype=np.uint64),
                        np.array([0, 1, (1 << n) - 1], dtype=np.uint64)])
    with S.State(ctx, n, dtype) as st:
        st.reset(x)
        st.run(W.qft(n), fuse_k=fuse_k)
        got = st.amplitudes(y)
        shots = st.sample(4096, SEED + 1)
    ph = ((np.uint64(x) * y) & np.uint64((1 << n) - 1)).astype(np.float64) / float(1 << n)
    want = np.exp(2j * np.pi * ph) / math.sqrt(1 << n)
    if dtype == "c128":
        assert np.max(np.abs(got - want)) <= 1e-12
    else:
        # relative error per amplitude for a state whose infidelity is <= 1e-5
        assert np.max(np.abs(got - want)) <= math.sqrt(1e-5) * 2 ** (-n / 2) * 10
    # the QFT of a basis state is uniform: top 4 bits of 4096 shots are balanced
    top = (shots >> np.uint64(n - 4)).astype(np.int64)
    counts = np.bincount(top, minlength=16)
    chi2 = float(np.sum((counts - 256.0) ** 2 / 256.0))
    assert chi2 < 60.0          # 15 dof; P(chi2 > 60) < 1e-6


@pytest.mark.parametrize("fuse_k", [0, -1])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qaoa_30q_p1_closed_form(ctx, S, dtype, fuse_k):
    n = 30
    ops, edges, terms = W.qaoa_maxcut(n, 1, seed=SEED + 4)
    gamma, beta = ops[n][2][0], ops[-1][2][0]
    want = qaoa_p1_edge_zz(gamma, beta, edges, n)
    with S.State(ctx, n, dtype) as st:
        st.run(ops, fuse_k=fuse_k)
        vals, energy = st.expect(terms)
    if dtype == "c128":
        assert np.max(np.abs(vals - want)) <= 1e-12
        assert abs(energy - want.sum()) <= 1e-10
    else:
        assert np.max(np.abs(vals - want)) <= 2 * math.sqrt(1e-5)


@pytest.fixture(scope="module")
def big_ctx(S):
    import torch

    c = S.Context(arena_bytes=140 << 30)
    yield c
    c.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fuse_k", [5, -1])
@pytest.mark.parametrize("n,dtype", [(33, "c128"), (34, "c64")])
def test_fused_cross_mirror_full_size(big_ctx, S, n, dtype, fuse_k):
    # fused blocks or tiled passes forward, one kernel per gate backward
    ops = W.brickwork(n, 10, seed=SEED + 2)
    with S.State(big_ctx, n, dtype) as st:
        st.run(S.ops_to_numpy(ops), fuse_k=fuse_k)
        st.run(S.ops_to_numpy(S.inverse_ops(ops)), fuse_k=0)
        a0 = st.amplitudes([0])[0]
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert 1.0 - abs(a0) ** 2 <= tol


def test_alias_rejects_more_than_32_qubits(big_ctx, S):
    # a table of 2^33 outcomes (36 B each) cannot fit next to its state; the
    # call fails with SV_E_INVALID before it allocates, and the state stays usable
    with S.State(big_ctx, 33, "c64") as st:
        with pytest.raises(S.SvError):
            st.sample_alias(10, 1)
        assert st.sample(4, 1).tolist() == [0, 0, 0, 0]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sampling_28q_coupled_to_oracle(ctx, S, O, dtype):
    # the inverse-CDF sampler at the measured size and shot count (4096 shots
    # of a 28-qubit brickwork state), against the oracle's inverse CDF of the
    # same state read back: both draw U01(seed, s) for shot s, so the outcomes
    # agree but where u lands between the two CDFs (expected count ~0)
    n, shots = 28, 4096
    with S.State(ctx, n, dtype) as st:
        st.run(W.brickwork(n, 6, seed=SEED))
        got = st.sample(shots, SEED + 1)
        psi = st.copy_out().astype(np.complex128)
    want = O.sample(psi, shots, SEED + 1)
    assert got.shape == (shots,) and np.all(got < (1 << n))
    assert int(np.count_nonzero(got != want)) <= 1


def test_alias_28q_table_and_draws(ctx, S, O):
    # the whole 2^28-entry alias table against the oracle's sweep over the same
    # state, and 10^5 draws. Tolerance on prob: a heavy entry's prob is
    # 1 - (D_k - E_j) with prefixes of up to N terms, so an ulp of difference
    # in the two squared norms moves it by up to about 2^-53 N per ulp; two
    # ulps are allowed
    n, shots = 28, 100000
    N = 1 << n
    with S.State(ctx, n, "c128") as st:
        st.run(W.brickwork(n, 6, seed=SEED))
        out, prob, alias = st.sample_alias(shots, SEED + 2, table=True)
        psi = st.copy_out()
    wp, wa = O.alias_build(psi)
    assert np.max(np.abs(prob - wp)) <= 1e-9 + 2 * 2.0**-53 * N
    assert int(np.count_nonzero(alias != wa)) <= 2 + N // 10**6
    p = np.abs(psi) ** 2
    assert np.all(prob[p == 0] == 0)
    ref = O.alias_sample(wp, wa, shots, SEED + 2)
    assert int(np.count_nonzero(out != ref)) <= 2
    assert np.all(out < N)
