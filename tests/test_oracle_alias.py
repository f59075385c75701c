"""Pins of the oracle's Walker alias sampler (Sec. III-C item 1): the defining
property of an alias table (the mass of every outcome, its own share plus
what other slots hand it, equals N p_i), a table worked out by hand, closed
forms for two outcomes and for a point mass, the histogram of the draws
against |psi|^2, and the prefix-sum form of the table (a partitioned merge of
the light deficits and heavy excesses, the form the device computes) against
the sweep, exactly, on inputs where FP64 arithmetic is exact."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O


def _masses(prob, alias):
    """m_i = prob_i + sum over slots j != i aliasing to i of (1 - prob_j)."""
    m = prob.astype(np.float64).copy()
    other = alias != np.arange(alias.size, dtype=np.uint64)
    np.add.at(m, alias[other].astype(np.int64), 1.0 - prob[other])
    return m


def test_hand_worked_table():
    # p = (0.1, 0.2, 0.3, 0.4): s = (0.4, 0.8, 1.2, 1.6); light 0 takes heavy 2,
    # which drops to 0.6 and takes heavy 3 (now 1.2); light 1 takes heavy 3 (now 1.0)
    psi = np.sqrt(np.array([0.1, 0.2, 0.3, 0.4])).astype(np.complex128)
    prob, alias = O.alias_build(psi)
    assert np.allclose(prob, [0.4, 0.8, 0.6, 1.0], atol=1e-15)
    assert alias.tolist() == [2, 3, 3, 3]


@pytest.mark.parametrize("a", [0.0, 0.13, 0.5 - 1e-9, 0.71, 1.0])
def test_two_outcomes_closed_form(a):
    psi = np.array([np.sqrt(a), np.sqrt(1 - a)], dtype=np.complex128)
    prob, alias = O.alias_build(psi)
    lo, hi = (0, 1) if a < 0.5 else (1, 0)
    plo = 2 * min(a, 1 - a)
    if plo < 1:
        assert abs(prob[lo] - plo) <= 1e-15 and alias[lo] == hi
    assert prob[hi] == 1.0 and alias[hi] == hi


def test_point_mass():
    n = 7
    psi = O.basis_state(n, 77)
    prob, alias = O.alias_build(psi)
    assert prob[77] == 1.0 and np.all(prob[np.arange(1 << n) != 77] == 0.0)
    assert np.all(alias == 77)
    assert np.all(O.alias_sample(prob, alias, 500, 3) == 77)


@pytest.mark.parametrize("n,seed", [(1, 1), (3, 2), (6, 3), (10, 4), (13, 5)])
def test_masses_reproduce_the_distribution(n, seed):
    psi = W.random_state(n, seed)
    # sparse and peaked entries too: zero some amplitudes, boost one
    rng = np.random.default_rng(seed)
    psi[rng.random(psi.size) < 0.3] = 0
    psi[int(rng.integers(0, psi.size))] *= 5
    if not np.any(psi):
        psi[0] = 1
    prob, alias = O.alias_build(psi)
    N = psi.size
    p = np.abs(psi) ** 2
    s = N * p / np.sum(p)
    assert np.all((prob >= 0) & (prob <= 1))
    assert np.all(alias < N)
    assert np.max(np.abs(_masses(prob, alias) - s)) <= 1e-12 * max(1, N)
    # zero-probability outcomes are never returned
    assert np.all(prob[p == 0] == 0)


def test_draws_follow_the_probabilities():
    n, shots = 5, 200000
    psi = W.random_state(n, 9)
    prob, alias = O.alias_build(psi)
    x = O.alias_sample(prob, alias, shots, 41)
    p = np.abs(psi) ** 2
    p /= p.sum()
    hist = np.bincount(x.astype(np.int64), minlength=1 << n) / shots
    sig = np.sqrt(p * (1 - p) / shots)
    assert np.all(np.abs(hist - p) <= 5 * sig + 1e-9)
    # the counter offset continues the stream
    assert np.array_equal(O.alias_sample(prob, alias, 100, 41, s0=50), x[50:150])


def _four_squares(d):
    """Up to four integers whose squares add up to d (Lagrange)."""
    r = int(np.sqrt(d)) + 1
    for a in range(r):
        for b in range(a, r):
            for c in range(b, r):
                e2 = d - a * a - b * b - c * c
                if e2 < 0:
                    break
                e = int(round(np.sqrt(e2)))
                if e * e == e2:
                    return [x for x in (a, b, c, e) if x]
    raise AssertionError(d)


def _dyadic_state(n, rng, mode):
    """Amplitudes (x_i + i y_i) / 1024 with small integers whose squares add up
    to a power of two, so that |psi_i|^2, the norm and every s_i = N p_i / W
    are exact in FP64 and the oracle's sweep runs in exact arithmetic."""
    N = 1 << n
    x = rng.integers(0, 4, N)
    if mode == "sparse":
        x[rng.random(N) < 0.6] = 0
    elif mode == "outlier":
        x[:] = 1
        x[int(rng.integers(N))] = 7
    elif mode == "uniform":
        x[:] = 1
    x[0] = max(x[0], 1)
    tot = int(np.sum(x * x))
    target = 1 << (tot - 1).bit_length()
    y = np.zeros(N, dtype=np.int64)
    fill = _four_squares(target - tot) if target > tot else []
    for k, v in zip(rng.permutation(N)[:len(fill)], fill):
        y[k] = v
    assert int(np.sum(x * x + y * y)) == target
    return (x + 1j * y).astype(np.complex128) / 1024.0


def _merge_form(s, width):
    """The alias table from prefix sums, as a partitioned merge: D (light
    deficits) and E (heavy excesses) in index order, merged with a light entry
    first on ties; `width` merge items per part. Light k takes heavy
    #{j: E_j < D_(k-1)} (light 0 takes heavy 0); heavy j, with i = #{k: D_k <=
    E_j}, is exhausted by light i and keeps 1 - (D_i - E_j), unless it is the
    last heavy entry or i = (number of lights). Exact arithmetic."""
    from fractions import Fraction as Fr
    N = len(s)
    lights = [i for i in range(N) if s[i] < 1]
    heavies = [i for i in range(N) if not s[i] < 1]
    nl, nh = len(lights), len(heavies)
    D, E = [], []
    acc = Fr(0)
    for i in lights:
        acc += 1 - s[i]
        D.append(acc)
    acc = Fr(0)
    for i in heavies:
        acc += s[i] - 1
        E.append(acc)
    prob = [Fr(1) if not s[i] < 1 else s[i] for i in range(N)]
    alias = list(range(N))
    if nh == 0:
        return [Fr(1)] * N, alias
    nparts = (N + width - 1) // width

    def part(d):   # lights among the first d merge items
        lo, hi = max(0, d - nh), min(d, nl)
        while lo < hi:
            mid = (lo + hi) // 2
            if D[mid] > E[d - 1 - mid]:
                hi = mid
            else:
                lo = mid + 1
        return lo

    cuts = [part(min(w * width, N)) for w in range(nparts + 1)]
    if nl:
        alias[lights[0]] = heavies[0]
    for w in range(nparts):
        d0, d1 = w * width, min(w * width + width, N)
        i0, i1 = cuts[w], cuts[w + 1]
        h0, h1 = d0 - i0, d1 - i1
        assert 0 <= i1 - i0 and h0 <= h1 and (i1 - i0) + (h1 - h0) == d1 - d0
        for i in range(i0, i1):
            if i + 1 < nl:
                h = h0 + sum(1 for j in range(h0, h1) if E[j] < D[i])
                alias[lights[i + 1]] = heavies[min(h, nh - 1)]
        for j in range(h0, h1):
            if j + 1 >= nh:
                continue
            i = i0 + sum(1 for k in range(i0, i1) if D[k] <= E[j])
            if i >= nl:
                continue
            prob[heavies[j]] = 1 - (D[i] - E[j])
            alias[heavies[j]] = heavies[j + 1]
    return prob, alias


@pytest.mark.parametrize("mode", ["random", "sparse", "outlier", "uniform"])
def test_prefix_merge_form_gives_the_sweep_table(mode):
    # the prefix-sum (merge) form of the table, the form the device computes,
    # equals the oracle's sweep exactly on inputs where FP64 is exact
    from fractions import Fraction as Fr
    rng = np.random.default_rng({"random": 1, "sparse": 2, "outlier": 3, "uniform": 4}[mode])
    checked = 0
    for trial in range(40):
        n = int(rng.integers(2, 7))
        psi = _dyadic_state(n, rng, mode)
        N = 1 << n
        p = [Fr(float(x.real)) ** 2 + Fr(float(x.imag)) ** 2 for x in psi]
        W = sum(p)
        s = [N * x / W for x in p]
        assert sum(s) == N
        wp, wa = O.alias_build(psi)
        for width in (1, 2, 3, 5, 8):
            prob, alias = _merge_form(s, width)
            assert [float(x) for x in prob] == wp.tolist()
            assert alias == wa.tolist()
        checked += 1
    assert checked == 40
