"""Pins of the oracle's Walker alias sampler (Sec. III-C item 1): the defining
property of an alias table (the mass of every outcome, its own share plus
what other slots hand it, equals N p_i), a table worked out by hand, closed
forms for two outcomes and for a point mass, and the histogram of the draws
against |psi|^2."""
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
