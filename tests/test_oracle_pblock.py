"""Pins of the p-block oracle (Sec. II, p-block; Sec. III-E) against what the
mathematics fixes: a product of blocks must equal the full state-vector
simulation (a different code path: one 2^n vector, no merges), measured
circuits must follow the full-state trajectory, the teleportation protocol
must deliver its input state, the remote CNOT must act as a CNOT, the
partition of small hand-made circuits is written out, per-block sampling
reproduces |psi|^2, and a Pauli string's expectation on a product state is the
one of the full vector. Conditional gates in the full-state oracle are pinned
by circuits whose outcomes are certain."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O
from oracle import pblock as PB


def _local_circuit(n, ngates, seed, span=3):
    """Random gates whose qubits lie within `span` of each other: blocks grow locally."""
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(ngates):
        r = rng.random()
        a = int(rng.integers(0, n))
        if r < 0.55 or n < 2:
            ops.append(("u3", (a,), tuple(rng.uniform(0, 2 * np.pi, 3))))
            continue
        cand = [q for q in range(max(0, a - span), min(n, a + span + 1)) if q != a]
        b = int(rng.choice(cand))
        if r < 0.9 or n < 3:
            name = ["cx", "cz", "cp", "swap", "rzz", "cy"][int(rng.integers(0, 6))]
            p = (float(rng.uniform(0, 6.28)),) if name in ("cp", "rzz") else ()
            ops.append((name, (a, b), p))
        else:
            c = int(rng.choice([q for q in cand if q != b] or [b]))
            if c != b:
                ops.append(("ccx", (a, b, c), ()))
    return ops


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (5, 3), (9, 4), (12, 5)])
def test_product_of_blocks_is_the_full_state(n, seed):
    ops = _local_circuit(n, 6 * n, seed, span=2)
    _, st = PB.run(ops, n)
    full = O.run(ops, n)
    assert np.max(np.abs(st.full_state() - full)) <= 1e-12
    for i in np.random.default_rng(seed).integers(0, 1 << n, 20):
        assert abs(st.amplitude(int(i)) - full[int(i)]) <= 1e-12


def test_partition_of_a_hand_made_circuit():
    ops = [("h", (0,), ()), ("cx", (0, 1), ()), ("h", (2,), ()), ("cz", (2, 3), ()), ("x", (5,), ())]
    _, st = PB.run(ops, 6)
    assert st.partition().tolist() == [0, 0, 1, 1, 2, 3]
    # a three-qubit gate joins three blocks
    _, st = PB.run(ops + [("ccx", (1, 4, 3), ())], 6)
    assert st.partition().tolist() == [0, 0, 0, 0, 0, 1]
    assert sorted(len(q) for q, _ in st.blocks) == [1, 5]
    # a measured qubit leaves its block
    _, st = PB.run(ops + [("measure", (1, 0), ())], 6, seed=3)
    assert st.partition().tolist() == [0, 1, 2, 2, 3, 4]


@pytest.mark.parametrize("seed", range(6))
def test_measured_circuit_follows_the_full_trajectory(seed):
    n = 8
    rng = np.random.default_rng(seed)
    ops = _local_circuit(n, 40, seed, span=3)
    # measurements, resets and conditional gates at random places
    out = []
    for i, op in enumerate(ops):
        out.append(op)
        if rng.random() < 0.15:
            q = int(rng.integers(0, n))
            out.append(("measure", (q, i % 5), ()) if rng.random() < 0.7 else ("reset", (q,), ()))
        if rng.random() < 0.1:
            out.append(W.c_if(("x", (int(rng.integers(0, n)),), ()), int(rng.integers(0, 5)), int(rng.integers(0, 2))))
    cl_pb, st = PB.run(out, n, seed=100 + seed)
    cl_full, full, K = O.trajectory(out, n, 100 + seed)
    assert K > 0
    assert cl_pb == cl_full
    assert np.max(np.abs(st.full_state() - full)) <= 1e-12
    # and shot 0 of the full-state shot runner
    cl0, _ = O.run_shots(out, n, 1, 100 + seed)
    assert int(cl0[0]) == cl_full


@pytest.mark.parametrize("seed", range(5))
def test_teleportation_delivers_the_input(seed):
    # qubit 0 holds a random state; pair (1, 2); Bell measurement of (0, 1);
    # X on 2 if bit 1 is set, Z on 2 if bit 0 is set
    ang = tuple(np.random.default_rng(seed).uniform(0, 2 * np.pi, 3))
    ops = [("u3", (0,), ang), ("h", (1,), ()), ("cx", (1, 2), ()), ("cx", (0, 1), ()), ("h", (0,), ()),
           ("measure", (0, 0), ()), ("measure", (1, 1), ()),
           W.c_if(("x", (2,), ()), 1, 1), W.c_if(("z", (2,), ()), 0, 1)]
    cl, st = PB.run(ops, 3, seed=seed)
    assert st.partition().tolist() == [0, 1, 2]
    want = O.run([("u3", (0,), ang)], 1)
    got = [psi for qs, psi in st.blocks if qs == [2]][0]
    # equal up to a global phase
    ph = np.vdot(want, got)
    assert abs(abs(ph) - 1) <= 1e-12
    assert np.max(np.abs(got - ph * want)) <= 1e-12
    # the measured qubits hold their outcomes
    for q in (0, 1):
        b = [psi for qs, psi in st.blocks if qs == [q]][0]
        m = (cl >> q) & 1
        assert abs(abs(b[m]) - 1) <= 1e-12 and abs(b[1 - m]) <= 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_remote_cx_acts_as_a_cnot(seed):
    # two hosts of 2 qubits in random states, a remote CNOT 0 -> 3 through comm qubits 4, 5
    rng = np.random.default_rng(seed)
    prep = [("u3", (q,), tuple(rng.uniform(0, 2 * np.pi, 3))) for q in range(4)] + [("cx", (0, 1), ()),
                                                                                   ("cx", (2, 3), ())]
    ops = prep + W.remote_cx(0, 3, 4, 5, 0, 1)
    _, st = PB.run(ops, 6, seed=seed)
    want = O.run(prep + [("cx", (0, 3), ())], 6)
    got = st.full_state()
    ph = np.vdot(want, got)
    assert abs(abs(ph) - 1) <= 1e-12 and np.max(np.abs(got - ph * want)) <= 1e-12
    # the communication qubits ended in blocks of their own, in |0>
    assert st.partition()[4] != st.partition()[5] and len(set(st.partition()[:4])) == 1
    assert abs(st.amplitude(0b000000) - got[0]) <= 1e-12


def test_dqc_workload_keeps_communication_qubits_out():
    ops, n = W.dqc(2, 4, 3, [(0, 1)], seed=7)
    _, st = PB.run(ops, n, seed=11)
    part = st.partition()
    assert len(set(part[:8])) == 1                     # the two hosts entangled
    assert part[8] != part[0] and part[9] != part[0]  # the link qubits left
    assert st.state_bytes() == 16 * ((1 << 8) + 2 * 2)
    full_cl, full, _ = O.trajectory(ops, n, 11)
    assert np.max(np.abs(st.full_state() - full)) <= 1e-12


def test_sampling_reproduces_the_probabilities():
    # two entangled blocks: the joint histogram of per-block draws matches |psi|^2
    ops = [("ry", (0,), (0.7,)), ("cx", (0, 1), ()), ("ry", (2,), (1.9,)), ("ry", (3,), (2.6,)), ("cx", (3, 2), ())]
    _, st = PB.run(ops, 4)
    shots = 40000
    s = np.array(st.sample(shots, 21))
    p = np.abs(O.run(ops, 4)) ** 2
    hist = np.bincount(s, minlength=16) / shots
    sig = np.sqrt(p * (1 - p) / shots) + 1e-12
    assert np.all(np.abs(hist - p) <= 5 * sig + 1e-9)
    # per-block counters: block 0 (qubits 0, 1) uses counters 0.., block 1 counters shots..
    b0 = [psi for qs, psi in st.ordered()][0]
    loc = O.sample_at(b0, np.arange(shots, dtype=np.uint64), 21)
    q0 = st.ordered()[0][0]
    want = [sum(((int(v) >> j) & 1) << q for j, q in enumerate(q0)) for v in loc]
    assert [x & 0b11 for x in s.tolist()] == want


def test_sampling_of_basis_states_is_exact():
    ops = [("x", (1,), ()), ("x", (4,), ()), ("cx", (4, 5), ())]
    _, st = PB.run(ops, 7)
    assert set(st.sample(50, 3)) == {0b0110010}


@pytest.mark.parametrize("seed", range(4))
def test_expectations_on_the_product_state(seed):
    n = 8
    ops = _local_circuit(n, 30, seed, span=1)
    _, st = PB.run(ops, n)
    full = O.run(ops, n)
    for x, z, _ in W.random_paulis(n, 12, seed):
        assert abs(st.expect(x, z) - O.expect(full, x, z).real) <= 1e-12


def test_conditional_gates_in_the_full_oracle():
    # qubit 0 is |1> with certainty, qubit 1 |0>: the condition on bit 0 == 1 fires,
    # the one on bit 1 == 1 does not
    ops = [("x", (0,), ()), ("measure", (0, 0), ()), ("measure", (1, 1), ()),
           W.c_if(("x", (2,), ()), 0, 1), W.c_if(("x", (3,), ()), 1, 1), W.c_if(("x", (4,), ()), 1, 0)]
    cl, psi, K = O.trajectory(ops, 5, 9)
    assert cl == 0b01 and K == 2
    assert abs(psi[0b10101] - 1) <= 1e-15
    cls, smp = O.run_shots(ops, 5, 7, 9)
    assert np.all(cls == 1) and np.all(smp == 0b10101)


def test_blocks_hold_ascending_qubits_and_one_block_samples_like_the_full_state():
    # merges in every order: (3, 1), then (0, 5), then the two blocks via (5, 3),
    # then 2 and 4 joined last
    ops = [("h", (3,), ()), ("cx", (3, 1), ()), ("ry", (5,), (0.4,)), ("cx", (5, 0), ()), ("cz", (5, 3), ()),
           ("u3", (4,), (0.3, 1.0, 2.0)), ("swap", (4, 2), ()), ("cx", (2, 1), ()), ("ry", (0,), (1.3,))]
    _, st = PB.run(ops, 6)
    assert [qs for qs, _ in st.blocks] == [[0, 1, 2, 3, 4, 5]]
    full = O.run(ops, 6)
    assert np.max(np.abs(st.blocks[0][1] - full)) <= 1e-12
    assert np.array_equal(np.array(st.sample(2000, 17), dtype=np.uint64), O.sample(full, 2000, 17))
