"""Seeded gate-list generators for the workloads the state-vector path is measured on.

A circuit is a list of ops ``(name, qubits, params)``:

* ``name``   -- lower-case gate name (Qiskit naming, the paper's input format,
  Sec. III-A): ``h x y z s sdg t tdg sx rx ry rz p u3`` (one qubit),
  ``cx cy cz cp swap rzz`` (two qubits, the control first for ``c*`` gates),
  ``ccx`` (two controls, then the target).
* ``qubits`` -- tuple of qubit indices; qubit q is bit q of the amplitude index.
* ``params`` -- tuple of angles in radians (``rx ry rz p cp rzz``: one angle,
  ``u3``: theta, phi, lambda).

Only names, indices and angles live here; what a name means numerically is
defined separately by each consumer.
"""
from __future__ import annotations

import math

import numpy as np

GATES_1Q = ("h", "x", "y", "z", "s", "sdg", "t", "tdg", "sx", "rx", "ry", "rz", "p", "u3")
GATES_2Q = ("cx", "cy", "cz", "cp", "swap", "rzz")
GATES_3Q = ("ccx",)
N_PARAMS = {"rx": 1, "ry": 1, "rz": 1, "p": 1, "u3": 3, "cp": 1, "rzz": 1}

TWO_PI = 2.0 * math.pi


def _op(name, qubits, params=()):
    return (name, tuple(int(q) for q in qubits), tuple(float(p) for p in params))


def circuit_gate_count(ops) -> int:
    return len(ops)


def brickwork(n: int, layers: int, seed: int):
    """Random brickwork: per layer a U3 on every qubit (angles iid uniform
    [0, 2*pi), drawn qubit by qubit in the order theta, phi, lambda), then CNOTs
    on neighbour pairs (0,1),(2,3),... on even layers and (1,2),(3,4),... on odd
    layers, the lower index as control, no wrap-around."""
    rng = np.random.default_rng(seed)
    ops = []
    for layer in range(layers):
        ang = rng.uniform(0.0, TWO_PI, size=(n, 3))
        for q in range(n):
            ops.append(_op("u3", (q,), ang[q]))
        for c in range(layer % 2, n - 1, 2):
            ops.append(_op("cx", (c, c + 1)))
    return ops


def ghz(n: int):
    """H on qubit 0, then a CNOT chain q -> q+1."""
    ops = [_op("h", (0,))]
    for q in range(n - 1):
        ops.append(_op("cx", (q, q + 1)))
    return ops


def random_basis_state(n: int, seed: int) -> int:
    """A seeded basis index x in [0, 2^n)."""
    rng = np.random.default_rng(seed)
    return int(rng.integers(0, 1 << n, dtype=np.uint64)) if n < 64 else 0


def qft(n: int, swaps: bool = True):
    """Quantum Fourier transform gate list (textbook construction written for
    little-endian qubit order: the most significant qubit is n-1).

    For j = n-1 down to 0: H(j), then for every k < j a controlled phase of
    pi / 2^(j-k) with control k and target j. Finally the bit-reversal SWAPs
    (q, n-1-q) for q < n/2. n H + n(n-1)/2 CP + floor(n/2) SWAP gates."""
    ops = []
    for j in range(n - 1, -1, -1):
        ops.append(_op("h", (j,)))
        for k in range(j - 1, -1, -1):
            ops.append(_op("cp", (k, j), (math.pi / float(1 << (j - k)),)))
    if swaps:
        for q in range(n // 2):
            ops.append(_op("swap", (q, n - 1 - q)))
    return ops


def random_regular_graph(n: int, d: int, seed: int):
    """Seeded random d-regular simple graph by the configuration (pairing)
    model with rejection: shuffle n*d stubs, pair them up, and retry until the
    pairing has no self-loop and no repeated edge. Edges are (u, v) with u < v,
    sorted."""
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    rng = np.random.default_rng(seed)
    for _ in range(100000):
        stubs = np.repeat(np.arange(n), d)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        edges = {(int(min(a, b)), int(max(a, b))) for a, b in pairs}
        if len(edges) != len(pairs):
            continue
        return sorted(edges)
    raise RuntimeError("pairing model did not converge")


def qaoa_maxcut(n: int, p: int, seed: int, degree: int = 3):
    """QAOA MaxCut on a seeded random 3-regular graph: H on every qubit, then p
    layers of RZZ(gamma_l) on every edge followed by RX(beta_l) on every qubit,
    gamma_l, beta_l iid uniform [0, pi). Returns (ops, edges, terms) where
    terms are the Z_u Z_v Pauli terms of the cost as (xmask, zmask, coeff)."""
    edges = random_regular_graph(n, degree, seed)
    rng = np.random.default_rng(seed + 7919)
    ops = [_op("h", (q,)) for q in range(n)]
    angles = rng.uniform(0.0, math.pi, size=(p, 2))
    for layer in range(p):
        gamma, beta = angles[layer]
        for u, v in edges:
            ops.append(_op("rzz", (u, v), (gamma,)))
        for q in range(n):
            ops.append(_op("rx", (q,), (beta,)))
    terms = [(0, (1 << u) | (1 << v), 1.0) for u, v in edges]
    return ops, edges, terms


SERVING_GATES = ("h", "s", "t", "rx", "ry", "rz", "cx", "cz", "swap")
_SERVING_1Q = ("h", "s", "t", "rx", "ry", "rz")


def serving_circuit(n: int, depth: int, rng):
    """One circuit of the serving stream: per layer the qubits are shuffled and
    walked; at each step a gate is drawn uniformly from SERVING_GATES; a
    two-qubit gate takes the next two qubits in walk order (control first),
    and if only one qubit is left the draw is repeated from the one-qubit
    gates. Rotation angles are uniform [0, 2*pi)."""
    ops = []
    for _ in range(depth):
        order = rng.permutation(n)
        i = 0
        while i < n:
            g = SERVING_GATES[int(rng.integers(0, len(SERVING_GATES)))]
            if g in ("cx", "cz", "swap"):
                if i + 1 >= n:
                    g = _SERVING_1Q[int(rng.integers(0, len(_SERVING_1Q)))]
                else:
                    ops.append(_op(g, (order[i], order[i + 1])))
                    i += 2
                    continue
            if g in ("rx", "ry", "rz"):
                ops.append(_op(g, (order[i],), (rng.uniform(0.0, TWO_PI),)))
            else:
                ops.append(_op(g, (order[i],)))
            i += 1
    return ops


def serving_stream(count: int, seed: int, n_lo: int = 8, n_hi: int = 26,
                   d_lo: int = 5, d_hi: int = 40, shots: int = 1000):
    """The serving request mix: qubit count uniform in [n_lo, n_hi], depth
    uniform in [d_lo, d_hi], gates as in serving_circuit, `shots` shots each and
    a per-request sampling seed. Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(d_lo, d_hi + 1))
        ops = serving_circuit(n, d, rng)
        out.append({"id": r, "n": n, "depth": d, "ops": ops, "shots": shots,
                    "seed": int(seed * 1000003 + r) & ((1 << 63) - 1)})
    return out


def poisson_arrivals(count: int, rate: float, seed: int):
    """Arrival times (seconds, from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    return np.cumsum(gaps) - gaps[0]


def random_circuit(n: int, ngates: int, seed: int, names=None):
    """Uniformly random gates from `names` (default: every supported gate that
    fits n qubits) on random distinct qubits with angles uniform [0, 2*pi)."""
    rng = np.random.default_rng(seed)
    if names is None:
        names = list(GATES_1Q) + (list(GATES_2Q) if n >= 2 else []) + (list(GATES_3Q) if n >= 3 else [])
    ops = []
    for _ in range(ngates):
        g = names[int(rng.integers(0, len(names)))]
        nq = 1 if g in GATES_1Q else (2 if g in GATES_2Q else 3)
        qs = rng.choice(n, size=nq, replace=False)
        params = rng.uniform(0.0, TWO_PI, size=N_PARAMS.get(g, 0))
        ops.append(_op(g, qs, params))
    return ops


def random_state(n: int, seed: int) -> np.ndarray:
    """A seeded random complex128 vector of 2^n entries with unit 2-norm
    (iid normal real and imaginary parts, then divided by the norm)."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return (v / np.linalg.norm(v)).astype(np.complex128)


def random_unitary(k: int, seed: int) -> np.ndarray:
    """A seeded Haar-random 2^k x 2^k unitary (QR of a complex Gaussian
    matrix with the phases of R's diagonal divided out)."""
    rng = np.random.default_rng(seed)
    K = 1 << k
    A = rng.normal(size=(K, K)) + 1j * rng.normal(size=(K, K))
    Q, R = np.linalg.qr(A)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


def random_paulis(n: int, count: int, seed: int):
    """Seeded random Pauli strings as (xmask, zmask, coeff) with coeff in [-1, 1]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        x = int(rng.integers(0, 1 << n))
        z = int(rng.integers(0, 1 << n))
        out.append((x, z, float(rng.uniform(-1, 1))))
    return out


def c_if(op, clbit: int, value: int):
    """The gate `op` applied only when classical bit `clbit` holds `value`."""
    return (op[0], op[1], op[2], False, (int(clbit), int(value)))


def remote_cx(a: int, b: int, ca: int, cb: int, m1: int, m2: int):
    """CNOT from qubit a (one host) to qubit b (another host) through the
    communication qubits ca (on a's host) and cb (on b's host), both |0> on
    entry: an entangled pair on (ca, cb); the cat-entangler (CX a->ca, measure
    ca into classical bit m1, X on cb if it read 1); CX cb->b; the disentangler
    (H on cb, measure cb into m2, Z on a if it read 1); then both communication
    qubits reset to |0>."""
    return [_op("h", (ca,)), _op("cx", (ca, cb)), _op("cx", (a, ca)), ("measure", (ca, m1), ()),
            c_if(_op("x", (cb,)), m1, 1), _op("cx", (cb, b)), _op("h", (cb,)), ("measure", (cb, m2), ()),
            c_if(_op("z", (a,)), m2, 1), ("reset", (ca,), ()), ("reset", (cb,), ())]


def dqc(hosts: int, m: int, rounds: int, links, seed: int):
    """A distributed circuit (Sec. III-E): `hosts` hosts of m computational
    qubits (host h holds qubits h*m .. h*m+m-1) and two communication qubits per
    link (link l, between hosts links[l] = (h1, h2), owns qubits hosts*m + 2l
    and hosts*m + 2l + 1). Each round applies one brickwork layer inside every
    host (U3 on each qubit, angles iid uniform [0, 2*pi) drawn qubit by qubit
    as theta, phi, lambda, then CNOTs on neighbour pairs starting at offset
    round % 2) and then, for every link, a remote CNOT from qubit r % m of h1 to
    qubit (3r + 1) % m of h2 (r = round index) through the link's
    communication qubits, its two measurements into classical bits 2l % 64 and
    (2l + 1) % 64. Returns (ops, total qubits)."""
    rng = np.random.default_rng(seed)
    links = [tuple(x) for x in links]
    n = hosts * m + 2 * len(links)
    ops = []
    for r in range(rounds):
        for h in range(hosts):
            base = h * m
            ang = rng.uniform(0.0, TWO_PI, size=(m, 3))
            for q in range(m):
                ops.append(_op("u3", (base + q,), ang[q]))
            for c in range(r % 2, m - 1, 2):
                ops.append(_op("cx", (base + c, base + c + 1)))
        for l, (h1, h2) in enumerate(links):
            ca, cb = hosts * m + 2 * l, hosts * m + 2 * l + 1
            ops += remote_cx(h1 * m + r % m, h2 * m + (3 * r + 1) % m, ca, cb, (2 * l) % 64, (2 * l + 1) % 64)
    return ops, n
