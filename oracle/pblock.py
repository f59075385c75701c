"""TEST INFRASTRUCTURE ONLY -- plain p-block oracle.

Partitioned-block simulation (Sec. II, p-block; Sec. III-E, distributed
circuits): the state is kept as a list of blocks, each an ascending qubit list
and a complex128 state vector of those qubits (bit j of a block's index is its
j-th smallest qubit). Every qubit starts in a block of its own; a gate whose
qubits lie in several blocks first replaces them by their tensor product
(numpy.kron, then the index bits put in ascending qubit order); a
measured or reset qubit leaves its block, since the projected state is the
qubit's basis state times the rest. Gates, probabilities and projections are
the full-state oracle's routines applied to a block. Only the tests, the
smoke check and the benchmark's CPU-baseline leg use this module.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def _ascending(qs, psi):
    """The same state with its index bits reordered so that bit j is the j-th
    smallest qubit (bit j of psi's index is qubit qs[j] on entry)."""
    nb = len(qs)
    order = sorted(qs)
    t = psi.reshape([2] * nb)                    # axis a <-> bit nb-1-a
    axes = [nb - 1 - qs.index(order[nb - 1 - a]) for a in range(nb)]
    return order, np.ascontiguousarray(np.transpose(t, axes).reshape(-1))


class PBlockState:
    def __init__(self, n: int):
        self.n = n
        self.blocks = [([q], O.basis_state(1, 0)) for q in range(n)]

    def _find(self, q):
        for i, (qs, _) in enumerate(self.blocks):
            if q in qs:
                return i
        raise ValueError(q)

    def _merge(self, qubits):
        """Replace the blocks holding `qubits` by their tensor product; returns its index."""
        idx = []
        for q in qubits:
            i = self._find(q)
            if i not in idx:
                idx.append(i)
        if len(idx) == 1:
            return idx[0]
        qs, psi = self.blocks[idx[0]]
        for i in idx[1:]:
            qb, pb = self.blocks[i]
            # kron(pb, psi)[ib * 2^len(qs) + ia] = pb[ib] * psi[ia]: qs stay the low bits
            psi = np.kron(pb, psi)
            qs = qs + qb
        qs, psi = _ascending(qs, psi)
        keep = [b for i, b in enumerate(self.blocks) if i not in idx]
        self.blocks = keep + [(qs, psi)]
        return len(self.blocks) - 1

    def gate(self, op):
        i = self._merge(list(op[1]))
        qs, psi = self.blocks[i]
        local = tuple(qs.index(q) for q in op[1])
        O.apply_op(psi, (op[0], local, op[2]), adjoint=bool(len(op) > 3 and op[3]))

    def measure(self, q, u, reset=False):
        """Draw u decides the outcome (1 exactly when u*(p0+p1) >= p0); returns it."""
        i = self._find(q)
        qs, psi = self.blocks[i]
        j = qs.index(q)
        p0, p1 = O.qubit_probs(psi, j)
        m = 1 if u * (p0 + p1) >= p0 else 0
        O.collapse(psi, j, m, p1 if m else p0, reset=reset)
        if len(qs) > 1:
            keep = 0 if reset else m      # bit value that holds the amplitudes now
            nb = len(qs)
            rest = np.ascontiguousarray(psi.reshape(1 << (nb - 1 - j), 2, 1 << j)[:, keep, :].reshape(-1))
            single = O.basis_state(1, 0 if reset else m)
            self.blocks[i] = ([x for x in qs if x != q], rest)
            self.blocks.append(([q], single))
        return m

    def ordered(self):
        """Blocks in partition order (by smallest qubit)."""
        return sorted(self.blocks, key=lambda b: min(b[0]))

    def partition(self):
        out = np.zeros(self.n, dtype=np.int32)
        for b, (qs, _) in enumerate(self.ordered()):
            out[qs] = b
        return out

    def amplitude(self, i: int) -> complex:
        a = complex(1.0)
        for qs, psi in self.ordered():
            loc = sum(((i >> q) & 1) << j for j, q in enumerate(qs))
            a *= complex(psi[loc])
        return a

    def full_state(self) -> np.ndarray:
        """The tensor product of all blocks as one vector (small n only)."""
        out = np.ones(1, dtype=np.complex128)
        order = []
        for qs, psi in self.blocks:
            out = np.kron(psi, out)
            order = order + qs
        return _ascending(order, out)[1]

    def sample(self, shots: int, seed: int):
        """Block b (partition order) draws shot s at counter b*shots + s; the
        shot's bits are the union of the blocks' bits. Python ints."""
        out = [0] * shots
        for b, (qs, psi) in enumerate(self.ordered()):
            loc = O.sample_at(psi, b * shots + np.arange(shots, dtype=np.uint64), seed)
            for s in range(shots):
                v = int(loc[s])
                for j, q in enumerate(qs):
                    if (v >> j) & 1:
                        out[s] |= 1 << q
        return out

    def expect(self, xmask: int, zmask: int) -> float:
        """<P> on the product state: the product of each block's <P_b>."""
        val = 1.0
        for qs, psi in self.blocks:
            xl = sum(((xmask >> q) & 1) << j for j, q in enumerate(qs))
            zl = sum(((zmask >> q) & 1) << j for j, q in enumerate(qs))
            if xl or zl:
                val *= O.expect(psi, xl, zl).real
        return val

    def state_bytes(self, itemsize: int = 16) -> int:
        return sum(psi.size * itemsize for _, psi in self.blocks)


def run(ops, n: int, seed: int = 0, state: PBlockState | None = None, clbits: int = 0):
    """Run ops on a p-block state: the k-th measure/reset of the call draws
    u = U01(seed, k). Returns (clbits, state)."""
    st = PBlockState(n) if state is None else state
    k = 0
    for op in ops:
        if op[0] in ("measure", "reset"):
            m = st.measure(int(op[1][0]), O.u01(seed, k), reset=(op[0] == "reset"))
            if op[0] == "measure":
                b = 1 << int(op[1][1])
                clbits = (clbits | b) if m else (clbits & ~b)
            k += 1
        elif O.cond_met(op, clbits):
            st.gate(op)
    return clbits, st
