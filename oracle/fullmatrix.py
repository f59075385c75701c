"""TEST INFRASTRUCTURE ONLY -- brute-force full-unitary construction (n <= 8).

An independent check of the oracle's gate indexing: a k-qubit matrix is
embedded into the full 2^n x 2^n operator by the textbook tensor-product
construction (G (x) I on a virtual qubit order, then an axis permutation to the
real order), with no bit-insertion enumeration anywhere. Qubit q is bit q of
the index; bit j of G's row/column index belongs to qubits[j].
"""
from __future__ import annotations

import numpy as np


def controlled(U: np.ndarray, ncontrols: int) -> np.ndarray:
    """The 2^(k+c) matrix acting as U on the low k bits when all c high
    (control) bits are 1, and as the identity otherwise."""
    K = U.shape[0]
    D = K << ncontrols
    G = np.eye(D, dtype=np.complex128)
    G[D - K:, D - K:] = U
    return G


def embed(G: np.ndarray, qubits, n: int) -> np.ndarray:
    """Full 2^n x 2^n operator of G acting on `qubits` (bit j of G <-> qubits[j])."""
    qubits = [int(q) for q in qubits]
    m = len(qubits)
    if len(set(qubits)) != m or any(q < 0 or q >= n for q in qubits):
        raise ValueError("bad qubits")
    rest = [q for q in range(n) if q not in qubits]
    # virtual order: virtual bit v is qubits[v] for v < m, rest[v-m] after.
    # np.kron(A, B) makes B's index the fast (low) one, so G sits on the low bits.
    Fv = np.kron(np.eye(1 << (n - m), dtype=np.complex128), np.asarray(G, dtype=np.complex128))
    perm = qubits + rest                      # virtual bit -> real qubit
    virt_of = {q: v for v, q in enumerate(perm)}
    T = Fv.reshape((2,) * (2 * n))            # axis a <-> bit n-1-a (row axes, then column axes)
    axes = [0] * (2 * n)
    for q in range(n):
        axes[n - 1 - q] = n - 1 - virt_of[q]
        axes[n + n - 1 - q] = n + n - 1 - virt_of[q]
    return np.transpose(T, axes).reshape(1 << n, 1 << n)


def gate_full(U: np.ndarray, targets, controls, n: int) -> np.ndarray:
    return embed(controlled(np.asarray(U), len(controls)), list(targets) + list(controls), n)


def circuit_unitary(ops, n: int, matrix_of) -> np.ndarray:
    """Product of embedded gates, last gate leftmost. `matrix_of(name, params)`
    returns (U, k, ncontrols) with the op's qubits ordered controls first."""
    W = np.eye(1 << n, dtype=np.complex128)
    for name, qubits, params in ops:
        U, k, nc = matrix_of(name, params)
        W = gate_full(U, qubits[nc:], qubits[:nc], n) @ W
    return W
