"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This package holds gate LISTS only (gate name, qubit indices, angles) and
seeded random draws. It contains no gate matrix, no amplitude arithmetic and
no sampling or reduction code: the oracle and the HIP path each turn these
lists into numbers with their own code.
"""
from .circuits import (  # noqa: F401
    GATES_1Q,
    GATES_2Q,
    GATES_3Q,
    brickwork,
    ghz,
    qft,
    random_basis_state,
    random_regular_graph,
    qaoa_maxcut,
    random_circuit,
    serving_circuit,
    serving_stream,
    poisson_arrivals,
    circuit_gate_count,
    random_state,
    random_unitary,
    random_paulis,
    c_if,
    remote_cx,
    dqc,
)
