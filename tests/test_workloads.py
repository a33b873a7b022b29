"""The seeded workload generators produce the shapes the benchmark quotes
(no GPU): qubit counts, T counts, measurement counts and determinism."""
from __future__ import annotations

import workloads


def test_cultivation_42q_shape():
    w = workloads.config("cultivation_42q", seed=1)
    st = workloads.circuit_stats(w.text)
    assert st["qubits"] == 42 and st["t_count"] == 72 and st["t_support"] == 19
    assert st["measurements"] == 93
    assert 450 <= st["two_qubit_gates"] <= 650
    assert w.meta["r_z"] == 9 and w.meta["r_x"] == 9


def test_cultivation_15q_shape():
    st = workloads.circuit_stats(workloads.config("cultivation_15q", seed=1).text)
    assert st["qubits"] == 15 and st["t_count"] == 28 and st["t_support"] == 7


def test_clifford_t_8q_shape():
    w = workloads.config("clifford_t_8q", seed=1)
    st = workloads.circuit_stats(w.text)
    assert st["qubits"] == 8 and st["t_count"] == 6 and st["measurements"] == 8
    assert st["gates"] == 214
    assert w.text.count("DETECTOR") == 4
    assert w.noise == {"p1": 1e-3, "p2": 1e-3}


def test_generators_are_deterministic():
    for name in ("clifford_t_8q", "cultivation_15q", "cultivation_42q"):
        assert workloads.config(name, seed=5).text == workloads.config(name, seed=5).text
        assert workloads.config(name, seed=5).text != workloads.config(name, seed=6).text
