"""The Gaussian-weighted Ising QAOA p=1 workload on five graph families
(the paper's timing workload): graph shapes, the gate list, and the host
plans' step programs against the state vector."""
import math

import numpy as np
import pytest

import instances as I
from oracle import statevector as SV

from .test_plan_host import _prefix_check, _plan


@pytest.mark.parametrize("topology", I.ISING_TOPOLOGIES)
def test_graph_families(topology):
    for n in (16, 100, 476):
        if topology == "3reg" and n > 100:
            continue
        nn, edges = I.ising_graph(topology, n)
        assert abs(nn - n) <= max(4, n // 10)
        deg = np.zeros(nn, dtype=int)
        for u, v in edges:
            assert 0 <= u < v < nn
            deg[u] += 1
            deg[v] += 1
        assert len(set(edges)) == len(edges) and deg.min() >= 1
        cap = {"grid": 4, "heavy_hex": 3, "kings": 8, "chimera": 6, "3reg": 3}[topology]
        assert deg.max() <= cap
        if topology == "3reg":
            assert np.all(deg == 3)


def test_heavy_hex_structure():
    """Two lines of L qubits, bridges of degree 2 every fourth column."""
    n, edges = I.heavy_hex_graph(2, 9)
    deg = np.bincount(np.array(edges).ravel(), minlength=n)
    assert n == 2 * 9 + 3 and np.sum(deg == 2) >= 3
    assert len(edges) == 2 * 8 + 2 * 3


def test_chimera_cells():
    """One K_{4,4} cell: 16 edges; two cells side by side add 4 couplers;
    a 2 x 2 block adds 4 between each neighbouring pair (4 pairs)."""
    assert len(I.chimera_graph(1, 1)) == 16
    assert len(I.chimera_graph(1, 2)) == 2 * 16 + 4
    assert len(I.chimera_graph(2, 2)) == 4 * 16 + 2 * 4 + 2 * 4


def test_ising_gate_list():
    """RZZ(2 gamma J_ij) per edge, RZ(2 gamma h_i) per qubit, RX(2 beta)."""
    c = I.ising_qaoa_p1("grid", 16, 3)
    kinds = [g.kind for g in c.gates]
    n = c.n_qubits
    assert kinds[:n] == ["H"] * n and kinds[-n:] == ["RX"] * n
    assert kinds.count("RZZ") == len(c.edges) and kinds.count("RZ") == n
    rx = [g for g in c.gates if g.kind == "RX"]
    assert all(g.coeff == 2.0 and g.param == 1 for g in rx)
    assert len(c.theta) == 2 and all(0 <= t <= math.pi for t in c.theta)
    # another instance has other couplings
    c2 = I.ising_qaoa_p1("grid", 16, 4)
    assert [g.coeff for g in c.gates if g.kind == "RZZ"] != [g.coeff for g in c2.gates if g.kind == "RZZ"]


@pytest.mark.parametrize("topology", I.ISING_TOPOLOGIES)
def test_ising_step_programs_match_state_vector(topology):
    c = I.ising_qaoa_p1(topology, 14)
    assert c.n_qubits <= 16
    p = _plan(c)
    assert _prefix_check(c, p, np.random.default_rng(5), n_states=3) < 1e-12
    # and the dense runs of a BF16x3 plan hold the same products (in double)
    pb = _plan(c, precision="bf16x3")
    assert any(pb.export(k)["dense"] is not None for k in range(pb.n_steps()))
