"""Gate matrices, block structure and Kraus lists of the oracle."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from instances import Circuit, Gate, NoiseSite
from oracle import gates as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig1_gates.json")


def _circ(theta=(0.7, 1.9)):
    return Circuit(n_qubits=2, gates=[], theta=np.array(theta))


def test_rotations_match_matrix_exponential():
    c = _circ()
    for kind, P in [("RX", G.PX), ("RZ", G.PZ), ("RZZ", np.kron(G.PZ, G.PZ))]:
        q = (0, 1) if kind == "RZZ" else (0,)
        g = Gate(kind, q, param=0, coeff=1.3, offset=0.2)
        t = 1.3 * 0.7 + 0.2
        ref = scipy.linalg.expm(-0.5j * t * P)
        assert np.allclose(G.gate_matrix(c, g), ref, atol=1e-14)


def test_special_values():
    c = _circ((math.pi,))
    assert np.allclose(G.gate_matrix(c, Gate("RX", (0,), param=0)), -1j * G.PX)
    h = G.gate_matrix(c, Gate("H", (0,)))
    assert np.allclose(h @ h, np.eye(2))
    # RZZ(pi) = -i Z(x)Z, a Pauli product (used by closed-form checks at any n)
    assert np.allclose(G.gate_matrix(c, Gate("RZZ", (0, 1), param=0)), -1j * np.kron(G.PZ, G.PZ))


def test_derivatives_by_finite_differences():
    for kind, q in [("RX", (0,)), ("RZ", (0,)), ("RZZ", (0, 1)), ("CRX", (0, 1))]:
        g = Gate(kind, q, param=0)
        h = 1e-6
        dp = G.gate_matrix(_circ((0.9 + h,)), g)
        dm = G.gate_matrix(_circ((0.9 - h,)), g)
        assert np.allclose(G.gate_matrix_derivative(_circ((0.9,)), g), (dp - dm) / (2 * h), atol=1e-8)


def test_figure1_block_structure():
    fx = json.load(open(GOLDEN))["gates"]
    c = _circ((0.8, 0.3))
    iswap = np.array([[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]])
    mats = {
        "CNOT": G.gate_matrix(c, Gate("CNOT", (0, 1))),
        "iSWAP": G.gate_matrix(c, Gate("U2", (0, 1), matrix=tuple(iswap.ravel()))),
        "CRX": G.gate_matrix(c, Gate("CRX", (0, 1), param=0)),
        "FSIM": G.gate_matrix(c, Gate("FSIM", (0, 1), param=0, param2=1)),
    }
    for name, spec in fx.items():
        m = mats[name]
        nz = sorted(map(list, zip(*np.nonzero(m))))
        assert nz == sorted(spec["nonzero"]), name
        assert G.is_monomial(m) == spec["monomial"], name
        if "blocks" in spec:
            for blk in spec["blocks"]:
                for loc in blk:
                    assert G.block_decompose(m, loc) == blk, (name, loc)
        assert np.allclose(m.conj().T @ m, np.eye(4))


def test_monomial_permutation():
    c = _circ()
    m = G.gate_matrix(c, Gate("CNOT", (0, 1)))
    sig = G.monomial_permutation(m)
    assert list(sig) == [0, 1, 3, 2]
    assert not G.is_monomial(G.gate_matrix(c, Gate("RX", (0,), param=0)))
    assert G.is_diagonal(G.gate_matrix(c, Gate("RZZ", (0, 1), param=0)))


def test_propagate_x_identity():
    """Figure 5(b): an X propagated through a diagonal gate G gives the diagonal
    gate with its entries permuted: (X G X)[k,k] = G[1-k,1-k]."""
    d = np.diag([0.3 + 0.1j, -0.7j])
    xdx = G.conjugate_by_frame(d, (1,))
    assert np.allclose(np.diag(xdx), [d[1, 1], d[0, 0]])
    assert G.is_diagonal(xdx)
    # RZZ conjugated on one qubit flips the angle sign; on both, unchanged
    c = _circ((1.1,))
    rzz = G.gate_matrix(c, Gate("RZZ", (0, 1), param=0))
    rzzm = G.gate_matrix(_circ((-1.1,)), Gate("RZZ", (0, 1), param=0))
    assert np.allclose(G.conjugate_by_frame(rzz, (1, 0)), rzzm)
    assert np.allclose(G.conjugate_by_frame(rzz, (1, 1)), rzz)
    rx = G.gate_matrix(c, Gate("RX", (0,), param=0))
    assert np.allclose(G.conjugate_by_frame(rx, (1,)), rx)


@pytest.mark.parametrize("site", [
    NoiseSite(0, "DEPOL1", (0,), (0.03,)),
    NoiseSite(0, "DEPOL2", (0, 1), (0.05,)),
    NoiseSite(0, "AMPDAMP", (0,), (0.2,)),
    NoiseSite(0, "PHASEDAMP", (0,), (0.3,)),
    NoiseSite(0, "PAULI1", (0,), (0.01, 0.02, 0.05)),
])
def test_kraus_completeness_and_lsm(site):
    ks = G.kraus_full(site)
    d = ks[0].shape[0]
    assert np.allclose(sum(E.conj().T @ E for E in ks), np.eye(d))
    for fs in G.kraus_factors(site):
        for f in fs:
            nz = f != 0
            assert nz.sum(axis=0).max() <= 1 and nz.sum(axis=1).max() <= 1   # submonomial
    m = len(site.qubits)
    for t in range(2 ** m):
        bits = tuple((t >> (m - 1 - j)) & 1 for j in range(m))
        pr = G.branch_probabilities(G.kraus_factors(site), bits)
        assert abs(sum(pr) - 1.0) < 1e-14
        # Eq. (4) against <t|E^dag E|t> with the full operators
        for E, p in zip(ks, pr):
            assert abs(np.real((E.conj().T @ E)[t, t]) - p) < 1e-15


def test_amplitude_damping_textbook_values():
    site = NoiseSite(0, "AMPDAMP", (0,), (0.2,))
    # Pr(E1 | 1) = gamma, Pr(E1 | 0) = 0
    assert G.branch_probabilities(G.kraus_factors(site), (1,)) == pytest.approx([0.8, 0.2])
    assert G.branch_probabilities(G.kraus_factors(site), (0,)) == pytest.approx([1.0, 0.0])
