"""Circuits beyond QAOA on the host: CRX / fSim / CNOT / CZ / XX+YY /
Haar-random two-qubit gates (blocks {00},{01},{10,11} and {00},{01,10},{11},
four-element blocks, |S| = 2 candidate sets) and Trotterised Heisenberg and
transverse-field Ising chains: every step program, in the vector sweep form
and as BF16x3 dense runs, against the state vector."""
import numpy as np
import pytest

import instances as I
from oracle import gates as G
from oracle import statevector as SV

from . import plan_exec as X

E = pytest.importorskip("paper_2510_24218_amd")


def open_qubits(c, g):
    """The gate's non-diagonal qubits (first listed = most significant bit of
    the candidate index)."""
    mat = G.gate_matrix(c, g)
    nq = len(g.qubits)
    return [g.qubits[j] for j in range(nq)
            if not all(mat[o, i] == 0 for o in range(2 ** nq) for i in range(2 ** nq)
                       if ((o >> (nq - 1 - j)) & 1) != ((i >> (nq - 1 - j)) & 1))]


def reachable(c, gate, rng):
    s = rng.integers(0, 2, c.n_qubits)
    touched = {q for g in c.gates[:gate + 1] for q in g.qubits}
    for q in range(c.n_qubits):
        if q not in touched:
            s[q] = 0
    return s


def candidate_refs(c, gate, s, psi):
    opn = open_qubits(c, c.gates[gate])
    ref = []
    for v in range(2 ** len(opn)):
        y = s.copy()
        for kk, q in enumerate(opn):
            y[q] = (v >> (len(opn) - 1 - kk)) & 1
        ref.append(psi[sum(int(y[j]) << j for j in range(c.n_qubits))])
    return np.array(ref)


CIRCUITS = {"general": lambda: I.general_gate_circuit(), "heisenberg": lambda: I.trotter_heisenberg(),
            "tfim": lambda: I.trotter_tfim()}


@pytest.mark.parametrize("name", list(CIRCUITS))
def test_step_programs_beyond_qaoa(name):
    c = CIRCUITS[name]()
    p = E.Plan(c, host_only=True)
    pb = E.Plan(c, precision="bf16x3", host_only=True)
    rng = np.random.default_rng(6)
    sizes = set()
    for k in range(p.n_steps()):
        op, gate, m = p.step_info(k)
        psi = SV.state(c, gate + 1)
        ex, exb = p.export(k), pb.export(k)
        for _ in range(3):
            s = reachable(c, gate, rng)
            ref = candidate_refs(c, gate, s, psi)
            sizes.add(len(ref))
            got = X.eval_step(ex, s, plan=p)
            assert np.allclose(got, ref, atol=1e-13), (k, got, ref)
            if exb["dense"] is not None and exb["dense"]["op0"] == 0:
                gd = X.dense_step(exb, s, plan=pb)
                assert np.linalg.norm(gd - ref) <= 2e-4 * max(np.linalg.norm(ref), 1e-300)
    if name != "tfim":
        assert 4 in sizes     # two-qubit candidate sets are exercised
