"""State vector and density matrix against brute-force full operators."""
import numpy as np
import pytest

from instances import Circuit, Gate, NoiseSite, add_qaoa_noise, qaoa_maxcut, random_regular_graph
from oracle import gates as G
from oracle import statevector as SV


def _rand_unitary(d, rng):
    z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def test_apply_gate_matches_full_operator():
    rng = np.random.default_rng(3)
    n = 4
    psi = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
    for qubits in [(0,), (3,), (0, 1), (2, 0), (3, 1), (1, 3)]:
        U = _rand_unitary(2 ** len(qubits), rng)
        ref = SV.full_operator(n, U, qubits) @ psi
        assert np.allclose(SV.apply_gate(psi, n, U, qubits), ref)


def test_full_operator_bit_convention():
    # X on qubit 2 maps |0> to basis index 4; CNOT(0->1) maps |q0=1> (index 1) to index 3
    n = 3
    X = SV.full_operator(n, G.PX, (2,))
    assert X[4, 0] == 1
    c = Circuit(n, [], np.zeros(0))
    cn = SV.full_operator(n, G.gate_matrix(c, Gate("CNOT", (0, 1))), (0, 1))
    assert cn[3, 1] == 1 and cn[0, 0] == 1


def test_state_norm_and_circuit():
    edges = random_regular_graph(3, 8, 5)
    c = qaoa_maxcut(8, edges, [0.4], [1.1])
    psi = SV.state(c)
    assert abs(np.vdot(psi, psi) - 1) < 1e-12
    # product of full operators equals the gate-by-gate state
    U = np.eye(2 ** 8, dtype=complex)
    for g in c.gates:
        U = SV.full_operator(8, G.gate_matrix(c, g), g.qubits) @ U
    assert np.allclose(U[:, 0], psi)


def test_density_matrix_noiseless_is_pure():
    edges = random_regular_graph(3, 6, 9)
    c = qaoa_maxcut(6, edges, [0.7], [0.3])
    psi = SV.state(c)
    rho = SV.density_matrix(c)
    assert np.allclose(rho, np.outer(psi, psi.conj()))


def test_density_matrix_channel_against_kraus_sum():
    rng = np.random.default_rng(4)
    n = 3
    a = rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))
    rho = a @ a.conj().T
    rho /= np.trace(rho)
    for site in [NoiseSite(0, "DEPOL2", (2, 0), (0.1,)), NoiseSite(0, "AMPDAMP", (1,), (0.3,))]:
        out = SV.apply_channel_dm(rho, n, G.kraus_full(site), site.qubits)
        ref = np.zeros_like(rho)
        for E in G.kraus_full(site):
            F = SV.full_operator(n, E, site.qubits)
            ref += F @ rho @ F.conj().T
        assert np.allclose(out, ref)
        assert abs(np.trace(out) - 1) < 1e-12


def test_noisy_density_matrix_is_state():
    edges = random_regular_graph(3, 6, 11)
    c = add_qaoa_noise(qaoa_maxcut(6, edges, [0.5, 1.0], [0.9, 0.2]), depol2=0.05, ampdamp=0.05)
    rho = SV.density_matrix(c)
    assert abs(np.trace(rho) - 1) < 1e-12
    assert np.allclose(rho, rho.conj().T)
    assert np.linalg.eigvalsh(rho).min() > -1e-12
