"""State-vector gradients for score-function QAOA training.

For p_theta(x) = |<x|C(theta)|0>|^2 and a cost C(x):

* exact objective gradient by the adjoint method (Jones & Gacon, 2020):
  with phi_k = U_k..U_1|0>, lambda = H_C |psi_T> pulled back through the
  gates, dE/dtheta_j = sum_{k tied to j} 2 Re <lambda_k| dU_k |phi_{k-1}>;
* per-sample score d log p(x) / d theta_j = 2 Re(conj(psi(x)) d_j psi(x)) / |psi(x)|^2
  with d_j psi by forward-mode differentiation through the gates;
* central finite differences of log p in FP64 (test support).

The score-function identity grad E[C] = E[C grad log p] links the two and is
checked statistically in the tests.
"""
from __future__ import annotations

import numpy as np

from . import gates as G
from . import statevector as SV


def _gate_terms(circ):
    for g in circ.gates:
        yield g, G.gate_matrix(circ, g)


def objective_and_gradient(circ, cost: np.ndarray):
    """E = <psi|diag(cost)|psi> and dE/dtheta (adjoint method)."""
    n = circ.n_qubits
    phis = [SV.zero_state(n)]
    mats = []
    for g in circ.gates:
        m = G.gate_matrix(circ, g)
        mats.append(m)
        phis.append(SV.apply_gate(phis[-1], n, m, g.qubits))
    psi = phis[-1]
    E = float(np.real(np.vdot(psi, cost * psi)))
    lam = cost * psi
    grad = np.zeros(len(circ.theta))
    for k in range(len(circ.gates) - 1, -1, -1):
        g = circ.gates[k]
        if g.param >= 0:
            dU = G.gate_matrix_derivative(circ, g) * g.coeff
            v = SV.apply_gate(phis[k], n, dU, g.qubits)
            grad[g.param] += 2.0 * np.real(np.vdot(lam, v))
        lam = SV.apply_gate(lam, n, mats[k].conj().T, g.qubits)
    return E, grad


def state_and_derivatives(circ):
    """psi_T and d psi_T / d theta_j for all j (forward mode)."""
    n = circ.n_qubits
    P = len(circ.theta)
    psi = SV.zero_state(n)
    d = np.zeros((P, 2 ** n), dtype=np.complex128)
    for g in circ.gates:
        m = G.gate_matrix(circ, g)
        d = SV.apply_gate(d, n, m, g.qubits)
        if g.param >= 0:
            dU = G.gate_matrix_derivative(circ, g) * g.coeff
            d[g.param] += SV.apply_gate(psi, n, dU, g.qubits)
        psi = SV.apply_gate(psi, n, m, g.qubits)
    return psi, d


def score(circ, idx: np.ndarray) -> np.ndarray:
    """d log p(x) / d theta for basis indices idx: (len(idx), P)."""
    psi, d = state_and_derivatives(circ)
    a = psi[idx]
    da = d[:, idx].T
    return 2.0 * np.real(np.conj(a)[:, None] * da) / (np.abs(a) ** 2)[:, None]


def score_fd(circ, idx: np.ndarray, h: float = 1e-4) -> np.ndarray:
    """Central finite differences of log p(x) in FP64."""
    P = len(circ.theta)
    out = np.zeros((len(idx), P))
    for j in range(P):
        tp = circ.theta.copy()
        tp[j] += h
        tm = circ.theta.copy()
        tm[j] -= h
        pp = np.abs(SV.state(circ.with_theta(tp))[idx]) ** 2
        pm = np.abs(SV.state(circ.with_theta(tm))[idx]) ** 2
        out[:, j] = (np.log(pp) - np.log(pm)) / (2 * h)
    return out


def log_amp_gradient_pathsum(circ, y, h: float = 1e-4):
    """d log|amp(C, y)|^2 / d theta by central differences of path-sum
    amplitudes (for qubit counts beyond the state vector)."""
    from . import pathsum
    P = len(circ.theta)
    out = np.zeros(P)
    for j in range(P):
        tp = circ.theta.copy()
        tp[j] += h
        tm = circ.theta.copy()
        tm[j] -= h
        ap = pathsum.amplitude(circ.with_theta(tp), len(circ.gates), y)
        am = pathsum.amplitude(circ.with_theta(tm), len(circ.gates), y)
        out[j] = (np.log(abs(ap) ** 2) - np.log(abs(am) ** 2)) / (2 * h)
    return out
