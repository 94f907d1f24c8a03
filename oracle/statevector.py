"""Dense complex128 state vectors and density matrices.

The state after the first t gates is psi_t = U_t ... U_1 |0^n> (Section 2);
amp(C_t, i) = <i|C_t|0^n> is an entry of it.  The noisy output distribution
is diag(rho_T) where rho evolves by U rho U^dag for gates and by
sum_i E_i rho E_i^dag for a channel (Section 3).

Index convention: basis index x has qubit k in bit k (little-endian).  A gate
on (q0, q1) uses local index 2*b(q0) + b(q1).

Pinned by ``tests/test_oracle_statevector.py`` against full 2^n x 2^n
operators built by Kronecker products (brute force, tiny n).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import gates as G


def _axes(n: int, qubits: Sequence[int]):
    # C-order reshape to (2,)*n puts qubit n-1 on axis 0.
    return [n - 1 - q for q in qubits]


def apply_gate(psi: np.ndarray, n: int, mat: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """psi <- (mat on qubits) psi.  psi may carry a leading batch axis (B, 2^n)."""
    m = len(qubits)
    batched = psi.ndim == 2
    B = psi.shape[0] if batched else 1
    t = psi.reshape((B,) + (2,) * n)
    ax = [1 + a for a in _axes(n, qubits)]
    # move gate axes to the front (q0 first = most significant local bit)
    t = np.moveaxis(t, ax, list(range(1, m + 1)))
    shp = t.shape
    t = t.reshape(B, 2 ** m, -1)
    t = np.einsum("ij,bjk->bik", mat, t)
    t = t.reshape(shp)
    t = np.moveaxis(t, list(range(1, m + 1)), ax)
    out = t.reshape(B, 2 ** n)
    return out if batched else out[0]


def apply_gate_per_batch(psi: np.ndarray, n: int, mats: np.ndarray, qubits) -> np.ndarray:
    """Different matrix per batch row: mats (B, d, d)."""
    m = len(qubits)
    B = psi.shape[0]
    t = psi.reshape((B,) + (2,) * n)
    ax = [1 + a for a in _axes(n, qubits)]
    t = np.moveaxis(t, ax, list(range(1, m + 1)))
    shp = t.shape
    t = t.reshape(B, 2 ** m, -1)
    t = np.einsum("bij,bjk->bik", mats, t)
    t = t.reshape(shp)
    t = np.moveaxis(t, list(range(1, m + 1)), ax)
    return t.reshape(B, 2 ** n)


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def state(circ, t: int | None = None) -> np.ndarray:
    """psi_t for the first t gates of the (noise-free) gate list."""
    n = circ.n_qubits
    psi = zero_state(n)
    gl = circ.gates if t is None else circ.gates[:t]
    for g in gl:
        psi = apply_gate(psi, n, G.gate_matrix(circ, g), g.qubits)
    return psi


def full_operator(n: int, mat: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """The 2^n x 2^n operator of a gate, by brute force over basis states."""
    d = 2 ** n
    m = len(qubits)
    U = np.zeros((d, d), dtype=np.complex128)
    for x in range(d):
        loc_in = 0
        for q in qubits:
            loc_in = 2 * loc_in + ((x >> q) & 1)
        for loc_out in range(2 ** m):
            a = mat[loc_out, loc_in]
            if a == 0:
                continue
            y = x
            for j, q in enumerate(qubits):
                bit = (loc_out >> (m - 1 - j)) & 1
                y = (y & ~(1 << q)) | (bit << q)
            U[y, x] += a
    return U


# ---------------------------------------------------------------- density matrix

def apply_gate_dm(rho: np.ndarray, n: int, mat: np.ndarray, qubits) -> np.ndarray:
    """rho <- U rho U^dag using the vector routine on rows and columns."""
    r = apply_gate(rho.T.copy(), n, mat, qubits).T          # U acting on the row index
    r = apply_gate(r.conj(), n, mat, qubits).conj()         # (U r^* ...)^*: U^dag on columns
    return r


def apply_channel_dm(rho: np.ndarray, n: int, kraus, qubits) -> np.ndarray:
    out = np.zeros_like(rho)
    for E in kraus:
        out += apply_gate_dm(rho, n, E, qubits)
    return out


def density_matrix(circ) -> np.ndarray:
    """rho_T of the noisy circuit (gates and channels in execution order)."""
    n = circ.n_qubits
    rho = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    rho[0, 0] = 1.0
    for kind, idx in circ.ops():
        if kind == "gate":
            g = circ.gates[idx]
            rho = apply_gate_dm(rho, n, G.gate_matrix(circ, g), g.qubits)
        else:
            s = circ.noise[idx]
            rho = apply_channel_dm(rho, n, G.kraus_full(s), s.qubits)
    return rho
