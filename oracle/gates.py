"""Gate matrices, Kraus lists and the structural predicates of the paper.

* Rotations use R_P(t) = exp(-i t P / 2) (appendix on QAOA).
* Monomial = exactly one non-zero per row and column (Section 2, before
  Proposition 1); diagonal = all off-diagonal entries zero.
* BlockDecompose (Algorithm 1): connected components of the graph on local
  basis states with an edge {x, y} whenever A[x, y] != 0.
* Kraus operators of the local-submonomial channels (Section 3 and
  Appendix A): depolarizing, amplitude damping (Nielsen & Chuang 8.3.5),
  phase damping and unequal Pauli noise, each given as a list of
  per-qubit 2x2 factors (E_i = factor_0 (x) factor_1 ...).

Matrices are indexed [out, in]; a two-qubit gate on (q0, q1) uses local
index 2*b(q0) + b(q1).
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULIS = (I2, PX, PY, PZ)


def rotation(pauli: np.ndarray, t: float) -> np.ndarray:
    """exp(-i t P / 2) for a Pauli product P (P^2 = I)."""
    d = pauli.shape[0]
    return math.cos(t / 2) * np.eye(d, dtype=np.complex128) - 1j * math.sin(t / 2) * pauli


def gate_matrix(circ, g) -> np.ndarray:
    k = g.kind
    if k == "H":
        return np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
    if k == "X":
        return PX.copy()
    if k == "RX":
        return rotation(PX, circ.angle(g))
    if k == "RZ":
        return rotation(PZ, circ.angle(g))
    if k == "RZZ":
        return rotation(np.kron(PZ, PZ), circ.angle(g))
    if k == "CNOT":
        m = np.zeros((4, 4), dtype=np.complex128)
        for b0 in range(2):
            for b1 in range(2):
                m[2 * b0 + (b1 ^ b0), 2 * b0 + b1] = 1
        return m
    if k == "CZ":
        return np.diag([1, 1, 1, -1]).astype(np.complex128)
    if k == "CRX":
        m = np.zeros((4, 4), dtype=np.complex128)
        m[:2, :2] = I2
        m[2:, 2:] = rotation(PX, circ.angle(g))
        return m
    if k == "FSIM":
        th, ph = circ.angle(g), circ.angle2(g)
        m = np.zeros((4, 4), dtype=np.complex128)
        m[0, 0] = 1
        m[1, 1] = m[2, 2] = math.cos(th)
        m[1, 2] = m[2, 1] = -1j * math.sin(th)
        m[3, 3] = np.exp(1j * ph)       # Figure 1(c) convention
        return m
    if k in ("U1", "U2"):
        d = 2 if k == "U1" else 4
        return np.array(g.matrix, dtype=np.complex128).reshape(d, d)
    raise ValueError(f"unknown gate kind {k}")


def gate_matrix_derivative(circ, g) -> np.ndarray:
    """d(gate)/d(angle) for the single-angle rotations (times nothing: the
    caller multiplies by d(angle)/d(theta) = coeff)."""
    t = circ.angle(g)
    k = g.kind
    if k == "RX":
        return -0.5j * PX @ rotation(PX, t)
    if k == "RZ":
        return -0.5j * PZ @ rotation(PZ, t)
    if k == "RZZ":
        zz = np.kron(PZ, PZ)
        return -0.5j * zz @ rotation(zz, t)
    if k == "CRX":
        m = np.zeros((4, 4), dtype=np.complex128)
        m[2:, 2:] = -0.5j * PX @ rotation(PX, t)
        return m
    raise ValueError(f"no derivative for {k}")


def is_diagonal(a: np.ndarray) -> bool:
    return bool(np.all(a[~np.eye(a.shape[0], dtype=bool)] == 0))


def is_monomial(a: np.ndarray) -> bool:
    nz = a != 0
    return bool(np.all(nz.sum(axis=0) == 1) and np.all(nz.sum(axis=1) == 1))


def monomial_permutation(a: np.ndarray) -> np.ndarray:
    """sigma with A[sigma(x), x] != 0 (the image of basis state x)."""
    return np.argmax(a != 0, axis=0)


def block_decompose(a: np.ndarray, local: int) -> List[int]:
    """Connected component of ``local`` in the graph {x,y}: A[x,y] != 0 (ascending)."""
    d = a.shape[0]
    adj = (a != 0) | (a.T != 0)
    seen = {local}
    stack = [local]
    while stack:
        x = stack.pop()
        for y in range(d):
            if adj[x, y] and y not in seen:
                seen.add(y)
                stack.append(y)
    return sorted(seen)


def conjugate_by_frame(a: np.ndarray, frame_bits: Tuple[int, ...]) -> np.ndarray:
    """PropagateX: X_q A X_q for every qubit q of the gate whose frame bit is 1."""
    m = len(frame_bits)
    x = np.eye(1, dtype=np.complex128)
    for b in frame_bits:
        x = np.kron(x, PX if b else I2)
    assert x.shape[0] == 2 ** m
    return x @ a @ x


# ---------------------------------------------------------------- noise

def kraus_factors(site) -> List[List[np.ndarray]]:
    """Kraus list of a noise site; each operator is a list of 2x2 factors,
    one per qubit of the site (local-submonomial form)."""
    k = site.kind
    if k == "DEPOL1":
        p = site.p[0]
        w = [1.0 - p, p / 3.0, p / 3.0, p / 3.0]
        return [[math.sqrt(w[a]) * PAULIS[a]] for a in range(4)]
    if k == "PAULI1":
        px, py, pz = site.p
        w = [1.0 - px - py - pz, px, py, pz]
        return [[math.sqrt(w[a]) * PAULIS[a]] for a in range(4)]
    if k == "DEPOL2":
        p = site.p[0]
        out = []
        for a in range(4):
            for b in range(4):
                w = (1.0 - p) if (a == 0 and b == 0) else p / 15.0
                out.append([math.sqrt(w) * PAULIS[a], PAULIS[b].copy()])
        return out
    if k == "AMPDAMP":
        gm = site.p[0]
        e0 = np.array([[1, 0], [0, math.sqrt(1.0 - gm)]], dtype=np.complex128)
        e1 = np.array([[0, math.sqrt(gm)], [0, 0]], dtype=np.complex128)
        return [[e0], [e1]]
    if k == "PHASEDAMP":
        lam = site.p[0]
        e0 = np.array([[1, 0], [0, math.sqrt(1.0 - lam)]], dtype=np.complex128)
        e1 = np.array([[0, 0], [0, math.sqrt(lam)]], dtype=np.complex128)
        return [[e0], [e1]]
    raise ValueError(f"unknown noise kind {k}")


def kraus_full(site) -> List[np.ndarray]:
    """Kraus operators as full 2^m x 2^m matrices (kron of the factors)."""
    out = []
    for fs in kraus_factors(site):
        m = np.eye(1, dtype=np.complex128)
        for f in fs:
            m = np.kron(m, f)
        out.append(m)
    return out


def column_norm2(m: np.ndarray, t: int) -> float:
    """|column t of a 2x2 factor|^2, in a fixed FP64 evaluation order."""
    a = m[0, t]
    b = m[1, t]
    return (a.real * a.real + a.imag * a.imag) + (b.real * b.real + b.imag * b.imag)


def branch_probabilities(factors_list, true_bits: Tuple[int, ...]) -> List[float]:
    """Eq. (4): Pr(i | t) = <t| E_i^dag E_i |t> = prod_j |col_{t_j}(M_ij)|^2."""
    out = []
    for fs in factors_list:
        pr = column_norm2(fs[0], true_bits[0])
        for j in range(1, len(fs)):
            pr = pr * column_norm2(fs[j], true_bits[j])
        out.append(pr)
    return out
