"""QAOA p=1 MaxCut edge expectations in closed form.

For one QAOA layer with gate angles RZZ(g) on every edge and RX(b) on every
qubit after the Hadamard layer (R_P(t) = exp(-i t P / 2)), the published
analytic result for p = 1 (Wang, Hadfield, Jiang, Rieffel, PRA 97, 022304,
2018), rewritten in these gate conventions, reads

  <Z_u Z_v> = 1/2 sin(2b) sin(g) (cos^{d_u} g + cos^{d_v} g)
            + 1/2 sin^2(b) cos^{d_u + d_v - 2 l} g (1 - cos^{l}(2g))

with d_u = deg(u) - 1, d_v = deg(v) - 1 and l the number of triangles that
contain the edge (u, v).  The expected cut is sum_e (1 - <Z_u Z_v>)/2.
(Conversion: the reference works with exp(-i g' C), C = sum (1 - ZZ)/2 and
exp(-i b' X), i.e. g' = -g and b' = b/2 here.)

This formula is independent of the state-vector code and pins it.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple

import numpy as np


def _neighbours(n: int, edges):
    nb = [set() for _ in range(n)]
    for u, v in edges:
        nb[u].add(v)
        nb[v].add(u)
    return nb


def zz_expectation(n: int, edges: Sequence[Tuple[int, int]], gamma: float, beta: float) -> Dict:
    nb = _neighbours(n, edges)
    out = {}
    cg = math.cos(gamma)
    for u, v in edges:
        du = len(nb[u]) - 1
        dv = len(nb[v]) - 1
        lam = len(nb[u] & nb[v])
        t1 = 0.5 * math.sin(2 * beta) * math.sin(gamma) * (cg ** du + cg ** dv)
        t2 = 0.5 * math.sin(beta) ** 2 * cg ** (du + dv - 2 * lam) * (1 - math.cos(2 * gamma) ** lam)
        out[(u, v)] = t1 + t2
    return out


def expected_cut(n: int, edges, gamma: float, beta: float) -> float:
    zz = zz_expectation(n, edges, gamma, beta)
    return float(sum((1.0 - z) / 2.0 for z in zz.values()))


def expected_cut_gradient(n: int, edges, gamma: float, beta: float, h: float = 1e-6):
    """(dE/dgamma, dE/dbeta) of the closed form by central differences of the
    analytic expression (exact function, no sampling)."""
    dg = (expected_cut(n, edges, gamma + h, beta) - expected_cut(n, edges, gamma - h, beta)) / (2 * h)
    db = (expected_cut(n, edges, gamma, beta + h) - expected_cut(n, edges, gamma, beta - h)) / (2 * h)
    return np.array([dg, db])
