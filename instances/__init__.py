"""Seeded synthetic workloads for the pilot-wave sampler.

This module is shared by the GPU engine's callers (bench, tests) and by the
CPU oracle.  It holds *inputs only*: graphs, gate lists (kind, qubits,
parameter binding), noise-site lists, seeds and named workload configurations.
It contains none of the sampler's arithmetic: no gate matrices, no Kraus
operators, no probabilities.  Each side turns a gate kind and angle into a
matrix by itself.

Conventions (shared by every consumer):

* qubit ``k`` of a bitstring is bit ``k % 64`` of 64-bit word ``k // 64``;
* a two-qubit gate on ``(q0, q1)`` has local index ``2*b(q0) + b(q1)``
  (first listed qubit is the most significant local bit);
* the angle of a gate is ``coeff * theta[param] + offset`` (``param < 0``
  means ``offset`` alone);
* execution order (the "op list") is the gate list with every noise site
  inserted directly after the gate named by its ``after_gate`` field, sites
  sharing a gate keeping their list order.  The position of an operation in
  that merged list is its *op index*; the random draw made at an operation is
  keyed by it.

QAOA circuits follow the paper's appendix on QAOA: a Hadamard layer, then per
layer ``l`` one ZZ rotation per graph edge (edges sorted lexicographically
with ``u < v``) followed by one X rotation per qubit in ascending order.  The
workloads take gate angles ``RZZ(gamma_l)`` and ``RX(beta_l)`` literally with
``R_P(t) = exp(-i t P / 2)`` (unweighted MaxCut, J = 1, h = 0).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Gate kinds understood by both the engine and the oracle.
GATE_KINDS = ("H", "X", "RX", "RZ", "RZZ", "CNOT", "CZ", "U1", "U2", "CRX", "FSIM")
# Noise kinds (all local-submonomial channels).
NOISE_KINDS = ("DEPOL1", "DEPOL2", "AMPDAMP", "PHASEDAMP", "PAULI1")

GATE_KIND_ID = {k: i for i, k in enumerate(GATE_KINDS)}
NOISE_KIND_ID = {k: i for i, k in enumerate(NOISE_KINDS)}


@dataclasses.dataclass(frozen=True)
class Gate:
    kind: str
    qubits: Tuple[int, ...]
    param: int = -1          # index into theta, -1 = none
    coeff: float = 1.0
    offset: float = 0.0
    param2: int = -1         # second angle (FSIM phi), same binding rule
    coeff2: float = 1.0
    offset2: float = 0.0
    matrix: Optional[Tuple[complex, ...]] = None   # U1 / U2 only, row-major


@dataclasses.dataclass(frozen=True)
class NoiseSite:
    after_gate: int
    kind: str
    qubits: Tuple[int, ...]
    p: Tuple[float, ...]     # DEPOL*/AMPDAMP/PHASEDAMP: (p,), PAULI1: (px, py, pz)


@dataclasses.dataclass
class Circuit:
    n_qubits: int
    gates: List[Gate]
    theta: np.ndarray
    noise: List[NoiseSite] = dataclasses.field(default_factory=list)
    name: str = ""
    edges: Optional[List[Tuple[int, int]]] = None

    def angle(self, g: Gate) -> float:
        a = g.offset
        if g.param >= 0:
            a += g.coeff * float(self.theta[g.param])
        return a

    def angle2(self, g: Gate) -> float:
        a = g.offset2
        if g.param2 >= 0:
            a += g.coeff2 * float(self.theta[g.param2])
        return a

    def ops(self) -> List[Tuple[str, int]]:
        """Execution order: [("gate", gi) | ("noise", si)], op index = position."""
        by_gate: dict = {}
        for si, s in enumerate(self.noise):
            if not (0 <= s.after_gate < len(self.gates)):
                raise ValueError("noise site after_gate out of range")
            by_gate.setdefault(s.after_gate, []).append(si)
        out: List[Tuple[str, int]] = []
        for gi in range(len(self.gates)):
            out.append(("gate", gi))
            for si in by_gate.get(gi, []):
                out.append(("noise", si))
        return out

    def with_theta(self, theta) -> "Circuit":
        return dataclasses.replace(self, theta=np.asarray(theta, dtype=np.float64).copy())

    def without_noise(self) -> "Circuit":
        return dataclasses.replace(self, noise=[])


# ---------------------------------------------------------------- graphs

def grid_graph(rows: int, cols: int, index: str = "row") -> List[Tuple[int, int]]:
    """Nearest-neighbour grid.  ``index='row'``: q = cols*r + c; ``'col'``: q = rows*c + r."""
    def q(r, c):
        return cols * r + c if index == "row" else rows * c + r
    edges = []
    for r in range(rows):
        for c in range(cols):
            if c + 1 < cols:
                edges.append(tuple(sorted((q(r, c), q(r, c + 1)))))
            if r + 1 < rows:
                edges.append(tuple(sorted((q(r, c), q(r + 1, c)))))
    return sorted(set(edges))


def random_regular_graph(d: int, n: int, seed: int) -> List[Tuple[int, int]]:
    """Uniform simple d-regular graph by the pairing (configuration) model with rejection."""
    if (n * d) % 2 or d >= n:
        raise ValueError("no d-regular graph with these parameters")
    rng = np.random.default_rng(seed)
    for _ in range(100000):
        stubs = np.repeat(np.arange(n), d)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        es = {tuple(sorted((int(a), int(b)))) for a, b in pairs}
        if len(es) != len(pairs):
            continue
        return sorted(es)
    raise RuntimeError("pairing model did not produce a simple graph")


# ---------------------------------------------------------------- circuits

def qaoa_maxcut(n: int, edges: Sequence[Tuple[int, int]], gammas, betas,
                weights=None, fields=None, name: str = "") -> Circuit:
    """QAOA circuit with gate angles RZZ(w_e * gamma_l) and RX(beta_l).

    ``weights`` (optional, per edge) and ``fields`` (optional, per qubit, adds
    RZ(h_q * gamma_l) after the ZZ layer) give the weighted Ising variant.
    theta = [gamma_1..gamma_p, beta_1..beta_p].
    """
    gammas = np.asarray(gammas, dtype=np.float64)
    betas = np.asarray(betas, dtype=np.float64)
    p = len(gammas)
    assert len(betas) == p
    edges = sorted(tuple(sorted(e)) for e in edges)
    gates: List[Gate] = [Gate("H", (q,)) for q in range(n)]
    for l in range(p):
        for ei, (u, v) in enumerate(edges):
            w = 1.0 if weights is None else float(weights[ei])
            gates.append(Gate("RZZ", (u, v), param=l, coeff=w))
        if fields is not None:
            for q in range(n):
                if fields[q] != 0.0:
                    gates.append(Gate("RZ", (q,), param=l, coeff=float(fields[q])))
        for q in range(n):
            gates.append(Gate("RX", (q,), param=p + l, coeff=1.0))
    theta = np.concatenate([gammas, betas])
    return Circuit(n_qubits=n, gates=gates, theta=theta, name=name, edges=list(edges))


def add_qaoa_noise(c: Circuit, depol2: float = 0.0, ampdamp: float = 0.0,
                   depol1: float = 0.0) -> Circuit:
    """Two-qubit depolarizing after each RZZ, amplitude damping (and optional
    one-qubit depolarizing) after each RX."""
    sites: List[NoiseSite] = []
    for gi, g in enumerate(c.gates):
        if g.kind == "RZZ" and depol2 > 0:
            sites.append(NoiseSite(gi, "DEPOL2", g.qubits, (depol2,)))
        if g.kind == "RX":
            if depol1 > 0:
                sites.append(NoiseSite(gi, "DEPOL1", g.qubits, (depol1,)))
            if ampdamp > 0:
                sites.append(NoiseSite(gi, "AMPDAMP", g.qubits, (ampdamp,)))
    return dataclasses.replace(c, noise=sites)


def qaoa_angles(p: int, seed: int):
    rng = np.random.default_rng(seed)
    gammas = rng.uniform(0.0, math.pi, p)
    betas = rng.uniform(0.0, math.pi, p)
    return gammas, betas


# ---------------------------------------------------------------- named workloads
# Seeds: graph 1000k+1, angles 1000k+2, sampler 1000k+3 for workload k.

def workload_qaoa3reg12() -> Tuple[Circuit, int, int]:
    """Ideal QAOA p=1 MaxCut, seeded random 3-regular graph, 12 qubits, 2000 chains."""
    k = 1
    edges = random_regular_graph(3, 12, 1000 * k + 1)
    g, b = qaoa_angles(1, 1000 * k + 2)
    return qaoa_maxcut(12, edges, g, b, name="qaoa_3reg_n12_p1"), 2000, 1000 * k + 3


def workload_grid6x8(rows: int = 6, cols: int = 8) -> Tuple[Circuit, int, int]:
    """Ideal QAOA p=2 MaxCut on a rows x cols grid (q = cols*r + c), 4096 chains."""
    k = 2
    edges = grid_graph(rows, cols, "row")
    g, b = qaoa_angles(2, 1000 * k + 2)
    return (qaoa_maxcut(rows * cols, edges, g, b, name=f"qaoa_grid{rows}x{cols}_p2"),
            4096, 1000 * k + 3)


def workload_noisy3reg100(n: int = 100) -> Tuple[Circuit, int, int]:
    """Noisy QAOA p=2, 3-regular n=100, depol2 1e-3 after RZZ, AD 5e-4 after RX, 8192 chains."""
    k = 3
    edges = random_regular_graph(3, n, 1000 * k + 1)
    g, b = qaoa_angles(2, 1000 * k + 2)
    c = qaoa_maxcut(n, edges, g, b, name=f"qaoa_3reg_n{n}_p2_noisy")
    return add_qaoa_noise(c, depol2=1e-3, ampdamp=5e-4), 8192, 1000 * k + 3


def workload_grad3reg64(n: int = 64) -> Tuple[Circuit, int, int]:
    """QAOA p=3 on a 3-regular n=64 graph for score-function gradients, 16384 samples."""
    k = 4
    edges = random_regular_graph(3, n, 1000 * k + 1)
    g, b = qaoa_angles(3, 1000 * k + 2)
    return qaoa_maxcut(n, edges, g, b, name=f"qaoa_3reg_n{n}_p3"), 16384, 1000 * k + 3


def workload_ladder4x119(cols: int = 119) -> Tuple[Circuit, int, int]:
    """Ideal QAOA p=2 on a 4 x cols grid ladder (q = 4c + r), 16384 chains."""
    k = 5
    edges = grid_graph(4, cols, "col")
    g, b = qaoa_angles(2, 1000 * k + 2)
    return qaoa_maxcut(4 * cols, edges, g, b, name=f"qaoa_ladder4x{cols}_p2"), 16384, 1000 * k + 3


def workload_mixed_ladders(count: int = 32) -> List[Tuple[Circuit, int]]:
    """32 mixed instances 4 x W, W ~ U{25..100}, p ~ U{1,2}, 1536 chains each."""
    rng = np.random.default_rng(5000 + 4)
    out = []
    for i in range(count):
        w = int(rng.integers(25, 101))
        p = int(rng.integers(1, 3))
        g, b = qaoa_angles(p, 5000 + 100 + i)
        out.append((qaoa_maxcut(4 * w, grid_graph(4, w, "col"), g, b,
                                name=f"qaoa_ladder4x{w}_p{p}"), 1536))
    return out


def maxcut_value(edges, bits: np.ndarray) -> np.ndarray:
    """Cut size of each row of a (K, n) 0/1 array (an input statistic, not sampler arithmetic)."""
    bits = np.asarray(bits)
    e = np.asarray(edges, dtype=np.int64)
    return np.sum(bits[:, e[:, 0]] != bits[:, e[:, 1]], axis=1)


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """(K, n) 0/1 -> (K, ceil(n/64)) uint64, qubit k in bit k%64 of word k//64."""
    bits = np.asarray(bits, dtype=np.uint64)
    K, n = bits.shape
    W = (n + 63) // 64
    out = np.zeros((K, W), dtype=np.uint64)
    for k in range(n):
        out[:, k // 64] |= bits[:, k] << np.uint64(k % 64)
    return out


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    words = np.asarray(words, dtype=np.uint64)
    K = words.shape[0]
    out = np.zeros((K, n), dtype=np.uint8)
    for k in range(n):
        out[:, k] = ((words[:, k // 64] >> np.uint64(k % 64)) & np.uint64(1)).astype(np.uint8)
    return out
