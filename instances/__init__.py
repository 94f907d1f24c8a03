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
    # per-qubit probability that the measured bit is flipped (readout error,
    # a classical flip of the sampled bitstring after the last operation)
    readout: Optional[Tuple[float, ...]] = None

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
        return dataclasses.replace(self, noise=[], readout=None)


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


def kings_graph(rows: int, cols: int) -> List[Tuple[int, int]]:
    """King's graph: the rows x cols grid with its diagonals (q = rows*c + r)."""
    edges = set()
    for r in range(rows):
        for c in range(cols):
            for dr, dc in ((0, 1), (1, 0), (1, 1), (-1, 1)):
                r2, c2 = r + dr, c + dc
                if 0 <= r2 < rows and 0 <= c2 < cols:
                    edges.add(tuple(sorted((rows * c + r, rows * c2 + r2))))
    return sorted(edges)


def heavy_hex_graph(rows: int, length: int) -> Tuple[int, List[Tuple[int, int]]]:
    """Heavy-hex lattice: `rows` lines of `length` qubits; between lines r and
    r+1 a bridge qubit joins the two qubits at column c, for c = 0, 4, 8, ...
    (r even) or c = 2, 6, 10, ... (r odd).  Qubits are numbered column by
    column (a line qubit before the bridge below it).  Returns (n, edges)."""
    ids = {}
    n = 0
    for c in range(length):
        for r in range(rows):
            ids[("q", r, c)] = n
            n += 1
            if r + 1 < rows and c % 4 == (0 if r % 2 == 0 else 2):
                ids[("b", r, c)] = n
                n += 1
    edges = []
    for r in range(rows):
        for c in range(length - 1):
            edges.append((ids[("q", r, c)], ids[("q", r, c + 1)]))
    for (kind, r, c), b in ids.items():
        if kind == "b":
            edges.append((ids[("q", r, c)], b))
            edges.append((ids[("q", r + 1, c)], b))
    return n, sorted(tuple(sorted(e)) for e in edges)


def chimera_graph(m: int, n: int, t: int = 4) -> List[Tuple[int, int]]:
    """Chimera graph C(m, n, t): m x n cells of K_{t,t}; qubit (i, j, side,
    k) = ((j*m + i)*2 + side)*t + k.  Side 0 of a cell joins side 0 of the
    cell below, side 1 joins side 1 of the cell to the right."""
    def q(i, j, side, k):
        return ((j * m + i) * 2 + side) * t + k
    edges = []
    for i in range(m):
        for j in range(n):
            for a in range(t):
                for b in range(t):
                    edges.append((q(i, j, 0, a), q(i, j, 1, b)))
                if i + 1 < m:
                    edges.append((q(i, j, 0, a), q(i + 1, j, 0, a)))
                if j + 1 < n:
                    edges.append((q(i, j, 1, a), q(i, j + 1, 1, a)))
    return sorted(tuple(sorted(e)) for e in edges)


# ---------------------------------------------------------------- circuits

def qaoa_maxcut(n: int, edges: Sequence[Tuple[int, int]], gammas, betas,
                weights=None, fields=None, name: str = "", beta_coeff: float = 1.0) -> Circuit:
    """QAOA circuit with gate angles RZZ(w_e * gamma_l) and RX(beta_coeff * beta_l).

    ``weights`` (optional, per edge, in the order of ``edges``) and ``fields``
    (optional, per qubit, adds RZ(h_q * gamma_l) after the ZZ layer) give the
    weighted Ising variant.  theta = [gamma_1..gamma_p, beta_1..beta_p].
    """
    gammas = np.asarray(gammas, dtype=np.float64)
    betas = np.asarray(betas, dtype=np.float64)
    p = len(gammas)
    assert len(betas) == p
    order = sorted(range(len(edges)), key=lambda i: tuple(sorted(edges[i])))
    wsort = None if weights is None else [float(weights[i]) for i in order]
    edges = [tuple(sorted(edges[i])) for i in order]
    gates: List[Gate] = [Gate("H", (q,)) for q in range(n)]
    for l in range(p):
        for ei, (u, v) in enumerate(edges):
            w = 1.0 if wsort is None else wsort[ei]
            gates.append(Gate("RZZ", (u, v), param=l, coeff=w))
        if fields is not None:
            for q in range(n):
                if fields[q] != 0.0:
                    gates.append(Gate("RZ", (q,), param=l, coeff=float(fields[q])))
        for q in range(n):
            gates.append(Gate("RX", (q,), param=p + l, coeff=float(beta_coeff)))
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


# The simulated chip of the paper's noisy experiments (Section 4): one-qubit
# error probability 0.005, two-qubit 0.01, readout 0.05, gate lengths 30 ns
# and 80 ns, relaxation time 100 us, dephasing time 50 us.
CHIP = dict(p1=0.005, p2=0.01, readout=0.05, t1q_ns=30.0, t2q_ns=80.0, T1_us=100.0, T2_us=50.0)


def chip_damping(t_ns: float, T1_us: float, T2_us: float) -> Tuple[float, float]:
    """Channel parameters of a gate of length t: amplitude damping gamma =
    1 - exp(-t / T1), and phase damping lambda with (1 - gamma)(1 - lambda) =
    exp(-2 t / T2), i.e. lambda = 1 - exp(-2 t / T_phi) for the pure
    dephasing time 1 / T_phi = 1 / T2 - 1 / (2 T1) (so the coherence of the
    qubit decays as exp(-t / T2) under both channels)."""
    t, T1, T2 = t_ns * 1e-3, T1_us, T2_us
    if T2 > 2 * T1:
        raise ValueError("T2 exceeds 2 T1")
    gamma = 1.0 - math.exp(-t / T1)
    lam = 1.0 - math.exp(-2.0 * t * (1.0 / T2 - 0.5 / T1))
    return gamma, lam


def add_chip_noise(c: Circuit, p1: float = CHIP["p1"], p2: float = CHIP["p2"], readout: float = CHIP["readout"],
                   t1q_ns: float = CHIP["t1q_ns"], t2q_ns: float = CHIP["t2q_ns"], T1_us: float = CHIP["T1_us"],
                   T2_us: float = CHIP["T2_us"]) -> Circuit:
    """The chip noise model: after every one-qubit gate, one-qubit
    depolarising noise p1 then amplitude and phase damping for the gate's
    length; after every two-qubit gate, two-qubit depolarising noise p2 then
    amplitude and phase damping of both qubits; readout flips with
    probability `readout` on every qubit."""
    g1, l1 = chip_damping(t1q_ns, T1_us, T2_us)
    g2, l2 = chip_damping(t2q_ns, T1_us, T2_us)
    sites: List[NoiseSite] = []
    for gi, g in enumerate(c.gates):
        if len(g.qubits) == 1:
            if p1 > 0:
                sites.append(NoiseSite(gi, "DEPOL1", g.qubits, (p1,)))
            damp = [(g.qubits[0], g1, l1)]
        else:
            if p2 > 0:
                sites.append(NoiseSite(gi, "DEPOL2", g.qubits, (p2,)))
            damp = [(q, g2, l2) for q in g.qubits]
        for q, gm, lm in damp:
            if gm > 0:
                sites.append(NoiseSite(gi, "AMPDAMP", (q,), (gm,)))
            if lm > 0:
                sites.append(NoiseSite(gi, "PHASEDAMP", (q,), (lm,)))
    ro = tuple([float(readout)] * c.n_qubits) if readout > 0 else None
    return dataclasses.replace(c, noise=sites, readout=ro)


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


# Gaussian-weighted Ising QAOA at p = 1 (the paper's timing workload:
# couplings J_ij and fields h_i drawn from N(0, 1), gates RZZ(2 gamma J_ij),
# RZ(2 gamma h_i), RX(2 beta)) on five graph families.  Every family is laid
# out as a long strip (its qubits numbered along the strip), so that a
# column sweep keeps the contraction narrow; `n` asks for about that many
# qubits.
ISING_TOPOLOGIES = ("grid", "heavy_hex", "kings", "chimera", "3reg")


def ising_graph(topology: str, n: int) -> Tuple[int, List[Tuple[int, int]]]:
    """A graph of the family with about n nodes: (nodes, edges)."""
    if topology == "grid":
        rows = 4 if n >= 16 else 2
        cols = max(2, round(n / rows))
        return rows * cols, grid_graph(rows, cols, "col")
    if topology == "kings":
        rows = 4 if n >= 16 else 2
        cols = max(2, round(n / rows))
        return rows * cols, kings_graph(rows, cols)
    if topology == "heavy_hex":
        # two lines of `length` qubits and their bridges: n ~ 2.25 L
        length = max(3, round(n / 2.25))
        return heavy_hex_graph(2, length)
    if topology == "chimera":
        cols = max(1, round(n / 8))
        return 8 * cols, chimera_graph(1, cols)
    if topology == "3reg":
        nn = n + (n % 2)
        return nn, random_regular_graph(3, nn, 6000 + nn)
    raise ValueError(f"unknown topology {topology}")


def ising_qaoa_p1(topology: str, n: int, instance: int = 0) -> Circuit:
    """Instance `instance` of the family at about n qubits: seeded Gaussian
    couplings and fields, angles gamma, beta ~ U(0, pi)."""
    nn, edges = ising_graph(topology, n)
    seed = 7000 + 100 * ISING_TOPOLOGIES.index(topology) + instance
    rng = np.random.default_rng(seed)
    J = rng.standard_normal(len(edges))
    h = rng.standard_normal(nn)
    g, b = rng.uniform(0.0, math.pi, 2)
    return qaoa_maxcut(nn, edges, [g], [b], weights=2.0 * J, fields=2.0 * h, beta_coeff=2.0,
                       name=f"ising_p1_{topology}_n{nn}_i{instance}")


def workload_ising_p1(topology: str, n: int, instance: int = 0) -> Tuple[Circuit, int, int]:
    """Gaussian Ising QAOA p=1 on the family at about n qubits, 4096 chains."""
    return ising_qaoa_p1(topology, n, instance), 4096, 7003 + instance


# Circuits beyond QAOA (gates with blocks smaller than 2^|S| and two-qubit
# candidate blocks): explicit two-qubit matrices are part of the input.

def _xx_plus_yy(theta: float) -> Tuple[complex, ...]:
    """exp(-i theta (XX + YY) / 2), basis 00, 01, 10, 11 (row-major)."""
    c, s = math.cos(theta), -1j * math.sin(theta)
    return (1, 0, 0, 0, 0, c, s, 0, 0, s, c, 0, 0, 0, 0, 1)


def _heisenberg(dt: float) -> Tuple[complex, ...]:
    """exp(-i dt (XX + YY + ZZ)): e^{-i dt} on 00 and 11; on {01, 10}
    e^{i dt} (cos 2dt - i sin 2dt X)."""
    a = complex(math.cos(dt), -math.sin(dt))
    b = complex(math.cos(dt), math.sin(dt))
    c, s = b * math.cos(2 * dt), -1j * b * math.sin(2 * dt)
    return (a, 0, 0, 0, 0, c, s, 0, 0, s, c, 0, 0, 0, 0, a)


def _haar_unitary(d: int, rng) -> Tuple[complex, ...]:
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    q = q * (np.diag(r) / np.abs(np.diag(r)))
    return tuple(complex(x) for x in q.reshape(-1))


def general_gate_circuit(n: int = 8, n_gates: int = 40, seed: int = 8001) -> Circuit:
    """H on every qubit, then a seeded sequence of CRX, FSIM, CNOT, CZ,
    XX+YY rotations, Haar-random two-qubit unitaries, RZ and RX on random
    qubits: blocks {00},{01},{10,11} (CRX), {00},{01,10},{11} (FSIM, XX+YY),
    one 4-element block (random unitaries), monomial and diagonal gates."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = [Gate("H", (q,)) for q in range(n)]
    theta = rng.uniform(0.2, math.pi - 0.2, 4)
    kinds = ["CRX", "FSIM", "CNOT", "CZ", "XXYY", "HAAR", "RZ", "RX"]
    for _ in range(n_gates):
        k = kinds[int(rng.integers(len(kinds)))]
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        if k == "CRX":
            gates.append(Gate("CRX", (a, b), param=0))
        elif k == "FSIM":
            gates.append(Gate("FSIM", (a, b), param=1, param2=2))
        elif k in ("CNOT", "CZ"):
            gates.append(Gate(k, (a, b)))
        elif k == "XXYY":
            gates.append(Gate("U2", (a, b), matrix=_xx_plus_yy(float(rng.uniform(0.3, 2.8)))))
        elif k == "HAAR":
            gates.append(Gate("U2", (a, b), matrix=_haar_unitary(4, rng)))
        elif k == "RZ":
            gates.append(Gate("RZ", (a,), param=3))
        else:
            gates.append(Gate("RX", (a,), param=3, coeff=0.5))
    return Circuit(n, gates, theta, name=f"general_n{n}_g{n_gates}")


def trotter_heisenberg(n: int = 10, steps: int = 3, dt: float = 0.3, field: float = 0.7) -> Circuit:
    """Trotterised Heisenberg chain with a transverse field: from |+...+> (H
    layer), per step exp(-i dt (XX+YY+ZZ)) on the even then the odd bonds,
    then RX(2 dt h) on every qubit."""
    gates: List[Gate] = [Gate("H", (q,)) for q in range(n)]
    for _ in range(steps):
        for start in (0, 1):
            for q in range(start, n - 1, 2):
                gates.append(Gate("U2", (q, q + 1), matrix=_heisenberg(dt)))
        for q in range(n):
            gates.append(Gate("RX", (q,), param=0, coeff=2 * dt))
    return Circuit(n, gates, np.array([field]), name=f"heisenberg_n{n}_s{steps}")


def trotter_tfim(n: int = 10, steps: int = 3, dt: float = 0.3, J: float = 1.0, h: float = 0.9) -> Circuit:
    """Trotterised transverse-field Ising chain from |0...0>: per step
    RZZ(2 dt J) on every bond, then RX(2 dt h) on every qubit."""
    gates: List[Gate] = []
    for _ in range(steps):
        for q in range(n - 1):
            gates.append(Gate("RZZ", (q, q + 1), param=0, coeff=2 * dt))
        for q in range(n):
            gates.append(Gate("RX", (q,), param=1, coeff=2 * dt))
    return Circuit(n, gates, np.array([J, h]), name=f"tfim_n{n}_s{steps}")


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
