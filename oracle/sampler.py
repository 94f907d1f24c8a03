"""Gate-by-gate (pilot-wave) samplers, written from Algorithms 1 and 2.

Algorithm 1 (ideal): the classical state s starts at 0^n; for every gate in
order, a monomial gate moves s deterministically (s[q] <- sigma(s[q])), a
non-monomial gate takes the block of s[q] (BlockDecompose) and draws the new
s among the block's members with probability |amp(C_t, y)|^2 normalised over
the block (Section 2, the transition rule before Eq. (1)'s proof).
Amplitudes come from the complex128 state vector of the prefix circuit; in
the ideal case it is shared by all chains.

Algorithm 2 (noisy): an X-frame x rides along.  Each added gate G is
replaced by PropagateX(x, G) = X^x G X^x; a noise site draws its Kraus branch
from Eq. (4), flips the frame on every anti-diagonal factor (M <- M sigma_X)
and adds the now-diagonal factors, conjugated by the new frame, to the
prefix circuit C''.  The result is s XOR x.  The Kraus draw uses the true
bit (s XOR x)[q]: Eq. (4) evaluated on the state the channel acts on, which
is X^x applied to the chain's C''-basis state (reading recorded in the
design notes; the literal s[q] does not reproduce diag(rho)).

Fixed choices shared with the GPU engine (the paper is silent on them):
candidates in ascending local index; p_v = re^2 + im^2 in FP64; P = sum in
ascending v; u from Philox4x64-10 with counter (op, chain, 0, 0) and key
(seed, 0); choose the smallest v with u*P < C_v (C_v the inclusive prefix
sum); P == 0 keeps s; if rounding leaves no v, take the last v with p_v > 0.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import gates as G
from . import statevector as SV
from .philox import uniform53


def apply_readout(circ, bits: np.ndarray, chain_ids: np.ndarray, seed: int) -> np.ndarray:
    """Readout error of the simulated chip (Section 4): after the last
    operation each measured bit flips with its probability r_q, drawn from
    u = U53(Philox4x64-10, counter (n_ops + q, chain), key seed); flip when
    u < r_q."""
    ro = getattr(circ, "readout", None)
    if not ro:
        return bits
    out = bits.copy()
    n_ops = len(circ.ops())
    for q, r in enumerate(ro):
        if r > 0:
            u = uniform53(n_ops + q, chain_ids, seed)
            out[:, q] ^= (u < r).astype(out.dtype)
    return out


def draw_index(p: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Rows of p (K, m) are candidate weights; returns the chosen column per row,
    or -1 where the total is zero."""
    K, m = p.shape
    P = p[:, 0].copy()
    for v in range(1, m):
        P = P + p[:, v]
    target = u * P
    choice = np.full(K, -1, dtype=np.int64)
    C = np.zeros(K, dtype=np.float64)
    for v in range(m):
        C = C + p[:, v]
        hit = (choice < 0) & (target < C)
        choice[hit] = v
    # rounding fallback: last v with p_v > 0
    miss = (choice < 0) & (P > 0)
    if np.any(miss):
        for r in np.nonzero(miss)[0]:
            nz = np.nonzero(p[r] > 0)[0]
            choice[r] = nz[-1]
    return choice


def _local_index(bits: np.ndarray, qubits) -> np.ndarray:
    loc = np.zeros(bits.shape[0], dtype=np.int64)
    for q in qubits:
        loc = 2 * loc + bits[:, q].astype(np.int64)
    return loc


def _set_local(bits: np.ndarray, qubits, loc: np.ndarray) -> None:
    m = len(qubits)
    for j, q in enumerate(qubits):
        bits[:, q] = (loc >> (m - 1 - j)) & 1


def _basis_index(bits: np.ndarray) -> np.ndarray:
    n = bits.shape[1]
    idx = np.zeros(bits.shape[0], dtype=np.int64)
    for q in range(n):
        idx |= bits[:, q].astype(np.int64) << q
    return idx


def _update_state(mat: np.ndarray, qubits, s: np.ndarray, amp_of, u_of, choose=None) -> None:
    """UpdateState of Algorithm 1 for one gate on every chain (in place).

    ``amp_of(rows, y_bits)`` returns amp(C_t, y) for the given chains;
    ``u_of(rows)`` returns their uniforms; ``choose(rows, p, u, ch)``
    (optional) may replace the draws ch (a test hook)."""
    if G.is_diagonal(mat):
        return
    if G.is_monomial(mat):
        sigma = G.monomial_permutation(mat)
        loc = _local_index(s, qubits)
        _set_local(s, qubits, sigma[loc])
        return
    d = mat.shape[0]
    loc = _local_index(s, qubits)
    # group chains by their block (BlockDecompose on s[q])
    blocks = {}
    for l in range(d):
        blocks[l] = tuple(G.block_decompose(mat, l))
    rows_by_block = {}
    for r in range(s.shape[0]):
        rows_by_block.setdefault(blocks[int(loc[r])], []).append(r)
    for blk, rows in rows_by_block.items():
        rows = np.asarray(rows, dtype=np.int64)
        if len(blk) == 1:
            _set_local_rows(s, rows, qubits, blk[0])
            continue
        p = np.zeros((len(rows), len(blk)), dtype=np.float64)
        for j, l in enumerate(blk):
            y = s[rows].copy()
            _set_local(y, qubits, np.full(len(rows), l, dtype=np.int64))
            a = amp_of(rows, y)
            p[:, j] = a.real * a.real + a.imag * a.imag
        u = u_of(rows)
        ch = draw_index(p, u)
        if choose is not None:
            ch = choose(rows, p, u, ch)
        keep = ch < 0      # zero-mass block: s unchanged
        newloc = np.array([blk[c] if c >= 0 else -1 for c in ch], dtype=np.int64)
        upd = rows[~keep]
        if len(upd):
            y = s[upd]
            _set_local(y, qubits, newloc[~keep])
            s[upd] = y


def _set_local_rows(s, rows, qubits, l):
    y = s[rows]
    _set_local(y, qubits, np.full(len(rows), l, dtype=np.int64))
    s[rows] = y


def sample_ideal(circ, n_chains: int, seed: int, record: bool = False,
                 chains: Optional[np.ndarray] = None):
    """Algorithm 1 with one shared complex128 state vector.

    Returns (K, n) uint8 bitstrings; with ``record`` also the list of states
    after every op (index = op index)."""
    assert not circ.noise
    n = circ.n_qubits
    chain_ids = np.arange(n_chains, dtype=np.uint64) if chains is None else np.asarray(chains, np.uint64)
    K = len(chain_ids)
    s = np.zeros((K, n), dtype=np.uint8)
    psi = SV.zero_state(n)
    traj: List[np.ndarray] = []
    for op, (kind, gi) in enumerate(circ.ops()):
        g = circ.gates[gi]
        mat = G.gate_matrix(circ, g)
        psi = SV.apply_gate(psi, n, mat, g.qubits)

        def amp_of(rows, y, _psi=psi):
            return _psi[_basis_index(y)]

        def u_of(rows, _op=op):
            return uniform53(_op, chain_ids[rows], seed)

        _update_state(mat, g.qubits, s, amp_of, u_of)
        if record:
            traj.append(s.copy())
    s = apply_readout(circ, s, chain_ids, seed)
    return (s, traj) if record else s


def sample_noisy(circ, n_chains: int, seed: int, chains: Optional[np.ndarray] = None,
                 return_frame: bool = False):
    """Algorithm 2 with one complex128 trajectory state vector of C'' per chain."""
    n = circ.n_qubits
    chain_ids = np.arange(n_chains, dtype=np.uint64) if chains is None else np.asarray(chains, np.uint64)
    K = len(chain_ids)
    s = np.zeros((K, n), dtype=np.uint8)
    x = np.zeros((K, n), dtype=np.uint8)
    psi = np.zeros((K, 2 ** n), dtype=np.complex128)
    psi[:, 0] = 1.0
    for op, (kind, idx) in enumerate(circ.ops()):
        if kind == "gate":
            g = circ.gates[idx]
            mat = G.gate_matrix(circ, g)
            fr = _local_index(x, g.qubits)
            m = len(g.qubits)
            mats = np.empty((K, 2 ** m, 2 ** m), dtype=np.complex128)
            for f in range(2 ** m):
                bits = tuple((f >> (m - 1 - j)) & 1 for j in range(m))
                mats[fr == f] = G.conjugate_by_frame(mat, bits)
            psi = SV.apply_gate_per_batch(psi, n, mats, g.qubits)
            # UpdateState per frame group (G' differs between groups)
            for f in range(2 ** m):
                rows = np.nonzero(fr == f)[0]
                if len(rows) == 0:
                    continue
                bits = tuple((f >> (m - 1 - j)) & 1 for j in range(m))
                gp = G.conjugate_by_frame(mat, bits)
                sub = s[rows].copy()

                def amp_of(r_local, y, _rows=rows):
                    return psi[_rows[r_local], _basis_index(y)]

                def u_of(r_local, _op=op, _rows=rows):
                    return uniform53(_op, chain_ids[_rows[r_local]], seed)

                _update_state(gp, g.qubits, sub, amp_of, u_of)
                s[rows] = sub
        else:
            site = circ.noise[idx]
            flist = G.kraus_factors(site)
            q = site.qubits
            true_bits = (s[:, list(q)] ^ x[:, list(q)]).astype(np.int64)
            pr = np.zeros((K, len(flist)), dtype=np.float64)
            for r in range(K):
                pr[r] = G.branch_probabilities(flist, tuple(int(b) for b in true_bits[r]))
            ch = draw_index(pr, uniform53(op, chain_ids, seed))
            if np.any(ch < 0):
                raise FloatingPointError("zero-probability noise site")
            for j, qj in enumerate(q):
                diag = np.empty((K, 2), dtype=np.complex128)
                for r in range(K):
                    M = flist[ch[r]][j]
                    if M[0, 0] == 0 and M[1, 1] == 0:      # M sigma_X is diagonal
                        x[r, qj] ^= 1
                        M = M @ G.PX
                    if x[r, qj]:
                        M = G.PX @ M @ G.PX                # PropagateX with the new frame
                    diag[r] = (M[0, 0], M[1, 1])
                mats = np.zeros((K, 2, 2), dtype=np.complex128)
                mats[:, 0, 0] = diag[:, 0]
                mats[:, 1, 1] = diag[:, 1]
                psi = SV.apply_gate_per_batch(psi, n, mats, (qj,))
    out = apply_readout(circ, s ^ x, chain_ids, seed)
    return (out, s, x) if return_frame else out


def sample_noisy_pathsum(circ, chain: int, seed: int, choose=None, record: bool = False):
    """Algorithm 2 for one chain with every candidate amplitude from a path
    sum of the chain's prefix circuit C'' (each gate conjugated by the frame
    it meets, PropagateX, and each drawn Kraus branch's diagonal factors,
    conjugated by the new frame, AddGate), in execution order: the oracle's
    noisy sampler for qubit counts beyond a state vector per chain.  Same
    draws and random stream as ``sample_noisy``.

    ``choose(op, p, u, v)`` (optional, a test hook) sees the candidate
    weights p, the uniform u and the draw v of every gate step and returns
    the candidate to take; the Kraus branches are always drawn here.
    Returns the output bits (n,) and, with ``record``, the list of
    (op, s, x) after every op."""
    import instances as INS
    from . import pathsum as PS
    n = circ.n_qubits
    cid = np.array([chain], dtype=np.uint64)
    s = np.zeros((1, n), dtype=np.uint8)
    x = np.zeros((1, n), dtype=np.uint8)
    cpp: List = []          # C'': explicit-matrix gates
    traj = []

    def add(mat, qubits):
        cpp.append(INS.Gate("U1" if len(qubits) == 1 else "U2", tuple(qubits),
                            matrix=tuple(complex(v) for v in np.asarray(mat).reshape(-1))))

    for op, (kind, idx) in enumerate(circ.ops()):
        if kind == "gate":
            g = circ.gates[idx]
            gp = G.conjugate_by_frame(G.gate_matrix(circ, g), tuple(int(x[0, q]) for q in g.qubits))
            add(gp, g.qubits)
            cc = INS.Circuit(n, list(cpp), np.zeros(0))

            def amp_of(rows, y, _cc=cc):
                return np.array([PS.amplitude(_cc, len(_cc.gates), y[i]) for i in range(len(rows))],
                                dtype=np.complex128)

            def u_of(rows, _op=op):
                return uniform53(_op, cid[rows], seed)

            hook = None
            if choose is not None:
                def hook(rows, p, u, ch, _op=op):
                    return np.array([choose(_op, p[0], u[0], int(ch[0]))], dtype=np.int64)
            _update_state(gp, g.qubits, s, amp_of, u_of, hook)
        else:
            site = circ.noise[idx]
            flist = G.kraus_factors(site)
            q = site.qubits
            t = tuple(int(s[0, qq] ^ x[0, qq]) for qq in q)
            pr = np.array([G.branch_probabilities(flist, t)], dtype=np.float64)
            ch = draw_index(pr, uniform53(op, cid, seed))
            if ch[0] < 0:
                raise FloatingPointError("zero-probability noise site")
            for j, qj in enumerate(q):
                M = flist[int(ch[0])][j]
                if M[0, 0] == 0 and M[1, 1] == 0:      # M sigma_X is diagonal
                    x[0, qj] ^= 1
                    M = M @ G.PX
                if x[0, qj]:
                    M = G.PX @ M @ G.PX                # conjugated by the new frame
                add(np.diag([M[0, 0], M[1, 1]]), (qj,))
        if record:
            traj.append((op, s[0].copy(), x[0].copy()))
    out = apply_readout(circ, s ^ x, cid, seed)[0]
    return (out, traj) if record else out


def exact_distribution(circ) -> np.ndarray:
    """|psi_T|^2 (ideal) or diag(rho_T) (noisy), indexed by basis index,
    followed by the readout flips (each qubit independently)."""
    if circ.noise:
        p = np.real(np.diag(SV.density_matrix(circ))).copy()
    else:
        psi = SV.state(circ)
        p = psi.real ** 2 + psi.imag ** 2
    ro = getattr(circ, "readout", None)
    if ro:
        idx = np.arange(len(p))
        for q, r in enumerate(ro):
            if r > 0:
                p = (1.0 - r) * p + r * p[idx ^ (1 << q)]
    return p


def basis_index(bits: np.ndarray) -> np.ndarray:
    return _basis_index(bits)


def sample_ideal_pathsum(circ, n_chains: int, seed: int, chains: Optional[np.ndarray] = None,
                         record: bool = False):
    """Algorithm 1 with every candidate amplitude from a path sum of the
    prefix circuit (per chain, no state vector): the oracle's sampler for
    qubit counts beyond a state vector.  Same draw rule and random stream as
    ``sample_ideal``."""
    from . import pathsum as PS
    assert not circ.noise
    n = circ.n_qubits
    chain_ids = np.arange(n_chains, dtype=np.uint64) if chains is None else np.asarray(chains, np.uint64)
    K = len(chain_ids)
    s = np.zeros((K, n), dtype=np.uint8)
    traj = []
    for op, (kind, gi) in enumerate(circ.ops()):
        g = circ.gates[gi]
        mat = G.gate_matrix(circ, g)

        def amp_of(rows, y, _gi=gi):
            return np.array([PS.amplitude(circ, _gi + 1, y[i]) for i in range(len(rows))],
                            dtype=np.complex128)

        def u_of(rows, _op=op):
            return uniform53(_op, chain_ids[rows], seed)

        _update_state(mat, g.qubits, s, amp_of, u_of)
        if record:
            traj.append(s.copy())
    s = apply_readout(circ, s, chain_ids, seed)
    return (s, traj) if record else s
