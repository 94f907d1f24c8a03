"""Prefix-circuit amplitudes for many qubits, by summing over paths.

amp(C_t, y) = <y|U_t ... U_1|0^n> is the sum, over one basis value per qubit
"segment", of the product of gate entries (Feynman path sum).  A segment of
qubit q ends at every gate that is not diagonal on q; a gate that is diagonal
on q (all entries with in_q != out_q zero) keeps q on the same segment, so
its in and out legs are one variable (the leg identification of Appendix A).
The first segment of every qubit is fixed to 0 and the last one to y[q]
(or left open for the candidate qubits).

The sum is evaluated exactly by variable elimination (bucket elimination):
eliminate one variable at a time, multiplying the factors that contain it and
summing it out.  The elimination order (greedy smallest-new-factor) changes
only rounding, not the value.  Pinned against the state vector on prefixes of
the 12-qubit and 4x4-grid circuits and against the gamma = 0 product state at
48 qubits (``tests/test_oracle_closed_form_grad.py``); the sampler built on it
is pinned against the state-vector sampler chain for chain
(``tests/test_oracle_pathsum_sampler.py``).
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import gates as G


def _gate_tensor(mat: np.ndarray, m: int) -> np.ndarray:
    """mat[out_local, in_local] -> tensor with axes (out_0..out_{m-1}, in_0..in_{m-1})."""
    return mat.reshape((2,) * (2 * m))


def _diag_on(mat: np.ndarray, m: int, j: int) -> bool:
    t = _gate_tensor(mat, m)
    for idx in np.ndindex(*t.shape):
        if idx[j] != idx[m + j] and t[idx] != 0:
            return False
    return True


def build_factors(circ, n_gates: int, y: Sequence[int], open_qubits: Sequence[int] = (),
                  extra_diag: Dict[Tuple[int, int], np.ndarray] | None = None):
    """Factor list [(vars, array)] of the prefix network; fixed variables are sliced."""
    n = circ.n_qubits
    seg = [0] * n
    # variable id = (q, segment)
    factors: List[Tuple[Tuple, np.ndarray]] = []
    for gi in range(n_gates):
        g = circ.gates[gi]
        mat = G.gate_matrix(circ, g)
        m = len(g.qubits)
        t = _gate_tensor(mat, m)
        legs_out = []
        legs_in = []
        diag = [_diag_on(mat, m, j) for j in range(m)]
        for j, q in enumerate(g.qubits):
            legs_in.append((q, seg[q]))
            if not diag[j]:
                seg[q] += 1
            legs_out.append((q, seg[q]))
        # merge identified legs: build the tensor over distinct variables
        all_legs = legs_out + legs_in
        uniq: List[Tuple[int, int]] = []
        for v in all_legs:
            if v not in uniq:
                uniq.append(v)
        arr = np.zeros((2,) * len(uniq), dtype=np.complex128)
        for idx in np.ndindex(*arr.shape):
            val = dict(zip(uniq, idx))
            arr[idx] = t[tuple(val[v] for v in all_legs)]
        factors.append((tuple(uniq), arr))
    if extra_diag:
        for (q, s_), d in extra_diag.items():
            factors.append((((q, s_),), np.asarray(d, dtype=np.complex128)))
    fixed = {}
    for q in range(n):
        fixed[(q, 0)] = 0
    for q in range(n):
        if q in open_qubits:
            continue
        last = (q, seg[q])
        if last in fixed and fixed[last] != int(y[q]):
            # segment 0 is also the output: the amplitude vanishes unless y[q] = 0
            fixed[last] = -1
        else:
            fixed[last] = int(y[q])
    for q in open_qubits:
        if seg[q] == 0:
            raise ValueError("open qubit has no gate acting on it")
    out = []
    zero = any(v < 0 for v in fixed.values())
    for vars_, arr in factors:
        sl = []
        keep = []
        for v in vars_:
            if v in fixed:
                if fixed[v] < 0:
                    zero = True
                    sl.append(0)
                else:
                    sl.append(fixed[v])
            else:
                sl.append(slice(None))
                keep.append(v)
        out.append((tuple(keep), arr[tuple(sl)]))
    open_vars = [(q, seg[q]) for q in open_qubits]
    return out, open_vars, zero


def contract(factors, open_vars) -> np.ndarray:
    """Variable elimination; returns the tensor over open_vars (in order)."""
    scalar = np.complex128(1.0)
    fac: Dict[int, Tuple[Tuple, np.ndarray]] = {}
    for v, a in factors:
        if len(v) == 0:
            scalar = scalar * a
        else:
            fac[len(fac)] = (v, a)
    nid = len(fac)
    open_set = set(open_vars)
    where: Dict = {}
    for fid, (v, _) in fac.items():
        for x in v:
            where.setdefault(x, set()).add(fid)
    free = set(where) - open_set
    while free:
        best = None
        for var in free:
            un = set()
            for fid in where[var]:
                un.update(fac[fid][0])
            key = (len(un) - 1, var)
            if best is None or key < best:
                best = key
        var = best[1]
        bucket_ids = sorted(where[var])
        bucket = [fac.pop(fid) for fid in bucket_ids]
        for fid, (v, _) in zip(bucket_ids, bucket):
            for x in v:
                where[x].discard(fid)
        del where[var]
        free.discard(var)
        allv: List = []
        for v, _ in bucket:
            for x in v:
                if x not in allv:
                    allv.append(x)
        outv = [x for x in allv if x != var]
        ids = {x: i for i, x in enumerate(allv)}
        args = []
        for v, a in bucket:
            args.append(a)
            args.append([ids[x] for x in v])
        args.append([ids[x] for x in outv])
        newa = np.einsum(*args, optimize=False)
        if len(outv) == 0:
            scalar = scalar * newa
        else:
            fac[nid] = (tuple(outv), newa)
            for x in outv:
                where[x].add(nid)
            nid += 1
    # multiply remaining factors over the open variables
    res = np.array(scalar, dtype=np.complex128)
    resv: List = []
    for fid in sorted(fac):
        v, a = fac[fid]
        allv = list(resv)
        for x in v:
            if x not in allv:
                allv.append(x)
        ids = {x: i for i, x in enumerate(allv)}
        res = np.einsum(res, [ids[x] for x in resv], a, [ids[x] for x in v], [ids[x] for x in allv])
        resv = allv
    if open_vars:
        for x in open_vars:
            if x not in resv:
                res = np.multiply.outer(res, np.ones(2, dtype=np.complex128))
                resv = resv + [x]
        perm = [resv.index(x) for x in open_vars]
        res = np.transpose(res, perm)
    return res


def amplitude(circ, n_gates: int, y: Sequence[int], open_qubits: Sequence[int] = ()):
    """amp(C_t, y) with C_t the first n_gates gates; open qubits give an array
    over their values (first open qubit = most significant axis)."""
    fac, open_vars, zero = build_factors(circ, n_gates, y, open_qubits)
    if zero:
        return np.zeros((2,) * len(open_qubits), dtype=np.complex128) if open_qubits else np.complex128(0)
    return contract(fac, open_vars)
