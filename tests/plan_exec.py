"""Test-side interpreter of the engine's exported step programs (numpy).

It evaluates the leaf and node descriptors that the device kernels execute
(factor sources, output modes, strides, contraction-offset tables, root
indexing, index slices) in complex128, without exponent renormalisation, so
that host planning can be checked against the oracle on a machine without a
GPU.  It shares no code with the engine or with the oracle."""
from __future__ import annotations

import numpy as np

SRC_FREE, SRC_CONST, SRC_CHAIN, SRC_SLICE = 0, 1, 2, 3


def _gate_mats(ex):
    mats = []
    for g in ex["gates"]:
        d = 2 ** g["nq"]
        v = np.array(g["mat"], dtype=np.float64)
        mats.append((v[0::2] + 1j * v[1::2]).reshape(d, d))
    return mats


def sweep_prefix(ex, s_bits, n_ops, mats=None):
    """Running tensor of a sweep-form step after its first n_ops ops, for chain
    bits s_bits (cells that hold no data are NaN)."""
    mats = _gate_mats(ex) if mats is None else mats
    vals_by_leaf = [_leaf_values(lf, np.asarray(s_bits), 0, mats) for lf in ex["leaves"]]
    T = np.full(2 ** ex["sw_width"], np.nan + 0j)
    T[0] = 1.0
    sweep_ops(ex, vals_by_leaf, 0, n_ops, T, s_bits)
    return T


def eval_step(ex, s_bits, mats=None, plan=None):
    """Candidate amplitudes (2^nS,) of an exported step for chain bits s_bits (n,).
    A two-sided step (its sweep contracted with an anchor step's kept tensor)
    needs `plan` (the Plan that exported it) to rebuild that tensor."""
    mats = _gate_mats(ex) if mats is None else mats
    s_bits = np.asarray(s_bits)
    for q in ex["zero_q"]:
        if s_bits[q]:
            return np.zeros(2 ** ex["nS"], dtype=np.complex128)
    acc = np.zeros(2 ** ex["nS"], dtype=np.complex128)
    # the flat element list covers every (step-local leaf, element) pair once
    el = np.array(ex["elems"], dtype=np.int64).reshape(-1, 2)
    want = [(i, e) for i, lf in enumerate(ex["leaves"]) for e in range(2 ** lf["nfree"])]
    assert sorted(map(tuple, el.tolist())) == want
    size = max(ex["arena_elems"], 2) + 64
    for sl in range(2 ** ex["n_slice_bits"]):
        vals_by_leaf = [_leaf_values(lf, s_bits, sl, mats) for lf in ex["leaves"]]
        m = 2 ** ex["nS"]
        if ex.get("sweep"):
            R = None
            if ex.get("merge"):
                assert plan is not None, "two-sided step: pass the plan"
                m = ex["merge"]
                # the anchor's running tensor after m["op"] ops, for the same
                # chain bits (its leaves read none that changed since it ran)
                R = sweep_prefix(plan.export(m["step"]), s_bits, m["op"])
            acc += _run_sweep(ex, vals_by_leaf, s_bits, R)
            continue
        arena = np.full(size, np.nan + 0j)
        for lf, vals in zip(ex["leaves"], vals_by_leaf):
            arena[lf["off"]:lf["off"] + len(vals)] = vals
        for nd in ex["nodes"]:
            _run_node(nd, arena)
        acc += np.array([arena[ex["root_off"] + ex["root_index"][v]] for v in range(m)])
    return acc * step_scalar(ex, s_bits, mats)


def step_scalar(ex, s_bits, mats=None):
    """Product of the step's fixed-leg factors: one scalar per chain, common
    to every candidate (draws skip it, amplitudes carry it)."""
    mats = _gate_mats(ex) if mats is None else mats
    acc = 1.0 + 0j
    for (kind, gid, nq, frame, so0, so1, si0, si1) in ex.get("scalars", []):
        def fbit(src):
            t, pl = src >> 24, src & 0xFFFFFF
            assert t in (SRC_CONST, SRC_CHAIN)
            return pl if t == SRC_CONST else int(s_bits[pl])
        out = inn = 0
        for j in range(nq):
            out = 2 * out + fbit([so0, so1][j])
            inn = 2 * inn + fbit([si0, si1][j])
        acc = acc * mats[gid][out, inn]
    return acc


def _leaf_values(lf, s_bits, sl, mats):
    """Elements of one leaf: the product of its factors (checked against the
    stored table of its chain variant when the leaf is tabulated)."""
    ne = 2 ** lf["nfree"]
    vals = np.ones(ne, dtype=np.complex128)
    table = None
    if lf["tab_off"] >= 0:
        v = 0
        for k, code in enumerate(lf["var"]):
            t, pl = code >> 24, code & 0xFFFFFF
            assert t in (0, 1), "interpreter covers chain and slice variant bits"
            b = int(s_bits[pl]) if t == 0 else (sl >> pl) & 1
            v |= b << k
        tv = np.array(lf["tab"], dtype=np.float64)
        tv = tv[0::2] + 1j * tv[1::2]
        table = tv[v * ne:(v + 1) * ne]
    for (kind, gid, nq, frame, so0, so1, si0, si1) in lf["factors"]:
        assert kind == 0 and frame == 0, "interpreter covers ideal gate factors"
        e = np.arange(ne)

        def bit(src):
            t, pl = src >> 24, src & 0xFFFFFF
            if t == SRC_FREE:
                return (e >> pl) & 1
            if t == SRC_CONST:
                return np.full(ne, pl)
            if t == SRC_CHAIN:
                return np.full(ne, int(s_bits[pl]))
            return np.full(ne, (sl >> pl) & 1)

        srcs_out = [so0, so1][:nq]
        srcs_in = [si0, si1][:nq]
        out = np.zeros(ne, dtype=np.int64)
        inn = np.zeros(ne, dtype=np.int64)
        for j in range(nq):
            out = 2 * out + bit(srcs_out[j])
            inn = 2 * inn + bit(srcs_in[j])
        vals = vals * mats[gid][out, inn]
    if table is not None:
        # the stored variant must equal the product of the leaf's factors
        assert np.allclose(table, vals, rtol=1e-14, atol=1e-15)
        vals = table
    return vals


_KEEP, _SUM, _NEW, _REPLACE = 0, 1, 2, 3


def _run_sweep(ex, vals_by_leaf, s_bits=None, R=None):
    """Sweep form: leaves absorbed one by one into a running tensor with
    sw_width bit positions, updated in place group by group.  Cells that the
    program must never read (free positions at 1) hold NaN.  A two-sided step
    ends with the contraction of that tensor with the kept tensor R over the
    shared legs (position here, position in R)."""
    W = ex["sw_width"]
    T = np.full(2 ** W, np.nan + 0j)
    T[0] = 1.0
    sweep_ops(ex, vals_by_leaf, 0, len(ex["sweeps"]), T, s_bits)
    m = 2 ** ex["nS"]
    if ex.get("merge"):
        pairs = ex["merge"]["pairs"]
        out = np.zeros(m, dtype=np.complex128)
        for b in range(2 ** len(pairs)):
            it = sum(((b >> k) & 1) << pt for k, (pt, pr) in enumerate(pairs))
            ir = sum(((b >> k) & 1) << pr for k, (pt, pr) in enumerate(pairs))
            for v in range(m):
                out[v] += T[it | ex["root_index"][v]] * R[ir]
    else:
        out = np.array([T[ex["root_index"][v]] for v in range(m)])
    assert not np.any(np.isnan(out))
    return out


def _folded_entry(me, s_bits):
    """A matrix entry in the folded form the kernels read: constant times the
    chain-dependent terms looked up by the chain bits they name."""
    v = complex(me[0], me[1])
    for term in me[3]:
        pos, tab = term[0], term[1:]
        var = sum(int(s_bits[q]) << k for k, q in enumerate(pos))
        v *= complex(tab[2 * var], tab[2 * var + 1])
    return v


def sweep_ops(ex, vals_by_leaf, lo, hi, T, s_bits=None):
    """Apply the step's sweep ops [lo, hi) to the running tensor T in place.
    With the chain bits s_bits, every folded matrix entry (constants folded on
    the host, chain-dependent terms tabulated) is checked against the product
    of its codes."""
    W = ex["sw_width"]
    for so in ex["sweeps"][lo:hi]:
        L = vals_by_leaf[so["leaf"]]
        k_np, pos, role, legs = so["np"], so["pos"], so["role"], so["leg"]
        assert len(L) == 2 ** len(legs)
        n = 1 << k_np
        # the op's matrix from its entry codes: each entry is a product of
        # factors, each a leaf element (summed over the leaf's internal legs)
        codes = so["mtab"]
        nt = len(codes) // (n if so["diag"] == 1 else n * n)
        assert nt * (n if so["diag"] == 1 else n * n) == len(codes)
        M = np.zeros((n, n), dtype=np.complex128)
        single = True
        for idx in range(len(codes) // nt):
            o, i = (idx, idx) if so["diag"] == 1 else divmod(idx, n)
            val = 1.0 + 0j
            for t in range(nt):
                code = codes[idx * nt + t] & 0xFFFFFFFF
                if code & 0x80000000:
                    val = 0.0
                    break
                if code & 0x40000000:
                    continue
                if t > 0:
                    single = False
                e0, im = (code >> 16) & 15, (code >> 20) & 15
                Lf = vals_by_leaf[code & 0xFFFF]
                val = val * sum(Lf[e0 | sub] for sub in range(16) if sub & im == sub)
            # structural zeros: kept positions equal, created inputs and summed outputs at 0
            if not ((so["out_mask"] >> o) & 1 and (so["in_mask"] >> i) & 1) or any(
                    role[j] == _KEEP and ((o >> j) & 1) != ((i >> j) & 1) for j in range(k_np)):
                assert val == 0
            M[o, i] = val
            if s_bits is not None and "ment" in so and not so["ment"][idx][2]:
                fv = _folded_entry(so["ment"][idx], s_bits)
                assert abs(fv - val) <= 1e-13 * max(1.0, abs(val)), (idx, fv, val)
        if so["diag"] == 2:
            assert k_np == 2 and role[1] == _KEEP and role[0] != _KEEP
        assert (so["diag"] == 1) == all(r == _KEEP for r in role)
        if single:
            # one factor: the entry codes must follow from the roles and leg codes
            internal = [k for k, code in enumerate(legs) if code & 16]
            M1 = np.zeros((n, n), dtype=np.complex128)
            for o in range(n):
                if not (so["out_mask"] >> o) & 1:
                    continue
                for i in range(n):
                    if not (so["in_mask"] >> i) & 1:
                        continue
                    if any(role[j] == _KEEP and ((o >> j) & 1) != ((i >> j) & 1) for j in range(k_np)):
                        continue
                    for t in range(2 ** len(internal)):
                        e = 0
                        for k, code in enumerate(legs):
                            if code & 16:
                                b = (t >> internal.index(k)) & 1
                            else:
                                b = (((o if code & 8 else i) >> (code & 7)) & 1)
                            e |= b << k
                        M1[o, i] += L[e]
            assert np.array_equal(M, M1), "matrix entry codes disagree with the op's roles and legs"
        outer = [q for q in range(W) if (so["outer_mask"] >> q) & 1]
        assert len(outer) == so["n_outer"] and so["outer_mask"] < 2 ** W
        assert not set(outer) & set(pos[:k_np]), "an op position is also an outer position"
        g = np.arange(2 ** so["n_outer"], dtype=np.int64)
        base = np.zeros_like(g)
        for t, q in enumerate(outer):
            base |= ((g >> t) & 1) << q
        idx = base[:, None] + np.array([sum(((x >> j) & 1) << pos[j] for j in range(k_np)) for x in range(n)],
                                       dtype=np.int64)[None, :]
        assert idx.max() < len(T) and len(np.unique(idx)) == idx.size, "groups overlap"
        rd = [i for i in range(n) if (so["in_mask"] >> i) & 1]
        wr = [o for o in range(n) if (so["out_mask"] >> o) & 1]
        vin = T[idx[:, rd]]
        assert not np.any(np.isnan(vin)), "sweep op read a cell that holds no data"
        T[idx[:, wr]] = vin @ M[np.ix_(wr, rd)].T
        # a closed leg's 1-half holds no data from here on
        gone = [o for o in range(n) if not (so["out_mask"] >> o) & 1]
        T[idx[:, gone]] = np.nan


def _run_node(nd, arena):
    """One node: generic (lanes over all output legs), blocked (lanes over
    the output legs of operand A, registers over the N legs) or matrix-core
    tiles (16 rows of A-only legs by 16 columns of B-only legs per tile)."""
    P = 2 ** nd["p_bits"]
    p = np.arange(P)
    offA = np.zeros(P, dtype=np.int64)
    offB = np.zeros(P, dtype=np.int64)
    offO = np.zeros(P, dtype=np.int64)
    rem = p.copy()
    for (w, sa, sb, so) in nd["modes"]:
        v = rem & ((1 << w) - 1)
        rem >>= w
        offA += v * sa
        offB += v * sb
        offO += v * so
    kt = np.array(nd["ktab"], dtype=np.int64).reshape(-1, 2)
    nout = 2 ** nd["out_bits"]
    out = np.full(nout, np.nan + 0j)
    if nd["kind"] == 2:
        # matrix-core tiles: offA / offB / offO are the tiles' offsets
        tt = np.array(nd["ntab"], dtype=np.int64).reshape(4, 16)
        rowA, rowO, colB, colO = tt
        for t in range(P):
            A = arena[nd["a"] + offA[t] + rowA[:, None] + kt[None, :, 0]]          # 16 x K
            B = arena[nd["b"] + offB[t] + colB[None, :] + kt[:, 1][:, None]]       # K x 16
            idx = offO[t] + rowO[:, None] + colO[None, :]
            assert np.all(np.isnan(out[idx])), "output written twice"
            out[idx] = A @ B
    elif nd["kind"] == 1:
        nt = np.array(nd["ntab"], dtype=np.int64).reshape(-1, 2)
        A = arena[nd["a"] + offA[:, None] + kt[None, :, 0]]
        for (nb, no) in nt:
            B = arena[nd["b"] + offB[:, None] + nb + kt[None, :, 1]]
            idx = offO + no
            assert np.all(np.isnan(out[idx])), "output written twice"
            out[idx] = np.sum(A * B, axis=1)
    else:
        assert np.array_equal(offO, p), "generic node output must be in lane order"
        A = arena[nd["a"] + offA[:, None] + kt[None, :, 0]]
        B = arena[nd["b"] + offB[:, None] + kt[None, :, 1]]
        out[:] = np.sum(A * B, axis=1)
    assert not np.any(np.isnan(out)), "node left an output unwritten or read an unwritten cell"
    arena[nd["out"]:nd["out"] + nout] = out


def _bf16_value(h):
    """Value of a bf16 encoding (the high half of an FP32 encoding)."""
    return np.array([h << 16], dtype=np.uint32).view(np.float32)[0].astype(np.float64)


def dense_table(d, r, var):
    """F of run r for chain-bit variant var, 16 x 16 complex.  FP32 tables:
    entry (u, w) as the words re, im at 2 (16 w + u).  bf16 tables: entry
    (u, w) is hi + lo; part p (0: hi, 1: lo) of the pair (Re F[u][w],
    -Im F[u][w]) sits in word 256 p + 4 (16 (w // 4) + u) + w % 4, the real
    part in the low half."""
    w = np.array(r["F"][var * 512:(var + 1) * 512], dtype=np.uint64).astype(np.uint32)
    if not d["bf16"]:
        v = w.view(np.float32).astype(np.float64)
        return (v[0::2] + 1j * v[1::2]).reshape(16, 16).T
    F = np.zeros((16, 16), dtype=np.complex128)
    for u in range(16):
        for col in range(16):
            re = im = 0.0
            for p in range(2):
                q = int(w[256 * p + 4 * (16 * (col // 4) + u) + col % 4])
                re += _bf16_value(q & 0xFFFF)
                im -= _bf16_value(q >> 16)
            F[u, col] = re + 1j * im
    return F


def dense_runs(ex, s_bits, T=None, start=None):
    """Dense-run form of a sweep step: each run is one 16 x 16 complex matrix
    F (the table of this chain's variant) applied to the running tensor viewed
    as 16 rows (the run's four positions, row bit b at pos[b]) by the columns
    of the other live positions.  Free cells hold zeros here (as on the
    device).  T: the tensor at the first run applied (default: the tensor of
    a fresh step, 1 at cell 0); start: index of that run.  Returns T after the
    last run."""
    d = ex["dense"]
    W = d["w"]
    if T is None:
        T = np.zeros(2 ** W, dtype=np.complex128)
        T[0] = 1.0
    runs = d["runs"][start or 0:]
    for r in runs:
        pos = r["pos"]
        assert len(set(pos)) == 4 and max(pos) < W
        outer = [q for q in range(W) if (r["outer_mask"] >> q) & 1]
        assert len(outer) == r["n_outer"] and not set(outer) & set(pos)
        var = sum(int(s_bits[q]) << b for b, q in enumerate(r["qubits"]))
        F = dense_table(d, r, var)
        rows = np.array([sum(((v >> b) & 1) << pos[b] for b in range(4)) for v in range(16)], dtype=np.int64)
        g = np.arange(2 ** len(outer), dtype=np.int64)
        cols = np.zeros_like(g)
        for t, q in enumerate(outer):
            cols |= ((g >> t) & 1) << q
        idx = rows[:, None] | cols[None, :]
        assert len(np.unique(idx)) == idx.size
        T[idx] = F @ T[idx]
    return T


def dense_step(ex, s_bits, plan=None):
    """Candidate amplitudes of a step through its dense runs (the runs must
    start at op 0; a two-sided step needs `plan` for the anchor's tensor),
    times the step's fixed-leg scalar."""
    d = ex["dense"]
    assert d["op0"] == 0
    m = 2 ** ex["nS"]
    for q in ex["zero_q"]:          # qubits no non-diagonal gate has touched
        if s_bits[q]:
            return np.zeros(m, dtype=np.complex128)
    T = dense_runs(ex, s_bits)
    sc = step_scalar(ex, s_bits)
    if ex.get("merge"):
        mg = ex["merge"]
        R = sweep_prefix(plan.export(mg["step"]), s_bits, mg["op"])
        out = np.zeros(m, dtype=np.complex128)
        for b in range(2 ** len(mg["pairs"])):
            it = sum(((b >> k) & 1) << pt for k, (pt, pr) in enumerate(mg["pairs"]))
            ir = sum(((b >> k) & 1) << pr for k, (pt, pr) in enumerate(mg["pairs"]))
            for v in range(m):
                out[v] += T[it | ex["root_index"][v]] * R[ir]
        return out * sc
    return np.array([T[ex["root_index"][v]] for v in range(m)]) * sc
