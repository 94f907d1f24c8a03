"""Host planning (no GPU): the emitted step programs, interpreted in numpy,
reproduce the oracle's prefix amplitudes; Proposition 2 (noisy networks keep
the shape of the noiseless ones); slicing; the library loads and exports every
symbol of include/pws.h."""
import ctypes
import os
import re

import numpy as np
import pytest

import instances as I
from oracle import pathsum as PS
from oracle import statevector as SV

from .plan_exec import eval_step, sweep_prefix

E = pytest.importorskip("paper_2510_24218_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _plan(c, **kw):
    return E.Plan(c, host_only=True, **kw)


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "pws.h")).read()
    declared = set(re.findall(r"\b(pws_[a-z_0-9]+)\s*\(", hdr))
    assert {"pws_plan", "pws_amplitudes", "pws_sample", "pws_grad"} <= declared
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2510_24218_amd", "libpws.so"))
    for name in sorted(declared):
        assert hasattr(lib, name), name


def _prefix_check(c, plan, rng, n_states=6, use_sv=True):
    n = c.n_qubits
    worst = 0.0
    for k in range(plan.n_steps()):
        op, gate, m = plan.step_info(k)
        ex = plan.export(k)
        g = c.gates[gate]
        psi = SV.state(c, gate + 1) if use_sv else None
        for _ in range(n_states):
            s = rng.integers(0, 2, n)
            # untouched qubits are 0 in any reachable state
            touched = {q for gg in c.gates[:gate + 1] for q in gg.qubits}
            for q in range(n):
                if q not in touched:
                    s[q] = 0
            got = eval_step(ex, s, plan=plan)
            q = g.qubits[0]
            if use_sv:
                base = sum(int(s[j]) << j for j in range(n)) & ~(1 << q)
                ref = np.array([psi[base], psi[base | (1 << q)]])
            else:
                ref = PS.amplitude(c, gate + 1, s, open_qubits=(q,))
            scale = max(np.abs(ref).max(), 1e-300)
            worst = max(worst, np.abs(got - ref).max() / scale)
    return worst


@pytest.mark.parametrize("planner", [0, 1, 2])
def test_step_programs_match_state_vector_qaoa12(planner, monkeypatch):
    """Node form (contraction trees from each planner)."""
    monkeypatch.setenv("PWS_SWEEP", "0")
    c, _, _ = I.workload_qaoa3reg12()
    p = _plan(c, planner=planner)
    assert all(not p.export(k)["sweep"] for k in range(p.n_steps()))
    assert _prefix_check(c, p, np.random.default_rng(1)) < 1e-12


def test_sweep_programs_match_state_vector_qaoa12():
    """Sweep form (leaves absorbed into an on-chip running tensor)."""
    c, _, _ = I.workload_qaoa3reg12()
    p = _plan(c)
    assert all(p.export(k)["sweep"] for k in range(p.n_steps() - 1))
    assert _prefix_check(c, p, np.random.default_rng(1)) < 1e-12


@pytest.mark.parametrize("sweep", ["0", "13"])
def test_step_programs_match_state_vector_grid4x4(sweep, monkeypatch):
    monkeypatch.setenv("PWS_SWEEP", sweep)
    c, _, _ = I.workload_grid6x8(4, 4)
    assert _prefix_check(c, _plan(c), np.random.default_rng(2), n_states=3) < 1e-12


def test_matrix_core_nodes_match_state_vector(monkeypatch):
    """Node form of FP32 plans: contractions with at least four legs of each
    operand alone run as 16 x 16 matrix-core tiles (kind 2); FP64 plans keep
    the vector forms.  Interpreted in numpy against the state vector."""
    monkeypatch.setenv("PWS_SWEEP", "0")
    c = I.qaoa_maxcut(20, I.random_regular_graph(3, 20, 77), [0.4, 0.9], [0.7, 0.3], name="3reg20_p2")
    p = _plan(c)
    steps = [k for k in range(p.n_steps()) if any(nd["kind"] == 2 for nd in p.export(k)["nodes"])]
    assert len(steps) >= 3, steps
    rng = np.random.default_rng(3)
    for k in steps:
        op, gate, m = p.step_info(k)
        q = c.gates[gate].qubits[0]
        touched = {qq for gg in c.gates[:gate + 1] for qq in gg.qubits}
        s = np.array([rng.integers(0, 2) if qq in touched else 0 for qq in range(c.n_qubits)])
        got = eval_step(p.export(k), s, plan=p)
        ref = PS.amplitude(c, gate + 1, s, open_qubits=(q,))
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), k
    p64 = _plan(c, precision="fp64")
    assert all(nd["kind"] != 2 for k in range(p64.n_steps()) for nd in p64.export(k)["nodes"])


@pytest.mark.parametrize("which", ["grid4x4", "ladder4x4"])
def test_two_sided_steps_match_state_vector(which):
    """Two-sided steps: an anchor step keeps its running tensor at several
    points and later steps contract a sweep of their other leaves with one of
    them over the shared legs; every step still matches the state vector."""
    c = I.workload_grid6x8(4, 4)[0] if which == "grid4x4" else I.workload_ladder4x119(4)[0]
    p = _plan(c)
    exs = [p.export(k) for k in range(p.n_steps() - 1)]
    merges = [ex for ex in exs if ex["merge"]]
    assert merges and any(ex["snaps"] for ex in exs)
    for ex in merges:   # the snapshot comes from an earlier anchor step
        m = ex["merge"]
        assert 0 <= m["step"] and [m["op"], m["slot"]] in [[o, s] for o, s, w in exs[m["step"]]["snaps"]]
    assert _prefix_check(c, p, np.random.default_rng(9), n_states=3) < 1e-12


def _general_circuit(th):
    gates = [I.Gate("H", (0,)), I.Gate("H", (1,)), I.Gate("RX", (2,), param=2),
             I.Gate("CRX", (0, 2), param=0), I.Gate("FSIM", (1, 2), param=1, param2=3),
             I.Gate("RZ", (3,), param=1), I.Gate("H", (3,)), I.Gate("CNOT", (3, 0)),
             I.Gate("CRX", (2, 1), param=2), I.Gate("FSIM", (0, 1), param=0, param2=1)]
    return I.Circuit(4, gates, th)


def test_step_programs_general_gates():
    c = _general_circuit(np.array([0.7, 1.1, 2.0, 0.4]))
    _general_check(c, _plan(c))


def _general_check(c, p):
    rng = np.random.default_rng(3)
    for k in range(p.n_steps()):
        op, gate, m = p.step_info(k)
        g = c.gates[gate]
        ex = p.export(k)
        psi = SV.state(c, gate + 1)
        for _ in range(5):
            s = rng.integers(0, 2, 4)
            got = eval_step(ex, s, plan=p)
            # open qubits: the gate's non-diagonal qubits, first listed = MSB of v
            from oracle import gates as G
            mat = G.gate_matrix(c, g)
            nq = len(g.qubits)
            opn = [g.qubits[j] for j in range(nq)
                   if not all(mat[o, i] == 0 for o in range(2 ** nq) for i in range(2 ** nq)
                              if ((o >> (nq - 1 - j)) & 1) != ((i >> (nq - 1 - j)) & 1))]
            assert len(got) == 2 ** len(opn)
            ref = []
            for v in range(2 ** len(opn)):
                y = s.copy()
                for kk, q in enumerate(opn):
                    y[q] = (v >> (len(opn) - 1 - kk)) & 1
                ref.append(psi[sum(int(y[j]) << j for j in range(4))])
            assert np.allclose(got, ref, atol=1e-13)


def _structure(ex):
    """The plan of a step without its angle-dependent numbers (leaf tables,
    folded constants and term values of the matrix entries)."""
    def op(so):
        d = {k: v for k, v in so.items() if k != "ment"}
        d["ment"] = [(e[2], [t[0] for t in e[3]]) for e in so.get("ment", [])]
        return d
    top = {k: v for k, v in ex.items() if k not in ("leaves", "gates", "sweeps")}
    top["sweeps"] = [op(so) for so in ex.get("sweeps", [])]
    return top, [{k: v for k, v in lf.items() if k != "tab"} for lf in ex["leaves"]]


def test_set_theta_retabulates_without_replanning():
    """New angles: every step program at the new theta matches the state
    vector there (the interpreter also checks each stored leaf table against
    the product of its factors), and the contraction plan is unchanged."""
    import dataclasses
    c, _, _ = I.workload_qaoa3reg12()
    p = _plan(c)
    before = [_structure(p.export(k)) for k in range(p.n_steps())]
    th2 = c.theta + np.array([0.31, -0.22, 0.17, -0.4, 0.05, 0.9])[:len(c.theta)]
    p.set_theta(th2)
    c2 = dataclasses.replace(c, theta=th2)
    assert _prefix_check(c2, p, np.random.default_rng(21), n_states=3) < 1e-12
    assert [_structure(p.export(k)) for k in range(p.n_steps())] == before
    # two-angle gates (FSIM) and controlled rotations
    cg = _general_circuit(np.array([0.7, 1.1, 2.0, 0.4]))
    pg = _plan(cg)
    th3 = np.array([1.3, -0.6, 0.25, 2.2])
    pg.set_theta(th3)
    _general_check(dataclasses.replace(cg, theta=th3), pg)


def test_set_theta_rejects_structure_change():
    """A mixer angle of zero turns RX into the identity (diagonal): the plan
    no longer fits the circuit, the call fails and the old angles stay."""
    c, _, _ = I.workload_qaoa3reg12()
    p = _plan(c)
    bad = c.theta.copy()
    n_layers = len(bad) // 2
    bad[n_layers] = 0.0
    with pytest.raises(E.PwsError):
        p.set_theta(bad)
    with pytest.raises(ValueError):
        p.set_theta(c.theta[:-1])
    assert _prefix_check(c, p, np.random.default_rng(22), n_states=2) < 1e-12


@pytest.mark.parametrize("which", ["grid4x4", "ladder8"])
def test_kept_tensor_equals_next_steps_prefix(which):
    """A step keeps its running tensor after ops [0, store_op) for the next
    step, which restores it instead of running its own ops [0, load_op): both
    prefixes must give the same tensor whatever the chain draws at the first
    step (the drawn qubits, and any others the prefix must not read, get
    different values on the two sides)."""
    c = I.workload_grid6x8(4, 4)[0] if which == "grid4x4" else I.workload_ladder4x119(8)[0]
    p = _plan(c)
    rng = np.random.default_rng(31)
    n, pairs = c.n_qubits, 0
    for k in range(p.n_steps() - 2):
        a, b = p.export(k), p.export(k + 1)
        if a["store_op"] < 0:
            assert b["load_op"] < 0
            continue
        assert b["load_op"] >= 0 and a["store_w"] == b["load_w"]
        pairs += 1
        g = c.gates[a["gate"]]
        s0 = rng.integers(0, 2, n)
        touched = {q for gg in c.gates[:b["gate"] + 1] for q in gg.qubits}
        for q in range(n):
            if q not in touched:
                s0[q] = 0
        for trial in range(2):
            s1 = s0.copy()
            for q in g.qubits:
                s1[q] = rng.integers(0, 2)
            ta = sweep_prefix(a, s0, a["store_op"])
            tb = sweep_prefix(b, s1, b["load_op"])
            w = 2 ** a["store_w"]
            # same cells hold data; values equal up to rounding (the two steps
            # may fold diagonal ops differently around their cache points)
            assert np.array_equal(np.isnan(ta[:w]), np.isnan(tb[:w])), (k, trial)
            ok = ~np.isnan(ta[:w])
            scale = np.abs(ta[:w][ok]).max()
            assert np.abs(ta[:w][ok] - tb[:w][ok]).max() <= 1e-13 * scale, (k, trial)
    assert pairs >= 3


@pytest.mark.parametrize("sweep", ["0", "13"])
def test_step_programs_match_pathsum_grid6x8_sampled(sweep, monkeypatch):
    monkeypatch.setenv("PWS_SWEEP", sweep)
    c, _, _ = I.workload_grid6x8()
    p = _plan(c)
    rng = np.random.default_rng(4)
    steps = [0, 47, 60, 95, 100, 143]
    n = c.n_qubits
    for k in steps:
        op, gate, m = p.step_info(k)
        ex = p.export(k)
        touched = {q for gg in c.gates[:gate + 1] for q in gg.qubits}
        s = rng.integers(0, 2, n)
        for q in range(n):
            if q not in touched:
                s[q] = 0
        got = eval_step(ex, s, plan=p)
        ref = PS.amplitude(c, gate + 1, s, open_qubits=(c.gates[gate].qubits[0],))
        assert np.allclose(got, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_full_network_amplitude():
    c, _, _ = I.workload_qaoa3reg12()
    p = _plan(c)
    ex = p.export(-1)
    psi = SV.state(c)
    rng = np.random.default_rng(5)
    for _ in range(8):
        y = rng.integers(0, 2, 12)
        got = eval_step(ex, y)
        assert got.shape == (1,)
        assert abs(got[0] - psi[sum(int(y[j]) << j for j in range(12))]) < 1e-14


def test_slicing_preserves_amplitudes(monkeypatch):
    c, _, _ = I.workload_grid6x8(4, 4)
    # device-memory form with a budget small enough that arenas must be sliced
    monkeypatch.setenv("PWS_NO_LDS", "1")
    monkeypatch.setenv("PWS_SWEEP", "0")
    p = _plan(c, hbm_budget_bytes=1024 * 4 * 8 * 2 * 256)
    assert p.stats()["n_slices"] > p.n_steps()
    assert _prefix_check(c, p, np.random.default_rng(6), n_states=2) < 1e-12


def test_lds_slicing_preserves_amplitudes(monkeypatch):
    c, _, _ = I.workload_grid6x8(4, 4)
    # LDS form with a small on-chip capacity: every step sliced to fit
    monkeypatch.setenv("PWS_FORM", "lds")
    monkeypatch.setenv("PWS_SWEEP", "0")
    monkeypatch.setenv("PWS_LDS_BYTES", "10240")
    p = _plan(c)
    assert p.stats()["n_slices"] > p.n_steps()
    assert max(p.export(k)["arena_elems"] for k in range(p.n_steps())) * 8 <= 10240
    assert _prefix_check(c, p, np.random.default_rng(7), n_states=2) < 1e-12


@pytest.mark.parametrize("sweep", ["0", "13"])
def test_noisy_plan_has_noiseless_shape(sweep, monkeypatch):
    """Proposition 2: with local-submonomial noise every step's network has the
    shape (and hence the contraction cost) of the noiseless one.  (Tensors
    kept between steps are off here: noise records change between steps, so a
    noisy plan may restore shorter prefixes than the noiseless one.)"""
    monkeypatch.setenv("PWS_SWEEP", sweep)
    monkeypatch.setenv("PWS_SWEEP_CACHE", "0")
    c, _, _ = I.workload_noisy3reg100(n=24)
    pn = _plan(c)
    p0 = _plan(c.without_noise())
    assert pn.n_steps() == p0.n_steps()
    assert pn.stats()["flops_per_sample"] == p0.stats()["flops_per_sample"]
    for k in [0, pn.n_steps() // 2, pn.n_steps() - 1]:
        a, b = pn.export(k), p0.export(k)
        assert [l["nfree"] for l in a["leaves"]] == [l["nfree"] for l in b["leaves"]]
        assert [(d["out_bits"], d["k_bits"]) for d in a["nodes"]] == [(d["out_bits"], d["k_bits"]) for d in b["nodes"]]
        # same ops and entry codes (how an entry is evaluated may differ: noise
        # records make entries chain-dependent)
        strip = lambda ops: [{k: v for k, v in so.items() if k != "ment"} for so in ops]
        assert a["sweep"] == b["sweep"] and strip(a["sweeps"]) == strip(b["sweeps"])


def test_step_count_is_qsize():
    """Proposition 1: one amplitude step per non-monomial gate (qsize)."""
    c, _, _ = I.workload_grid6x8(4, 4)
    p = _plan(c)
    nonmono = sum(1 for g in c.gates if g.kind in ("H", "RX"))
    assert p.n_steps() == nonmono
    assert all(p.step_info(k)[2] == 2 for k in range(p.n_steps()))


def test_plan_rejects_bad_input():
    c = I.Circuit(3, [I.Gate("RX", (5,), param=0)], np.array([0.3]))
    with pytest.raises(E.PwsError) as ei:
        _plan(c)
    assert ei.value.status == 1


def test_sample_batch_rejects_bad_arguments():
    """pws_sample_batch validates its arguments before touching a device."""
    lib = E.load_library()
    assert lib.pws_sample_batch(0, None, None, None, None) == 1   # PWS_ERR_ARG
    c, _, _ = I.workload_qaoa3reg12()
    p = _plan(c)   # host-only: it has no device tables to sample with
    hs = (ctypes.c_void_p * 1)(p._h.value)
    ks = (ctypes.c_int64 * 1)(-1)
    ss = (ctypes.c_uint64 * 1)(1)
    bs = (E._ffi.pws_bits * 1)()
    assert lib.pws_sample_batch(1, hs, ks, ss, bs) == 1           # negative chain count
    out = np.zeros((4, 1), dtype=np.uint64)
    ks[0] = 4
    bs[0] = p._bits_struct(out, 4)
    assert lib.pws_sample_batch(1, hs, ks, ss, bs) != 0           # no device tables


def test_fresh_qubit_steps_are_marked():
    """Steps whose one-qubit gate acts on a qubit no earlier gate touched (the
    QAOA H layer) are drawn from the gate's column 0 in sampling passes; no
    other step is, and the option switches it off."""
    c, _, _ = I.workload_qaoa3reg12()
    p = _plan(c)
    fresh = [p.export(k)["fresh"] for k in range(p.n_steps())]
    kinds = [c.gates[p.step_info(k)[1]].kind for k in range(p.n_steps())]
    assert fresh == [1 if kd == "H" else 0 for kd in kinds] and sum(fresh) == 12
    c2 = I.Circuit(2, [I.Gate("H", (0,)), I.Gate("CNOT", (0, 1)), I.Gate("H", (1,)), I.Gate("H", (0,))],
                   np.zeros(0))
    p2 = _plan(c2)
    assert [p2.export(k)["fresh"] for k in range(p2.n_steps())] == [1, 0, 0]


def test_fresh_qubit_steps_option(monkeypatch):
    monkeypatch.setenv("PWS_FRESH", "0")
    c, _, _ = I.workload_qaoa3reg12()
    p = _plan(c)
    assert not any(p.export(k)["fresh"] for k in range(p.n_steps()))
