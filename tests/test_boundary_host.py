"""The C ABI's planning inputs on the host: a caller's contraction tree for
the full-circuit amplitude network (SSA pairs over the leaves that
pws_plan_export reports), forced sliced legs, and plan options given as
(key, value) pairs instead of defaults."""
import numpy as np
import pytest

import instances as I
from oracle import sampler as S
from oracle import statevector as SV

from .plan_exec import eval_step

E = pytest.importorskip("paper_2510_24218_amd")


def _full_amp(ex, bits):
    return eval_step(ex, np.asarray(bits))[0]


def test_explicit_tree_round_trip_and_left_deep():
    c, _, _ = I.workload_qaoa3reg12()
    p = E.Plan(c, precision="fp64", host_only=True)
    net = p.export(-1)["network"]
    L = len(net["legs"])
    assert len(net["pairs"]) == L - 1
    psi = SV.state(c)
    rng = np.random.default_rng(3)
    bits = rng.integers(0, 2, (6, 12))
    ref = psi[S.basis_index(bits)]
    # the internal tree handed back, and a left-deep order over the leaves
    left_deep = [[0, 1]] + [[L + k - 1, k + 1] for k in range(1, L - 1)]
    for tree in (net["pairs"], left_deep):
        q = E.Plan(c, precision="fp64", host_only=True, tree=tree)
        exq = q.export(-1)
        assert exq["network"]["pairs"] == [list(t) for t in tree]
        got = np.array([_full_amp(exq, b) for b in bits])
        assert np.allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("tree", [[[0, 1]], [[0, 0]], [[0, 1], [1, 2]], [[0, 99]]])
def test_bad_trees_are_rejected(tree):
    c, _, _ = I.workload_qaoa3reg12()
    L = len(E.Plan(c, host_only=True).export(-1)["network"]["legs"])
    full = [list(t) for t in tree] + [[L + k - 1, k + 1] for k in range(len(tree), L - 1)] if len(tree) > 1 else tree
    with pytest.raises(E.PwsError) as e:
        E.Plan(c, host_only=True, tree=full)
    assert "ERR_ARG" in str(e.value)


def test_forced_sliced_legs():
    """Legs the caller asks to slice are sliced in every node-form network
    that contracts them, and the step programs still give the state
    vector's amplitudes."""
    c, _, _ = I.workload_grid6x8(3, 3)
    base = E.Plan(c, host_only=True, options={"sweep_width": 0})
    net = base.export(-1)["network"]
    inner = sorted({l for legs in net["legs"] for l in legs})
    pick = inner[len(inner) // 2: len(inner) // 2 + 2]
    p = E.Plan(c, host_only=True, options={"sweep_width": 0}, sliced=pick)
    n_sliced = [p.export(k)["n_slice_bits"] for k in range(p.n_steps())]
    assert max(n_sliced) >= 1
    rng = np.random.default_rng(4)
    for k in range(p.n_steps()):
        op, gate, m = p.step_info(k)
        q = c.gates[gate].qubits[0]
        psi = SV.state(c, gate + 1)
        touched = {qq for g in c.gates[:gate + 1] for qq in g.qubits}
        s = rng.integers(0, 2, c.n_qubits)
        for qq in range(c.n_qubits):
            if qq not in touched:
                s[qq] = 0
        got = eval_step(p.export(k), s, plan=p)
        base_i = S.basis_index(s[None, :])[0] & ~(1 << q)
        assert np.allclose(got, [psi[base_i], psi[base_i | (1 << q)]], atol=1e-13)
    with pytest.raises(E.PwsError):
        E.Plan(c, host_only=True, sliced=[10 ** 6])


def test_plan_options():
    c, _, _ = I.workload_grid6x8(4, 4)
    node = E.Plan(c, host_only=True, options={"sweep_width": 0})
    assert not any(node.export(k)["sweep"] for k in range(node.n_steps()))
    sweep = E.Plan(c, host_only=True)
    assert all(sweep.export(k)["sweep"] for k in range(sweep.n_steps()))
    nofresh = E.Plan(c, host_only=True, options={"fresh": 0})
    assert sum(nofresh.export(k)["fresh"] for k in range(nofresh.n_steps())) == 0
    import ctypes as C
    from paper_2510_24218_amd import _ffi
    lib = _ffi.load()
    bad = (_ffi.pws_option * 1)(_ffi.pws_option(999, 1))
    sl = _ffi.pws_slices(0, 0, 1, None, 0, 1, 0, 1, 0, bad)
    h = C.c_void_p()
    st = lib.pws_plan(None, None, None, C.byref(sl), C.byref(h))
    assert st == _ffi.PWS_ERR_ARG and b"unknown plan option" in lib.pws_last_error()
