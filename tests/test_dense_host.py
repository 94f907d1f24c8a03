"""Dense-run form of the sweep steps, checked on the host: the runs' F tables
(products of the ops' matrices for each value of the chain bits they read),
applied by the test-side interpreter, give the state vector's candidate
amplitudes at every step; the runs cover the ops from op 0 and start again
where a sampling pass restores a kept tensor."""
import numpy as np
import pytest

import instances as I
from oracle import sampler as S
from oracle import statevector as SV

from . import plan_exec as X

E = pytest.importorskip("paper_2510_24218_amd")


def _plan(c, **kw):
    return E.Plan(c, host_only=True, **kw)


def _reachable(c, gate, rng):
    s = rng.integers(0, 2, c.n_qubits)
    touched = {q for g in c.gates[:gate + 1] for q in g.qubits}
    for q in range(c.n_qubits):
        if q not in touched:
            s[q] = 0
    return s


@pytest.mark.parametrize("name", ["qaoa12", "grid4x4", "ladder4x4"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_dense_runs_match_state_vector(name, prec):
    c = {"qaoa12": I.workload_qaoa3reg12()[0], "grid4x4": I.workload_grid6x8(4, 4)[0],
         "ladder4x4": I.workload_ladder4x119(4)[0]}[name]
    p = _plan(c, precision=prec, dense=True)
    rng = np.random.default_rng(3)
    n_dense = 0
    worst = 0.0
    for k in range(p.n_steps()):
        ex = p.export(k)
        if ex["dense"] is None:
            assert ex["fresh"] or not ex["sweep"]
            continue
        n_dense += 1
        op, gate, m = p.step_info(k)
        psi = SV.state(c, gate + 1)
        q = c.gates[gate].qubits[0]
        for _ in range(4):
            s = _reachable(c, gate, rng)
            got = X.dense_step(ex, s, plan=p)
            base = S.basis_index(s[None, :])[0] & ~(1 << q)
            ref = np.array([psi[base], psi[base | (1 << q)]])
            worst = max(worst, np.linalg.norm(got - ref) / np.linalg.norm(ref))
            # the runs from the restore point on, started from the kept
            # prefix (the VALU sweep's tensor after load_op ops), agree too
            if ex["load_op"] > 0:
                T = X.sweep_prefix(ex, s, ex["load_op"])
                T = np.where(np.isnan(T), 0, T)
                T = np.concatenate([T, np.zeros(2 ** ex["dense"]["w"] - len(T))])
                start = ex["dense"]["load"]
                runs = ex["dense"]["runs"]
                # the restore point starts a run, or no run is left after it
                assert start == len(runs) or runs[start]["op"] == ex["load_op"]
                assert all(r["op"] < ex["load_op"] for r in runs[:start])
                T = X.dense_runs(ex, s, T, start)
                if not ex.get("merge"):
                    got2 = np.array([T[ex["root_index"][v]] for v in range(2 ** ex["nS"])]) * X.step_scalar(ex, s)
                    assert np.linalg.norm(got2 - ref) <= (1e-5 if prec == "fp32" else 2e-4) * np.linalg.norm(ref)
    assert n_dense > 0
    # the tables hold the products formed in double, rounded once to FP32
    # or to a bf16 pair (about 16 bits)
    assert worst < (1e-5 if prec == "fp32" else 2e-4), worst


def test_dense_runs_fewer_than_ops():
    """Runs merge consecutive ops (6x8 grid: several ops per run)."""
    c = I.workload_grid6x8()[0]
    p = _plan(c, precision="bf16x3")
    n_ops = n_runs = 0
    for k in range(p.n_steps()):
        ex = p.export(k)
        if ex["dense"] is None:
            continue
        n_ops += len(ex["sweeps"]) - ex["dense"]["op0"]
        n_runs += len(ex["dense"]["runs"])
        for r in ex["dense"]["runs"]:
            assert len(r["F"]) == 512 * 2 ** len(r["qubits"])
    assert n_runs > 0 and n_ops > 2.5 * n_runs, (n_ops, n_runs)


def test_noisy_plans_keep_the_vector_form():
    c = I.add_qaoa_noise(I.workload_grid6x8(3, 3)[0], depol2=0.05, ampdamp=0.05)
    p = _plan(c, precision="bf16x3")
    assert all(p.export(k)["dense"] is None for k in range(p.n_steps()))


def test_dense_tables_follow_new_angles():
    """pws_set_theta rewrites the dense runs' tables in place: the same runs,
    and tables equal to those of a plan made at the new angles."""
    c = I.workload_grid6x8(4, 4)[0]
    theta2 = np.array([0.31, 1.7, 2.2, 0.45])
    p = _plan(c, precision="bf16x3")
    p.set_theta(theta2)
    q = _plan(c.with_theta(theta2), precision="bf16x3")
    for k in range(p.n_steps()):
        a, b = p.export(k)["dense"], q.export(k)["dense"]
        assert (a is None) == (b is None)
        if a is None:
            continue
        assert [r["op"] for r in a["runs"]] == [r["op"] for r in b["runs"]]
        for ra, rb in zip(a["runs"], b["runs"]):
            assert ra["F"] == rb["F"]
