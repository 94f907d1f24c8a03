"""Closed form (QAOA p=1), path sums and gradients of the oracle."""
import math

import numpy as np
import pytest

import instances as I
from oracle import closed_form as CF
from oracle import gradient as GR
from oracle import pathsum as PS
from oracle import sampler as S
from oracle import statevector as SV


def _zz_from_sv(c, u, v):
    psi = SV.state(c)
    p = psi.real ** 2 + psi.imag ** 2
    idx = np.arange(len(p))
    z = (1 - 2 * ((idx >> u) & 1)) * (1 - 2 * ((idx >> v) & 1))
    return float(np.sum(p * z))


@pytest.mark.parametrize("name,n,edges", [
    ("3reg12", 12, I.random_regular_graph(3, 12, 1001)),
    ("K4", 4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]),
    ("triangle_tail", 5, [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4)]),
    ("cube", 8, [(0, 1), (1, 3), (3, 2), (2, 0), (4, 5), (5, 7), (7, 6), (6, 4),
                 (0, 4), (1, 5), (2, 6), (3, 7)]),
])
def test_p1_closed_form_matches_state_vector(name, n, edges):
    for g, b in [(0.37, 1.21), (2.5, 0.4), (1.0, 2.9)]:
        c = I.qaoa_maxcut(n, edges, [g], [b])
        zz = CF.zz_expectation(n, c.edges, g, b)
        for (u, v), val in zz.items():
            assert abs(_zz_from_sv(c, u, v) - val) < 1e-12


def test_pathsum_matches_state_vector_prefixes():
    rng = np.random.default_rng(5)
    for c in [I.workload_qaoa3reg12()[0], I.workload_grid6x8(4, 4)[0]]:
        n = c.n_qubits
        for t in rng.integers(1, len(c.gates) + 1, 12):
            psi = SV.state(c, int(t))
            y = rng.integers(0, 2, n)
            q = int(rng.integers(0, n))
            # only ask for open qubits that a gate has touched
            touched = {qq for g in c.gates[:t] for qq in g.qubits}
            if q not in touched:
                continue
            a = PS.amplitude(c, int(t), y, open_qubits=(q,))
            base = sum(int(y[k]) << k for k in range(n)) & ~(1 << q)
            assert np.allclose(a, [psi[base], psi[base | (1 << q)]], atol=1e-14)
            full = PS.amplitude(c, int(t), y)
            assert abs(full - psi[sum(int(y[k]) << k for k in range(n))]) < 1e-14


def test_pathsum_gamma_zero_product_state():
    """gamma = 0: the state is a product, amp(y) = prod_q <y_q| RX(b) H |0>."""
    c = I.qaoa_maxcut(48, I.grid_graph(6, 8), [0.0, 0.0], [0.7, 0.5])
    rng = np.random.default_rng(1)
    y = rng.integers(0, 2, 48)
    b = 0.7 + 0.5
    one = [(math.cos(b / 2) - 1j * math.sin(b / 2)) / math.sqrt(2)] * 2
    ref = np.prod([one[int(v)] for v in y])
    assert abs(PS.amplitude(c, len(c.gates), y) - ref) < 1e-14 * 1e3 * abs(ref) + 1e-30


def test_adjoint_gradient_matches_finite_differences():
    edges = I.random_regular_graph(3, 10, 4001)
    c = I.qaoa_maxcut(10, edges, [0.4, 1.3, 0.2], [1.1, 0.5, 2.0])
    allbits = ((np.arange(2 ** 10)[:, None] >> np.arange(10)) & 1)
    cost = I.maxcut_value(c.edges, allbits).astype(float)
    E, g = GR.objective_and_gradient(c, cost)
    h = 1e-5
    for j in range(6):
        tp = c.theta.copy(); tp[j] += h
        tm = c.theta.copy(); tm[j] -= h
        Ep, _ = GR.objective_and_gradient(c.with_theta(tp), cost)
        Em, _ = GR.objective_and_gradient(c.with_theta(tm), cost)
        assert abs((Ep - Em) / (2 * h) - g[j]) < 1e-7


def test_adjoint_gradient_matches_p1_closed_form():
    n = 12
    edges = I.random_regular_graph(3, n, 1001)
    gm, bt = 0.63, 1.9
    c = I.qaoa_maxcut(n, edges, [gm], [bt])
    allbits = ((np.arange(2 ** n)[:, None] >> np.arange(n)) & 1)
    cost = I.maxcut_value(c.edges, allbits).astype(float)
    E, g = GR.objective_and_gradient(c, cost)
    assert abs(E - CF.expected_cut(n, c.edges, gm, bt)) < 1e-12
    assert np.allclose(g, CF.expected_cut_gradient(n, c.edges, gm, bt), atol=1e-7)


def test_per_sample_score_matches_finite_differences():
    edges = I.random_regular_graph(3, 8, 4002)
    c = I.qaoa_maxcut(8, edges, [0.4, 1.3, 0.2], [1.1, 0.5, 2.0])
    idx = np.array([0, 5, 77, 200, 255])
    sc = GR.score(c, idx)
    fd = GR.score_fd(c, idx)
    assert np.allclose(sc, fd, rtol=1e-6, atol=1e-6)


def test_score_function_identity_and_estimator():
    """E[d log p] = 0 and the score estimator of grad E[C] agrees with the
    adjoint gradient within 4 standard errors."""
    n = 10
    edges = I.random_regular_graph(3, n, 4003)
    c = I.qaoa_maxcut(n, edges, [0.5, 0.9], [1.2, 0.3])
    bits = S.sample_ideal(c, 20000, 4003)
    idx = S.basis_index(bits)
    sc = GR.score(c, idx)
    se0 = sc.std(axis=0) / math.sqrt(len(idx))
    assert np.all(np.abs(sc.mean(axis=0)) < 4 * se0)
    cost = I.maxcut_value(c.edges, bits).astype(float)
    allbits = ((np.arange(2 ** n)[:, None] >> np.arange(n)) & 1)
    _, g = GR.objective_and_gradient(c, I.maxcut_value(c.edges, allbits).astype(float))
    terms = (cost - cost.mean())[:, None] * sc
    est = terms.mean(axis=0)
    se = terms.std(axis=0) / math.sqrt(len(idx))
    assert np.all(np.abs(est - g) < 4 * se + 1e-3)


def test_pathsum_log_amp_gradient_matches_score():
    edges = I.random_regular_graph(3, 8, 4004)
    c = I.qaoa_maxcut(8, edges, [0.4, 1.3], [1.1, 0.5])
    y = np.array([1, 0, 1, 1, 0, 0, 1, 0])
    idx = np.array([sum(int(y[k]) << k for k in range(8))])
    assert np.allclose(GR.log_amp_gradient_pathsum(c, y), GR.score(c, idx)[0], rtol=1e-5, atol=1e-6)


def test_golden_20q_p3_scores_two_ways():
    """The stored per-sample scores of the 20-qubit p=3 instance (written by
    tests/golden/make_grad_3reg20_p3.py from the oracle only): forward-mode
    state-vector derivatives and FP64 central differences agree to the
    difference error (h^2 terms and rounding / h), and the stored
    bitstrings are the oracle's Algorithm 1 chains for that seed."""
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "grad_3reg20_p3.json")))
    score = np.array(d["score"])
    fd = np.array(d["score_fd"])
    assert score.shape == (64, 6) and np.all(np.isfinite(score))
    rel = np.linalg.norm(score - fd, axis=1) / np.linalg.norm(score, axis=1)
    assert rel.max() < 1e-5
    # not a trivial fixture: the per-sample scores are O(1) and differ across samples
    assert np.median(np.abs(score)) > 0.1 and np.std(score[:, 0]) > 0.1
    c, _, seed = I.workload_grad3reg64(20)
    assert seed == d["seed"]
    bits = S.sample_ideal(c, 8, seed)
    assert np.array_equal(bits, np.array(d["bits"][:8]))
