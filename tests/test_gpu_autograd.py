"""GPU: new angles without re-planning (pws_set_theta) and the autograd layer
(log-probability with adjoint backward, score-function expectation) against
the oracle's state vector and adjoint gradients."""
import dataclasses

import numpy as np
import pytest

import instances as I
from oracle import gradient as GR
from oracle import sampler as S
from oracle import statevector as SV

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2510_24218_amd")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_24218_amd import autograd as AG  # noqa: E402


def _circuit10(p=3, seed=4005):
    edges = I.random_regular_graph(3, 10, seed)
    g = [0.4, 1.3, 0.2][:p]
    b = [1.1, 0.5, 2.0][:p]
    return I.qaoa_maxcut(10, edges, g, b)


def _cut_cost(edges):
    e = torch.tensor(edges, dtype=torch.int64, device="cuda")

    def cost(x):
        w = x[:, 0]
        return (((w[:, None] >> e[None, :, 0]) ^ (w[:, None] >> e[None, :, 1])) & 1).sum(1).to(torch.float64)
    return cost


def _cut_vector(c):
    idx = np.arange(2 ** c.n_qubits)
    bits = ((idx[:, None] >> np.arange(c.n_qubits)[None, :]) & 1)
    return I.maxcut_value(c.edges, bits).astype(np.float64)


def test_set_theta_sampling_and_amplitudes_follow_new_angles():
    """Captured sampling graph and lazily built amplitude program keep working
    after new angles: FP64 chains stay bit-exact with the oracle at theta2."""
    c, _, seed = I.workload_qaoa3reg12()
    p = E.Plan(c, precision="fp64")
    rng = np.random.default_rng(31)
    bits = rng.integers(0, 2, (200, 12))
    a1, e1 = p.amplitudes(I.pack_bits(bits))
    assert np.array_equal(I.unpack_bits(p.sample(500, seed), 12), S.sample_ideal(c, 500, seed))
    th2 = c.theta * 0.7 + 0.05
    c2 = c.with_theta(th2)
    p.set_theta(th2)
    out = torch.zeros((500, 1), dtype=torch.int64, device="cuda")
    for r in range(3):   # graph replays with the rewritten tables
        p.sample(500, seed + r, out=out)
        torch.cuda.synchronize()
        got = I.unpack_bits(out.cpu().numpy().view(np.uint64), 12)
        assert np.array_equal(got, S.sample_ideal(c2, 500, seed + r))
    m, ex = p.amplitudes(I.pack_bits(bits))
    ref = SV.state(c2)[S.basis_index(bits)]
    assert np.max(np.abs(m * np.exp2(ex.astype(float)) - ref) / np.abs(ref)) < 1e-12
    # a structure change is refused and the plan keeps theta2
    bad = th2.copy()
    bad[len(bad) // 2] = 0.0
    with pytest.raises(E.PwsError):
        p.set_theta(bad)
    assert np.array_equal(I.unpack_bits(p.sample(300, seed), 12), S.sample_ideal(c2, 300, seed))


@pytest.mark.parametrize("prec,tol_f,tol_b", [("fp64", 1e-11, 1e-9), ("fp32", 5e-5, 1e-3)])
def test_log_probability_forward_backward(prec, tol_f, tol_b):
    c = _circuit10()
    p = E.Plan(c, precision=prec)
    bits = S.sample_ideal(c, 300, 41)
    idx = S.basis_index(bits)
    x = torch.tensor(I.pack_bits(bits).view(np.int64), device="cuda")
    theta = torch.tensor(c.theta, dtype=torch.float64, requires_grad=True)
    logp = AG.log_probability(p, theta, x)
    ref = np.log(np.abs(SV.state(c)[idx]) ** 2)
    assert np.max(np.abs(logp.detach().cpu().numpy() - ref)) < tol_f
    w = np.random.default_rng(5).normal(size=len(idx))
    (logp * torch.tensor(w, device="cuda")).sum().backward()
    want = w @ GR.score(c, idx)
    got = theta.grad.numpy()
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < tol_b


def test_gradient_matches_central_differences_fp64():
    """pws_grad against central differences of the engine's own FP64
    log-probabilities, re-evaluated at theta +- h through pws_set_theta."""
    c = _circuit10()
    p = E.Plan(c, precision="fp64")
    bits = S.sample_ideal(c, 64, 43)
    xb = I.pack_bits(bits)
    g = p.grad(xb)
    h = 1e-4

    def logp(th):
        p.set_theta(th)
        m, ex = p.amplitudes(xb)
        return np.log(np.abs(m) ** 2) + 2 * np.log(2.0) * ex
    fd = np.zeros_like(g)
    for j in range(len(c.theta)):
        tp = c.theta.copy()
        tp[j] += h
        tm = c.theta.copy()
        tm[j] -= h
        fd[:, j] = (logp(tp) - logp(tm)) / (2 * h)
    p.set_theta(c.theta)
    rel = np.linalg.norm(g - fd, axis=1) / np.linalg.norm(fd, axis=1)
    assert rel.max() < 1e-6
    # and the gradient program was rewritten too: at theta2 it matches the oracle
    th2 = c.theta + 0.1
    p.set_theta(th2)
    g2 = p.grad(xb)
    ref2 = GR.score(c.with_theta(th2), S.basis_index(bits))
    assert np.max(np.linalg.norm(g2 - ref2, axis=1) / np.linalg.norm(ref2, axis=1)) < 1e-9


def test_sampled_expectation_estimator():
    """The estimator equals mean((f - b) * score) on the returned samples and
    is centred on (K-1)/K times the exact gradient (within 5 standard errors)."""
    c = _circuit10(p=2, seed=4011)
    p = E.Plan(c, precision="fp64")
    theta = torch.tensor(c.theta, dtype=torch.float64, requires_grad=True)
    K = 20000
    val, x = AG.sampled_expectation(p, theta, _cut_cost(c.edges), K, 77)
    val.backward()
    bits = I.unpack_bits(x.cpu().numpy().view(np.uint64), 10)
    assert np.array_equal(bits, S.sample_ideal(c, K, 77))
    f = I.maxcut_value(c.edges, bits).astype(np.float64)
    assert abs(val.item() - f.mean()) < 1e-12
    sc = GR.score(c, S.basis_index(bits))
    terms = (f - f.mean())[:, None] * sc
    assert np.allclose(theta.grad.numpy(), terms.mean(0), rtol=1e-9, atol=1e-12)
    _, exact = GR.objective_and_gradient(c, _cut_vector(c))
    se = terms.std(0) / np.sqrt(K)
    assert np.all(np.abs(terms.mean(0) - (K - 1) / K * exact) < 5 * se + 1e-12)


def test_training_loop_raises_expected_cut():
    c = _circuit10(p=2, seed=4013)
    p = E.Plan(c, precision="fp32")
    cost = _cut_cost(c.edges)
    theta = torch.tensor(c.theta, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([theta], lr=0.05)
    cut = _cut_vector(c)
    e0, _ = GR.objective_and_gradient(c, cut)
    for it in range(20):
        opt.zero_grad()
        loss, _ = AG.sampled_expectation(p, theta, lambda x: -cost(x), 2048, 100 + it)
        loss.backward()
        opt.step()
    e1, _ = GR.objective_and_gradient(c.with_theta(theta.detach().numpy()), cut)
    assert e1 > e0 + 0.1
