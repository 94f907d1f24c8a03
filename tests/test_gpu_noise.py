"""GPU parity of the noisy sampler (Algorithm 2) beyond depolarising +
amplitude damping at small sizes:

* the simulated chip of the paper's noisy experiments (one- and two-qubit
  depolarising errors, amplitude and phase damping per gate length from T1
  and T2, readout errors) and unequal Pauli noise: FP64 chains bit-exact
  against the oracle's Algorithm 2 in both contraction forms, FP32 samples
  against diag(rho) followed by the readout flips;
* the full 6x8 grid at 4096 chains, FP32 and FP64, in the timed launch
  shapes (the noisy entries of the one-wave and four-wave steps of 2^9 to
  2^12 elements included): for chains at both ends of the launch and in
  both halves of a wave, the oracle runs Algorithm 2 for that chain alone
  with path-sum amplitudes of its C'' (its own Kraus branches from s XOR x
  and the chain's Philox stream), and every traced draw must equal the
  oracle's, up to near-ties the precision cannot resolve, where the oracle
  follows the traced value."""
import dataclasses

import numpy as np
import pytest
from scipy import stats

import instances as I
from oracle import sampler as S

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2510_24218_amd")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


@pytest.fixture(params=["sweep", "node"])
def form(request, monkeypatch):
    if request.param == "node":
        monkeypatch.setenv("PWS_SWEEP", "0")
    return request.param


def _qaoa10():
    return I.qaoa_maxcut(10, I.random_regular_graph(3, 10, 3002), [0.8, 1.7], [0.6, 2.1])


def _chi2_p(counts, prob, K):
    exp = prob * K
    order = np.argsort(exp)
    ob, eb, ao, ae = [], [], 0.0, 0.0
    for i in order:
        ao += counts[i]; ae += exp[i]
        if ae >= 5:
            ob.append(ao); eb.append(ae); ao = ae = 0.0
    ob[-1] += ao; eb[-1] += ae
    ob, eb = np.array(ob), np.array(eb)
    return stats.chi2.sf(np.sum((ob - eb) ** 2 / eb), len(ob) - 1)


def test_chip_noise_fp64_bit_exact(form):
    """The chip model at the paper's rates and at raised rates."""
    for c in [I.add_chip_noise(_qaoa10()),
              I.add_chip_noise(_qaoa10(), p1=0.05, p2=0.08, readout=0.1, T1_us=0.5, T2_us=0.6)]:
        p = E.Plan(c, precision="fp64")
        K = 1200
        print(f"chip noise {len(c.noise)} sites, {K} FP64 chains", flush=True)
        got = I.unpack_bits(p.sample(K, 41), 10)
        assert np.array_equal(got, S.sample_noisy(c, K, 41))


def test_pauli_and_phase_noise_fp64_bit_exact(form):
    """Unequal Pauli errors after two-qubit gates, phase damping after
    one-qubit gates, readout errors on half the qubits."""
    c = _qaoa10()
    sites = []
    for gi, g in enumerate(c.gates):
        if len(g.qubits) == 2:
            sites.append(I.NoiseSite(gi, "PAULI1", (g.qubits[0],), (0.04, 0.01, 0.07)))
            sites.append(I.NoiseSite(gi, "PAULI1", (g.qubits[1],), (0.02, 0.05, 0.0)))
        else:
            sites.append(I.NoiseSite(gi, "PHASEDAMP", g.qubits, (0.1,)))
    c = dataclasses.replace(c, noise=sites, readout=tuple([0.07, 0.0] * 5))
    p = E.Plan(c, precision="fp64")
    got = I.unpack_bits(p.sample(1000, 43), 10)
    assert np.array_equal(got, S.sample_noisy(c, 1000, 43))


def test_chip_noise_fp32_distribution():
    """8-qubit twin, chip model at raised rates, FP32 samples against diag(rho)
    followed by the readout flips."""
    c = I.qaoa_maxcut(8, I.random_regular_graph(3, 8, 3001), [0.8, 1.7], [0.6, 2.1])
    c = I.add_chip_noise(c, p1=0.02, p2=0.04, readout=0.05, T1_us=2.0, T2_us=2.0)
    p = E.Plan(c, precision="fp32")
    K = 1 << 15
    bits = I.unpack_bits(p.sample(K, 47), 8)
    counts = np.bincount(S.basis_index(bits), minlength=256).astype(float)
    assert _chi2_p(counts, S.exact_distribution(c), K) > 1e-3


@pytest.mark.parametrize("prec,margin,chip", [("fp64", 1e-12, False), ("fp32", 1e-4, False), ("fp64", 1e-12, True)])
def test_noisy_grid6x8_traced_draws(prec, margin, chip):
    """Full noisy 6x8 grid at 4096 chains (the bench's noisy workload:
    depolarising 1e-3 after each RZZ, amplitude damping 5e-4 after each RX;
    or the chip model), traced draws of chains at both ends of the launch and
    in both halves of a wave against the oracle's Algorithm 2 for that chain."""
    c, K, seed = I.workload_grid6x8()
    if chip:
        c = I.add_chip_noise(c)
        chains = [0, 4095]
    else:
        c = I.add_qaoa_noise(c, depol2=1e-3, ampdamp=5e-4)
        chains = [0, 1, 2049, K - 1]
    p = E.Plan(c, precision=prec)
    out, trace = p.sample_trace(K, seed)
    ns = p.n_steps()
    op_to_step = {p.step_info(k)[0]: k for k in range(ns)}
    near = 0
    for chain in chains:
        print(f"noisy grid {prec} chip={chip}: chain {chain}", flush=True)

        def follow(op, pv, u, v, _chain=chain):
            nonlocal near
            k = op_to_step[op]
            t = int(trace[k, _chain])
            if t != v:
                P = float(np.sum(pv))
                C0 = float(pv[0])
                assert abs(u * P - C0) < margin * P, (_chain, k, t, v)
                near += 1
            return t

        bits = S.sample_noisy_pathsum(c, chain, seed, choose=follow)
        assert np.array_equal(bits, I.unpack_bits(out[chain:chain + 1], c.n_qubits)[0]), chain
    assert near <= 2
