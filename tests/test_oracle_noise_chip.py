"""The simulated chip's noise model in the oracle (Section 4's noisy
experiments: one- and two-qubit depolarising errors, amplitude and phase
damping for each gate's length from T1 and T2, readout errors), pinned
against independent formulations: readout errors against bit-flip channels
in the density matrix, the damping parameters against the decay of a
qubit's population and coherence, Algorithm 2 against diag(rho), and the
path-sum noisy sampler against the state-vector one, chain for chain."""
import dataclasses
import math

import numpy as np
import pytest
from scipy import stats

import instances as I
from oracle import sampler as S
from oracle import statevector as SV


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


def test_readout_equals_bit_flip_channels():
    """Readout errors r_q after the last operation give the distribution of
    the density matrix with a bit-flip channel (Pauli X with probability r_q)
    on every qubit at the end."""
    c = I.add_qaoa_noise(I.qaoa_maxcut(5, [(0, 1), (1, 2), (2, 3), (3, 4), (0, 4)], [0.7], [1.2]),
                         depol2=0.03, ampdamp=0.02)
    r = (0.05, 0.1, 0.0, 0.2, 0.07)
    with_ro = dataclasses.replace(c, readout=r)
    last = len(c.gates) - 1
    flips = [I.NoiseSite(last, "PAULI1", (q,), (r[q], 0.0, 0.0)) for q in range(5)]
    as_channels = dataclasses.replace(c, noise=list(c.noise) + flips)
    a = S.exact_distribution(with_ro)
    b = np.real(np.diag(SV.density_matrix(as_channels)))
    assert np.allclose(a, b, atol=1e-14)


def test_readout_flips_in_sampled_chains():
    c, _, _ = I.workload_qaoa3reg12()
    c = dataclasses.replace(c, readout=tuple([0.05] * 12))
    K = 1 << 15
    bits = S.sample_ideal(c, K, 77)
    counts = np.bincount(S.basis_index(bits), minlength=4096).astype(float)
    assert _chi2_p(counts, S.exact_distribution(c), K) > 1e-3
    # the readout draws use their own counters: without them, the chains agree
    plain = S.sample_ideal(dataclasses.replace(c, readout=None), K, 77)
    frac = np.mean(bits != plain)
    assert abs(frac - 0.05) < 0.005


@pytest.mark.parametrize("t_ns", [30.0, 80.0, 5000.0])
def test_chip_damping_decays(t_ns):
    """Amplitude damping gamma then phase damping lambda for a gate of length
    t: from |1> the population of |1> is exp(-t / T1); from |+> the
    coherence is exp(-t / T2) / 2 (density matrix with the channels'
    Kraus operators)."""
    T1, T2 = 100.0, 50.0
    g, l = I.chip_damping(t_ns, T1, T2)
    t = t_ns * 1e-3
    for prep, check in [("X", lambda rho: abs(rho[1, 1] - math.exp(-t / T1))),
                        ("H", lambda rho: abs(rho[0, 1] - 0.5 * math.exp(-t / T2)))]:
        c = I.Circuit(1, [I.Gate(prep, (0,))], np.zeros(0),
                      noise=[I.NoiseSite(0, "AMPDAMP", (0,), (g,)), I.NoiseSite(0, "PHASEDAMP", (0,), (l,))])
        assert check(SV.density_matrix(c)) < 1e-14


def test_chip_noise_model_sites():
    c = I.add_chip_noise(I.qaoa_maxcut(4, [(0, 1), (1, 2), (2, 3)], [0.5], [0.9]))
    kinds = [s.kind for s in c.noise]
    n1 = sum(1 for g in c.gates if len(g.qubits) == 1)
    n2 = sum(1 for g in c.gates if len(g.qubits) == 2)
    assert kinds.count("DEPOL1") == n1 and kinds.count("DEPOL2") == n2
    assert kinds.count("AMPDAMP") == kinds.count("PHASEDAMP") == n1 + 2 * n2
    assert c.readout == (0.05,) * 4
    assert [s.p[0] for s in c.noise if s.kind == "DEPOL2"][0] == 0.01


def test_chip_noise_sampler_matches_density_matrix():
    """Algorithm 2 with the chip model at raised rates (so every channel is
    visible at 2^13 chains) against diag(rho) followed by the readout flips."""
    c = I.qaoa_maxcut(6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (0, 5), (1, 4)], [0.8, 1.9], [0.6, 2.2])
    c = I.add_chip_noise(c, p1=0.05, p2=0.1, readout=0.08, T1_us=0.6, T2_us=0.5)
    K = 1 << 13
    bits = S.sample_noisy(c, K, 3)
    counts = np.bincount(S.basis_index(bits), minlength=64).astype(float)
    assert _chi2_p(counts, S.exact_distribution(c), K) > 1e-3


def test_noisy_pathsum_sampler_equals_statevector_sampler():
    """One chain at a time with path-sum amplitudes of its C'' (frame-
    conjugated gates, drawn diagonal Kraus factors) gives the same chains,
    bit for bit, as the state-vector trajectories (raised rates, chip model
    with readout errors, and depolarising + amplitude damping)."""
    base = I.workload_grid6x8(3, 3)[0]
    for c in [I.add_qaoa_noise(base, depol2=0.05, ampdamp=0.05),
              I.add_chip_noise(base, p1=0.05, p2=0.08, readout=0.1, T1_us=0.5, T2_us=0.6)]:
        ref = S.sample_noisy(c, 16, 5)
        got = np.array([S.sample_noisy_pathsum(c, k, 5) for k in range(16)])
        assert np.array_equal(ref, got)
