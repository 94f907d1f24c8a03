"""Algorithms 1 and 2 of the oracle against exact distributions.

Eq. (1) makes the chain marginal equal |psi_t|^2 at every t; the noisy sampler
must reproduce diag(rho_T).  Chi-square tests with fixed seeds (p > 1e-3)."""
import numpy as np
import pytest
from scipy import stats

import instances as I
from oracle import gates as G
from oracle import sampler as S
from oracle import statevector as SV


def _chi2_pvalue(counts, probs, min_expected=5.0):
    """Pearson chi-square with bins of small expectation pooled together."""
    counts = np.asarray(counts, dtype=np.float64)
    N = counts.sum()
    exp = probs * N
    order = np.argsort(exp)
    obs_b, exp_b = [], []
    acc_o = acc_e = 0.0
    for i in order:
        acc_o += counts[i]
        acc_e += exp[i]
        if acc_e >= min_expected:
            obs_b.append(acc_o)
            exp_b.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 and exp_b:
        obs_b[-1] += acc_o
        exp_b[-1] += acc_e
    obs_b = np.array(obs_b)
    exp_b = np.array(exp_b)
    chi2 = np.sum((obs_b - exp_b) ** 2 / exp_b)
    return stats.chi2.sf(chi2, len(obs_b) - 1)


def test_qaoa12_cut_histogram_and_zz():
    c, K, seed = I.workload_qaoa3reg12()
    bits = S.sample_ideal(c, K, seed)
    prob = S.exact_distribution(c)
    n = c.n_qubits
    allbits = ((np.arange(2 ** n)[:, None] >> np.arange(n)) & 1).astype(np.uint8)
    cut_all = I.maxcut_value(c.edges, allbits)
    cut_s = I.maxcut_value(c.edges, bits)
    m = len(c.edges)
    p_cut = np.bincount(cut_all, weights=prob, minlength=m + 1)
    obs = np.bincount(cut_s, minlength=m + 1)
    assert _chi2_pvalue(obs, p_cut) > 1e-3
    # per-edge <ZZ> z-tests
    z_all = 1 - 2 * allbits.astype(float)
    z_s = 1 - 2 * bits.astype(float)
    worst = 0.0
    for u, v in c.edges:
        ex = np.sum(prob * z_all[:, u] * z_all[:, v])
        est = np.mean(z_s[:, u] * z_s[:, v])
        se = np.sqrt(max(1 - ex ** 2, 1e-12) / K)
        worst = max(worst, abs(est - ex) / se)
    assert worst < 4.0


def test_full_distribution_many_chains():
    """Oracle self-test: 2^16 chains, full 4096-bin chi-square (pooled)."""
    c, _, _ = I.workload_qaoa3reg12()
    K = 1 << 16
    bits = S.sample_ideal(c, K, 777)
    idx = S.basis_index(bits)
    counts = np.bincount(idx, minlength=2 ** c.n_qubits)
    assert _chi2_pvalue(counts, S.exact_distribution(c)) > 1e-3


def test_marginal_at_every_step():
    """Eq. (1): after every op the chain states follow |psi_t|^2."""
    edges = I.random_regular_graph(3, 8, 21)
    c = I.qaoa_maxcut(8, edges, [0.9, 0.4], [0.5, 1.2])
    K = 6000
    _, traj = S.sample_ideal(c, K, 99, record=True)
    for t in [3, 8, 20, len(c.gates) // 2, len(c.gates) - 1]:
        psi = SV.state(c, t + 1)
        p = psi.real ** 2 + psi.imag ** 2
        counts = np.bincount(S.basis_index(traj[t]), minlength=2 ** 8)
        assert _chi2_pvalue(counts, p) > 1e-3, t


def test_transition_rows_sum_to_one_and_block_mass():
    """Block-mass conservation (proof of Eq. (1)) and normalised transition rows."""
    edges = I.random_regular_graph(3, 8, 23)
    c = I.qaoa_maxcut(8, edges, [1.3], [0.8])
    n = 8
    psi_prev = SV.zero_state(n)
    rng = np.random.default_rng(0)
    for g in c.gates:
        mat = G.gate_matrix(c, g)
        psi = SV.apply_gate(psi_prev, n, mat, g.qubits)
        if not G.is_monomial(mat):
            for _ in range(10):
                x = int(rng.integers(0, 2 ** n))
                q = g.qubits[0]
                blk = [x & ~(1 << q), x | (1 << q)]
                before = sum(abs(psi_prev[b]) ** 2 for b in blk)
                after = sum(abs(psi[b]) ** 2 for b in blk)
                assert abs(before - after) < 1e-14
                if after > 0:
                    rows = [abs(psi[b]) ** 2 / after for b in blk]
                    assert abs(sum(rows) - 1) < 1e-14
        psi_prev = psi


def test_monomial_gates_are_deterministic():
    c = I.Circuit(4, [I.Gate("X", (0,)), I.Gate("CNOT", (0, 2)), I.Gate("CZ", (2, 3)),
                      I.Gate("X", (3,)), I.Gate("CNOT", (3, 1))], np.zeros(0))
    bits = S.sample_ideal(c, 50, 5)
    assert np.all(bits == np.array([1, 1, 1, 1], dtype=np.uint8))


def test_nontrivial_blocks_fsim_crx():
    """Gates with blocks smaller than 2^|q| (Figure 1(c)) sample |psi|^2."""
    th = np.array([0.7, 1.1, 2.0, 0.4])
    gates = [I.Gate("H", (0,)), I.Gate("H", (1,)), I.Gate("RX", (2,), param=2),
             I.Gate("CRX", (0, 2), param=0), I.Gate("FSIM", (1, 2), param=1, param2=3),
             I.Gate("CRX", (2, 1), param=2), I.Gate("FSIM", (0, 1), param=0, param2=1)]
    c = I.Circuit(3, gates, th)
    bits = S.sample_ideal(c, 20000, 31)
    counts = np.bincount(S.basis_index(bits), minlength=8)
    assert _chi2_pvalue(counts, S.exact_distribution(c)) > 1e-3


def _noisy_twin(n=8, rate=0.05, seed=3001):
    edges = I.random_regular_graph(3, n, seed)
    c = I.qaoa_maxcut(n, edges, [0.8, 1.7], [0.6, 2.1])
    return I.add_qaoa_noise(c, depol2=rate, ampdamp=rate)


def test_noisy_sampler_matches_density_matrix():
    c = _noisy_twin()
    bits = S.sample_noisy(c, 6000, 4242)
    counts = np.bincount(S.basis_index(bits), minlength=2 ** c.n_qubits)
    p = S.exact_distribution(c)
    assert _chi2_pvalue(counts, p) > 1e-3


def test_noisy_sampler_with_config_rates():
    c = _noisy_twin(rate=0.0)
    c = I.add_qaoa_noise(c.without_noise(), depol2=1e-3, ampdamp=5e-4)
    bits = S.sample_noisy(c, 4000, 99)
    counts = np.bincount(S.basis_index(bits), minlength=2 ** c.n_qubits)
    assert _chi2_pvalue(counts, S.exact_distribution(c)) > 1e-3


def test_literal_sbit_reading_is_detected():
    """Planted mistake: choosing the Kraus branch from s[q] instead of the true
    bit (s xor x)[q] must be caught by the distribution test."""
    c = _noisy_twin(n=6, rate=0.25, seed=3003)
    bits = _sample_noisy_sbit(c, 6000, 5)
    counts = np.bincount(S.basis_index(bits), minlength=2 ** c.n_qubits)
    assert _chi2_pvalue(counts, S.exact_distribution(c)) < 1e-6
    good = S.sample_noisy(c, 6000, 5)
    counts = np.bincount(S.basis_index(good), minlength=2 ** c.n_qubits)
    assert _chi2_pvalue(counts, S.exact_distribution(c)) > 1e-3


def _sample_noisy_sbit(circ, K, seed):
    """Copy of the noisy sampler's control flow with the literal s[q] bit."""
    from oracle.philox import uniform53
    n = circ.n_qubits
    chain_ids = np.arange(K, dtype=np.uint64)
    s = np.zeros((K, n), dtype=np.uint8)
    x = np.zeros((K, n), dtype=np.uint8)
    psi = np.zeros((K, 2 ** n), dtype=np.complex128)
    psi[:, 0] = 1.0
    for op, (kind, idx) in enumerate(circ.ops()):
        if kind == "gate":
            g = circ.gates[idx]
            mat = G.gate_matrix(circ, g)
            fr = S._local_index(x, g.qubits)
            m = len(g.qubits)
            mats = np.empty((K, 2 ** m, 2 ** m), dtype=np.complex128)
            for f in range(2 ** m):
                bits = tuple((f >> (m - 1 - j)) & 1 for j in range(m))
                mats[fr == f] = G.conjugate_by_frame(mat, bits)
            psi = SV.apply_gate_per_batch(psi, n, mats, g.qubits)
            for f in range(2 ** m):
                rows = np.nonzero(fr == f)[0]
                if len(rows) == 0:
                    continue
                bits = tuple((f >> (m - 1 - j)) & 1 for j in range(m))
                gp = G.conjugate_by_frame(mat, bits)
                sub = s[rows].copy()
                S._update_state(gp, g.qubits, sub,
                                lambda r, y, _rows=rows: psi[_rows[r], S._basis_index(y)],
                                lambda r, _op=op, _rows=rows: uniform53(_op, chain_ids[_rows[r]], seed))
                s[rows] = sub
        else:
            site = circ.noise[idx]
            flist = G.kraus_factors(site)
            q = site.qubits
            wrong_bits = s[:, list(q)].astype(np.int64)          # <- the planted mistake
            pr = np.array([G.branch_probabilities(flist, tuple(int(b) for b in wrong_bits[r]))
                           for r in range(K)])
            ch = S.draw_index(pr, uniform53(op, chain_ids, seed))
            for j, qj in enumerate(q):
                mats = np.zeros((K, 2, 2), dtype=np.complex128)
                for r in range(K):
                    M = flist[ch[r]][j]
                    if M[0, 0] == 0 and M[1, 1] == 0:
                        x[r, qj] ^= 1
                        M = M @ G.PX
                    if x[r, qj]:
                        M = G.PX @ M @ G.PX
                    mats[r, 0, 0], mats[r, 1, 1] = M[0, 0], M[1, 1]
                psi = SV.apply_gate_per_batch(psi, n, mats, (qj,))
    return s ^ x


def test_draw_rule():
    p = np.array([[0.25, 0.75], [0.0, 1.0], [0.0, 0.0], [0.5, 0.5]])
    u = np.array([0.2499, 0.0, 0.3, 0.5])
    assert list(S.draw_index(p, u)) == [0, 1, -1, 1]
