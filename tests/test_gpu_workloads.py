"""GPU parity on circuits beyond the QAOA MaxCut workloads:

* gates with blocks smaller than 2^|S| and two-qubit candidate sets (CRX,
  fSim, CNOT, CZ, XX+YY, Haar-random two-qubit unitaries; Figure 1 of the
  paper) and Trotterised Heisenberg / transverse-field Ising chains: FP64
  chains bit-exact against the oracle's Algorithm 1 in both contraction
  forms, FP32 and BF16x3 candidate amplitudes against the state vector;
* the paper's timing workload, Gaussian-weighted Ising QAOA p=1 on grid,
  heavy-hex, King's, Chimera and random 3-regular graphs at about 18 qubits:
  FP64 chains bit-exact for the ten instances of every family, candidate
  amplitudes for two of them."""
import numpy as np
import pytest

import instances as I
from oracle import sampler as S
from oracle import statevector as SV

from .test_general_host import candidate_refs, reachable

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2510_24218_amd")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

BARS = {"fp32": 1e-5, "bf16x3": 1e-3}


@pytest.fixture(params=["sweep", "node"])
def form(request, monkeypatch):
    if request.param == "node":
        monkeypatch.setenv("PWS_SWEEP", "0")
    return request.param


CIRCUITS = {"general": lambda: I.general_gate_circuit(), "heisenberg": lambda: I.trotter_heisenberg(),
            "tfim": lambda: I.trotter_tfim()}
ISING = [(t, i) for t in I.ISING_TOPOLOGIES for i in range(10)]
ISING_AMPS = [(t, i) for t in I.ISING_TOPOLOGIES for i in (0, 1)]


def _circ(name):
    if name in CIRCUITS:
        return CIRCUITS[name]()
    t, i = name
    return I.ising_qaoa_p1(t, 18, i)


def _bit_exact(c, K=1000, seed=31):
    p = E.Plan(c, precision="fp64")
    print(f"{c.name}: {K} FP64 chains", flush=True)
    got = I.unpack_bits(p.sample(K, seed), c.n_qubits)
    assert np.array_equal(got, S.sample_ideal(c, K, seed))


def _amplitudes(c, prec):
    p = E.Plan(c, precision=prec)
    rng = np.random.default_rng(8)
    worst = 0.0
    for k in range(p.n_steps()):
        op, gate, m = p.step_info(k)
        s = np.stack([reachable(c, gate, rng) for _ in range(8)])
        gm, ge = p.step_amplitudes(k, I.pack_bits(s))
        got = gm * np.exp2(ge.astype(np.float64))[:, None]
        psi = SV.state(c, gate + 1)
        for i in range(len(s)):
            ref = candidate_refs(c, gate, s[i], psi)
            nr = np.linalg.norm(ref)
            if nr == 0:
                assert np.all(got[i] == 0)
                continue
            worst = max(worst, np.linalg.norm(got[i] - ref) / nr)
    print(f"{c.name} {prec}: worst {worst:.3e}", flush=True)
    assert worst < BARS[prec]


@pytest.mark.parametrize("name", list(CIRCUITS))
def test_beyond_qaoa_fp64_chains_bit_exact(name, form):
    _bit_exact(_circ(name))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name", list(CIRCUITS))
def test_beyond_qaoa_amplitudes(name, prec):
    _amplitudes(_circ(name), prec)


@pytest.mark.parametrize("name", ISING, ids=[f"{t}-{i}" for t, i in ISING])
def test_ising_p1_fp64_chains_bit_exact(name):
    _bit_exact(_circ(name))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name", ISING_AMPS[::2], ids=[t for t, i in ISING_AMPS[::2]])
def test_ising_p1_amplitudes(name, prec):
    _amplitudes(_circ(name), prec)
