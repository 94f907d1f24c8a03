"""pws_sample_noalloc (the sampling pass with the library's static device
workspace, for callers that cannot allocate) against pws_sample, through the
C ABI: two calls in a row on each plan, the second with fewer chains, equal
bit for bit to pws_sample's chains (and, in FP64, to the oracle's
Algorithm 1)."""
import numpy as np
import pytest

import instances as I
from oracle import sampler as S

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2510_24218_amd")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _dev_out(p, k):
    return torch.full((k, p.words), -1, dtype=torch.int64, device="cuda")


@pytest.mark.parametrize("case", ["qaoa12_fp64", "grid4x4_fp32", "ladder4x30_fp32", "ladder4x30_bf16x3"])
def test_noalloc_equals_sample_twice(case):
    if case == "qaoa12_fp64":
        c, _, seed = I.workload_qaoa3reg12()
        prec, ks = "fp64", (1000, 333)
    elif case == "grid4x4_fp32":
        c, _, seed = I.workload_grid6x8(4, 4)
        prec, ks = "fp32", (2048, 777)
    else:
        c, _, seed = I.workload_ladder4x119(30)
        prec, ks = case.split("_")[1], (200, 100)
    p = E.Plan(c, precision=prec)
    for i, k in enumerate(ks):
        print(f"{case}: call {i}, {k} chains, seed {seed + i}", flush=True)
        out = _dev_out(p, k)
        p.sample_noalloc(k, seed + i, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint64)
        ref = p.sample(k, seed + i)
        assert np.array_equal(got, ref), (case, i)
        if prec == "fp64":
            assert np.array_equal(I.unpack_bits(got, c.n_qubits), S.sample_ideal(c, k, seed + i))


def test_noalloc_rejects_a_workspace_beyond_the_static_array():
    c, _, seed = I.workload_grid6x8()
    p = E.Plan(c, precision="fp32")
    k = 1 << 16          # kept running tensors alone: 2^16 chains x 2^12 x 8 bytes
    out = _dev_out(p, k)
    with pytest.raises(E.PwsError) as ei:
        p.sample_noalloc(k, seed, out)
    assert "static workspace" in str(ei.value)
    # the plan stays usable, and the static array serves a call that fits
    out2 = _dev_out(p, 64)
    p.sample_noalloc(64, seed, out2)
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy().view(np.uint64), p.sample(64, seed))
