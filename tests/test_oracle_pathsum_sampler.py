"""Pin of the path-sum sampler (the CPU baseline's sampler).

Algorithm 1 is a function of the candidate amplitudes, the draw rule and the
random stream only, so the sampler that takes every candidate amplitude from
a path sum of the prefix circuit must produce the same chains, bit for bit,
as the sampler that reads them from one shared state vector; any slip in the
prefix length, the candidate order or the counter would split them."""
import numpy as np

import instances as I
from oracle import sampler as S


def _same_chains(c, K, seed):
    a, ta = S.sample_ideal_pathsum(c, K, seed, record=True)
    b, tb = S.sample_ideal(c, K, seed, record=True)
    assert np.array_equal(a, b)
    # the whole trajectory, op by op, not only the end state
    assert len(ta) == len(tb)
    for k, (x, y) in enumerate(zip(ta, tb)):
        assert np.array_equal(x, y), f"op {k}"


def test_pathsum_sampler_equals_statevector_sampler_qaoa12():
    c, _, seed = I.workload_qaoa3reg12()
    _same_chains(c, 200, seed)


def test_pathsum_sampler_equals_statevector_sampler_grid4x4():
    c, _, seed = I.workload_grid6x8(4, 4)
    _same_chains(c, 200, seed)


def test_pathsum_sampler_chain_ids_key_the_stream():
    """Chains 7, 8, 9 of a run equal chains 0, 1, 2 of a run with those ids."""
    c, _, seed = I.workload_qaoa3reg12()
    full = S.sample_ideal(c, 10, seed)
    sub = S.sample_ideal_pathsum(c, 3, seed, chains=np.array([7, 8, 9], np.uint64))
    assert np.array_equal(full[7:10], sub)
