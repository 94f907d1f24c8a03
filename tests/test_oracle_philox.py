"""Philox4x64-10 of the oracle against numpy's library implementation."""
import numpy as np
import pytest

from oracle.philox import philox4x64, philox4x64_scalar, uniform53

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _numpy_block(ctr, key):
    # numpy's Philox increments its counter before producing a block, so the
    # block for counter c is produced from the state c - 1 (with borrow).
    c = [int(v) for v in ctr]
    i = 0
    while True:
        c[i] = (c[i] - 1) % (1 << 64)
        if c[i] != (1 << 64) - 1:
            break
        i += 1
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return tuple(int(v) for v in g.random_raw(4))


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((7, 3, 0, 0), (12345, 0)),
    ((0, 5, 0, 0), (2003, 0)),                 # borrow across words in numpy's state
    ((2**64 - 1, 2**40, 0, 0), (2**63 + 17, 0)),
    ((123456789, 987654321, 0, 0), (0xDEADBEEFCAFEF00D, 0)),
])
def test_scalar_matches_numpy(ctr, key):
    assert philox4x64_scalar(ctr, key) == _numpy_block(ctr, key)


def test_vectorised_matches_scalar():
    rng = np.random.default_rng(1)
    ops = rng.integers(0, 2**63, 50, dtype=np.uint64)
    chains = rng.integers(0, 2**63, 50, dtype=np.uint64)
    seed = 0x1234567890ABCDEF
    w = philox4x64(ops, chains, seed)
    for i in range(50):
        ref = philox4x64_scalar((int(ops[i]), int(chains[i]), 0, 0), (seed, 0))
        assert tuple(int(x[i]) for x in w) == ref


def test_uniform53_definition():
    u = uniform53(42, np.arange(1000, dtype=np.uint64), 7)
    assert np.all(u >= 0) and np.all(u < 1)
    w0 = philox4x64_scalar((42, 3, 0, 0), (7, 0))[0]
    assert u[3] == (w0 >> 11) * 2.0 ** -53
    # uniformity sanity: mean and variance of 1000 draws
    assert abs(u.mean() - 0.5) < 0.05
    assert abs(u.var() - 1 / 12) < 0.02
