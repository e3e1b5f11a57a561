"""The host definition of the output digest, pinned to the published SplitMix64
test vectors, and the properties the chunk log relies on (split invariance,
sensitivity to every bit, position dependence)."""
import numpy as np

from tests.digest_ref import G, digest, splitmix64


def test_splitmix64_published_vectors():
    # SplitMix64 (Steele, Lea and Flood 2014; the public-domain reference
    # generator) from state 1234567 and from state 0
    got = [int(v) for v in splitmix64(1234567, 5)]
    assert got == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]
    assert int(splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF


def test_digest_of_zeros_is_a_splitmix64_sum():
    # zeros at global index e0.. give the outputs of SplitMix64 from state G e0
    for e0, n in ((0, 7), (1000, 33)):
        with np.errstate(over="ignore"):
            seed = int(np.uint64(e0) * G)
        ref = int(np.sum(splitmix64(seed, n), dtype=np.uint64))
        assert digest(np.zeros(n), e0) == ref


def test_digest_split_invariance():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(1000)
    full = digest(x)
    for cut in (0, 1, 517, 999, 1000):
        assert (digest(x[:cut]) + digest(x[cut:], cut)) % 2**64 == full


def test_digest_sees_every_bit_and_position():
    rng = np.random.default_rng(4)
    x = rng.standard_normal(64)
    d0 = digest(x)
    b = x.view(np.uint64).copy()
    for bit in (0, 31, 52, 63):
        y = b.copy()
        y[17] ^= np.uint64(1 << bit)
        assert digest(y.view(np.float64)) != d0
    assert digest(x[::-1].copy()) != d0
    assert digest(np.array([0.0])) != digest(np.array([-0.0]))
    assert digest(x, 1) != d0
