"""Host definition of the output digest (numpy, uint64 arithmetic wraps mod 2^64).

D = sum_e mix(bits(x_e) + G (e0 + e + 1)) mod 2^64, G = 0x9E3779B97F4A7C15, mix the
SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014).  Not part of the
integral method: it checks the library's chunk digest of streamed output.
"""
import numpy as np

G = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed, n):
    """First n outputs of SplitMix64 from state `seed` (the state advances by G before each output)."""
    k = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix(np.uint64(seed) + G * k)


def digest(x, e0=0):
    """Digest of the float64 array x whose first element has global index e0."""
    b = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64).ravel()
    idx = np.arange(e0 + 1, e0 + 1 + b.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return int(np.sum(mix(b + G * idx), dtype=np.uint64))
