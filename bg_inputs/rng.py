"""Counter-based random numbers from the SplitMix64 mixer.

SplitMix64 is the generator of Steele, Lea and Flood, "Fast splittable
pseudorandom number generators" (OOPSLA 2014): a Weyl sequence with increment
0x9E3779B97F4A7C15 followed by the 64-bit finaliser
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
    z ^= z >> 27; z *= 0x94D049BB133111EB;
    z ^= z >> 31.
Here it is used as a keyed hash: draw k of counter c under seed s is
    mix64(mix64(s + GAMMA * (c + 1)) + GAMMA * (k + 1))
so any (counter, draw) pair can be regenerated independently, and a run can
be resumed at any counter.  Doubles in the open interval (0, 1) take the top
53 bits: ((z >> 11) + 0.5) * 2**-53.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)
_S30 = np.uint64(30)
_S27 = np.uint64(27)
_S31 = np.uint64(31)
_S11 = np.uint64(11)


def mix64(z):
    """SplitMix64 finaliser on a uint64 array (wrap-around arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _S30)) * _C1
        z = (z ^ (z >> _S27)) * _C2
    return z ^ (z >> _S31)


def splitmix64_bits(seed, counters, n_draws):
    """uint64 array [len(counters), n_draws] of keyed draws."""
    c = np.asarray(counters, dtype=np.uint64).reshape(-1, 1)
    k = np.arange(1, n_draws + 1, dtype=np.uint64).reshape(1, -1)
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        base = mix64(s + GAMMA * (c + np.uint64(1)))
        return mix64(base + GAMMA * k)


def splitmix64_uniform(seed, counters, n_draws):
    """float64 array [len(counters), n_draws] of uniforms in (0, 1)."""
    bits = splitmix64_bits(seed, counters, n_draws)
    return ((bits >> _S11).astype(np.float64) + 0.5) * (2.0 ** -53)
