"""SplitMix64 as a counter-based generator (oracle side).

Definition (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the state advances by the odd constant
GAMMA = 0x9E3779B97F4A7C15 and each state is finalised by the mix function
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)
all modulo 2^64.  The i-th output (i = 0, 1, ...) of a stream started from
state s is mix(s + (i + 1) * GAMMA); we use it with s = mix(seed) and i a
particle/axis counter.  Uniform doubles are (x >> 11) * 2^-53 in [0, 1).

This file is written with plain Python integers (exact, slow) for scalars and
numpy uint64 (wrap-around multiply) for arrays.
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK = (1 << 64) - 1


def mix_int(z):
    z &= MASK
    z = ((z ^ (z >> 30)) * M1) & MASK
    z = ((z ^ (z >> 27)) * M2) & MASK
    return z ^ (z >> 31)


def stream_key(seed, species):
    """Per-(seed, species) stream origin: mix of the seed with the species
    folded into the upper bits."""
    return mix_int((int(seed) & MASK) ^ ((int(species) & 0xFF) << 56))


def mix_u64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def uniform(key, counter):
    """Uniform double in [0,1) for stream origin ``key`` and uint64 ``counter``
    (array): mix(key + (counter + 1) * GAMMA) >> 11, times 2^-53."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        s = np.uint64(key) + (c + np.uint64(1)) * np.uint64(GAMMA)
    x = mix_u64(s) >> np.uint64(11)
    return x.astype(np.float64) * (2.0 ** -53)
