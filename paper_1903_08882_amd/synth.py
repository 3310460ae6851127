"""Seeded synthetic inputs shared by the GPU library's callers and the oracle.

This module holds random numbers only: no lattice Boltzmann arithmetic.  Every
draw is a counter-based splitmix64 value (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) of ``key(seed, stream) + n``,
with n the node's linear index (x fastest), mapped to a double in [-1, 1) from
its top 53 bits.  The same (seed, stream, N) always gives the same array.

Field arrays have shape (N, N, N) indexed [z][y][x].
"""
import numpy as np

SEED0 = 190308882  # the paper's arXiv number, used as the base seed

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """splitmix64 finaliser of uint64 array ``x`` (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed, stream, count):
    """``count`` doubles in [-1, 1) for (seed, stream)."""
    key = splitmix64(np.uint64(seed) ^ (np.uint64(stream) << np.uint64(40)))
    with np.errstate(over="ignore"):
        ctr = key + np.arange(count, dtype=np.uint64)
    bits = splitmix64(ctr) >> np.uint64(11)
    return bits.astype(np.float64) * (2.0 / 9007199254740992.0) - 1.0


def noise_field(N, seed, stream, amplitude):
    """amplitude * U[-1, 1) on an N^3 grid, shape (N, N, N) [z][y][x]."""
    return (amplitude * uniform(seed, stream, N ** 3)).reshape(N, N, N)


def rest_with_noise(N, seed=SEED0, amplitude=1e-3):
    """Fluid at rest with seeded temperature noise: fields [u, v, w, T].

    u = v = w = 0 and T = amplitude * U[-1, 1) per node: the initial state of
    the side-heated and Rayleigh-Benard runs (temperatures are measured from
    the mean of the two wall temperatures).
    """
    f = np.zeros((4, N, N, N))
    f[3] = noise_field(N, seed, 0, amplitude)
    return f


def rich_fields(N, seed=SEED0 + 100, u_amp=0.05, T_amp=0.5, rho_amp=1e-3):
    """A state that excites every moment: returns (rho, [u, v, w, T]).

    rho = 1 + rho_amp * U, u_a = u_amp * U, T = T_amp * U, independent streams.
    """
    uvwT = np.empty((4, N, N, N))
    for a in range(3):
        uvwT[a] = noise_field(N, seed, 1 + a, u_amp)
    uvwT[3] = noise_field(N, seed, 4, T_amp)
    rho = 1.0 + noise_field(N, seed, 5, rho_amp)
    return rho, uvwT


def population_noise(N, seed=SEED0 + 100, nq=26):
    """U[-1, 1) per (population, node): shape (nq, N, N, N)."""
    return np.stack([noise_field(N, seed, 16 + q, 1.0) for q in range(nq)])


def sweep_cavities(K=64, seed=SEED0 + 3, sizes=(33, 49, 65), ra_range=(1e4, 1e7),
                   prandtl=(0.71, 7.0)):
    """K side-heated cavity set-ups for a training sweep: N uniform over
    `sizes`, Ra log-uniform over `ra_range`, Pr uniform over `prandtl`, and a
    noise seed per cavity.  Returns a list of dicts (N, Ra, Pr, seed)."""
    a = (uniform(seed, 0, K) + 1.0) / 2.0          # [0, 1)
    b = (uniform(seed, 1, K) + 1.0) / 2.0
    c = (uniform(seed, 2, K) + 1.0) / 2.0
    lo, hi = np.log10(ra_range[0]), np.log10(ra_range[1])
    out = []
    for k in range(K):
        out.append({"N": int(sizes[min(int(a[k] * len(sizes)), len(sizes) - 1)]),
                    "Ra": float(10.0 ** (lo + (hi - lo) * b[k])),
                    "Pr": float(prandtl[min(int(c[k] * len(prandtl)), len(prandtl) - 1)]),
                    "seed": int(seed * 1000 + k)})
    return out
