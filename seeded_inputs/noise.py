"""Counter-based Gaussian noise for the initial EPD potential fields.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used in counter mode, draw k = mix(seed +
(k+1)*0x9E3779B97F4A7C15), turned into uniforms with 53 random bits, and
Box-Muller (Box and Muller 1958) for normal deviates: draws 2p and 2p+1 form
the pair p; element 2p takes the cosine branch and element 2p+1 the sine
branch.  Element order is species (A, B, S), then row y, then column x.

The paper starts from a homogeneous mixture perturbed by a tiny random noise
(Sec. III, closed-system setup); the noise amplitude and its Gaussian form are
workload choices, not part of the method.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_uniforms(seed, count, offset=0):
    """Uniform deviates in (0, 1]: ((bits >> 11) + 1) * 2**-53 for draws offset..offset+count-1."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * _GAMMA
        bits = _mix(z)
    return ((bits >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def gaussian_noise(seed, count):
    """`count` standard normal deviates (Box-Muller over SplitMix64 counter draws)."""
    npairs = (count + 1) // 2
    u = splitmix64_uniforms(seed, 2 * npairs)
    u1 = u[0::2]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    out = np.empty(2 * npairs, dtype=np.float64)
    out[0::2] = r * np.cos(ang)
    out[1::2] = r * np.sin(ang)
    return out[:count]


def initial_omega(nx, ny, seed, sigma):
    """Initial potentials omega_I = sigma * xi, shape (3, ny, nx), species order A, B, S."""
    return sigma * gaussian_noise(seed, 3 * nx * ny).reshape(3, ny, nx)
