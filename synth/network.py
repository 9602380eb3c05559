"""Random inputs of the learned interpolant's network: Fourier frequencies and
test parameter vectors.  Only random draws live here (Box-Muller normals from
the counter-based generator); the network itself is computed elsewhere."""
import numpy as np

from .rng import uniform01

N_FREQ = 64
N_PARAMS = 68112


def normals(seed: int, stream: int, n: int) -> np.ndarray:
    """n standard normals (Box-Muller on pairs of counter-based uniforms)."""
    u = uniform01(seed, stream, 2 * n)
    u1 = np.maximum(u[0::2], 1e-300)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u[1::2])


def fourier_frequencies(seed: int = 31, scale: float = 0.25) -> np.ndarray:
    """(64, 2) float32 frequencies, each component normal with std `scale`
    (cycles per unit of the in-square offset; the interpolation weights are
    smooth over a square, so low frequencies serve best)."""
    return (normals(seed, 11, 2 * N_FREQ) * scale).reshape(N_FREQ, 2).astype(np.float32)


def random_parameters(seed: int, scale: float = 0.1) -> np.ndarray:
    """N_PARAMS float32 numbers, normal with std `scale` (for checks)."""
    return (normals(seed, 12, N_PARAMS) * scale).astype(np.float32)
