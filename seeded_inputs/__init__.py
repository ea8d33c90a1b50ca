"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method itself (no Dirac operator, no
contour, no solver).  It only draws the inputs the method is applied to:

* SU(3) gauge links U = exp(i A) with A = r * sum_k a_k lambda_k, where
  lambda_k are the eight Gell-Mann matrices (tr lambda_a lambda_b = 2 delta_ab)
  and a_k are iid standard normal numbers.  ``r`` (the "roughness") controls
  how far the field is from the free field U = 1.  This stands in for the
  quenched Wilson-action ensemble the paper uses (Numerical experiments
  section), which is not available; a smaller r gives a smoother field and a
  larger spectral gap of H_W.
* Complex Gaussian source vectors (real and imaginary parts iid N(0, 1)),
  the "random vector" of the sign-function quality measure sigma.

External layouts (row-major, complex128):
  gauge  : [4][Lt][Lz][Ly][Lx][3][3]   (mu = 0..3 is x, y, z, t)
  spinor : [n][Lt][Lz][Ly][Lx][4][3]   (spin index, then colour)
"""
import numpy as np

__all__ = ["gell_mann", "gauge_field", "unit_gauge", "gaussian_sources",
           "random_su3_direction"]


def gell_mann():
    """The eight Gell-Mann matrices, shape [8][3][3] complex128."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1] = -1j
    g[1][1, 0] = 1j
    g[2][0, 0], g[2][1, 1] = 1, -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2] = -1j
    g[4][2, 0] = 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2] = -1j
    g[6][2, 1] = 1j
    g[7][0, 0] = g[7][1, 1] = 1 / np.sqrt(3)
    g[7][2, 2] = -2 / np.sqrt(3)
    return g


def _exp_i_hermitian(A):
    """exp(i A) for a batch of hermitian 3x3 matrices, via eigh."""
    e, W = np.linalg.eigh(A)
    return np.einsum("...ij,...j,...kj->...ik", W, np.exp(1j * e), W.conj())


def gauge_field(dims, roughness=0.3, seed=0):
    """Seeded SU(3) field, complex128 [4][Lt][Lz][Ly][Lx][3][3].

    dims = (Lx, Ly, Lz, Lt).  The coefficients are drawn as one array
    [4][Lt][Lz][Ly][Lx][8] from numpy.random.default_rng(seed).
    """
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((4, Lt, Lz, Ly, Lx, 8))
    A = roughness * np.einsum("...k,kij->...ij", a, gell_mann())
    return np.ascontiguousarray(_exp_i_hermitian(A))


def unit_gauge(dims):
    """The free field U = 1, complex128 [4][Lt][Lz][Ly][Lx][3][3]."""
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    U = np.zeros((4, Lt, Lz, Ly, Lx, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1
    return U


def gaussian_sources(dims, n, first_seed=1000):
    """n complex Gaussian spinor fields, complex128 [n][Lt][Lz][Ly][Lx][4][3].

    Source i is drawn from numpy.random.default_rng(first_seed + i): first the
    real parts, then the imaginary parts, each of shape [Lt][Lz][Ly][Lx][4][3].
    """
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    shape = (Lt, Lz, Ly, Lx, 4, 3)
    out = np.empty((n,) + shape, dtype=np.complex128)
    for i in range(n):
        rng = np.random.default_rng(first_seed + i)
        re = rng.standard_normal(shape)
        im = rng.standard_normal(shape)
        out[i] = re + 1j * im
    return out


def random_su3_direction(dims, seed):
    """A random Lie-algebra direction on every link, normalised to unit norm.

    Returns real coefficients omega[4][Lt][Lz][Ly][Lx][8] (Gaussian, then
    divided by their global 2-norm); the link perturbation is
    U -> exp(i h sum_k omega_k lambda_k / 2) U.
    """
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((4, Lt, Lz, Ly, Lx, 8))
    return w / np.linalg.norm(w)
