"""Free-field (U = 1) closed forms in momentum space, for any lattice size.

With unit links the hopping term is diagonal in momentum.  A plane wave
e^{i p.x} chi (chi a 4-spinor, times any colour vector) is mapped by the
operator of ``oracle.wilson`` to e^{i p.x} H(p) chi with

  H(p) = gamma5 D(p),
  D(p) = [ -m0 + sum_mu (1 - cos p_mu) + i sum_mu gamma_mu sin p_mu ] / (4 - m0),

where p_mu = 2 pi (n_mu + theta_mu) / L_mu, theta_mu = 0 for a periodic and
1/2 for an antiperiodic direction.  Since gamma5 D(p) gamma5 = D(p)^dag,
H(p)^2 = D(p)^dag D(p) = E(p)^2 with
E(p) = sqrt(M(p)^2 + sum_mu sin^2 p_mu) / (4 - m0), M(p) = -m0 + sum_mu (1 - cos p_mu),
so the eigenvalues are +E(p) and -E(p), each twice in spin and three times in
colour.  A function f of H_W therefore acts per momentum as the 4x4 matrix
f(H(p)), computed here by a 4x4 eigendecomposition.
"""
import numpy as np

from .gamma import gammas, gamma5


def _theta(bc):
    return np.array([0.0 if b > 0 else 0.5 for b in bc])


def momenta(dims, bc=(1, 1, 1, -1)):
    """p[mu] arrays broadcastable over [Lt][Lz][Ly][Lx] (FFT index order)."""
    Lx, Ly, Lz, Lt = dims
    th = _theta(bc)
    nt, nz, ny, nx = np.indices((Lt, Lz, Ly, Lx))
    return [2 * np.pi * (n + th[mu]) / L for mu, (n, L) in
            enumerate(zip((nx, ny, nz, nt), (Lx, Ly, Lz, Lt)))]


def h_of_p(p, m0):
    """H(p) as [...][4][4] for momentum arrays p[0..3]."""
    g = gammas()
    g5 = gamma5()
    M = -m0 + sum(1.0 - np.cos(pm) for pm in p)
    D = M[..., None, None] * np.eye(4)
    for mu in range(4):
        D = D + 1j * np.sin(p[mu])[..., None, None] * g[mu]
    return np.einsum("ab,...bc->...ac", g5, D) / (4.0 - m0)


def energies(dims, m0, bc=(1, 1, 1, -1)):
    """E(p) for every momentum, shape [Lt][Lz][Ly][Lx]."""
    p = momenta(dims, bc)
    M = -m0 + sum(1.0 - np.cos(pm) for pm in p)
    return np.sqrt(M ** 2 + sum(np.sin(pm) ** 2 for pm in p)) / (4.0 - m0)


def spectrum(dims, m0, bc=(1, 1, 1, -1)):
    """All 12V eigenvalues of the free H_W, sorted."""
    E = energies(dims, m0, bc).ravel()
    return np.sort(np.concatenate([np.repeat(E, 6), np.repeat(-E, 6)]))


def plane_wave(dims, n, chi, colour, bc=(1, 1, 1, -1)):
    """e^{i p.x} chi (x) colour as a spinor [Lt][Lz][Ly][Lx][4][3]; n = (nx, ny, nz, nt)."""
    Lx, Ly, Lz, Lt = dims
    th = _theta(bc)
    t, z, y, x = np.indices((Lt, Lz, Ly, Lx))
    ph = np.zeros(x.shape)
    for mu, (coord, L) in enumerate(zip((x, y, z, t), (Lx, Ly, Lz, Lt))):
        ph = ph + 2 * np.pi * (n[mu] + th[mu]) / L * coord
    return np.exp(1j * ph)[..., None, None] * np.einsum("a,i->ai", chi, colour)


def _twist(dims, bc, sign):
    Lx, Ly, Lz, Lt = dims
    th = _theta(bc)
    t, z, y, x = np.indices((Lt, Lz, Ly, Lx))
    ph = sum(2 * np.pi * th[mu] * c / L for mu, (c, L) in
             enumerate(zip((x, y, z, t), (Lx, Ly, Lz, Lt))))
    return np.exp(sign * 1j * ph)


def apply_function(b, dims, m0, f, bc=(1, 1, 1, -1)):
    """f(H_W) b for the free field; b has shape [Lt][Lz][Ly][Lx][4][3].

    f maps an array of real eigenvalues to complex values.
    """
    b = np.asarray(b, dtype=np.complex128)
    tw = _twist(dims, bc, -1)[..., None, None]
    bt = np.fft.fftn(b * tw, axes=(0, 1, 2, 3))
    Hp = h_of_p(momenta(dims, bc), m0)
    lam, W = np.linalg.eigh(Hp)
    fl = f(lam)
    # W f W^dag acting on the spin index, colour untouched
    M = np.einsum("...ak,...k,...bk->...ab", W, fl, W.conj())
    st = np.einsum("...ab,...bi->...ai", M, bt)
    return np.fft.ifftn(st, axes=(0, 1, 2, 3)) * _twist(dims, bc, +1)[..., None, None]
