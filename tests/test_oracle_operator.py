"""Pins of the oracle's H_W against closed forms and invariants (CPU)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import seeded_inputs as si
from oracle import freefield as ff
from oracle.gamma import gammas, gamma5
from oracle.wilson import hermitian_wilson, kappa


def test_gamma_clifford_algebra():
    g = gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4), atol=1e-15)
    g5 = gamma5()
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    for mu in range(4):
        assert np.allclose(g5 @ g[mu] + g[mu] @ g5, 0)


@pytest.mark.parametrize("dims,r", [((2, 2, 2, 4), 0.3), ((4, 4, 4, 4), 0.4), ((3, 2, 4, 2), 0.2)])
def test_hw_hermitian(dims, r):
    H = hermitian_wilson(si.gauge_field(dims, r, seed=3), 1.4)
    assert abs(H - H.getH()).max() < 1e-15


@pytest.mark.parametrize("m0", [1.0, 1.4])
def test_free_spectrum_closed_form(m0):
    dims = (2, 2, 2, 4)
    H = hermitian_wilson(si.unit_gauge(dims), m0)
    ev = np.linalg.eigvalsh(H.toarray())
    assert np.abs(ev - ff.spectrum(dims, m0)).max() < 1e-13


def test_free_spectrum_periodic_time():
    dims = (2, 2, 2, 4)
    bc = (1, 1, 1, 1)
    H = hermitian_wilson(si.unit_gauge(dims), 1.4, bc=bc)
    ev = np.linalg.eigvalsh(H.toarray())
    assert np.abs(ev - ff.spectrum(dims, 1.4, bc=bc)).max() < 1e-13


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 3, 2, 4), (3, 1, 0, 5)])
def test_free_plane_wave(n):
    """H_W e^{ipx} chi (x) c = e^{ipx} H(p) chi (x) c with H(p) = gamma5 D(p)."""
    dims = (4, 4, 4, 6)
    H = hermitian_wilson(si.unit_gauge(dims), 1.4)
    rng = np.random.default_rng(sum(n))
    chi = rng.normal(size=4) + 1j * rng.normal(size=4)
    col = rng.normal(size=3) + 1j * rng.normal(size=3)
    pw = ff.plane_wave(dims, n, chi, col)
    L = (4, 4, 4, 6)
    th = (0, 0, 0, 0.5)
    p = [np.array(2 * np.pi * (n[m] + th[m]) / L[m]) for m in range(4)]
    # D(p) written directly from the hopping sum on a plane wave:
    # (1 - gamma) e^{ip} forward + (1 + gamma) e^{-ip} backward
    g = gammas()
    D = np.eye(4, dtype=complex)
    for mu in range(4):
        D -= kappa(1.4) * ((np.eye(4) - g[mu]) * np.exp(1j * p[mu]) +
                           (np.eye(4) + g[mu]) * np.exp(-1j * p[mu]))
    Hp = gamma5() @ D
    assert np.allclose(Hp, ff.h_of_p(p, 1.4), atol=1e-15)
    lhs = (H @ pw.ravel()).reshape(pw.shape)
    rhs = ff.plane_wave(dims, n, Hp @ chi, col)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_gauge_covariance():
    dims = (2, 4, 2, 4)
    U = si.gauge_field(dims, 0.3, seed=1)
    gtr = si.gauge_field(dims, 1.0, seed=9)[0]          # one SU(3) matrix per site
    Lx, Ly, Lz, Lt = dims
    Ug = np.empty_like(U)
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        gn = np.roll(gtr, -1, axis=ax)                  # g(x + mu)
        Ug[mu] = np.einsum("...ij,...jk,...lk->...il", gtr, U[mu], gn.conj())
    H = hermitian_wilson(U, 1.4)
    Hg = hermitian_wilson(Ug, 1.4)
    rng = np.random.default_rng(0)
    v = (rng.normal(size=(Lt, Lz, Ly, Lx, 4, 3)) + 1j * rng.normal(size=(Lt, Lz, Ly, Lx, 4, 3)))
    gv = np.einsum("...ij,...sj->...si", gtr, v)
    lhs = (Hg @ gv.ravel()).reshape(v.shape)
    rhs = np.einsum("...ij,...sj->...si", gtr, (H @ v.ravel()).reshape(v.shape))
    assert np.abs(lhs - rhs).max() < 1e-13


@pytest.mark.parametrize("r", [0.2, 0.4])
def test_norm_bound(r):
    """||H_W|| <= 1 + 4/(4 - m0): each direction's hop is a unitary times 2."""
    m0 = 1.4
    H = hermitian_wilson(si.gauge_field((4, 4, 4, 4), r, seed=0), m0)
    top = spla.eigsh(H, k=1, which="LM", return_eigenvectors=False)[0]
    assert abs(top) <= 1 + 4 / (4 - m0) + 1e-12
    assert abs(top) > 1.5            # and the bound is not vacuous
