"""Pins of the oracle's quadrature, sign function, D_ov and force (CPU)."""
import json
import os

import numpy as np
import pytest

import seeded_inputs as si
from oracle import contour, freefield as ff
from oracle.force import action, force
from oracle.sign import eigh_dense, gamma5_flat, overlap, sigma, sign_by_eigh, sign_by_solves
from oracle.wilson import hermitian_wilson

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


@pytest.mark.parametrize("nq", [8, 32, 64, 128])
def test_circle_filter_closed_form(nq):
    """On a circle (alpha = 1) the trapezoidal sum over N points with
    theta_j = 2 pi (j - 1/2)/N equals 1/(1 + ((lam - g)/rho)^N) exactly,
    because the scaled nodes are the N roots of -1."""
    g, rho = 1.3, 1.2999
    z, c = contour.nodes(nq, g, rho, 1.0)
    lam = np.linspace(-3, 3, 601) + 0.013
    Fp = np.sum(c[:nq, None] / (z[:nq, None] - lam[None, :]), axis=0)
    exact = 1.0 / (1.0 + ((lam - g) / rho) ** nq)
    assert np.abs(Fp - exact).max() < 1e-13


def test_filter_odd_real_and_zero_at_zero():
    """sgn_N(lam) = F+(lam) - F+(-lam) for even N: odd, real on the real
    axis, and exactly 0 at lam = 0 (zero modes drop out, eq. (3))."""
    for (g, rho, a) in [(1.3, 1.2999, 1.0), (1.2, 1.1999, 0.1)]:
        z, c = contour.nodes(64, g, rho, a)
        lam = np.linspace(-2.5, 2.5, 1001)
        f = contour.scalar_filter(lam, z, c)
        assert np.abs(f.imag).max() < 1e-13
        assert np.abs(f + contour.scalar_filter(-lam, z, c)).max() < 1e-13
        assert abs(contour.scalar_filter(np.array([0.0]), z, c)[0]) < 1e-14


def test_single_contour_form():
    """2 P_+ - 1 agrees with the two-contour filter on the spectrum away from
    zero (the circle closed form gives both); at lam = 0 it gives 2 F_+(0) - 1
    (towards -1) where the two-contour filter gives exactly 0."""
    from oracle.contour import nodes, nodes_single, scalar_filter
    gamma, rho, alpha = 1.3, 1.2999, 1.0
    nq = 64
    z1, c1, c0 = nodes_single(nq, gamma, rho, alpha)
    assert len(z1) == nq and c0 == -1.0
    lam = np.concatenate([np.linspace(0.05, 2.5, 200), -np.linspace(0.05, 2.5, 200)])
    f1 = 2 * scalar_filter(lam, z1, c1 / 2) + c0          # 2 F_+ - 1
    # closed form of the circle filter F_+(lam) = 1 / (1 + ((lam - gamma)/rho)^N)
    fp = 1.0 / (1.0 + ((lam - gamma) / rho) ** nq)
    assert np.abs(f1 - (2 * fp - 1)).max() < 1e-13
    z2, c2 = nodes(nq, gamma, rho, alpha)
    f2 = scalar_filter(lam, z2, c2)
    # same function up to F_+(lam) + F_+(-lam) - 1, tiny away from 0 and the
    # spectrum's ends (where the filter itself departs from sgn)
    diff = np.abs(f1 - f2)
    assert diff.max() < 1e-2 and np.median(diff) < 1e-8
    # at lam = 0 the two-contour filter is exactly 0 (odd in lam); the
    # one-contour form gives 2 F_+(0) - 1, which tends to -1 with N, fast
    # when 0 lies well outside Gamma_+ (closed form on a circle with margin)
    zero = np.array([0.0])
    assert abs(scalar_filter(zero, z2, c2)[0]) < 1e-15
    for g, r in ((1.3, 1.2999), (1.3, 1.2)):
        zs, cs, c0s = nodes_single(nq, g, r, 1.0)
        f0 = scalar_filter(zero, zs, cs)[0] + c0s
        assert abs(f0 - (2.0 / (1.0 + (g / r) ** nq) - 1.0)) < 1e-12
    assert f0.real < -0.98


def test_paper_contour_counts_per_contour_points():
    """With the paper's ellipse, N_qtot >= 500 gives sigma <= 1e-14 (Results
    summary).  The filter error on the spectrum range reaches that only if
    N_qtot counts the points of one contour: at N = 500 per contour the error
    is ~1e-15, while 250 per contour (500 in total) is ~1e-11."""
    p = json.load(open(GOLDEN))
    a, rho, g = p["contour"]["alpha"], p["contour"]["rho"], p["contour"]["gamma"]
    lam = np.concatenate([np.linspace(0.02, 2.33, 3000), -np.linspace(0.02, 2.33, 3000)])
    err = {}
    for n in (100, 250, 500):
        z, c = contour.nodes(n, g, rho, a)
        err[n] = np.abs(contour.scalar_filter(lam, z, c) - np.sign(lam)).max()
    assert err[500] < p["summary_claim"]["sigma_at_most"]
    assert err[250] > 1e-12
    assert err[100] > 1e-6
    # the contour encloses (0.0001, 2.3999) and the normalised free operator fits
    z, _ = contour.nodes(500, g, rho, a)
    assert z.real.max() == pytest.approx(g + rho * np.cos(np.pi / 500), abs=1e-12)
    assert z[:500].real.min() == pytest.approx(g - rho * np.cos(np.pi / 500), abs=1e-12)
    m0 = p["m0"]
    assert 1 + 4 / (4 - m0) < g + rho


@pytest.fixture(scope="module")
def small_system():
    dims = (2, 2, 2, 4)
    U = si.gauge_field(dims, 0.2, seed=0)       # spectral gap 0.163
    H = hermitian_wilson(U, 1.4)
    b = si.gaussian_sources(dims, 1)[0].ravel()
    return dims, U, H, b, eigh_dense(H)


def test_solves_match_spectral_filter(small_system):
    """Independent per-node solves agree with V F(lam) V^dag b (eq. (2))."""
    dims, U, H, b, eig = small_system
    z, c = contour.nodes(32, 1.3, 1.2999, 1.0)
    s_solve = sign_by_solves(H, b, z, c, method="dense")
    s_filt, _ = sign_by_eigh(H, b, z, c, eig=eig)
    assert np.linalg.norm(s_solve - s_filt) / np.linalg.norm(s_filt) < 1e-13
    s_gm = sign_by_solves(H, b, z, c, method="gmres", rtol=1e-14)
    assert np.linalg.norm(s_gm - s_filt) / np.linalg.norm(s_filt) < 1e-12


def test_quadrature_error_bound(small_system):
    """||sgn_N b - sgn b|| <= max_lam |F(lam) - sgn(lam)| ||b|| (H normal)."""
    dims, U, H, b, eig = small_system
    lam = eig[0]
    for nq in (32, 128, 400):
        z, c = contour.nodes(nq, 1.3, 1.2999, 1.0)
        s_n = sign_by_solves(H, b, z, c, method="dense")
        _, s_ex = sign_by_eigh(H, b, eig=eig)
        bound = np.abs(contour.scalar_filter(lam, z, c) - np.sign(lam)).max()
        err = np.linalg.norm(s_n - s_ex) / np.linalg.norm(b)
        assert err <= bound * (1 + 1e-6) + 1e-14
    assert err < 1e-12           # N = 400 per contour is exact to double precision


def test_sign_squared_and_sigma(small_system):
    """sgn(H)^2 = 1 and sigma = 0 for the exact sign; the quadrature form
    meets both to within its filter error at large N (Numerical experiments:
    the GW relation is equivalent to sgn^2 = 1)."""
    dims, U, H, b, eig = small_system
    _, s = sign_by_eigh(H, b, eig=eig)
    _, s2 = sign_by_eigh(H, s, eig=eig)
    assert np.linalg.norm(s2 - b) / np.linalg.norm(b) < 1e-13
    assert sigma(b, s) < 1e-14
    z, c = contour.nodes(400, 1.3, 1.2999, 1.0)
    sn = sign_by_solves(H, b, z, c, method="dense")
    sn2 = sign_by_solves(H, sn, z, c, method="dense")
    assert np.linalg.norm(sn2 - b) / np.linalg.norm(b) < 1e-12
    assert sigma(b, sn) < 1e-13
    z, c = contour.nodes(8, 1.3, 1.2999, 1.0)        # a poor quadrature is detected
    assert sigma(b, sign_by_solves(H, b, z, c, method="dense")) > 1e-4


def _dense_overlap(eig, mq):
    lam, Vv = eig
    eps = (Vv * np.sign(lam)) @ Vv.conj().T
    n = eps.shape[0]
    g5 = np.diag(np.tile([1, 1, 1, 1, 1, 1, -1, -1, -1, -1, -1, -1], n // 12)).astype(complex)
    return 0.5 * (1 + mq) * np.eye(n) + 0.5 * (1 - mq) * g5 @ eps, g5


def test_ginsparg_wilson_factor_two(small_system):
    """For D = (1 + gamma5 sgn)/2 (eq. (1) at m_q = 0) the identity equivalent
    to sgn^2 = 1 is {D, gamma5} = 2 D gamma5 D; the relation as printed in
    the Numerical experiments section lacks the factor 2 for this
    normalisation (reading documented with the oracle)."""
    dims, U, H, b, eig = small_system
    D, g5 = _dense_overlap(eig, 0.0)
    lhs = D @ g5 + g5 @ D
    assert np.abs(lhs - 2 * D @ g5 @ D).max() < 1e-12
    assert np.abs(lhs - D @ g5 @ D).max() > 0.1


def test_overlap_spectrum_on_circle(small_system):
    """gamma5 sgn(H) is unitary, so D_ov(0) has its spectrum on |l - 1/2| = 1/2."""
    dims, U, H, b, eig = small_system
    D, _ = _dense_overlap(eig, 0.0)
    ev = np.linalg.eigvals(D)
    assert np.abs(np.abs(ev - 0.5) - 0.5).max() < 1e-12


def test_overlap_formula_matches_dense(small_system):
    dims, U, H, b, eig = small_system
    _, s = sign_by_eigh(H, b, eig=eig)
    D, _ = _dense_overlap(eig, 0.05)
    assert np.allclose(overlap(b, s, 0.05), D @ b, atol=1e-13)
    assert np.allclose(gamma5_flat(gamma5_flat(b)), b)


def test_free_field_fft_route_matches_solves():
    """The momentum-space filter (any size) equals independent solves."""
    dims = (4, 4, 4, 4)
    H = hermitian_wilson(si.unit_gauge(dims), 1.4)
    b = si.gaussian_sources(dims, 1)[0]
    z, c = contour.nodes(16, 1.3, 1.2999, 1.0)
    s_fft = ff.apply_function(b, dims, 1.4, lambda l: contour.scalar_filter(l, z, c))
    s_sol = sign_by_solves(H, b.ravel(), z, c, method="gmres", rtol=1e-14, processes=4)
    assert np.linalg.norm(s_fft.ravel() - s_sol) / np.linalg.norm(s_sol) < 1e-12


def test_sign_gauge_covariant(small_system):
    dims, U, H, b, eig = small_system
    gtr = si.gauge_field(dims, 1.0, seed=4)[0]
    Ug = np.empty_like(U)
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        Ug[mu] = np.einsum("...ij,...jk,...lk->...il", gtr, U[mu], np.roll(gtr, -1, axis=ax).conj())
    z, c = contour.nodes(16, 1.3, 1.2999, 1.0)
    bb = b.reshape(dims[::-1] + (4, 3))
    gb = np.einsum("...ij,...sj->...si", gtr, bb).ravel()
    s1 = sign_by_solves(hermitian_wilson(Ug, 1.4), gb, z, c, method="dense")
    s0 = sign_by_solves(H, b, z, c, method="dense").reshape(bb.shape)
    assert np.abs(s1 - np.einsum("...ij,...sj->...si", gtr, s0).ravel()).max() < 1e-12


def test_force_matches_finite_differences():
    """Brute force: central differences of the dense action along a random
    complex link direction (G) and along a random su(3) direction (F)."""
    dims = (2, 2, 2, 4)
    m0, mq = 1.4, 0.1
    U = si.gauge_field(dims, 0.3, seed=0)
    phi = si.gaussian_sources(dims, 1)[0].ravel()
    z, c = contour.nodes(16, 1.3, 1.2999, 1.0)
    G, F, S = force(U, phi, m0, mq, z, c, method="dense")
    assert S == pytest.approx(action(hermitian_wilson(U, m0), phi, z, c, mq, "dense"), rel=1e-13)
    rng = np.random.default_rng(5)
    E = rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape)
    h = 1e-5
    Sp = action(hermitian_wilson(U + h * E, m0), phi, z, c, mq, "dense")
    Sm = action(hermitian_wilson(U - h * E, m0), phi, z, c, mq, "dense")
    an = np.sum((G.conj() * E).real)
    assert abs((Sp - Sm) / (2 * h) - an) / abs(an) < 1e-8
    om = si.random_su3_direction(dims, 7)
    Om = np.einsum("...k,kij->...ij", om, si.gell_mann()) / 2

    def expi(hh):
        e, W = np.linalg.eigh(hh * Om)
        return np.einsum("...ij,...j,...kj->...ik", W, np.exp(1j * e), W.conj())

    Up = np.einsum("...ij,...jk->...ik", expi(h), U)
    Um = np.einsum("...ij,...jk->...ik", expi(-h), U)
    fd = (action(hermitian_wilson(Up, m0), phi, z, c, mq, "dense") -
          action(hermitian_wilson(Um, m0), phi, z, c, mq, "dense")) / (2 * h)
    an = np.einsum("...ij,...ji->...", Om, F).sum().real
    assert abs(fd - an) < 1e-7 * abs(an)
    assert np.abs(F - np.conj(np.swapaxes(F, -1, -2))).max() < 1e-14
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-14
