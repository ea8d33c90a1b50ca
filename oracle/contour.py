"""Quadrature nodes and weights of the contour-integral projectors (eq. (7)).

For one ellipse with centre gamma, radius rho and vertical scaling alpha,
eq. (7) takes theta_j = 2 pi (j - 1/2)/N_q, j = 1..N_q,
z_j = gamma + rho (cos theta_j + i alpha sin theta_j) and the weight
rho w_j / N_q with w_j = alpha cos theta_j + i sin theta_j, which is the
trapezoidal rule for the integral of dz/(2 pi i) around the ellipse.

sgn(H) = P_+ - P_- (eq. (3)): Gamma_+ has centre +gamma and Gamma_- centre
-gamma; the weights of Gamma_- are negated.  Reading taken: N_q counts the
points of ONE contour, so a sign application uses 2 N_q shifted systems.
The paper's own contour (Supplemental Material, numerical setup) is
alpha = 0.1, rho = 1.1999, gamma = 1.2.
"""
import numpy as np


def nodes(nq, gamma, rho, alpha):
    """(z, c): complex128 arrays of length 2*nq, Gamma_+ nodes first."""
    nq = int(nq)
    if nq < 1:
        raise ValueError("nq must be positive")
    j = np.arange(1, nq + 1)
    theta = 2.0 * np.pi * (j - 0.5) / nq
    w = alpha * np.cos(theta) + 1j * np.sin(theta)
    ell = rho * (np.cos(theta) + 1j * alpha * np.sin(theta))
    z = np.concatenate([gamma + ell, -gamma + ell])
    c = np.concatenate([rho * w / nq, -rho * w / nq])
    return z, c


def nodes_single(nq, gamma, rho, alpha):
    """(z, c, c0) of the one-contour form sgn(H) = 2 P_+ - 1, which holds when
    H has no exact zero mode (P_+ + P_- = 1, eq. (3)): the Gamma_+ nodes
    with twice their weights, and the constant term c0 = -1."""
    z, c = nodes(nq, gamma, rho, alpha)
    nq = int(nq)
    return z[:nq], 2.0 * c[:nq], -1.0


def scalar_filter(lam, z, c):
    """sum_j c_j / (z_j - lam): the scalar function the quadrature applies
    to each eigenvalue lam of H_W (the resolvent expansion under eq. (4))."""
    lam = np.asarray(lam, dtype=np.complex128)
    return np.sum(c[:, None] / (z[:, None] - lam.ravel()[None, :]), axis=0).reshape(lam.shape)
