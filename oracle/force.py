"""Derivative of S = phi^dag D_ov^dag D_ov phi with respect to the links.

The paper gives no force; this follows from eq. (1) and the resolvent form
under eq. (4).  The sign is the quadrature's rational function
eps(H) = sum_j c_j G_j with G_j = (z_j - H)^-1, so S is an exact function of
the links and

  dS  = 2 Re[ psi^dag d(eps) phi ],   psi = b_m gamma5 D_ov phi,  b_m = (1-m_q)/2,
  d(eps) = sum_j c_j G_j dH G_j       (d(A^-1) = -A^-1 dA A^-1 with dA = -dH),
  dS  = 2 Re sum_j c_j X_j^dag dH Y_j, Y_j = G_j phi,  X_j = G_j^dag psi = (conj(z_j) - H)^-1 psi.

A link U_mu(x) (boundary phase ph) enters H in two blocks:
row x, column x+mu: -kappa ph gamma5 (1 - gamma_mu) U, and row x+mu, column x:
-kappa ph gamma5 (1 + gamma_mu) U^dag.  Writing every link as an unconstrained
complex 3x3 matrix gives

  dS = Re sum_links sum_ab conj(G_ab) dU_ab,    G = conj(A) + B^T,
  A_ab = -2 kappa ph sum_j c_j sum_{s,s'} conj(X_j(x)_{s a}) M_{s s'} Y_j(x+mu)_{s' b},      M  = gamma5 (1 - gamma_mu)
  B_cd = -2 kappa ph sum_j c_j sum_{s,s'} conj(X_j(x+mu)_{s c}) M'_{s s'} Y_j(x)_{s' d},     M' = gamma5 (1 + gamma_mu)

G is the complex gradient (PyTorch's convention for a real function of a
complex tensor: dS = Re sum conj(G) dU).  For a move along SU(3),
U -> exp(i h Omega) U with Omega hermitian traceless, dS/dh = sum_links
tr(Omega F) with the traceless hermitian force
F = TH[(Z + Z^dag)/2], Z = i U G^dag, TH removing the trace.
"""
import numpy as np

from .gamma import gammas, gamma5
from .sign import sign_by_solves, overlap, gamma5_flat, _solve_one
from .wilson import hermitian_wilson, kappa


def action(H, phi, z, c, mq, method="splu", rtol=1e-14):
    """S = || D_ov(m_q) phi ||^2 with every shifted system solved on its own."""
    s = sign_by_solves(H, phi, z, c, method=method, rtol=rtol)
    d = overlap(phi, s, mq)
    return float(np.vdot(d, d).real)


def _shift(field, mu, step):
    """field[..., t, z, y, x, 4, 3] -> field at x + step*mu (periodic index shift)."""
    axis = {0: -3, 1: -4, 2: -5, 3: -6}[mu]
    return np.roll(field, -step, axis=axis)


def force(U, phi, m0, mq, z, c, bc=(1, 1, 1, -1), method="splu", rtol=1e-14):
    """(G, F, S): complex gradient, SU(3) force and action.

    U: [4][Lt][Lz][Ly][Lx][3][3]; phi: spinor [Lt][Lz][Ly][Lx][4][3] or flat.
    G and F have the shape of U.
    """
    U = np.asarray(U, dtype=np.complex128)
    Lt, Lz, Ly, Lx = U.shape[1:5]
    sshape = (Lt, Lz, Ly, Lx, 4, 3)
    H = hermitian_wilson(U, m0, bc)
    phi = np.asarray(phi, dtype=np.complex128).ravel()
    s = sign_by_solves(H, phi, z, c, method=method, rtol=rtol)
    dphi = overlap(phi, s, mq)
    S = float(np.vdot(dphi, dphi).real)
    psi = 0.5 * (1.0 - mq) * gamma5_flat(dphi)
    k = kappa(m0)
    g = gammas()
    g5 = gamma5()
    one4 = np.eye(4)
    G = np.zeros_like(U)
    for j in range(len(z)):
        Y = _solve_one(H, z[j], phi, method, rtol)[0].reshape(sshape)
        X = _solve_one(H, np.conj(z[j]), psi, method, rtol)[0].reshape(sshape)
        for mu in range(4):
            L = (Lx, Ly, Lz, Lt)[mu]
            coord = np.indices((Lt, Lz, Ly, Lx))[3 - mu]
            ph = np.where(coord == L - 1, bc[mu], 1.0)[..., None, None]
            M = g5 @ (one4 - g[mu])
            Mp = g5 @ (one4 + g[mu])
            Yf = _shift(Y, mu, 1)
            Xf = _shift(X, mu, 1)
            K1 = np.einsum("...sa,st,...tb->...ab", X.conj(), M, Yf)
            K2 = np.einsum("...sc,st,...td->...cd", Xf.conj(), Mp, Y)
            A = -2.0 * k * ph * c[j] * K1
            B = -2.0 * k * ph * c[j] * K2
            G[mu] += np.conj(A) + np.swapaxes(B, -1, -2)
    Z = 1j * np.einsum("...ab,...cb->...ac", U, G.conj())
    F = 0.5 * (Z + np.conj(np.swapaxes(Z, -1, -2)))
    tr = np.trace(F, axis1=-2, axis2=-1)
    F = F - tr[..., None, None] * np.eye(3) / 3.0
    return G, F, S
