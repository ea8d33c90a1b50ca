"""The hermitian Wilson-Dirac operator H_W = gamma5 D_W(-m0) as a CSR matrix.

Definition (paper: eq. (1) and the text that follows it, which only names
D_W(-m0) with m0 > 0).  Readings taken where the paper is silent:

* normalisation: D_W = 1 - kappa * sum_mu [ (1 - gamma_mu) U_mu(x) delta_{x+mu,y}
  + (1 + gamma_mu) U_mu(x-mu)^dag delta_{x-mu,y} ],  kappa = 1/(2(4 - m0)).
  This is the Wilson operator with mass -m0 divided by (4 - m0).  It is the
  reading under which the paper's contour (Supplemental Material, numerical
  setup: centres +-1.2, radius 1.1999) encloses the whole spectrum at m0 = 1,
  since ||H_W|| <= 1 + 4/(4 - m0) = 7/3 < 2.3999.
* (1 - gamma_mu) goes with the forward hop.
* chiral gamma basis (``oracle.gamma``).
* boundary: a hop that wraps around direction mu is multiplied by bc[mu]
  (default periodic x, y, z and antiperiodic t).

Index convention: site = x + Lx*(y + Ly*(z + Lz*t)); row = 12*site + 3*spin +
colour, which is the row-major flattening of a spinor [Lt][Lz][Ly][Lx][4][3].
Links are U[mu][t][z][y][x][3][3].
"""
import numpy as np
import scipy.sparse as sp

from .gamma import gammas, gamma5


def kappa(m0):
    return 1.0 / (2.0 * (4.0 - m0))


def _site(dims):
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.indices((Lt, Lz, Ly, Lx))
    return x, y, z, t


def _flat(x, y, z, t, dims):
    Lx, Ly, Lz, Lt = dims
    return (x + Lx * (y + Ly * (z + Lz * t))).ravel()


def hermitian_wilson(U, m0, bc=(1, 1, 1, -1)):
    """H_W as a complex128 scipy CSR matrix of size 12V x 12V.

    U: complex128 [4][Lt][Lz][Ly][Lx][3][3].  Every lattice extent must be >= 2.
    """
    U = np.asarray(U, dtype=np.complex128)
    Lt, Lz, Ly, Lx = U.shape[1:5]
    dims = (Lx, Ly, Lz, Lt)
    if min(dims) < 2:
        raise ValueError("every lattice extent must be at least 2")
    V = Lx * Ly * Lz * Lt
    k = kappa(m0)
    g = gammas()
    g5 = gamma5()
    one4 = np.eye(4, dtype=np.complex128)
    x, y, z, t = _site(dims)
    here = _flat(x, y, z, t, dims)
    coord = [x, y, z, t]

    def blocks(spin, col3):
        # [V][12][12] blocks kron(spin, colour_v)
        return np.einsum("ab,vij->vaibj", spin, col3).reshape(V, 12, 12)

    rows, cols, vals = [], [], []

    def add(r_site, c_site, blk):
        rr = (12 * r_site)[:, None, None] + np.arange(12)[None, :, None]
        cc = (12 * c_site)[:, None, None] + np.arange(12)[None, None, :]
        rows.append(np.broadcast_to(rr, blk.shape).ravel())
        cols.append(np.broadcast_to(cc, blk.shape).ravel())
        vals.append(blk.ravel())

    # diagonal term: gamma5 * 1
    add(here, here, blocks(g5, np.broadcast_to(np.eye(3), (V, 3, 3))))
    for mu in range(4):
        L = dims[mu]
        fwd = [c.copy() for c in coord]
        fwd[mu] = (coord[mu] + 1) % L
        bwd = [c.copy() for c in coord]
        bwd[mu] = (coord[mu] - 1) % L
        wrap_f = (coord[mu] == L - 1).ravel()
        wrap_b = (coord[mu] == 0).ravel()
        ph_f = np.where(wrap_f, bc[mu], 1.0)
        ph_b = np.where(wrap_b, bc[mu], 1.0)
        Umu = U[mu].reshape(V, 3, 3)
        # U_mu(x - mu) for every x, as a [V][3][3] array in x order
        Ub = U[mu][bwd[3], bwd[2], bwd[1], bwd[0]].reshape(V, 3, 3)
        Ub_dag = np.conj(np.swapaxes(Ub, -1, -2))
        sf = g5 @ (one4 - g[mu])
        sb = g5 @ (one4 + g[mu])
        add(here, _flat(*fwd, dims), -k * ph_f[:, None, None] * blocks(sf, Umu))
        add(here, _flat(*bwd, dims), -k * ph_b[:, None, None] * blocks(sb, Ub_dag))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    keep = vals != 0
    H = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(12 * V, 12 * V))
    return H.tocsr()

