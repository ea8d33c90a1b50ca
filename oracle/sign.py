"""sgn(H_W) b and D_ov(m_q) b in plain FP64 (eqs. (1)-(7)).

``sign_by_solves`` is the definition of the quadrature written out: every
shifted system (z_j I - H_W) y_j = b of eq. (6) is solved on its own, and
s = sum_j c_j y_j (eqs. (5) and (7)).  It does not use a shifted (multi-shift)
Krylov method; it is the slow, obviously correct form.

``sign_by_eigh`` is eq. (2): a dense eigendecomposition H = V diag(lam) V^dag,
giving both the quadrature's result V diag(F(lam)) V^dag b and the exact sign
V diag(sgn(lam)) V^dag b (sgn(0) = 0, as the paper defines it).
"""
import multiprocessing as mp

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .contour import scalar_filter


def _solve_one(H, zj, b, method, rtol):
    n = H.shape[0]
    A = (zj * sp.identity(n, dtype=np.complex128, format="csr") - H).tocsc()
    if method == "dense":
        y = sla.solve(A.toarray(), b)
    elif method == "splu":
        y = spla.splu(A).solve(b)
    elif method == "gmres":
        # GMRES(m), m = min(n, 100): scipy preallocates the m-vector basis, and
        # these shifted systems converge without stagnation under restarts.
        # The Arnoldi residual estimate can stall a little above rtol near
        # machine precision, so the acceptance test is the true residual below.
        m = min(n, 100)
        y, info = spla.gmres(A.tocsr(), b, rtol=rtol, atol=0.0, restart=m, maxiter=200)
    else:
        raise ValueError(method)
    res = np.linalg.norm(b - A @ y) / np.linalg.norm(b)
    if method == "gmres" and res > 10 * rtol:
        raise RuntimeError(f"GMRES true residual {res:.3e} above 10*rtol (rtol={rtol})")
    return y, res


_pool_H = None


def _pool_init(H):
    global _pool_H
    _pool_H = H
    try:  # one BLAS thread per worker: the pool already spans the cores
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _pool_task(args):
    zj, b, method, rtol = args
    return _solve_one(_pool_H, zj, b, method, rtol)


def sign_by_solves(H, b, z, c, method="splu", rtol=1e-14, processes=1, return_parts=False):
    """s = sum_j c_j (z_j I - H)^-1 b, one independent solve per node.

    b: complex128 vector of length H.shape[0].  Returns s (and, with
    return_parts, the list of y_j and their relative true residuals).
    The sum runs in node order j = 0 .. len(z)-1.
    """
    b = np.asarray(b, dtype=np.complex128).ravel()
    if processes > 1:
        ctx = mp.get_context("fork")
        with ctx.Pool(processes, initializer=_pool_init, initargs=(H,)) as pool:
            results = pool.map(_pool_task, [(zj, b, method, rtol) for zj in z], chunksize=1)
    else:
        results = [_solve_one(H, zj, b, method, rtol) for zj in z]
    s = np.zeros_like(b)
    for cj, (y, _) in zip(c, results):
        s += cj * y
    if return_parts:
        return s, [y for y, _ in results], np.array([r for _, r in results])
    return s


def eigh_dense(H):
    """Dense eigendecomposition of the hermitian matrix H (eq. (2))."""
    Hd = H.toarray() if sp.issparse(H) else np.asarray(H)
    return np.linalg.eigh(Hd)


def sign_by_eigh(H, b, z=None, c=None, eig=None):
    """(s_filter, s_exact): V F(lam) V^dag b and V sgn(lam) V^dag b."""
    lam, Vv = eig if eig is not None else eigh_dense(H)
    bt = Vv.conj().T @ np.asarray(b, dtype=np.complex128)
    s_exact = Vv @ (np.sign(lam) * bt)
    s_filter = None
    if z is not None:
        s_filter = Vv @ (scalar_filter(lam, z, c) * bt)
    return s_filter, s_exact


def gamma5_flat(v):
    """gamma5 = diag(1, 1, -1, -1) on a flat vector with row = 12 site + 3 spin + colour."""
    w = np.array(v, dtype=np.complex128, copy=True).reshape(-1, 4, 3)
    w[:, 2:, :] *= -1
    return w.reshape(np.shape(v))


def overlap(b, s, mq):
    """D_ov(m_q) b = (1+m_q)/2 b + (1-m_q)/2 gamma5 s, with s = sgn(H_W) b (eq. (1))."""
    return 0.5 * (1.0 + mq) * np.asarray(b) + 0.5 * (1.0 - mq) * gamma5_flat(s)


def sigma(y, s):
    """Sign-function quality |s^dag s - y^dag y| / y^dag y for s = sgn(H_W) y
    (the measure defined in the Numerical experiments section)."""
    yy = np.vdot(y, y).real
    return abs(np.vdot(s, s).real - yy) / yy
