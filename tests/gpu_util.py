"""Helpers for the GPU tests: contexts on cuda:0 fed from the seeded inputs,
and cached oracle results."""
import functools
import os

import numpy as np

import seeded_inputs as si
from oracle.contour import nodes
from oracle.sign import sign_by_solves
from oracle.wilson import hermitian_wilson

CIRCLE = (1.3, 1.2999, 1.0)   # gamma, rho, alpha: encloses (1e-4, 2.5999)
NPROC = min(16, len(os.sched_getaffinity(0)))


def relerr(a, b):
    """Relative 2-norm error ||a - b|| / ||b|| over the whole array."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxerr(a, b):
    """Element-wise relative error max_i |a_i - b_i| / max_i |b_i|: an error
    confined to a few elements (a padded tile, a boundary wrap, one block) is
    not diluted by the size of the array, as it is in relerr."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.abs(a - b).max() / np.abs(b).max())


def assert_close(a, b, tol, what=""):
    """Both the relative 2-norm error and the element-wise error below tol."""
    e2, em = relerr(a, b), maxerr(a, b)
    print(f"{what}: rel 2-norm {e2:.2e}, element-wise {em:.2e} (tol {tol:.0e})")
    assert e2 < tol and em < tol, (what, e2, em, tol)
    return e2, em


def make_ctx(dims, U, m0=1.4, mq=0.1, nq=None, contour=CIRCLE, precision=0, form=1,
             tol=1e-12, maxiter=3000, bc=(1, 1, 1, -1), switch_res=0.0):
    import torch
    from paper_2204_01583_amd import ovl
    ctx = ovl.Context(dims, bc=bc, device=0)
    ctx.set_gauge(torch.from_numpy(np.ascontiguousarray(U)).to("cuda:0"))
    ctx.set_masses(m0, mq)
    if nq is not None:
        ctx.set_contour(nq, *contour)
    ctx.set_solver(precision, form, tol=tol, maxiter=maxiter, switch_res=switch_res)
    return ctx


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@functools.lru_cache(maxsize=None)
def gauge(dims, r, seed):
    return si.gauge_field(dims, r, seed)


@functools.lru_cache(maxsize=None)
def oracle_H(dims, r, seed, m0):
    return hermitian_wilson(gauge(dims, r, seed), m0)


@functools.lru_cache(maxsize=None)
def oracle_sign(dims, r, seed, m0, nq, contour, src_seed):
    """sum_j c_j (z_j - H)^-1 b by independent GMRES solves (rtol 1e-14)."""
    H = oracle_H(dims, r, seed, m0)
    b = si.gaussian_sources(dims, 1, first_seed=src_seed)[0]
    z, c = nodes(nq, *contour)
    return sign_by_solves(H, b.ravel(), z, c, method="gmres", rtol=1e-14, processes=NPROC)
