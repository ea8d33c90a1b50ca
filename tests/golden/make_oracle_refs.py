"""Writes the stored oracle results used by the GPU parity tests.

Calls only the oracle (and the seeded input generator).  Each file holds
s = sum_j c_j (z_j - H_W)^-1 b for one seeded workload, every shifted system
solved on its own by GMRES to a relative true residual of 1e-14, as a
complex128 vector in the row order of a spinor [Lt][Lz][Ly][Lx][4][3].

    python tests/golden/make_oracle_refs.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import seeded_inputs as si                          # noqa: E402
from oracle.contour import nodes                    # noqa: E402
from oracle.sign import sign_by_solves              # noqa: E402
from oracle.wilson import hermitian_wilson          # noqa: E402

CIRCLE = (1.3, 1.2999, 1.0)

# name -> (dims, roughness, gauge seed, m0, nq per contour, contour, source seed)
REFS = {
    "sign_8x8x8x8_r0.3_m1.4_nq64_circle_src1000":
        ((8, 8, 8, 8), 0.3, 0, 1.4, 64, CIRCLE, 1000),
}


def path(name):
    return os.path.join(HERE, name + ".npy")


def make(name, processes):
    dims, r, seed, m0, nq, contour, src = REFS[name]
    H = hermitian_wilson(si.gauge_field(dims, r, seed), m0)
    b = si.gaussian_sources(dims, 1, first_seed=src)[0].ravel()
    z, c = nodes(nq, *contour)
    t = time.time()
    s, _, res = sign_by_solves(H, b, z, c, method="gmres", rtol=1e-14, processes=processes,
                               return_parts=True)
    print(f"{name}: {len(z)} solves in {time.time() - t:.1f}s, max true residual {res.max():.2e}")
    np.save(path(name), s)


if __name__ == "__main__":
    nproc = len(os.sched_getaffinity(0))
    for name in REFS:
        make(name, nproc)
