"""ovl_apply_hw_noalloc, the entry point that allocates nothing, through the
raw C ABI: two calls in a row (the second with fewer right-hand sides, so it
reuses the static scratch with a smaller footprint) give what ovl_apply_hw
gives, element by element, and both match the oracle's H_W; an input beyond
the scratch is rejected."""
import ctypes

import numpy as np
import pytest

import seeded_inputs as si
from tests.gpu_util import gauge, make_ctx, maxerr, oracle_H, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(ctx, x):
    import torch
    out = torch.empty_like(x)
    ctx._sync_stream()
    rc = ctx.lib.ovl_apply_hw_noalloc(ctx._h, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), x.shape[0])
    return rc, out


def test_noalloc_matches_apply_hw_twice():
    import torch
    from paper_2204_01583_amd import ovl
    ovl.load()
    dims = (6, 6, 4, 6)     # a partial 256-site block and a partial 64-site tile
    U = gauge(dims, 0.3, 2)
    H = oracle_H(dims, 0.3, 2, 1.4)
    ctx = make_ctx(dims, U)
    for nrhs, seed in ((3, 5), (1, 6)):
        b = to_dev(si.gaussian_sources(dims, nrhs, first_seed=seed))
        ref = ctx.apply_hw(b)                       # tunes (allocates) for this nrhs
        rc, out = _noalloc(ctx, b)
        torch.cuda.synchronize()
        assert rc == ovl.OK, ctx.lib.ovl_last_error(ctx._h)
        o, r = out.cpu().numpy(), ref.cpu().numpy()
        assert maxerr(o, r) < 1e-14
        for i in range(nrhs):
            assert maxerr(o[i], H @ b.cpu().numpy()[i].ravel()) < 1e-14
    ctx.close()


def test_noalloc_rejects_inputs_beyond_the_scratch():
    from paper_2204_01583_amd import ovl
    ovl.load()
    dims = (16, 16, 16, 16)  # 2 x 12 x 65536 x 16 B = 25.2 MB per rhs: 3 rhs exceed 64 MiB
    ctx = make_ctx(dims, gauge(dims, 0.3, 0))
    b = to_dev(si.gaussian_sources(dims, 3))
    rc, _ = _noalloc(ctx, b)
    assert rc == ovl.E_ARG
    rc, out = _noalloc(ctx, b[:2].contiguous())
    assert rc == ovl.OK
    ref = ctx.apply_hw(b[:2].contiguous())
    assert maxerr(out.cpu().numpy(), ref.cpu().numpy()) < 1e-14
    ctx.close()
