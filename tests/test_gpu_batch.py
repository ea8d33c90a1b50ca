"""Batched solves over uneven lattices (one job-table launch per stage,
graph-captured chunks), the two-pass form, and graph replay against eager
launches."""
import os

import numpy as np
import pytest

import seeded_inputs as si
from tests.gpu_util import CIRCLE, gauge, make_ctx, relerr, to_dev

pytestmark = pytest.mark.gpu
REF8 = os.path.join(os.path.dirname(__file__), "golden",
                    "sign_8x8x8x8_r0.3_m1.4_nq64_circle_src1000.npy")


def setup_module(module):
    from paper_2204_01583_amd import ovl
    ovl.load()


@pytest.mark.parametrize("precision,form", [(0, 1), (0, 0), (1, 2), (1, 3)])
def test_graph_replay_equals_eager(precision, form, monkeypatch):
    """Every solve replays its captured 16-iteration graph many times; the
    result must equal the eagerly launched solve bit for bit (same kernels,
    deterministic reductions), on two applies in a row."""
    dims = (4, 4, 4, 6)
    U = gauge(dims, 0.3, 3)
    b = to_dev(si.gaussian_sources(dims, 2, first_seed=21))
    ctx = make_ctx(dims, U, nq=16, precision=precision, form=form)
    g1, st = ctx.apply_sign(b)
    g2, _ = ctx.apply_sign(b)
    monkeypatch.setenv("OVL_GRAPHS", "0")
    e1, _ = ctx.apply_sign(b)
    print(f"prec {precision} form {form}: iterations {st.iterations}")
    assert st.iterations > 32            # several chunk replays
    assert bool((g1 == e1).all()) and bool((g2 == e1).all())
    ctx.close()


@pytest.mark.parametrize("precision,form", [(1, 2), (1, 3), (0, 1), (0, 2)])
def test_lookahead_equals_chunk_by_chunk(precision, form):
    """Normally the solver keeps one chunk queued ahead of the state poll
    (away from the precision switch and convergence), and each chunk graph
    ends by exporting the state to pinned host memory; with profiling on it
    polls every chunk before queueing the next.  Results, iteration counts
    and the FP64/FP32 split must agree bit for bit, with a tolerance that
    ends the solve several chunks in."""
    dims = (4, 4, 4, 6)
    U = gauge(dims, 0.3, 3)
    b = to_dev(si.gaussian_sources(dims, 2, first_seed=21))
    ctx = make_ctx(dims, U, nq=16, precision=precision, form=form)
    a, sa = ctx.apply_sign(b)
    ctx.set_profiling(True)
    p, sp = ctx.apply_sign(b)
    ctx.set_profiling(False)
    a2, _ = ctx.apply_sign(b)
    print(f"prec {precision} form {form}: iterations {sa.iterations} ({sa.fp32_iterations} FP32)")
    assert sa.iterations > 128           # many chunks, look-ahead on for most
    assert (sa.iterations, sa.fp32_iterations) == (sp.iterations, sp.fp32_iterations)
    assert bool((a == p).all()) and bool((a2 == p).all())
    ctx.close()


def test_init_partials_beyond_the_update_grid():
    """A lattice whose initial ||b||^2 reduction runs more blocks per source
    (up to 512) than the basis forms' update kernel (256 plus one per shift
    slice): the reduction's partials have a buffer of their own size, and
    the basis and two-pass forms, batched and alone, agree with the FP64
    sweep form (a regression test for partials once sized by the update
    grid)."""
    from paper_2204_01583_amd import ovl
    dims = (16, 16, 16, 6)  # 12 V / 1024 = 288 > 256 blocks
    U = gauge(dims, 0.3, 4)
    b = to_dev(si.gaussian_sources(dims, 2, first_seed=500))
    ref_ctx = make_ctx(dims, U, nq=16, precision=0, form=1)
    ref, _ = ref_ctx.apply_sign(b)
    ref = ref.cpu().numpy()
    ref_ctx.close()
    for form in (2, 3):
        ctx = make_ctx(dims, U, nq=16, precision=0, form=form)
        s, _ = ctx.apply_sign(b)
        err = relerr(s.cpu().numpy(), ref)
        print(f"form {form} against the sweep form: {err:.2e}")
        assert err < 1e-12
        outs, _ = ovl.apply_sign_batched([ctx], [b])
        assert relerr(outs[0].cpu().numpy(), ref) < 1e-12
        ctx.close()


def test_twopass_equals_basis():
    dims = (8, 8, 8, 8)
    U = gauge(dims, 0.3, 0)
    b = to_dev(si.gaussian_sources(dims, 2, first_seed=1000))
    ctx = make_ctx(dims, U, 1.4, 0.05, 64, precision=1, form=2)
    s_basis, st1 = ctx.apply_sign(b)
    ctx.set_solver(1, 3, tol=1e-12, maxiter=3000)
    s_two, st2 = ctx.apply_sign(b)
    err = relerr(s_two.cpu().numpy(), s_basis.cpu().numpy())
    print(f"two-pass vs basis (mixed): {err:.2e}, iterations {st1.iterations} {st2.iterations}")
    assert st1.iterations == st2.iterations
    assert err < 1e-13
    ctx.close()


@pytest.mark.parametrize("precision,form", [(1, 3), (0, 2)])
def test_batched_uneven_lattices(precision, form):
    """A batch of fields of different sizes and roughness, several sources
    each, in one solve: every job equals its own unbatched solve, and the
    job carrying the stored 8^4 workload matches the oracle."""
    from paper_2204_01583_amd import ovl
    specs = [((8, 8, 8, 8), 0.3, 0), ((4, 4, 6, 6), 0.2, 1), ((6, 6, 6, 8), 0.4, 2),
             ((4, 4, 4, 4), 0.3, 3), ((3, 5, 4, 6), 0.3, 4)]    # the last with a partial layout tile
    nq = 64
    ctxs, ins = [], []
    for dims, r, seed in specs:
        c = make_ctx(dims, gauge(dims, r, seed), 1.4, 0.05, nq, precision=precision, form=form)
        ctxs.append(c)
        ins.append(to_dev(si.gaussian_sources(dims, 3, first_seed=1000)))
    outs, st = ovl.apply_sign_batched(ctxs, ins)
    print(f"batched: iterations {st.iterations}, fp32 {st.fp32_iterations}")
    tol = 1e-10 if precision else 1e-11
    ref8 = np.load(REF8)
    assert relerr(outs[0][0].cpu().numpy(), ref8) < tol
    # FP64: the same kernels and reductions, so the jobs agree to rounding;
    # mixed: every job switches to FP32 on its own residuals.  The switch
    # falls on a chunk boundary, which may come one 16-iteration chunk
    # earlier in the batch (its polls wait for every job to be far from its
    # switch before queueing ahead), so the FP32 split agrees to within a chunk.
    same = 1e-12 if precision == 0 else 1e-10
    for c, x, o in zip(ctxs, ins, outs):
        bst = c.stats()
        single, sst = c.apply_sign(x)
        err = relerr(o.cpu().numpy(), single.cpu().numpy())
        print(f"  {c.dims}: batched vs single {err:.2e}, iterations {bst.iterations} / "
              f"{sst.iterations}, fp32 {bst.fp32_iterations} / {sst.fp32_iterations}")
        assert err < same
        assert abs(bst.iterations - sst.iterations) <= 2
        assert abs(bst.fp32_iterations - sst.fp32_iterations) <= 16 + 2
    for c in ctxs:
        c.close()


def test_batched_rejects_bad_arguments():
    from paper_2204_01583_amd import ovl
    dims = (4, 4, 4, 4)
    c = make_ctx(dims, gauge(dims, 0.3, 0), nq=8)
    x = to_dev(si.gaussian_sources(dims, 1))
    with pytest.raises(ovl.OvlError):
        ovl.apply_sign_batched([c, c], [x, x])          # the same context twice
    d = ovl.Context(dims)                                # no gauge field
    with pytest.raises(ovl.OvlError):
        ovl.apply_sign_batched([c, d], [x, x])
    c.close()
    d.close()


def test_batched_single_contour_matches_single_solves():
    """The lead context's node set, here the one-contour form with its
    constant term, applies to every job of a batch: each batched output
    equals that context's own solve with the same settings."""
    from paper_2204_01583_amd import ovl
    sizes = [(4, 4, 4, 4), (4, 4, 2, 6)]
    ctxs, ins = [], []
    for i, dims in enumerate(sizes):
        c = make_ctx(dims, gauge(dims, 0.3, 10 + i), precision=0, form=2)
        c.set_contour_single(16, *CIRCLE)
        ctxs.append(c)
        ins.append(to_dev(si.gaussian_sources(dims, 2, first_seed=81)))
    outs, _ = ovl.apply_sign_batched(ctxs, ins)
    for c, x, o in zip(ctxs, ins, outs):
        ref, st = c.apply_sign(x)
        assert st.n_shifts == 16
        assert relerr(o.cpu().numpy(), ref.cpu().numpy()) < 1e-13
    for c in ctxs:
        c.close()


@pytest.mark.timeout(900)
def test_batch_each_size_class_against_the_oracle():
    """One batched mixed-precision two-pass solve over one field of each size
    class of the uneven workload (8^4, 12^4, 16^3x32; roughness 0.2, 0.27,
    0.4) with the lead's node set: 4 stratified nodes of the 2 x 64 circle
    with their eq. (7) weights.  Every job against the oracle's independent
    solves on the same nodes, relative 2-norm and element-wise, to 1e-10."""
    from oracle.contour import nodes
    from oracle.sign import sign_by_solves
    from tests.gpu_util import NPROC, assert_close, oracle_H
    from paper_2204_01583_amd import ovl
    z, c = nodes(64, *CIRCLE)
    pick = np.array([5, 37, 69, 101])
    jobs = [((8, 8, 8, 8), 0.2, 0), ((12, 12, 12, 12), 0.2 + 0.2 / 3, 11),
            ((16, 16, 16, 32), 0.4, 23)]
    ctxs, ins, refs = [], [], []
    for dims, r, seed in jobs:
        U = gauge(dims, r, seed)
        b = si.gaussian_sources(dims, 1, first_seed=1000)
        ctx = make_ctx(dims, U, precision=1, form=3, tol=1e-12, switch_res=1e-4)
        ctxs.append(ctx)
        ins.append(to_dev(b))
        refs.append(sign_by_solves(oracle_H(dims, r, seed, 1.4), b[0].ravel(), z[pick], c[pick],
                                   method="gmres", rtol=1e-14, processes=min(NPROC, 4)))
    ctxs[0].set_nodes(z[pick], c[pick])
    outs, st = ovl.apply_sign_batched(ctxs, ins)
    assert st.n_active_end == 0 and st.fp32_iterations > 0
    for (dims, _, _), o, ref in zip(jobs, outs, refs):
        assert_close(o.cpu().numpy()[0], ref, 1e-10, f"batched {dims}")
    for ctx in ctxs:
        ctx.close()


@pytest.mark.parametrize("form", [2, 3])
def test_batch_jobs_finishing_at_very_different_times(form):
    """Jobs leave the batch grids as they finish: a zero source (done before
    the first iteration), a smooth field that converges early and a rough one
    that converges late, mixed precision.  Every job equals its own solve,
    the zero source gives zero, and a second batched call (grids laid out
    afresh, graphs captured again) repeats the first bit for bit."""
    from paper_2204_01583_amd import ovl
    specs = [((4, 4, 4, 4), 0.2, 3, True), ((4, 4, 4, 6), 0.1, 4, False),
             ((6, 4, 4, 4), 0.45, 5, False)]
    ctxs, ins = [], []
    for dims, r, seed, zero in specs:
        c = make_ctx(dims, gauge(dims, r, seed), 1.4, 0.1, 32, precision=1, form=form, tol=1e-12,
                     switch_res=1e-3)
        x = to_dev(si.gaussian_sources(dims, 2, first_seed=90))
        ctxs.append(c)
        ins.append(x * 0 if zero else x)
    outs, st = ovl.apply_sign_batched(ctxs, ins)
    iters = [c.stats().iterations for c in ctxs]
    print(f"form {form}: per-job iterations {iters}")
    assert iters[1] + 32 < iters[2]          # they leave the grids chunks apart
    assert float(outs[0].abs().max()) == 0.0
    outs2, _ = ovl.apply_sign_batched(ctxs, ins)
    for o, o2 in zip(outs, outs2):
        assert bool((o == o2).all())
    for c, x, o in zip(ctxs[1:], ins[1:], outs[1:]):
        single, _ = c.apply_sign(x)
        assert relerr(o.cpu().numpy(), single.cpu().numpy()) < 1e-10
    for c in ctxs:
        c.close()
