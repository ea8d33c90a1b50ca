"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle."""
import os

import numpy as np
import pytest

import seeded_inputs as si
from oracle import freefield as ff
from oracle.contour import nodes, scalar_filter
from oracle.sign import overlap
from tests.gpu_util import (CIRCLE, NPROC, assert_close, gauge, make_ctx, maxerr, oracle_H,
                             oracle_sign, relerr, to_dev)

pytestmark = pytest.mark.gpu


def setup_module(module):
    import torch
    from paper_2204_01583_amd import ovl
    ovl.load()                      # fails loudly if the library was not built
    assert torch.cuda.is_available()


# ---------------------------------------------------------------- stencil
@pytest.mark.parametrize("dims,r", [((4, 4, 4, 4), 0.3), ((8, 8, 8, 8), 0.3),
                                    ((3, 5, 4, 6), 0.4), ((2, 2, 2, 2), 0.2),
                                    ((16, 16, 16, 16), 0.3)])
def test_hw_matches_oracle(dims, r):
    U = gauge(dims, r, 0)
    ctx = make_ctx(dims, U)
    b = si.gaussian_sources(dims, 3)
    out = ctx.apply_hw(to_dev(b)).cpu().numpy()
    H = oracle_H(dims, r, 0, 1.4)
    for i in range(3):
        ref = H @ b[i].ravel()
        err = float(np.abs(out[i].ravel() - ref).max() / np.abs(ref).max())
        assert err < 1e-14, err
    ctx.close()


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 5, 4, 6), (16, 16, 16, 16)])
def test_hw_fp32_matches_oracle(dims):
    """The FP32 stencil of the mixed solver against the FP64 oracle, element
    by element.  Rounding the inputs and links to FP32 and ~100 FP32
    operations per element give ~3e-7 (an FP32 emulation of the CSR product
    measures 2-4e-7), hence the 1e-6 bound."""
    U = gauge(dims, 0.3, 0)
    ctx = make_ctx(dims, U)
    b = si.gaussian_sources(dims, 2)
    out = ctx.apply_hw_fp32(to_dev(b)).cpu().numpy()
    H = oracle_H(dims, 0.3, 0, 1.4)
    for i in range(2):
        ref = H @ b[i].ravel()
        err = maxerr(out[i], ref)
        print(f"{dims} rhs {i}: FP32 H_W element-wise error {err:.2e}")
        assert err < 1e-6, err
    ctx.close()


def test_gauge_nonfinite_rejected():
    """A NaN or an infinity anywhere in the field (here in the third row of
    one link, the row the two-row link form would rebuild) is rejected: the
    context then has no gauge field until a finite one is set."""
    from paper_2204_01583_amd import ovl
    dims = (4, 4, 4, 4)
    U = gauge(dims, 0.3, 0)
    b = to_dev(si.gaussian_sources(dims, 1))
    ctx = make_ctx(dims, U, nq=16)
    for bad_value in (float("nan"), float("inf")):
        Ub = U.copy()
        Ub[3, 1, 2, 0, 3, 2, 1] = bad_value
        with pytest.raises(ovl.OvlError) as e:
            ctx.set_gauge(to_dev(Ub))
        assert e.value.status == ovl.E_NONFINITE
        with pytest.raises(ovl.OvlError) as e:
            ctx.apply_hw(b)
        assert e.value.status == ovl.E_STATE
        with pytest.raises(ovl.OvlError) as e:
            ctx.apply_sign(b)
        assert e.value.status == ovl.E_STATE
    ctx.set_gauge(to_dev(U))
    out = ctx.apply_hw(b).cpu().numpy()
    ref = oracle_H(dims, 0.3, 0, 1.4) @ b.cpu().numpy()[0].ravel()
    assert maxerr(out[0], ref) < 1e-14
    ctx.close()


def test_hw_periodic_time_and_other_mass():
    dims = (4, 4, 2, 6)
    U = gauge(dims, 0.3, 2)
    ctx = make_ctx(dims, U, m0=1.0, bc=(1, -1, 1, 1))
    b = si.gaussian_sources(dims, 1)
    out = ctx.apply_hw(to_dev(b)).cpu().numpy()
    from oracle.wilson import hermitian_wilson
    ref = hermitian_wilson(U, 1.0, bc=(1, -1, 1, 1)) @ b[0].ravel()
    assert_close(out[0], ref, 1e-14, "H_W, antiperiodic y, m0 = 1")
    ctx.close()


def test_hw_free_plane_wave_16():
    dims = (16, 16, 16, 16)
    ctx = make_ctx(dims, si.unit_gauge(dims))
    rng = np.random.default_rng(3)
    for n in [(0, 0, 0, 0), (3, 7, 11, 5), (15, 1, 8, 12)]:
        chi = rng.normal(size=4) + 1j * rng.normal(size=4)
        col = rng.normal(size=3) + 1j * rng.normal(size=3)
        pw = ff.plane_wave(dims, n, chi, col)
        p = [np.array(2 * np.pi * (n[m] + (0.5 if m == 3 else 0)) / 16) for m in range(4)]
        ref = ff.plane_wave(dims, n, ff.h_of_p(p, 1.4) @ chi, col)
        out = ctx.apply_hw(to_dev(pw)).cpu().numpy()
        # the reference's own phases 2 pi n x / L carry ~1e-14 relative rounding
        err = float(np.abs(out - ref).max() / np.abs(ref).max())
        assert err < 5e-14, err
    ctx.close()


# ---------------------------------------------------------------- sign
CFG0 = dict(dims=(4, 4, 4, 4), r=0.3, seed=0, m0=1.4, mq=0.1, nq=32)


@pytest.mark.parametrize("form", [0, 1, 2, 3])
def test_sign_4x4_fp64_all_forms(form):
    c = CFG0
    U = gauge(c["dims"], c["r"], c["seed"])
    ctx = make_ctx(c["dims"], U, c["m0"], c["mq"], c["nq"], form=form)
    b = si.gaussian_sources(c["dims"], 1)[0]
    s, st = ctx.apply_sign(to_dev(b))
    ref = oracle_sign(c["dims"], c["r"], c["seed"], c["m0"], c["nq"], CIRCLE, 1000)
    assert_close(s.cpu().numpy(), ref, 1e-11, f"form {form}, {st.iterations} iterations")
    assert st.n_active_end == 0 and st.max_est_rel_res <= 1e-12
    ctx.close()


@pytest.mark.parametrize("form", [1, 2, 3])
def test_sign_4x4_mixed(form):
    c = CFG0
    U = gauge(c["dims"], c["r"], c["seed"])
    ctx = make_ctx(c["dims"], U, c["m0"], c["mq"], c["nq"], precision=1, form=form)
    b = si.gaussian_sources(c["dims"], 1)[0]
    s, st = ctx.apply_sign(to_dev(b))
    ref = oracle_sign(c["dims"], c["r"], c["seed"], c["m0"], c["nq"], CIRCLE, 1000)
    assert st.fp32_iterations > 0
    assert_close(s.cpu().numpy(), ref, 1e-10,
                 f"mixed form {form}, {st.iterations} iterations ({st.fp32_iterations} FP32)")
    ctx.close()


def test_dov_4x4_multi_rhs():
    c = CFG0
    U = gauge(c["dims"], c["r"], c["seed"])
    ctx = make_ctx(c["dims"], U, c["m0"], c["mq"], c["nq"], form=1)
    b = si.gaussian_sources(c["dims"], 2)
    d, st = ctx.apply_dov(to_dev(b))
    d = d.cpu().numpy()
    for i in range(2):
        s_ref = oracle_sign(c["dims"], c["r"], c["seed"], c["m0"], c["nq"], CIRCLE, 1000 + i)
        ref = overlap(b[i].ravel(), s_ref, c["mq"])
        assert_close(d[i], ref, 1e-11, f"D_ov rhs {i}")
    ctx.close()


REF8 = os.path.join(os.path.dirname(__file__), "golden",
                    "sign_8x8x8x8_r0.3_m1.4_nq64_circle_src1000.npy")


@pytest.mark.parametrize("precision,form,tol", [(0, 1, 1e-11), (0, 2, 1e-11), (1, 2, 1e-10),
                                                (0, 3, 1e-11), (1, 3, 1e-10)])
def test_sign_8x8(precision, form, tol):
    """8^4, 2 x 64 nodes, against the stored oracle result (make_oracle_refs.py)."""
    dims, nq = (8, 8, 8, 8), 64
    U = gauge(dims, 0.3, 0)
    ctx = make_ctx(dims, U, 1.4, 0.05, nq, precision=precision, form=form)
    b = si.gaussian_sources(dims, 1)[0]
    s, st = ctx.apply_sign(to_dev(b))
    ref = np.load(REF8)
    assert_close(s.cpu().numpy(), ref, tol,
                 f"8^4 prec {precision} form {form}, {st.iterations} iterations "
                 f"({st.fp32_iterations} FP32), {st.seconds:.3f}s")
    ctx.close()


def test_sign_free_field_16_fft():
    """16^4 unit links: against the momentum-space oracle at full size."""
    dims, nq = (16, 16, 16, 16), 32
    ctx = make_ctx(dims, si.unit_gauge(dims), 1.4, 0.1, nq, form=2)
    b = si.gaussian_sources(dims, 1)[0]
    s, st = ctx.apply_sign(to_dev(b))
    z, c = nodes(nq, *CIRCLE)
    ref = ff.apply_function(b, dims, 1.4, lambda l: scalar_filter(l, z, c))
    assert_close(s.cpu().numpy(), ref, 1e-11, f"16^4 free field, {st.iterations} iterations")
    ctx.close()


# ---------------------------------------------------------------- errors
def test_error_paths():
    from paper_2204_01583_amd import ovl
    dims = (4, 4, 4, 4)
    U = gauge(dims, 0.3, 0)
    b = to_dev(si.gaussian_sources(dims, 1))
    ctx = ovl.Context(dims)
    with pytest.raises(ovl.OvlError) as e:
        ctx.apply_hw(b)
    assert e.value.status == ovl.E_STATE
    ctx.set_gauge(to_dev(U))
    ctx.set_masses(1.4, 0.1)
    with pytest.raises(ovl.OvlError) as e:
        ctx.apply_sign(b)
    assert e.value.status == ovl.E_STATE
    with pytest.raises(ovl.OvlError) as e:
        ctx.set_contour(33, *CIRCLE)
    assert e.value.status == ovl.E_ARG
    with pytest.raises(ovl.OvlError):
        ctx.set_masses(4.5, 0.0)
    with pytest.raises(ovl.OvlError):
        ctx.set_nodes([1.0 + 0j], [1.0 + 0j])       # node on the real axis
    ctx.set_contour(16, *CIRCLE)
    ctx.set_solver(0, 1, tol=1e-12, maxiter=1)
    s, st = ctx.apply_sign(b, allow_not_converged=True)
    assert st.iterations == 1 and st.n_active_end > 0
    with pytest.raises(ovl.OvlError) as e:
        ctx.apply_sign(b)
    assert e.value.status == ovl.NOT_CONVERGED
    ctx.set_solver(0, 1, tol=1e-12, maxiter=500)
    bad = b.clone()
    bad[0, 1, 2, 3, 0, 1, 2] = float("nan")
    with pytest.raises(ovl.OvlError) as e:
        ctx.apply_sign(bad)
    assert e.value.status == ovl.E_NONFINITE
    # aliasing in/out through the raw ABI
    import ctypes
    rc = ctx.lib.ovl_apply_hw(ctx._h, ctypes.c_void_p(b.data_ptr()),
                              ctypes.c_void_p(b.data_ptr()), 1)
    assert rc == ovl.E_ARG
    # host pointer rejected
    hb = b.cpu()
    rc = ctx.lib.ovl_apply_hw(ctx._h, ctypes.c_void_p(hb.data_ptr()),
                              ctypes.c_void_p(b.data_ptr()), 1)
    assert rc == ovl.E_ARG
    # zero source gives zero
    z0 = b * 0
    s, st = ctx.apply_sign(z0)
    assert float(s.abs().max()) == 0.0
    # shift limits: 2048 in all, 1024 for the sweep forms
    with pytest.raises(ovl.OvlError) as e:
        ctx.set_contour(1026, *CIRCLE)
    assert e.value.status == ovl.E_ARG
    ctx.set_contour(600, *CIRCLE)
    ctx.set_solver(0, 1, tol=1e-12, maxiter=500)
    with pytest.raises(ovl.OvlError) as e:
        ctx.apply_sign(b)
    assert e.value.status == ovl.E_ARG
    ctx.close()


def test_deterministic():
    c = CFG0
    U = gauge(c["dims"], c["r"], c["seed"])
    ctx = make_ctx(c["dims"], U, c["m0"], c["mq"], c["nq"], form=2)
    b = to_dev(si.gaussian_sources(c["dims"], 2))
    s1, _ = ctx.apply_sign(b)
    s2, _ = ctx.apply_sign(b)
    assert bool((s1 == s2).all())
    ctx.close()


@pytest.mark.parametrize("form", [0, 2])
def test_true_residual_single_node(form):
    """With one node and weight 1 the output is x = (z - H)^-1 b itself, so
    the true residual the library reports can be recomputed here from the
    oracle's H; loose tolerance so the residual is far above rounding."""
    dims = (4, 4, 4, 4)
    U = gauge(dims, 0.3, 0)
    ctx = make_ctx(dims, U, form=form, tol=1e-6)
    z = 0.3 + 0.4j
    ctx.set_nodes([z], [1.0])
    ctx.set_residual_check(1)
    b = si.gaussian_sources(dims, 2, first_seed=21)
    out, st = ctx.apply_sign(to_dev(b))
    x = out.cpu().numpy()
    H = oracle_H(dims, 0.3, 0, 1.4)
    mine = 0.0
    for n in range(2):
        bv, xv = b[n].ravel(), x[n].ravel()
        mine = max(mine, np.linalg.norm(bv - (z * xv - H @ xv)) / np.linalg.norm(bv))
    assert 1e-9 < mine < 1e-5, mine
    assert abs(st.max_true_rel_res - mine) <= 1e-6 * mine, (st.max_true_rel_res, mine)
    ctx.close()


@pytest.mark.parametrize("precision,form", [(0, 2), (0, 0), (1, 2), (0, 1)])
def test_true_residual_contour(precision, form):
    """On the full contour the recurrence's residual estimates track the true
    residuals of the shifts it reports worst (FP64), and the mixed path stays
    within a small factor of the tolerance; forms that keep no x_j report -1."""
    dims = (4, 4, 4, 8)
    U = gauge(dims, 0.3, 3)
    tol = 1e-10
    ctx = make_ctx(dims, U, nq=32, precision=precision, form=form, tol=tol)
    ctx.set_residual_check(3)
    b = si.gaussian_sources(dims, 2, first_seed=31)
    _, st = ctx.apply_sign(to_dev(b))
    print("true", st.max_true_rel_res, "est", st.max_est_rel_res, "iters", st.iterations)
    if form == 1:
        assert st.max_true_rel_res == -1.0
    elif precision == 0:
        assert 0.5 * st.max_est_rel_res < st.max_true_rel_res < 2.0 * st.max_est_rel_res + 1e-14
        assert st.max_true_rel_res < 2 * tol
    else:
        assert 0.0 < st.max_true_rel_res < 100 * tol
    ctx.close()


@pytest.mark.parametrize("links", ["two-row", "full"])
@pytest.mark.parametrize("variant", list(range(28)))
def test_stencil_variants(variant, links, monkeypatch):
    """Every stencil variant the autotuner may pick gives the oracle's H_W,
    including an odd number of right-hand sides (the two-rhs tail), and the
    same sign function in both precisions; SU(3) fields in the two-row link
    form (third row rebuilt, boundary sign applied) and in the full form."""
    monkeypatch.setenv("OVL_STENCIL_VARIANT", str(variant))
    if links == "full":
        monkeypatch.setenv("OVL_LINKS", "full")
    dims = (4, 6, 4, 8)
    U = gauge(dims, 0.3, 1)
    # the sweep form runs the two-kernel iteration, whose stencil is the forced variant
    ctx = make_ctx(dims, U, nq=16, precision=1, form=1)
    H = oracle_H(dims, 0.3, 1, 1.4)
    for nrhs in (1, 3):
        b = si.gaussian_sources(dims, nrhs, first_seed=7)
        out = ctx.apply_hw(to_dev(b)).cpu().numpy()
        for i in range(nrhs):
            ref = H @ b[i].ravel()
            err = float(np.abs(out[i].ravel() - ref).max() / np.abs(ref).max())
            assert err < 1e-14, (nrhs, i, err)
        out32 = ctx.apply_hw_fp32(to_dev(b)).cpu().numpy()
        for i in range(nrhs):
            ref = H @ b[i].ravel()
            assert maxerr(out32[i], ref) < 1e-6, ("fp32", nrhs, i)
    b = si.gaussian_sources(dims, 3, first_seed=7)
    s, st = ctx.apply_sign(to_dev(b))
    fmt = 0 if links == "full" else 1
    assert st.stencil_variant64 == variant + 28 * fmt
    assert st.stencil_variant32 == variant + 28 * fmt
    ref = oracle_sign(dims, 0.3, 1, 1.4, 16, CIRCLE, 7)
    assert_close(s[0].cpu().numpy(), ref, 1e-10, f"mixed sign, variant {variant} {links}")
    ctx.close()
    # a volume that is not a multiple of the 256-site tile (ragged last block)
    dims = (6, 6, 4, 6)
    U = gauge(dims, 0.3, 2)
    ctx = make_ctx(dims, U, nq=16, precision=1, form=2)
    H = oracle_H(dims, 0.3, 2, 1.4)
    b = si.gaussian_sources(dims, 3, first_seed=9)
    out = ctx.apply_hw(to_dev(b)).cpu().numpy()
    for i in range(3):
        ref = H @ b[i].ravel()
        err = float(np.abs(out[i].ravel() - ref).max() / np.abs(ref).max())
        assert err < 1e-14, ("ragged", i, err)
    ctx.close()


@pytest.mark.parametrize("variant", [v for v in range(24) if not v & 4])
def test_stencil_plane_patch(variant, monkeypatch):
    """Rhs-fastest variants on a lattice of whole 16 x 16 (z, t) planes, where
    each XCD's run of planes is mapped to a (z, t) patch: H_W in both
    precisions against the oracle, element by element, and the FP64 shifted
    solve (job-table stencil, whose block partials sit at the permuted site
    blocks' indices) against the same solve with the site-fastest twin
    variant, whose blocks are not permuted."""
    dims = (16, 16, 4, 8)
    U = gauge(dims, 0.3, 5)
    H = oracle_H(dims, 0.3, 5, 1.4)
    b = si.gaussian_sources(dims, 3, first_seed=11)
    sols = []
    for v in (variant, variant | 4):
        monkeypatch.setenv("OVL_STENCIL_VARIANT", str(v))
        ctx = make_ctx(dims, U, nq=16, precision=0, form=2)
        if v == variant:
            out = ctx.apply_hw(to_dev(b)).cpu().numpy()
            out32 = ctx.apply_hw_fp32(to_dev(b)).cpu().numpy()
            for i in range(3):
                ref = H @ b[i].ravel()
                assert maxerr(out[i], ref) < 1e-14, ("fp64", i)
                assert maxerr(out32[i], ref) < 1e-6, ("fp32", i)
        s, st = ctx.apply_sign(to_dev(b))
        assert st.stencil_variant64 == v + 28  # two-row links (SU(3) field)
        sols.append(s.cpu().numpy())
        ctx.close()
    assert_close(sols[0], sols[1], 1e-12, f"sign, variant {variant} against {variant | 4}")


def test_single_contour_against_oracle():
    """The one-contour form 2 P_+ - 1 (opt-in) against the oracle's direct
    solves with the same nodes and constant term, in FP64 and mixed."""
    from oracle.contour import nodes_single
    from oracle.sign import sign_by_solves
    c = CFG0
    U = gauge(c["dims"], c["r"], c["seed"])
    b = si.gaussian_sources(c["dims"], 2, first_seed=41)
    H = oracle_H(c["dims"], c["r"], c["seed"], c["m0"])
    z, w, c0 = nodes_single(32, *CIRCLE)
    refs = [sign_by_solves(H, b[n].ravel(), z, w, method="gmres", processes=NPROC)
            + c0 * b[n].ravel() for n in range(2)]
    for precision, form, tol in ((0, 2, 1e-11), (1, 2, 1e-10), (0, 1, 1e-11)):
        ctx = make_ctx(c["dims"], U, precision=precision, form=form)
        ctx.set_contour_single(32, *CIRCLE)
        s, st = ctx.apply_sign(to_dev(b))
        assert st.n_shifts == 32
        for n in range(2):
            assert_close(s[n].cpu().numpy(), refs[n], tol, f"single contour {precision} {form} {n}")
        ctx.close()


def test_spectral_bounds_and_suggested_contour():
    """Ritz values of the seed recurrence bound H_W's spectrum (oracle eigh at
    4^4), and the contour suggested from them reaches sgn^2 = 1 to the target."""
    from oracle.sign import eigh_dense
    from paper_2204_01583_amd import ovl
    c = CFG0
    U = gauge(c["dims"], c["r"], c["seed"])
    lam = np.linalg.eigvalsh(oracle_H(c["dims"], c["r"], c["seed"], c["m0"]).toarray())
    b = si.gaussian_sources(c["dims"], 1, first_seed=51)
    ctx = make_ctx(c["dims"], U, nq=32, form=2, tol=1e-12)
    ctx.apply_sign(to_dev(b))
    lo, hi, gap = ctx.spectral_bounds(0)
    true_gap = np.abs(lam).min()
    print("ritz", lo, hi, gap, "eig", lam[0], lam[-1], true_gap)
    assert abs(lo - lam[0]) < 1e-8 and abs(hi - lam[-1]) < 1e-8
    assert true_gap * (1 - 1e-10) <= gap < 1.01 * true_gap
    lmax = max(-lo, hi)
    nq, g, r = ovl.suggest_contour(gap, lmax, 1e-10)
    ctx.set_contour(nq, g, r, 1.0)
    s, _ = ctx.apply_sign(to_dev(b))
    s2, _ = ctx.apply_sign(s)
    err = relerr(s2.cpu().numpy(), b)
    assert err < 1e-9, (nq, err)
    ctx.close()


def test_non_su3_links_keep_full_form():
    """A field that is not SU(3) (scaled links) cannot use the two-row form:
    the library must detect it, and H_W and sgn must still match the oracle
    built from the same links."""
    from oracle.wilson import hermitian_wilson
    dims = (4, 4, 4, 4)
    U = gauge(dims, 0.3, 0) * 1.001
    ctx = make_ctx(dims, U, nq=32, form=2)
    H = hermitian_wilson(U, 1.4)
    b = si.gaussian_sources(dims, 2, first_seed=61)
    out = ctx.apply_hw(to_dev(b)).cpu().numpy()
    for n in range(2):
        ref = H @ b[n].ravel()
        assert float(np.abs(out[n].ravel() - ref).max() / np.abs(ref).max()) < 1e-14
    ctx.close()


def test_sign_ragged_lattice_below_one_tile():
    """sgn on a lattice of 192 sites (one partial 256-site tile) and on one of
    384 sites (a tile and a half), FP64 and mixed, against the oracle."""
    from oracle.sign import sign_by_solves
    from oracle.contour import nodes
    for dims in ((4, 4, 2, 6), (6, 4, 4, 4)):
        U = gauge(dims, 0.3, 4)
        H = oracle_H(dims, 0.3, 4, 1.4)
        b = si.gaussian_sources(dims, 1, first_seed=71)
        z, c = nodes(16, *CIRCLE)
        ref = sign_by_solves(H, b[0].ravel(), z, c, method="gmres", processes=NPROC)
        for precision, tol in ((0, 1e-11), (1, 1e-10)):
            ctx = make_ctx(dims, U, nq=16, precision=precision, form=2)
            s, _ = ctx.apply_sign(to_dev(b))
            assert_close(s[0].cpu().numpy(), ref, tol, f"{dims} precision {precision}")
            ctx.close()


def test_sign_partial_layout_tile_two_sources():
    """Volumes that are not a multiple of the 64-site layout tile (360 and 180
    sites: 24 and 12 padding sites in the last tile), two sources (so the
    second one starts 12 Vt elements in), basis, two-pass and fused forms in
    FP64 and mixed precision, against the oracle."""
    from oracle.sign import sign_by_solves
    from oracle.contour import nodes
    for dims in ((3, 5, 4, 6), (5, 3, 3, 4)):
        U = gauge(dims, 0.3, 5)
        H = oracle_H(dims, 0.3, 5, 1.4)
        b = si.gaussian_sources(dims, 2, first_seed=81)
        z, c = nodes(16, *CIRCLE)
        refs = [sign_by_solves(H, b[n].ravel(), z, c, method="gmres", processes=NPROC)
                for n in range(2)]
        mq = 0.1
        for precision, form, tol in ((0, 2, 1e-11), (1, 2, 1e-10), (1, 3, 1e-10), (0, 1, 1e-11)):
            ctx = make_ctx(dims, U, mq=mq, nq=16, precision=precision, form=form)
            s, _ = ctx.apply_sign(to_dev(b))
            d, _ = ctx.apply_dov(to_dev(b))
            for n in range(2):
                assert_close(s[n].cpu().numpy(), refs[n], tol, f"sgn {dims} {precision} {form} {n}")
                # D_ov b = (1 + mq)/2 b + (1 - mq)/2 gamma5 sgn b, gamma5 = diag(1, 1, -1, -1)
                g5s = refs[n].reshape(-1, 4, 3) * np.array([1, 1, -1, -1])[None, :, None]
                dref = 0.5 * (1 + mq) * b[n].ravel() + 0.5 * (1 - mq) * g5s.ravel()
                assert_close(d[n].cpu().numpy(), dref, tol, f"D_ov {dims} {precision} {form} {n}")
            ctx.close()


def test_sign_invariants_16x16x16x16_bench_configuration():
    """At the benchmark's size and launch configuration (16^4, roughness 0.3,
    4 sources, 2 x 128 circle nodes, mixed precision, basis form), properties
    that hold exactly for the rational function s = F(H) b: F(H) hermitian,
    <a, F b> = <F a, b>; F commutes with H, H F b = F H b; and the true
    residuals of the shifts active longest (in-band and two more, synchronous)
    stay within the mixed path's bound 10 eps32 switch_res, the drift its FP32
    phase adds to the tolerance the estimates meet, without an FP64 repeat."""
    import torch
    dims = (16, 16, 16, 16)
    U = gauge(dims, 0.3, 0)
    ctx = make_ctx(dims, U, nq=128, precision=1, form=2, tol=1e-12, switch_res=1e-4)
    ctx.set_residual_check(2)
    b = to_dev(si.gaussian_sources(dims, 4))
    s, st = ctx.apply_sign(b)
    print(f"16^4 mixed: true residual {st.max_true_rel_res:.3e}, estimate {st.max_est_rel_res:.3e}, "
          f"FP32 iterations {st.fp32_iterations} of {st.iterations}")
    bound = 10 * 2.0 ** -24 * 1e-4
    assert st.n_active_end == 0 and st.fp64_repeat == 0
    assert 0 < st.max_true_rel_res < bound, st.max_true_rel_res
    ctx.set_residual_check(0)
    # hermiticity: <b_i, F b_j> = <F b_i, b_j>
    B = b.reshape(4, -1)
    S = s.reshape(4, -1)
    g1 = torch.conj(B) @ S.T
    g2 = torch.conj(S) @ B.T
    assert float((g1 - g2).abs().max() / g1.abs().max()) < 1e-10
    # commutation: H (F b) = F (H b)
    hs = ctx.apply_hw(s)
    hb = ctx.apply_hw(b)
    shb, _ = ctx.apply_sign(hb)
    assert float((hs - shb).norm() / hs.norm()) < 1e-10
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_ginsparg_wilson_relation(precision):
    """At m_q = 0, D = (1 + gamma5 sgn(H_W))/2 (eq. (1)) satisfies
    {D, gamma5} = 2 D gamma5 D when sgn^2 = 1, the relation the Numerical
    experiments section checks (with the factor 2 that eq. (1)'s
    normalisation gives).  The paper's ellipse with 300 points per contour
    has a filter error of ~2e-13 on this field's spectrum, so the relation
    holds to the solver's accuracy."""
    dims = (4, 4, 4, 4)
    U = gauge(dims, 0.3, 0)
    ctx = make_ctx(dims, U, m0=1.4, mq=0.0, nq=300, contour=(1.2, 1.1999, 0.1),
                   precision=precision, form=2, tol=1e-13)
    b = si.gaussian_sources(dims, 1, first_seed=91)[0]
    g5 = np.array([1, 1, -1, -1], dtype=np.complex128)[:, None]
    g5b = b * g5
    d, _ = ctx.apply_dov(to_dev(np.stack([b, g5b])))
    d = d.cpu().numpy()
    db, dg5b = d[0], d[1]
    dg5db, _ = ctx.apply_dov(to_dev(g5 * db))
    lhs = dg5b + g5 * db
    rhs = 2.0 * dg5db.cpu().numpy()
    err = relerr(lhs, rhs)
    print(f"precision {precision}: GW defect {err:.2e}, element-wise {maxerr(lhs, rhs):.2e}")
    assert err < 1e-10 and maxerr(lhs, rhs) < 1e-10
    ctx.close()


@pytest.mark.timeout(900)
def test_sign_16x16x16x16_oracle_node_sample():
    """The benchmark's configuration (16^4, roughness 0.3, m0 = 1.4, 4
    Gaussian sources, the 2 x 128 circle nodes, basis form, tolerance 1e-12)
    against the oracle on a stratified sample of the nodes: every 32nd node,
    4 on each contour, with their eq. (7) weights.  Both sides compute
    sum_j c_j (z_j - H_W)^-1 b over the same 8 nodes, the oracle by 32
    independent GMRES solves to a true residual of 1e-14; FP64 to 1e-11 and
    mixed precision (switch at 1e-4) to 1e-10, as relative 2-norm and
    element-wise errors per source."""
    from oracle.contour import nodes
    from oracle.sign import sign_by_solves
    dims = (16, 16, 16, 16)
    U = gauge(dims, 0.3, 0)
    b = si.gaussian_sources(dims, 4, first_seed=1000)
    z, c = nodes(128, *CIRCLE)
    pick = np.arange(8, 256, 32)
    H = oracle_H(dims, 0.3, 0, 1.4)
    refs = [sign_by_solves(H, b[n].ravel(), z[pick], c[pick], method="gmres", rtol=1e-14,
                           processes=NPROC) for n in range(4)]
    bd = to_dev(b)
    for precision, tol in ((0, 1e-11), (1, 1e-10)):
        ctx = make_ctx(dims, U, mq=0.1, precision=precision, form=2, tol=1e-12,
                       switch_res=1e-4)
        ctx.set_nodes(z[pick], c[pick])
        s, st = ctx.apply_sign(bd)
        s = s.cpu().numpy()
        assert st.n_active_end == 0
        for n in range(4):
            assert_close(s[n], refs[n], tol, f"16^4 precision {precision} source {n} "
                         f"({st.iterations} iterations, {st.fp32_iterations} FP32)")
        ctx.close()


def test_inband_residual_check_matches_synchronous_check():
    """The in-band check (basis form, default on) rebuilds every source's
    worst shifted solution inside the final basis sum and reports its FP64
    true residual; the synchronous diagnostic of the same worst shift gives
    the same value, and -1 turns both off."""
    dims = (4, 4, 4, 8)
    U = gauge(dims, 0.3, 3)
    b = to_dev(si.gaussian_sources(dims, 2, first_seed=31))
    ctx = make_ctx(dims, U, nq=32, precision=0, form=2, tol=1e-10)
    _, st0 = ctx.apply_sign(b)
    assert 0.0 < st0.max_true_rel_res < 2e-10, st0.max_true_rel_res
    ctx.set_residual_check(1)
    _, st1 = ctx.apply_sign(b)
    assert abs(st1.max_true_rel_res - st0.max_true_rel_res) <= 1e-6 * st0.max_true_rel_res
    ctx.set_residual_check(-1)
    _, st2 = ctx.apply_sign(b)
    assert st2.max_true_rel_res == -1.0
    assert st0.fp64_repeat == 0 and st0.mixed_true_rel_res == -1.0
    ctx.close()


def test_mixed_repeats_in_fp64_when_the_check_fails():
    """Mixed precision switched to FP32 very early (at 1e-2) drifts to a true
    residual of about eps32 * 1e-2: within the default bound (max(10 tol,
    10 eps32 switch)) no repeat happens; with the bound set to 10 tol = 1e-13
    the in-band check sees the drift, the apply is solved again in FP64, and
    the result is the FP64 one (oracle parity at 1e-11).  With the default
    switch at tol 1e-12 no repeat is needed."""
    c = CFG0
    U = gauge(c["dims"], c["r"], c["seed"])
    b = si.gaussian_sources(c["dims"], 1)[0]
    ref = oracle_sign(c["dims"], c["r"], c["seed"], c["m0"], c["nq"], CIRCLE, 1000)
    ctx = make_ctx(c["dims"], U, c["m0"], c["mq"], c["nq"], precision=1, form=2, tol=1e-14,
                   switch_res=1e-2)
    s, st = ctx.apply_sign(to_dev(b))
    eps32 = 2.0 ** -24
    print(f"switch 1e-2: iterations {st.iterations} ({st.fp32_iterations} FP32), true residual "
          f"{st.max_true_rel_res:.3e}, estimate {st.max_est_rel_res:.3e}, stencils "
          f"{st.stencil_variant64} / {st.stencil_variant32}")
    assert st.fp32_iterations > 0
    assert st.fp64_repeat == 0 and 1e-13 < st.max_true_rel_res <= 10 * eps32 * 1e-2
    ctx.set_check_bound(1e-13)
    s, st = ctx.apply_sign(to_dev(b))
    print("repeat", st.fp64_repeat, "mixed true res", st.mixed_true_rel_res,
          "final", st.max_true_rel_res)
    assert st.fp64_repeat == 1 and st.mixed_true_rel_res > 1e-13
    assert st.fp32_iterations == 0 and st.max_true_rel_res <= 1e-13
    assert_close(s.cpu().numpy(), ref, 1e-11, "after the FP64 repeat")
    ctx.set_check_bound(0.0)
    ctx.set_solver(1, 2, tol=1e-12, switch_res=1e-4)
    s, st = ctx.apply_sign(to_dev(b))
    assert st.fp64_repeat == 0 and st.fp32_iterations > 0 and st.max_true_rel_res < 1e-11
    ctx.close()


@pytest.mark.parametrize("links", ["two-row", "full"])
@pytest.mark.parametrize("variant", [0, 1, 17, 21])
def test_inband_check_sees_the_fp32_drift(variant, links, monkeypatch):
    """Mixed precision switched to FP32 at 1e-2 on 4^4 (2 x 32 nodes, tol
    1e-14): the result moves about 3e-10 from the FP64 one, and the in-band
    check must see the drift behind it for every stencil the tuner may pick.
    All converged shifts end with estimates just below tol; the check takes
    the shift active longest (most FP32 iterations), not the largest
    estimate, which had picked shifts that stopped in the FP64 phase (true
    residual 1e-14) for about half the variants."""
    monkeypatch.setenv("OVL_STENCIL_VARIANT", str(variant))
    if links == "full":
        monkeypatch.setenv("OVL_LINKS", "full")
    c = CFG0
    U = gauge(c["dims"], c["r"], c["seed"])
    b = to_dev(si.gaussian_sources(c["dims"], 1)[0])
    ctx = make_ctx(c["dims"], U, c["m0"], c["mq"], c["nq"], precision=1, form=2, tol=1e-14,
                   switch_res=1e-2)
    s, st = ctx.apply_sign(b)
    ctx.set_solver(0, 2, tol=1e-14)
    s64, _ = ctx.apply_sign(b)
    err = float((s - s64).norm() / s64.norm())
    print(f"variant {variant} {links}: FP32 iterations {st.fp32_iterations}, true residual "
          f"{st.max_true_rel_res:.3e}, estimate {st.max_est_rel_res:.3e}, vs FP64 {err:.2e}")
    assert st.fp32_iterations > 0 and err > 1e-11
    assert st.max_true_rel_res > 1e-11, "the check missed the FP32 drift"
    ctx.close()


@pytest.mark.parametrize("links", ["two-row", "full"])
@pytest.mark.parametrize("variant", list(range(8)))
def test_fused_iteration_variants(variant, links, monkeypatch):
    """Every variant of the fused one-kernel iteration (hops per loop step,
    block order, LDS tile of the block's r_k) in both link formats: basis and
    two-pass forms, FP64 and mixed, three sources, against the oracle; on a
    lattice with a partial 256-site block and one with a partial 64-site
    layout tile.  The two forms run the same iterations (the same count)
    and differ only in the order in which they sum s."""
    monkeypatch.setenv("OVL_FUSED", "1")
    monkeypatch.setenv("OVL_ITER_VARIANT", str(variant))
    if links == "full":
        monkeypatch.setenv("OVL_LINKS", "full")
    fmt = 0 if links == "full" else 1
    for dims, seed in (((6, 6, 4, 6), 2), ((3, 5, 4, 6), 5)):
        U = gauge(dims, 0.3, seed)
        H = oracle_H(dims, 0.3, seed, 1.4)
        b = si.gaussian_sources(dims, 3, first_seed=9)
        z, c = nodes(16, *CIRCLE)
        from oracle.sign import sign_by_solves
        refs = [sign_by_solves(H, b[n].ravel(), z, c, method="gmres", processes=NPROC)
                for n in range(3)]
        for precision, tol in ((0, 1e-11), (1, 1e-10)):
            outs, iters = [], []
            for form in (2, 3):
                ctx = make_ctx(dims, U, nq=16, precision=precision, form=form)
                s, st = ctx.apply_sign(to_dev(b))
                assert st.stencil_variant64 == 1000 + variant + 8 * fmt
                for n in range(3):
                    assert_close(s[n].cpu().numpy(), refs[n], tol,
                                 f"fused v{variant} {links} {dims} p{precision} f{form} {n}")
                outs.append(s.cpu().numpy())
                iters.append((st.iterations, st.fp32_iterations))
                ctx.close()
            assert iters[0] == iters[1]
            # mixed: the basis form stores the iterate at the switch in FP32,
            # the two-pass form adds it in FP64 (a difference of ~eps32 * switch)
            assert relerr(outs[1], outs[0]) < (1e-13 if precision == 0 else 1e-11)


@pytest.mark.parametrize("fused", ["0", "1"])
def test_basis_iteration_kinds_match_the_oracle(fused, monkeypatch):
    """The basis form on the default two-kernel iteration and on the opt-in
    fused one (OVL_FUSED=1) against the oracle, FP64 and mixed; the stats
    name which iteration ran."""
    monkeypatch.setenv("OVL_FUSED", fused)
    c = CFG0
    U = gauge(c["dims"], c["r"], c["seed"])
    b = si.gaussian_sources(c["dims"], 1)[0]
    ref = oracle_sign(c["dims"], c["r"], c["seed"], c["m0"], c["nq"], CIRCLE, 1000)
    for precision, tol in ((0, 1e-11), (1, 1e-10)):
        ctx = make_ctx(c["dims"], U, c["m0"], c["mq"], c["nq"], precision=precision, form=2)
        s, st = ctx.apply_sign(to_dev(b))
        assert (st.stencil_variant64 >= 1000) == (fused == "1")
        assert_close(s.cpu().numpy(), ref, tol, f"fused={fused} basis p{precision}")
        ctx.close()


@pytest.fixture(scope="module")
def eig_4x4():
    """Dense eigendecomposition of the 4^4 parity field's H_W (3072 x 3072)."""
    from oracle.sign import eigh_dense
    c = CFG0
    return eigh_dense(oracle_H(c["dims"], c["r"], c["seed"], c["m0"]))


@pytest.mark.parametrize("precision,form,nq", [(0, 2, 1024), (1, 2, 1024), (0, 3, 1024),
                                               (0, 1, 512), (1, 1, 512)])
def test_maximum_shift_counts_against_the_oracle(precision, form, nq, eig_4x4):
    """The largest node sets the library takes: 2 x 1024 = 2048 shifts (eight
    256-shift slices) in the basis and two-pass forms, 2 x 512 = 1024 in the
    sweep form, whose per-shift directions are limited to that.  The 4^4
    field (roughness 0.3) and two sources against the oracle's dense
    eigendecomposition route, s = V F(lam) V^dag b with the same nodes and
    weights, element by element."""
    from oracle.sign import sign_by_eigh
    c = CFG0
    U = gauge(c["dims"], c["r"], c["seed"])
    b = si.gaussian_sources(c["dims"], 2, first_seed=61)
    ctx = make_ctx(c["dims"], U, c["m0"], c["mq"], nq, precision=precision, form=form,
                   tol=1e-13 if precision == 0 else 1e-12)
    s, st = ctx.apply_sign(to_dev(b))
    assert st.n_shifts == 2 * nq and st.n_active_end == 0
    z, w = nodes(nq, *CIRCLE)
    H = oracle_H(c["dims"], c["r"], c["seed"], c["m0"])
    tol = 1e-11 if precision == 0 else 1e-10
    for i in range(2):
        ref, _ = sign_by_eigh(H, b[i].ravel(), z, w, eig=eig_4x4)
        assert_close(s[i].cpu().numpy(), ref, tol, f"{2 * nq} shifts, form {form}, prec {precision}")
    ctx.close()
