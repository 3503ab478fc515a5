"""Galerkin coarse operators on the GPU (R A P, 27 coefficients per vertex)
against the FP64 CPU oracle, through the C ABI.

Covers Galerkin throughout (first Galerkin level 1) and the hybrid
construction (re-discretized links above level g, R A P from g on), the
stencil itself, every level operation on a Galerkin level, the V-cycle, full
solves, the mixed-precision path and the truncated hierarchy with its inexact
coarse CG.  Sizes span several x and y tiles with ragged last tiles.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1604_07163_amd import gmg, inputs
from tests.gpu_util import rand_vec, rel_l2, rel_max, say, to_gpu, to_np

pytestmark = pytest.mark.gpu

CASES = [(17, 3, 1), (33, 4, 1), (81, 4, 2), (161, 5, 1), (161, 5, 3)]


def make(n, levels, galerkin, seed=2, precision="fp64", **kw):
    k = inputs.lognormal_k(n, seed, width=3.0)
    say(f"  case n={n} levels={levels} galerkin={galerkin} precision={precision} {kw}")
    s = gmg.Solver(*[to_gpu(a) for a in k], levels=levels, precision=precision, galerkin=galerkin, **kw)
    H = oracle.Hierarchy(*k, levels=levels, galerkin=galerkin)
    return k, s, H


@pytest.mark.parametrize("n,levels,g", CASES)
def test_galerkin_stencils(n, levels, g):
    k, s, H = make(n, levels, g)
    for l in range(1, levels):
        if l < g:
            with pytest.raises(gmg.GmgError):
                s.level_stencil(l)
            continue
        got, ref = to_np(s.level_stencil(l)), H.level_a27(l)
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-13 * scale, (l, np.abs(got - ref).max() / scale)
        assert np.all(got[0] == 0) and np.all(got[:, :, -1] == 0)
    with pytest.raises(gmg.GmgError):
        s.level_stencil(0)


@pytest.mark.parametrize("n,levels,g", CASES)
def test_galerkin_chebyshev_intervals(n, levels, g):
    """The Lanczos-estimated interval of every smoothed Galerkin level equals the
    oracle's (independent FP64 sums in another order); other levels keep the
    option interval."""
    k, s, H = make(n, levels, g)
    for l in range(levels):
        lo, hi = s.level_interval(l)
        lo_o, hi_o = H.level_interval(l)
        assert abs(hi - hi_o) <= 1e-12 * hi_o and abs(lo - lo_o) <= 1e-12 * hi_o, (l, lo, hi, lo_o, hi_o)
        if not (g <= l < levels - 1):
            assert (lo, hi) == (0.25, 2.0)


@pytest.mark.parametrize("n,levels,g", CASES)
def test_galerkin_level_operations(n, levels, g):
    k, s, H = make(n, levels, g)
    for l in range(max(g, 1), levels - 1):
        nl = H.level_n(l)
        b, x0 = rand_vec(nl, 10 + l), rand_vec(nl, 20 + l)
        assert rel_max(to_np(s.apply_operator(l, to_gpu(x0))), H.apply(l, x0)) <= 1e-13
        assert rel_max(to_np(s.smooth(l, to_gpu(b))), H.smooth(l, b)) <= 1e-12
        assert rel_max(to_np(s.smooth(l, to_gpu(b), to_gpu(x0))), H.smooth(l, b, x0)) <= 1e-12
        ref = oracle.restrict(b - H.apply(l, x0))
        assert rel_max(to_np(s.residual_restrict(l, to_gpu(b), to_gpu(x0))), ref) <= 1e-12
    nc = H.level_n(levels - 1)
    b = rand_vec(nc, 5)
    assert rel_max(to_np(s.coarse_solve(to_gpu(b))), H.coarse_solve(b)) <= 1e-11


@pytest.mark.parametrize("n,levels,g", CASES)
def test_galerkin_vcycle(n, levels, g):
    k, s, H = make(n, levels, g)
    r = rand_vec(n, 7)
    assert rel_max(to_np(s.vcycle(to_gpu(r))), H.vcycle(r)) <= 1e-10


@pytest.mark.parametrize("g", [1, 2])
def test_galerkin_solve_inclusions(g):
    n, levels = 65, 5
    kx, ky, kz, _ = inputs.inclusion_k(n, 4)
    f = inputs.uniform_rhs(n, 5)
    H = oracle.Hierarchy(kx, ky, kz, levels=levels, galerkin=g)
    xo, io = H.solve(f, rtol=1e-8, max_it=400)
    s = gmg.Solver(*[to_gpu(a) for a in (kx, ky, kz)], levels=levels, galerkin=g)
    fg = to_gpu(f)
    xg, ig = s.solve(fg, rtol=1e-8, max_it=400)
    say(f"    galerkin={g}: its gpu {ig['iterations']} oracle {io['iterations']}, true {ig['rel_res_true']:.2e}")
    assert ig["status"] == "GMG_OK" and abs(ig["iterations"] - io["iterations"]) <= 1
    assert ig["rel_res_true"] <= 1e-8
    xf, _ = s.solve(fg, rtol=0.0, max_it=io["iterations"])
    assert rel_l2(to_np(xf), xo) <= 1e-10
    # mixed precision: FP32 27-point levels, converges to the same tolerance
    sm = gmg.Solver(*[to_gpu(a) for a in (kx, ky, kz)], levels=levels, galerkin=g, precision="mixed")
    xm, im = sm.solve(fg, rtol=1e-8, max_it=400)
    say(f"    mixed: its {im['iterations']} restarts {im['restarts']} true {im['rel_res_true']:.2e}")
    assert im["status"] == "GMG_OK" and im["rel_res_true"] <= 1e-8
    assert im["iterations"] <= io["iterations"] + 2 + io["iterations"] // 10
    assert rel_l2(to_np(xm), xo) <= 1e-6


def test_galerkin_truncated_flexible():
    """Galerkin levels with the truncation arm: inexact Jacobi-CG on a large
    27-point coarsest level and flexible outer CG."""
    n, levels = 65, 3
    kx, ky, kz, _ = inputs.inclusion_k(n, 4)
    f = inputs.uniform_rhs(n, 5)
    H = oracle.Hierarchy(kx, ky, kz, levels=levels, galerkin=1, coarse_solver=1, coarse_rtol=1e-4,
                         coarse_max_it=500)
    xo, io = H.solve(f, rtol=1e-8, max_it=500, flexible=True)
    s = gmg.Solver(*[to_gpu(a) for a in (kx, ky, kz)], levels=levels, galerkin=1, coarse_solver="cg",
                   coarse_rtol=1e-4, coarse_max_it=500, flexible=True)
    fg = to_gpu(f)
    xg, ig = s.solve(fg, rtol=1e-8, max_it=500)
    say(f"    its gpu {ig['iterations']} oracle {io['iterations']}; coarse its gpu {ig['coarse_iterations']} "
        f"oracle {io['coarse_iterations']}")
    assert ig["status"] == "GMG_OK" and abs(ig["iterations"] - io["iterations"]) <= 1
    xf, _ = s.solve(fg, rtol=0.0, max_it=io["iterations"])
    assert rel_l2(to_np(xf), xo) <= 1e-10
    b = rand_vec(H.level_n(levels - 1), 7)
    assert rel_max(to_np(s.coarse_solve(to_gpu(b))), H.coarse_solve(b)) <= 1e-10


@pytest.mark.parametrize("g", [1, 3])
def test_galerkin_agglomerated_levels_identical(g):
    """Galerkin levels inside the persistent kernel (one workgroup, a team of 4,
    a team with a second switch level) give the grid path's iterates: the
    27-point row sum, the fused residual-restriction and the Chebyshev steps
    round in the same order on both paths."""
    n, levels = 129, 6
    kx, ky, kz, _ = inputs.inclusion_k(n, 4)
    kg = [to_gpu(a) for a in (kx, ky, kz)]
    f = to_gpu(inputs.uniform_rhs(n, 5))
    base = gmg.Solver(*kg, levels=levels, galerkin=g)
    x0, i0 = base.solve(f, rtol=1e-8, max_it=400)
    r = to_gpu(rand_vec(n, 3))
    z0 = base.vcycle(r)
    H = oracle.Hierarchy(kx, ky, kz, levels=levels, galerkin=g)
    assert rel_max(to_np(z0), H.vcycle(to_np(r))) <= 1e-10
    for kw in (dict(switch_n=17), dict(switch_n=33, persistent_wgs=4), dict(switch_n=33, persistent_wgs=4,
                                                                             switch2_n=9)):
        s = gmg.Solver(*kg, levels=levels, galerkin=g, **kw)
        z = s.vcycle(r)
        assert float((z - z0).abs().max()) <= 1e-14 * float(z0.abs().max()), kw
        x, info = s.solve(f, rtol=1e-8, max_it=400)
        say(f"    galerkin={g} {kw}: its {info['iterations']} (grid path {i0['iterations']})")
        assert info["iterations"] == i0["iterations"]
        assert float((x - x0).abs().max()) <= 1e-13 * float(x0.abs().max())
        s.close()
