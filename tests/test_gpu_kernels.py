"""Kernel-level parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Sizes span several x tiles (64 wide) and y tiles (4 rows), ragged last tiles
(N = 81, 161) and the small levels that the persistent kernel handles.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1604_07163_amd import gmg, inputs
from tests.gpu_util import bf16_rne, rand_vec, rel_max, say, to_gpu, to_np

pytestmark = pytest.mark.gpu

CASES = [(17, 4), (33, 5), (81, 5), (161, 6)]


def make(n, levels, seed=2, precision="fp64", **kw):
    k = inputs.lognormal_k(n, seed, width=3.0)
    say(f"  case n={n} levels={levels} precision={precision} {kw}")
    s = gmg.Solver(*[to_gpu(a) for a in k], levels=levels, precision=precision, **kw)
    H = oracle.Hierarchy(*k, levels=levels)
    return k, s, H


@pytest.mark.parametrize("n,levels", CASES)
def test_apply_fp64(n, levels):
    k, s, H = make(n, levels)
    u = rand_vec(n, 1)
    ref = oracle.apply(*k, u)
    for use64 in (True, False):
        got = to_np(s.apply_operator(0, to_gpu(u), use_fp64=use64))
        assert rel_max(got, ref) <= 1e-14, (use64, rel_max(got, ref))
        assert np.all(got[0] == 0) and np.all(got[:, :, -1] == 0)


def active_masks(n):
    """Links with at least one interior end point: transverse indices interior."""
    sx, sy, sz = inputs.face_shapes(n)
    mx, my, mz = np.zeros(sx, bool), np.zeros(sy, bool), np.zeros(sz, bool)
    mx[1:-1, 1:-1, :] = True
    my[1:-1, :, 1:-1] = True
    mz[:, 1:-1, 1:-1] = True
    return mx, my, mz


@pytest.mark.parametrize("n,levels", CASES)
def test_coarse_coefficients_bitwise(n, levels):
    k, s, H = make(n, levels)
    for l in range(levels):
        g = [to_np(t) for t in s.level_coefficients(l)]
        o = H.level_k(l)
        for a, b, m in zip(g, o, active_masks(H.level_n(l))):
            np.testing.assert_array_equal(a[m], b[m])
            assert np.all(a[~m] == 0)


@pytest.mark.parametrize("n,levels", CASES)
def test_level_operations_fp64(n, levels):
    k, s, H = make(n, levels)
    for l in range(levels - 1):
        nl = H.level_n(l)
        kl = H.level_k(l)
        b, x0 = rand_vec(nl, 10 + l), rand_vec(nl, 20 + l)
        # operator on level l
        got = to_np(s.apply_operator(l, to_gpu(x0)))
        assert rel_max(got, oracle.apply(*kl, x0)) <= 1e-14
        # smoothing from zero and from x0
        assert rel_max(to_np(s.smooth(l, to_gpu(b))), H.smooth(l, b)) <= 1e-13
        assert rel_max(to_np(s.smooth(l, to_gpu(b), to_gpu(x0))), H.smooth(l, b, x0)) <= 1e-13
        # residual + full weighting
        ref = oracle.restrict(b - H.apply(l, x0))
        assert rel_max(to_np(s.residual_restrict(l, to_gpu(b), to_gpu(x0))), ref) <= 1e-13
        # trilinear prolongation + correction
        e = rand_vec(H.level_n(l + 1), 30 + l)
        assert rel_max(to_np(s.prolong(l, to_gpu(e), to_gpu(x0))), oracle.prolong_add(e, x0)) <= 1e-15


@pytest.mark.parametrize("n,levels", [(17, 3), (33, 4), (81, 4), (161, 5), (33, 2)])
def test_coarsest_cholesky(n, levels):
    """The coarsest solve by the device-built Cholesky factor against the
    oracle's dense solve; (33, 2) has a 17^3 coarsest level, 3375 unknowns."""
    k, s, H = make(n, levels)
    nc = H.level_n(levels - 1)
    b = rand_vec(nc, 5)
    assert rel_max(to_np(s.coarse_solve(to_gpu(b))), H.coarse_solve(b)) <= 1e-12


@pytest.mark.parametrize("n,levels", CASES)
def test_vcycle_and_switch_invariance(n, levels):
    k, s, H = make(n, levels)
    r = rand_vec(n, 3)
    ref = H.vcycle(r)
    base = to_np(s.vcycle(to_gpu(r)))
    assert rel_max(base, ref) <= 1e-12, rel_max(base, ref)
    sizes = sorted({H.level_n(l) for l in range(1, levels)})
    for sw in sizes:
        for wgs, lds in ((1, True), (1, False), (4, True), (8, True)):
            sp = gmg.Solver(*[to_gpu(a) for a in k], levels=levels, switch_n=sw, persistent_wgs=wgs,
                            persistent_lds=lds)
            z = to_np(sp.vcycle(to_gpu(r)))
            d = rel_max(z, base)
            say(f"    switch {sw} team {wgs} lds {sp.persistent_lds_bytes}: max rel diff vs grid path {d:.3e} "
                f"(bitwise: {np.array_equal(z, base)})")
            assert np.array_equal(z, base)
            if wgs > 1 or not lds:
                assert sp.persistent_lds_bytes == 0
            elif sw <= 9:  # levels 9^3 and below always fit in 64 KiB of LDS
                assert sp.persistent_lds_bytes > 0
            sp.close()
    # multi-stage: a team on the middle levels, one workgroup below switch2
    if len(sizes) >= 3:
        sp = gmg.Solver(*[to_gpu(a) for a in k], levels=levels, switch_n=sizes[-1], persistent_wgs=4,
                        switch2_n=sizes[1])
        z = to_np(sp.vcycle(to_gpu(r)))
        say(f"    multi-stage switch {sizes[-1]} -> team 4 -> {sizes[1]} -> 1 wg: bitwise {np.array_equal(z, base)}")
        assert np.array_equal(z, base)


def test_bf16_coefficients_round_to_nearest_even():
    n, levels = 33, 5
    k, s, H = make(n, levels, precision="mixed")
    for l in range(levels):
        g = [to_np(t) for t in s.level_coefficients(l)]
        o = H.level_k(l)
        for a, b, m in zip(g, o, active_masks(H.level_n(l))):
            np.testing.assert_array_equal(a[m], bf16_rne(b[m]))


@pytest.mark.parametrize("n,levels", [(33, 5), (81, 5)])
def test_mixed_level_operations(n, levels):
    """FP32 arithmetic with BF16 links vs the FP64 oracle fed the same BF16 links."""
    k, s, H = make(n, levels, precision="mixed")
    for l in range(levels - 1):
        nl = H.level_n(l)
        kl = [to_np(t) for t in s.level_coefficients(l)]
        b = rand_vec(nl, 40 + l).astype(np.float32).astype(np.float64)
        x0 = rand_vec(nl, 50 + l).astype(np.float32).astype(np.float64)
        assert rel_max(to_np(s.apply_operator(l, to_gpu(x0))), oracle.apply(*kl, x0)) <= 2e-6
        ref = oracle.cheb(*kl, b, x0=x0)
        assert rel_max(to_np(s.smooth(l, to_gpu(b), to_gpu(x0))), ref) <= 2e-6
        ref = oracle.restrict(b - oracle.apply(*kl, x0))
        assert rel_max(to_np(s.residual_restrict(l, to_gpu(b), to_gpu(x0))), ref) <= 2e-6


@pytest.mark.parametrize("n,levels", [(17, 4), (33, 5), (81, 5), (161, 6), (257, 5)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pre_smoothing_and_residual_one_sweep_bitwise(n, levels, precision, monkeypatch):
    """Pre-smoothing and the residual's z-sums in one sweep (x1 and x2 kept in
    LDS) give the V-cycle of the separate sweeps to the bit, with and without
    agglomerated coarse levels, and the same solve."""
    k = inputs.lognormal_k(n, 9, width=3.0)
    kg = [to_gpu(a) for a in k]
    for sw in (0, 9):
        say(f"  pre-smoothing + residual n={n} levels={levels} {precision} switch={sw}")
        sf = gmg.Solver(*kg, levels=levels, precision=precision, switch_n=sw)
        monkeypatch.setenv("GMG_PRE_FUSED", "0")
        su = gmg.Solver(*kg, levels=levels, precision=precision, switch_n=sw)
        monkeypatch.delenv("GMG_PRE_FUSED")
        r = to_gpu(rand_vec(n, 15))
        zf, zu = to_np(sf.vcycle(r)), to_np(su.vcycle(r))
        say(f"    V-cycle bitwise {np.array_equal(zf, zu)}")
        np.testing.assert_array_equal(zf, zu)
        f = to_gpu(inputs.uniform_rhs(n, 16))
        xf, i_f = sf.solve(f, rtol=1e-10)
        xu, i_u = su.solve(f, rtol=1e-10)
        assert i_f["iterations"] == i_u["iterations"] and torch.equal(xf, xu)
        sf.close()
        su.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_one_sweep_kernels_independent_of_chunk_length(precision, monkeypatch):
    """The one-sweep kernels recompute x1 (and x2) on the halo planes of each
    z-chunk, so their results must not depend on where the chunks start: odd
    and even post-smoothing chunks and short pre-smoothing chunks give the
    default chunks' V-cycle to the bit, and the solve (whose r.z partial sums
    are grouped by chunk) to FP64 rounding."""
    n, levels = 257, 5
    k = inputs.lognormal_k(n, 13, width=3.0)
    kg = [to_gpu(a) for a in k]
    r = to_gpu(rand_vec(n, 17))
    f = to_gpu(inputs.uniform_rhs(n, 18))
    s0 = gmg.Solver(*kg, levels=levels, precision=precision, switch_n=9)
    z0 = to_np(s0.vcycle(r))
    x0, i0 = s0.solve(f, rtol=1e-10)
    x0 = to_np(x0)
    s0.close()
    for post, pre in ((5, 6), (7, 10), (13, 2)):
        say(f"  chunks n={n} {precision} post={post} pre={pre}")
        monkeypatch.setenv("GMG_POST_CHUNK", str(post))
        monkeypatch.setenv("GMG_PRE_CHUNK", str(pre))
        s = gmg.Solver(*kg, levels=levels, precision=precision, switch_n=9)
        monkeypatch.delenv("GMG_POST_CHUNK")
        monkeypatch.delenv("GMG_PRE_CHUNK")
        np.testing.assert_array_equal(to_np(s.vcycle(r)), z0)
        x, i = s.solve(f, rtol=1e-10)
        d = rel_max(to_np(x), x0)
        say(f"    V-cycle bitwise; solve its {i['iterations']} / {i0['iterations']}, max rel diff {d:.1e}")
        assert i["iterations"] == i0["iterations"] and d <= 1e-12
        s.close()


def test_bad_coefficients_after_set_are_reported_by_the_next_solve():
    """gmg_set_coefficients enqueues its checks without waiting; the next solve
    (and every one after it) returns GMG_ERR_COEFF until valid coefficients
    are set again."""
    n = 17
    k = inputs.const_k(n)
    kg = [to_gpu(a) for a in k]
    f = to_gpu(inputs.uniform_rhs(n, 1))
    s = gmg.Solver(*kg, levels=3)
    bad = kg[1].clone()
    bad[5, 3, 7] = 0.0
    s.set_coefficients(kg[0], bad, kg[2])  # returns: nothing checked yet on the host
    for _ in range(2):
        with pytest.raises(gmg.GmgError) as e:
            s.solve(f)
        assert e.value.status == 3
    s.set_coefficients(*kg)
    x, info = s.solve(f, rtol=1e-10)
    assert info["status"] == "GMG_OK" and info["rel_res_true"] <= 1e-10


def test_errors_are_reported():
    n = 17
    k = inputs.const_k(n)
    kg = [to_gpu(a) for a in k]
    o = gmg.Options()
    gmg.lib().gmg_default_options(o, n)
    o.levels = 6  # 16 not divisible by 32
    st, h = gmg.raw_create(o, *kg)
    assert st == 2 and not h.value
    o.levels = 3
    bad = k[0].copy()
    bad[4, 4, 4] = -1.0
    st, h = gmg.raw_create(o, to_gpu(bad), kg[1], kg[2])
    assert st == 3
    bad[4, 4, 4] = np.nan
    st, h = gmg.raw_create(o, to_gpu(bad), kg[1], kg[2])
    assert st == 3
    s = gmg.Solver(*kg, levels=3)
    x, info = s.solve(to_gpu(inputs.uniform_rhs(n, 1)), rtol=1e-12, max_it=1)
    assert info["status"] == "GMG_ERR_NOT_CONVERGED" and info["iterations"] == 1
    x, info = s.solve(torch.zeros((n, n, n), dtype=torch.float64, device="cuda"))
    assert info["status"] == "GMG_OK" and info["iterations"] == 0 and float(x.abs().max()) == 0.0
    with pytest.raises(gmg.GmgError):
        s.solve(to_gpu(np.full((n, n, n), np.nan)))


@pytest.mark.parametrize("n,levels", [(33, 5), (129, 7)])
def test_mixed_persistent_lds_identical(n, levels):
    """MIXED V-cycle: the agglomerated levels in LDS, in HBM/L2 and on the grid
    path give bitwise the same z; and the PCG iterates agree."""
    k, s, H = make(n, levels, precision="mixed")
    r = rand_vec(n, 4)
    base = to_np(s.vcycle(to_gpu(r)))
    f = to_gpu(inputs.uniform_rhs(n, 6))
    xb, ib = s.solve(f, rtol=1e-8)
    for sw in (9, 17):
        for lds in (True, False):
            sp = gmg.Solver(*[to_gpu(a) for a in k], levels=levels, precision="mixed", switch_n=sw,
                            persistent_lds=lds)
            z = to_np(sp.vcycle(to_gpu(r)))
            say(f"    mixed switch {sw} lds bytes {sp.persistent_lds_bytes}: bitwise {np.array_equal(z, base)}")
            assert np.array_equal(z, base)
            x, info = sp.solve(f, rtol=1e-8)
            assert info["iterations"] == ib["iterations"] and torch.equal(x, xb)
            sp.close()


@pytest.mark.parametrize("n,levels", [(17, 4), (33, 5), (81, 5), (161, 6)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_post_smoothing_one_sweep_bitwise(n, levels, precision):
    """The one-sweep post-smoothing (first Chebyshev iterate kept in LDS) gives
    the two-sweep values to the bit: the smoother hook on every grid level and
    whole V-cycles, with and without agglomerated coarse levels."""
    k = inputs.lognormal_k(n, 7, width=3.0)
    kg = [to_gpu(a) for a in k]
    for sw in (0, 9):
        say(f"  post-smoothing n={n} levels={levels} {precision} switch={sw}")
        sf = gmg.Solver(*kg, levels=levels, precision=precision, switch_n=sw, post_fused=True)
        su = gmg.Solver(*kg, levels=levels, precision=precision, switch_n=sw, post_fused=False)
        for l in range(levels - 1):
            nl = sf.level_n(l)
            b, x0 = to_gpu(rand_vec(nl, 60 + l)), to_gpu(rand_vec(nl, 70 + l))
            np.testing.assert_array_equal(to_np(sf.smooth(l, b, x0)), to_np(su.smooth(l, b, x0)))
        r = to_gpu(rand_vec(n, 5))
        zf, zu = to_np(sf.vcycle(r)), to_np(su.vcycle(r))
        say(f"    V-cycle bitwise {np.array_equal(zf, zu)}")
        np.testing.assert_array_equal(zf, zu)
        f = to_gpu(inputs.uniform_rhs(n, 8))
        xf, i_f = sf.solve(f, rtol=1e-10)
        xu, i_u = su.solve(f, rtol=1e-10)
        d = rel_max(to_np(xf), to_np(xu))
        say(f"    solve its {i_f['iterations']} / {i_u['iterations']}, max rel diff {d:.1e}")
        # the r.z partial sums are grouped by different tiles: FP64 rounding only
        assert i_f["iterations"] == i_u["iterations"] and d <= 1e-12
        sf.close()
        su.close()
