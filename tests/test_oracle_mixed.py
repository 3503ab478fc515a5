"""Pins of the oracle's reduced-precision preconditioner (the MIXED mode).

The mixed mode rounds the V-cycle's coefficients (links to bfloat16, 27-point
Galerkin stencils to FP32) and the V-cycle's input, output and the CG search
direction to FP32, and keeps the outer CG in FP64.  The references here do not
use the oracle's rounding code: bfloat16 rounding is checked against exact
rational arithmetic, FP32 rounding is numpy's, and the V-cycle against a dense
composition from the rounded matrices.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_1604_07163_amd import inputs
from tests import manufactured as mf
from tests.test_oracle_pins import a27_to_dense, rand_k, rand_vec

DEG = 2


def bf16_exact(v):
    """Nearest value with 8 significant bits, ties to the even last bit, by exact
    rational arithmetic."""
    if v == 0.0:
        return 0.0
    a = Fraction(abs(v))
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    ulp = Fraction(2) ** (e - 7)  # 2^e <= a < 2^(e+1): 8 bits from 2^e down to 2^(e-7)
    q = a / ulp
    lo = q.numerator // q.denominator
    rem = q - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    return math.copysign(float(lo * ulp), v)


def bf16_array(a):
    return np.vectorize(bf16_exact, otypes=[np.float64])(a)


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def test_bf16_rounding_is_nearest_even(oracle_mod):
    g = np.random.default_rng(7)
    vals = [np.exp(g.uniform(np.log(1e-6), np.log(1e6), 4000))]
    # exact midpoints between neighbouring bfloat16 values, both parities
    m = np.arange(128, 256, dtype=np.float64)
    for e in (-20, -3, 0, 1, 9, 30):
        vals.append((m + 0.5) * 2.0 ** (e - 7))
        vals.append(np.nextafter((m + 0.5) * 2.0 ** (e - 7), 0.0))
        vals.append(np.nextafter((m + 0.5) * 2.0 ** (e - 7), np.inf))
    vals.append(np.array([1000.0, 1.0, 2.0 ** -126, 255.5, 255.75, 1.0 / 3.0, np.pi]))
    v = np.concatenate(vals)
    v = np.concatenate([v, -v[:200]])
    got = oracle_mod.round_bf16(v)
    ref = bf16_array(v)
    np.testing.assert_array_equal(got, ref)
    # 1000 = 1111101000b needs 7 significant bits: the inclusion contrast is exact
    assert oracle_mod.round_bf16(np.array([1000.0]))[0] == 1000.0


def test_mixed_level_operators_use_rounded_coefficients(oracle_mod):
    n, levels = 17, 4
    k = inputs.lognormal_k(n, 21, width=3.0)
    H = oracle_mod.Hierarchy(*k, levels=levels)
    Hm = oracle_mod.Hierarchy(*k, levels=levels, precision="mixed")
    for l in range(levels):
        nl = H.level_n(l)
        kl = H.level_k(l)
        np.testing.assert_array_equal(Hm.level_k(l)[0], kl[0])  # the FP64 hierarchy is unchanged
        kr = [bf16_array(a) for a in kl]
        u, b = rand_vec(nl, 30 + l), rand_vec(nl, 40 + l)
        np.testing.assert_array_equal(Hm.apply(l, u), oracle_mod.apply(*kr, u))
        np.testing.assert_array_equal(H.apply(l, u), oracle_mod.apply(*kl, u))
        if l + 1 < levels:
            np.testing.assert_array_equal(Hm.smooth(l, b), oracle_mod.cheb(*kr, b))
            np.testing.assert_array_equal(Hm.smooth(l, b, u), oracle_mod.cheb(*kr, b, x0=u))
    # Galerkin levels: the 27-point stencils rounded to FP32
    Hg = oracle_mod.Hierarchy(*k, levels=levels, galerkin=2, precision="mixed")
    for l in (2, 3):
        nl = Hg.level_n(l)
        u = rand_vec(nl, 50 + l)
        np.testing.assert_array_equal(Hg.apply(l, u), oracle_mod.apply27(f32(Hg.level_a27(l)), u))


def dense_mixed_vcycle(smooth_mats, coarse_mat, ns, intervals, m=DEG):
    """Dense V-cycle with given per-level smoothing/residual matrices and the
    coarsest matrix solved exactly: E = p(K)(I - P B_c R A)p(K), B = (I - E) A^-1."""
    L = len(ns)

    def B(l):
        if l == L - 1:
            return np.linalg.inv(coarse_mat)
        A = smooth_mats[l]
        P = mf.prolongation_matrix(ns[l])
        K = np.diag(1.0 / np.diag(A)) @ A
        pK = mf.cheb_poly_matrix(K, m, *intervals[l])
        I = np.eye(A.shape[0])
        E = pK @ (I - P @ B(l + 1) @ (P.T / 8.0) @ A) @ pK
        return (I - E) @ np.linalg.inv(A)
    return B(0)


@pytest.mark.parametrize("n,levels,galerkin", [(9, 2, 0), (9, 3, 0), (17, 3, 0), (17, 3, 1), (17, 4, 2)])
def test_mixed_vcycle_matches_dense_composition(oracle_mod, n, levels, galerkin):
    """z = fl32(B fl32(r)), B composed from the rounded level matrices, with the
    coarsest level solved with its FP64 matrix."""
    k = rand_k(n, 60 + n + levels + galerkin)
    H = oracle_mod.Hierarchy(*k, levels=levels, galerkin=galerkin)
    Hm = oracle_mod.Hierarchy(*k, levels=levels, galerkin=galerkin, precision="mixed")
    ns = [H.level_n(l) for l in range(levels)]

    def mat(l, rounded):
        if galerkin and l >= galerkin:
            a = H.level_a27(l)
            return a27_to_dense(f32(a) if rounded else a)
        kl = H.level_k(l)
        return mf.dense_from_links(*[bf16_array(a) for a in kl] if rounded else kl)

    Bd = dense_mixed_vcycle([mat(l, True) for l in range(levels - 1)], mat(levels - 1, False), ns,
                            [H.level_interval(l) for l in range(levels)])
    r = rand_vec(n, 13)
    ref = Bd @ mf.interior(f32(r))
    z = Hm.vcycle(r)
    zi = mf.interior(z)
    np.testing.assert_array_equal(z, f32(z))  # an FP32 result
    np.testing.assert_array_equal(Hm.vcycle(f32(r)), z)  # of an FP32 input
    assert np.all(z[~mf.interior_mask(n)] == 0)
    # FP32 output rounding (half an ulp, 2^-24 relative) on an FP64 result
    assert np.all(np.abs(zi - ref) <= 2.0 ** -24 * np.abs(ref) + 1e-11 * np.abs(ref).max())
    # the rounding of the coefficients is visible: not the FP64 V-cycle
    z64 = mf.interior(H.vcycle(r))
    assert np.abs(z64 - zi).max() > 1e-5 * np.abs(z64).max()


def test_mixed_pcg_reaches_dense_solution(oracle_mod):
    """The outer CG keeps the FP64 operator: the reduced-precision preconditioner
    changes the iterates, not the solution it converges to."""
    n, levels = 9, 3
    k = rand_k(n, 71)
    f = inputs.uniform_rhs(n, 72)
    Hm = oracle_mod.Hierarchy(*k, levels=levels, precision="mixed")
    x, info = Hm.solve(f, rtol=1e-13, max_it=100)
    ref = np.linalg.solve(mf.dense_from_links(*k), mf.interior(f))
    assert info["status"] == "OK" and info["rel_res_true"] <= 1e-13
    np.testing.assert_allclose(mf.interior(x), ref, rtol=1e-10, atol=1e-11 * np.abs(ref).max())


def update_ratio(x0, x1, p):
    """x1 - x0 over p where p is not small: one scalar (the CG step length)
    if p is the direction that moved x0 to x1."""
    d, pi = mf.interior(x1) - mf.interior(x0), mf.interior(p)
    big = np.abs(pi) > 1e-3 * np.abs(pi).max()
    ratio = d[big] / pi[big]
    mid = np.median(ratio)
    return mid, np.abs(ratio - mid).max() / abs(mid)


def test_mixed_search_direction_is_fp32(oracle_mod):
    """The mixed CG moves x along an FP32 search direction: the direction the
    oracle leaves after m iterations is the one that takes x_m to x_{m+1}
    (x_{m+1} - x_m is a scalar multiple of it, to FP64 roundoff), and every
    value of it is an FP32 number.  The FP64 solve's direction is not, so the
    check would see a direction left unrounded."""
    n, levels = 17, 3
    k = rand_k(n, 81)
    f = inputs.uniform_rhs(n, 82)
    Hm = oracle_mod.Hierarchy(*k, levels=levels, precision="mixed")
    H = oracle_mod.Hierarchy(*k, levels=levels)
    for m in (1, 2, 3):
        xm, info = Hm.solve(f, rtol=0.0, max_it=m)
        assert info["iterations"] == m and info["restarts"] == 0
        p = Hm.last_direction()
        np.testing.assert_array_equal(p, f32(p))
        assert np.abs(mf.interior(p)).max() > 0
        x_next, _ = Hm.solve(f, rtol=0.0, max_it=m + 1)
        alpha, spread = update_ratio(xm, x_next, p)
        assert alpha > 0 and spread <= 1e-9, (m, spread)
        x64, _ = H.solve(f, rtol=0.0, max_it=m)
        p64 = H.last_direction()
        x64_next, _ = H.solve(f, rtol=0.0, max_it=m + 1)
        assert update_ratio(x64, x64_next, p64)[1] <= 1e-9
        assert not np.array_equal(p64, f32(p64))


@pytest.mark.parametrize("n,levels", [(33, 5), (65, 6)])
def test_mixed_pcg_iterations_match_fp64(oracle_mod, n, levels):
    """With coefficients that bfloat16 holds exactly on every level (constant k)
    only the FP32 roundings of r, z and p remain: the iteration count stays
    within one of the FP64 solve, and both reach the FP64 tolerance."""
    k = inputs.const_k(n, 3.0)
    f = inputs.uniform_rhs(n, 5)
    H = oracle_mod.Hierarchy(*k, levels=levels)
    Hm = oracle_mod.Hierarchy(*k, levels=levels, precision="mixed")
    for l in range(levels):
        for a in Hm.level_k(l):
            np.testing.assert_array_equal(oracle_mod.round_bf16(a), a)
    x, i64 = H.solve(f, rtol=1e-8)
    xm, imx = Hm.solve(f, rtol=1e-8)
    assert i64["status"] == "OK" and imx["status"] == "OK"
    assert abs(i64["iterations"] - imx["iterations"]) <= 1
    assert imx["rel_res_true"] <= 1e-8 and imx["restarts"] == 0
    assert np.linalg.norm(x - xm) <= 1e-7 * np.linalg.norm(x)


def test_mixed_rejects_links_outside_bf16_range(oracle_mod):
    n = 9
    kx, ky, kz = inputs.const_k(n)
    kx = kx.copy()
    kx[4, 4, 3] = 1e-40  # positive and normal in FP64, below the bfloat16 normal range
    oracle_mod.Hierarchy(kx, ky, kz, levels=2)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.Hierarchy(kx, ky, kz, levels=2, precision="mixed")
