"""gmg_solve_static (no allocation: the hierarchy in the library's static
device workspace) against gmg_create + gmg_solve on the same inputs, on two
calls in a row, the second with a smaller grid, plus the size limit."""
import numpy as np
import pytest
import torch

from paper_1604_07163_amd import gmg, inputs
from tests.gpu_util import say, to_gpu

pytestmark = pytest.mark.gpu

CASES = [  # (grid, levels, precision, switch level, k, f): the second call is smaller
    (65, 6, "mixed", 9, lambda n: inputs.lognormal_k(n, 2), lambda n: inputs.uniform_rhs(n, 3)),
    (33, 4, "fp64", 17, lambda n: inputs.const_k(n), lambda n: inputs.sine_rhs(n)),
]


def test_static_workspace_solve_equals_gmg_solve():
    for n, levels, prec, sw, kfun, ffun in CASES:
        k = [to_gpu(a) for a in kfun(n)]
        f = to_gpu(ffun(n))
        s = gmg.Solver(*k, levels=levels, precision=prec, switch_n=sw)
        xr, ir = s.solve(f, rtol=1e-8)
        s.close()
        xs, is_ = gmg.solve_static(*k, f, levels=levels, precision=prec, switch_n=sw, rtol=1e-8)
        d = float((xs - xr).abs().max())
        say(f"  {n}^3 {prec}: gmg_solve its {ir['iterations']}, static its {is_['iterations']}, max |diff| {d:.3e}")
        assert is_["status"] == "GMG_OK" and ir["status"] == "GMG_OK"
        assert is_["iterations"] == ir["iterations"] and is_["restarts"] == ir["restarts"]
        assert is_["rel_res_true"] <= 1e-8
        # same kernels, launch shapes and reduction order: the same iterates
        assert d == 0.0


def test_static_workspace_rejects_a_grid_that_does_not_fit():
    n = 129
    k = [to_gpu(a) for a in inputs.const_k(n)]
    f = to_gpu(inputs.uniform_rhs(n, 1))
    with pytest.raises(gmg.GmgError) as e:
        gmg.solve_static(*k, f)
    assert e.value.status == 2 and "static workspace" in str(e.value)
    # and a following call that fits still works
    n = 17
    k = [to_gpu(a) for a in inputs.const_k(n)]
    f = to_gpu(inputs.uniform_rhs(n, 1))
    x, info = gmg.solve_static(*k, f, rtol=1e-10)
    assert info["status"] == "GMG_OK" and info["rel_res_true"] <= 1e-10
