"""GPU checks of the mixed-precision path (FP32 state, reconstruction passes
and streaming; FP64 Newton solve and polishing update): L1 errors of density,
velocity and temperature against the FP64 results within the 1e-4 relative
budget, and conservation to FP32 rounding."""
import numpy as np
import pytest

import lelbm_inputs as li
from helpers import gpu_moments, primitives, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

BUDGET = 1e-4


def l1_errors(a, b, dim, K):
    """Relative L1 errors of rho, |u| and RT of state a against reference b:
    sum|x_a - x_b| / sum|x_b| (velocity as the vector norm of the difference
    over the sum of |u_b|)."""
    ra, uxa, uya, ta = primitives(a, dim, K)
    rb, uxb, uyb, tb = primitives(b, dim, K)
    e_rho = np.abs(ra - rb).sum() / np.abs(rb).sum()
    e_u = np.hypot(uxa - uxb, uya - uyb).sum() / np.hypot(uxb, uyb).sum()
    e_t = np.abs(ta - tb).sum() / np.abs(tb).sum()
    return e_rho, e_u, e_t


def _case(name):
    print("\n[gpu case] %s" % name, flush=True)


def test_mixed_vs_oracle_riemann1d():
    _case("mixed riemann1d seed 0 n=2000 200 steps")
    cfg, prim = li.riemann1d(0, n=2000)
    a, sa = run_gpu(cfg, prim, 200, precision=1)
    b, sb = run_oracle(cfg, prim, 200)
    errs = l1_errors(a, b, 1, cfg["K"])
    print("L1 rho/u/T", errs, "it", sa["it_mean_f"], sa["it_max_f"])
    assert max(errs) < BUDGET


@pytest.mark.parametrize("seed", [2, 4])
def test_mixed_vs_oracle_quadrants(seed):
    _case("mixed quadrants seed %d 72x56 100 steps" % seed)
    cfg, prim = li.quadrants(seed, n=72, ny=56)
    a, sa = run_gpu(cfg, prim, 100, precision=1)
    b, sb = run_oracle(cfg, prim, 100)
    errs = l1_errors(a, b, 2, cfg["K"])
    print("L1 rho/u/T", errs, "it", sa["it_mean_f"], sa["it_max_f"])
    assert max(errs) < BUDGET
    assert sa["q_max"] == sb["q_max"]


def test_mixed_conservation():
    _case("mixed conservation quadrants seed 4 64x64")
    import paper_2508_06911_amd as lb
    cfg, prim = li.quadrants(4, n=64)
    m = gpu_moments(cfg, prim)
    c = lb.Lelbm(cfg, m, precision=lb.MIXED)
    tot = np.array([m[0].sum(), m[1].sum(), m[2].sum(), (m[3] + m[5] + m[8]).sum()])
    st = c.step(20)
    c.close()
    new = np.array(st["sum"])
    assert abs(new[0] - tot[0]) / tot[0] < 2e-6
    assert np.all(np.abs(new[1:3] - tot[1:3]) / tot[0] < 2e-6)
    assert abs(new[3] - tot[3]) / tot[3] < 2e-6


def test_mixed_full_size_matches_fp64():
    """The benchmark workload (1024^2 four-quadrant input) after 60 steps:
    mixed path against the FP64 path (which matches the oracle to 1e-10)."""
    _case("mixed vs fp64 quadrants seed 0 1024x1024 60 steps")
    cfg, prim = li.quadrants(0, n=1024)
    a, sa = run_gpu(cfg, prim, 60, precision=1)
    b, sb = run_gpu(cfg, prim, 60, precision=0)
    errs = l1_errors(a, b, 2, cfg["K"])
    print("L1 rho/u/T", errs, "it mixed", sa["it_mean_f"], "fp64", sb["it_mean_f"])
    assert max(errs) < BUDGET
    # the FP32 path stops Newton at 1e-4 and then polishes (residual squared):
    # its errors stay at the rounding level of FP32 state, far inside the budget
    assert max(errs) < 1e-5
