"""GPU parity with the oracle for population paths reflected by solid cells
and slip walls (Sec. III.B), through the C ABI."""
import sys

import numpy as np
import pytest

import lelbm_inputs as li
from helpers import oracle_moments, rel_linf, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def _case(name):
    print("case:", name, flush=True)
    sys.stdout.flush()


def _fluid_rel_linf(a, b, solid):
    f = np.asarray(solid).ravel() == 0
    return rel_linf(a[:, f], b[:, f])


def test_channel_with_obstacles_parity():
    """Supersonic inflow past seeded ellipses, slip walls, outflow."""
    _case("channel seed 0 128x48 Mach 2.5, 60 steps")
    cfg, prim = li.channel(0, nx=128, ny=48, size_scale=0.08, pad=24, mach=2.5)
    a, _ = run_gpu(cfg, prim, 60)
    b, _ = run_oracle(cfg, prim, 60)
    err = _fluid_rel_linf(a, b, cfg["solid"])
    print("rel_linf", err)
    assert err < 1e-10
    assert np.abs(a[:, cfg["solid"].ravel() != 0]).max() == 0.0


@pytest.mark.parametrize("seed", [1, 2])
def test_random_solids_in_a_periodic_box_parity(seed):
    _case("random solids periodic 40x36 seed %d, 40 steps" % seed)
    cfg, prim = li.smooth_periodic(seed, n=40, ny=36)
    rng = np.random.default_rng(seed)
    cfg["solid"] = (rng.random((36, 40)) < 0.08).astype(np.uint8)
    m = oracle_moments(cfg, prim)
    a, _ = run_gpu(cfg, prim, 40, mom=m)
    b, _ = run_oracle(cfg, prim, 40, mom=m)
    err = _fluid_rel_linf(a, b, cfg["solid"])
    print("rel_linf", err)
    assert err < 1e-10


@pytest.mark.parametrize("seed,nx,ny,frac,walls", [(4, 33, 47, 0.12, True), (6, 29, 29, 0.20, False)])
def test_dense_random_solids_parity(seed, nx, ny, frac, walls):
    """Dense random solids (most tiles trace their paths, many paths reflect
    several times), with and without slip walls, on tiles that are cut by
    the domain edge; the walk cache is filled and then read."""
    _case("dense random solids %dx%d %.2f walls=%s, 25 steps" % (nx, ny, frac, walls))
    cfg, prim = li.smooth_periodic(seed, n=nx, ny=ny, RT=1.2)
    if walls:
        cfg["bc"] = ["periodic", "periodic", "slipwall", "slipwall"]
    rng = np.random.default_rng(seed)
    cfg["solid"] = (rng.random((ny, nx)) < frac).astype(np.uint8)
    m = oracle_moments(cfg, prim)
    a, _ = run_gpu(cfg, prim, 25, mom=m)
    b, _ = run_oracle(cfg, prim, 25, mom=m)
    err = _fluid_rel_linf(a, b, cfg["solid"])
    print("rel_linf", err)
    assert err < 1e-10


def test_narrow_slip_channel_reflects_twice():
    """A channel narrower than the stencil reach: paths reflect off both
    walls."""
    _case("narrow slip channel 48x5, 30 steps")
    cfg, prim = li.smooth_periodic(4, n=48, ny=5, RT=1.5)
    cfg["bc"] = ["periodic", "periodic", "slipwall", "slipwall"]
    a, _ = run_gpu(cfg, prim, 30)
    b, _ = run_oracle(cfg, prim, 30)
    err = rel_linf(a, b)
    print("rel_linf", err)
    assert err < 1e-10


def test_narrow_1d_slip_box_traces_paths():
    """A 1D box between two slip walls, narrower than twice the stencil
    reach: every tile traces its paths back (the 1D backward-walk gather and
    its cache, filled at the first step and read at the later ones)."""
    _case("1d slip box 12 cells, 40 steps")
    cfg, prim = li.riemann1d(2, n=12)
    cfg["bc"] = ["slipwall", "slipwall", "periodic", "periodic"]
    a, _ = run_gpu(cfg, prim, 40)
    b, _ = run_oracle(cfg, prim, 40)
    err = rel_linf(a, b)
    print("rel_linf", err)
    assert err < 1e-10


def test_gas_at_rest_around_obstacles_stays_at_rest():
    _case("rest state with obstacles 64x48")
    cfg, _ = li.hotbox(0.8, n=64, ny=48)
    rng = np.random.default_rng(5)
    cfg["solid"] = (rng.random((48, 64)) < 0.1).astype(np.uint8)
    shape = (48, 64)
    prim = {"rho": np.ones(shape), "ux": np.zeros(shape), "uy": np.zeros(shape), "RT": np.full(shape, 0.8)}
    m = oracle_moments(cfg, prim)
    a, st = run_gpu(cfg, prim, 5, mom=m)
    f = cfg["solid"].ravel() == 0
    err = (np.abs(a[:, f] - m[:, f]).max(axis=1) / np.maximum(np.abs(m[:, f]).max(axis=1), 1.0)).max()
    print("rest error", err)
    assert err < 1e-13
    assert np.abs(a[:, ~f]).max() == 0.0


def test_channel_mach6_parity():
    _case("channel seed 3 128x48 Mach 6, 30 steps")
    cfg, prim = li.channel(3, nx=128, ny=48, size_scale=0.08, pad=24, mach=6.0)
    a, _ = run_gpu(cfg, prim, 30)
    b, _ = run_oracle(cfg, prim, 30)
    err = _fluid_rel_linf(a, b, cfg["solid"])
    print("rel_linf", err)
    assert err < 1e-10


def test_channel_mixed_precision_errors():
    _case("channel seed 3 128x48 Mach 2.5 mixed, 60 steps")
    cfg, prim = li.channel(3, nx=128, ny=48, size_scale=0.08, pad=24, mach=2.5)
    a, _ = run_gpu(cfg, prim, 60, precision=1)
    b, _ = run_oracle(cfg, prim, 60)
    f = cfg["solid"].ravel() == 0
    rho_a, rho_b = a[0, f], b[0, f]
    l1 = np.abs(rho_a - rho_b).sum() / np.abs(rho_b).sum()
    print("L1 rho", l1)
    assert l1 < 1e-4


def test_reach_beyond_the_walk_cache_parity():
    """Hot fast gas around a solid block: RT 40 (R = 25) at u = (8, 3) gives a
    reach of 34 cells, beyond the largest reach whose backward walks are
    cached (31), so the tiles near the block walk every displacement at every
    step, and the blocker map of a wavefront's region is too large for its
    LDS share, so the walks read the mask from global memory."""
    _case("reach 34 around a solid block, 96x96 periodic, 6 steps")
    cfg, prim = li.hotbox(40.0, n=96, u=(8.0, 3.0))
    solid = np.zeros((96, 96), dtype=np.uint8)
    solid[40:52, 44:52] = 1
    cfg["solid"] = solid
    y = (np.arange(96) + 0.5)[:, None]
    x = (np.arange(96) + 0.5)[None, :]
    prim["rho"] = 1.0 + 0.02 * np.sin(2 * np.pi * x / 96) * np.cos(2 * np.pi * y / 96)
    m = oracle_moments(cfg, prim)
    a, st = run_gpu(cfg, prim, 6, mom=m)
    b, _ = run_oracle(cfg, prim, 6, mom=m)
    print("colat_max %.2f" % st["colat_max"])
    assert st["colat_max"] + 1 > 31
    err = _fluid_rel_linf(a, b, solid)
    print("rel_linf", err)
    assert err < 1e-10
