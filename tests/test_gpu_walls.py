"""No-slip walls by the extended bounce-back (Sec. III.B, Eqs. IIIB8-15) on
the HIP path: element-wise parity with the oracle (moving and static walls,
flow into a wall fast enough that its absorbed populations are reflected
specularly, open x faces with pads, a banded record scratch, both
precisions), exact mass per step, the gas at rest, a Couette profile, and the
reach errors the oracle reports."""
import numpy as np
import pytest

import lelbm_inputs as li
from helpers import gpu_moments, oracle_moments, rel_linf, run_oracle

pytestmark = pytest.mark.gpu


def _case(name):
    print("\n[gpu case] %s" % name, flush=True)


def _sheared(ny=24, nx=8, RT=0.5, U=0.07, u0=(0.3, 0.2)):
    """Walls on the y faces, the top one moving, over a density and x-velocity
    perturbation (so that every cell is off equilibrium after one step)."""
    cfg, prim = li.couette(ny=ny, nx=nx, RT=RT, U=U, u0=u0)
    y = (np.arange(ny) + 0.5)[:, None]
    x = (np.arange(nx) + 0.5)[None, :]
    prim["rho"] = 1.0 + 0.05 * np.sin(2 * np.pi * y / ny) + 0.02 * np.cos(2 * np.pi * x / nx)
    prim["ux"] = prim["ux"] + 0.05 * np.sin(2 * np.pi * y / ny) * np.ones((1, nx))
    return cfg, prim


def _run(cfg, prim, steps, precision=0, budget=None):
    import paper_2508_06911_amd as lb
    ctx = lb.Lelbm(cfg, gpu_moments(cfg, prim), precision=precision)
    if budget is not None:
        ctx.set_scratch_budget(budget)
    st = ctx.step(steps)
    out = ctx.read_moments()
    ctx.close()
    return out, st


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-6)])
def test_moving_wall_parity(prec, tol):
    _case("no-slip walls, top moving, precision %d, 6 steps" % prec)
    cfg, prim = _sheared()
    ref, _ = run_oracle(cfg, prim, 6)
    out, _ = _run(cfg, prim, 6, precision=prec)
    err = rel_linf(out, ref)
    print("rel Linf vs oracle %.3g" % err, flush=True)
    assert err < tol


def test_specular_fallback_parity():
    """Flow into the bottom wall at 1.5 cells per step: sources a few rows
    above it lose populations to the wall but no image population reaches
    back across it, so their absorbed populations are reflected."""
    _case("no-slip walls, flow into the wall at 1.5 cells per step, 1 step")
    cfg, prim = _sheared(u0=(0.2, -1.5))
    ref, _ = run_oracle(cfg, prim, 1)
    out, _ = _run(cfg, prim, 1)
    err = rel_linf(out, ref)
    print("rel Linf vs oracle %.3g" % err, flush=True)
    assert err < 1e-10
    assert abs(out[0].sum() / ref[0].sum() - 1) < 1e-13


def test_walls_with_open_x_faces():
    """Inflow on the left, outflow on the right: pad sources lose populations
    to the walls too, and image populations that land in a pad are dropped."""
    _case("no-slip walls with inflow/outflow x faces, 5 steps")
    cfg, prim = _sheared(ny=20, nx=24, RT=0.7, U=0.05, u0=(0.4, 0.0))
    cfg["bc"] = ["inflow", "outflow", "wall", "wall"]
    cfg["pad"] = 6
    cfg["in_rho"], cfg["in_u"], cfg["in_RT"] = 1.0, (0.4, 0.0), 0.7
    ref, _ = run_oracle(cfg, prim, 5)
    out, _ = _run(cfg, prim, 5)
    err = rel_linf(out, ref)
    print("rel Linf vs oracle %.3g" % err, flush=True)
    assert err < 1e-10


def test_walls_with_banded_scratch():
    """Records in bands of one tile row (a small scratch budget): each band's
    image populations are taken from its records before the slot is reused."""
    _case("no-slip walls, 96 x 40, banded scratch, 4 steps")
    cfg, prim = _sheared(ny=96, nx=40, RT=0.6, U=0.08, u0=(0.25, 0.1))
    ref, _ = run_oracle(cfg, prim, 4)
    out, _ = _run(cfg, prim, 4, budget=1 << 20)
    whole, _ = _run(cfg, prim, 4)
    err = rel_linf(out, ref)
    print("rel Linf vs oracle %.3g (banded), banded vs one band %.3g" % (err, rel_linf(out, whole)), flush=True)
    assert err < 1e-10
    assert np.array_equal(out, whole)


def test_mass_is_exact_each_step():
    import paper_2508_06911_amd as lb
    _case("no-slip walls: mass per step, 10 steps")
    cfg, prim = _sheared(ny=32, nx=16, RT=0.8, U=0.1, u0=(0.1, 0.3))
    ctx = lb.Lelbm(cfg, gpu_moments(cfg, prim))
    m0 = ctx.read_moments()[0].sum()
    for _ in range(10):
        st = ctx.step(1)
        assert abs(st["sum"][0] / m0 - 1) < 1e-13
    ctx.close()


def test_gas_at_rest_stays_at_rest():
    _case("no-slip walls: gas at rest, 5 steps")
    cfg, prim = li.couette(ny=20, nx=6, RT=0.8, U=0.0)
    m = gpu_moments(cfg, prim)
    out, _ = _run(cfg, prim, 5)
    assert np.abs(out - m).max() < 1e-13 * np.abs(m).max()


def test_couette_profile():
    """Steady Couette flow: linear and antisymmetric about the mid-plane, no
    normal flow, against the oracle's profile after the same steps."""
    _case("Couette flow 8 rows, 3000 steps")
    U, ny = 0.1, 8
    cfg, prim = li.couette(ny=ny, nx=4, RT=0.5, U=U, nu=0.05)
    ref, _ = run_oracle(cfg, prim, 3000)
    out, _ = _run(cfg, prim, 3000)
    ux = (out[1] / out[0]).reshape(ny, 4).mean(axis=1)
    uy = (out[2] / out[0]).reshape(ny, 4)
    y = np.arange(ny) + 0.5
    b, a = np.polyfit(y, ux, 1)
    print("profile", np.round(ux / U, 5), "rel Linf vs oracle %.3g" % rel_linf(out, ref), flush=True)
    assert np.abs(ux - (a + b * y)).max() < 5e-3 * U
    assert np.abs(ux + ux[::-1] - U).max() < 1e-4 * U
    assert np.abs(uy).max() < 1e-4 * U
    assert rel_linf(out, ref) < 1e-9


@pytest.mark.parametrize("what", ["image lands past the far wall", "refined stencil reaches a wall"])
def test_reach_errors_match_the_oracle(what):
    import oracle
    import paper_2508_06911_amd as lb
    _case("no-slip walls: %s" % what)
    if what.startswith("image"):
        cfg, prim = li.couette(ny=8, nx=4, RT=2.0, U=0.1, nu=0.5)
    else:
        cfg, prim = li.couette(ny=12, nx=4, RT=0.3, U=0.1, nu=0.05)
    st, _, stats, done = oracle.step(cfg, oracle_moments(cfg, prim), 1)
    assert st == oracle.EREACH
    ctx = lb.Lelbm(cfg, gpu_moments(cfg, prim))
    with pytest.raises(lb.LelbmError) as e:
        ctx.step(1)
    ctx.close()
    assert e.value.code == lb.EREACH
