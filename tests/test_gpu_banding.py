"""Banded population scratch (Sec. II.E: the moment fractions live only
within a step): with a scratch budget far below the records of the whole
domain, the library reconstructs bands of tile rows and gathers each
destination row as soon as the bands within its reach are done.  The fields
must equal the unbanded run's bit for bit (the gather's summation order does
not depend on where the records are stored), the scratch must stay within
the budget, and re-planning mid-run (bands outgrowing their slots as the gas
heats up, stencils reaching farther) must not change the result."""
import numpy as np
import pytest

import lelbm_inputs as li
from helpers import gpu_moments

pytestmark = pytest.mark.gpu


def _case(name):
    print("\n[gpu case] %s" % name, flush=True)


def _run(cfg, prim, steps, prec=0, budget=None, guess=0, chunks=1):
    import paper_2508_06911_amd as lb
    c = lb.Lelbm(cfg, gpu_moments(cfg, prim), precision=prec, guess=guess)
    if budget is not None:
        c.set_scratch_budget(budget)
    st = None
    for _ in range(chunks):
        st = c.step(steps // chunks)
    out = c.read_moments()
    _, scratch = c.memory()
    c.close()
    return out, st, scratch


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("seed", [2, 9])
def test_banded_quadrants_equal_unbanded(seed, prec):
    """Seed 2 (RT <= 1, reach ~6) fits bands of a few tile rows into a
    quarter of the unbanded scratch; seed 9 (RT up to 17, reach ~25, its hot
    tile rows several times the mean) needs bands of one row, whose largest
    then sets the scratch above that quarter (still below the unbanded)."""
    _case("banded quadrants seed %d 64x512 precision %d" % (seed, prec))
    cfg, prim = li.quadrants(seed, n=64, ny=512)
    a, sa, sc_a = _run(cfg, prim, 12, prec)
    budget = sc_a // 4                            # a quarter of the unbanded scratch
    b, sb, sc_b = _run(cfg, prim, 12, prec, budget=budget)
    print("unbanded scratch", sc_a, "banded", sc_b, "budget", budget, "q_max", sb["q_max"])
    assert np.array_equal(a, b)
    assert sb["arrivals"] == sa["arrivals"] and sb["point_passes"] == sa["point_passes"]
    if seed == 2:
        assert sc_b <= budget
    else:
        assert sc_b < sc_a


def test_banded_channel_with_obstacles_equal_unbanded():
    """Inflow and outflow pads, slip walls, solid cells (backward-walk gather
    near them), the gas heating up behind the bow shocks: the plan is redone
    as bands outgrow their slots."""
    _case("banded channel Mach 3 192x256 with obstacles")
    cfg, prim = li.channel(1, nx=192, ny=256, size_scale=0.15, pad=24, mach=3.0)
    a, sa, sc_a = _run(cfg, prim, 60)
    b, sb, sc_b = _run(cfg, prim, 60, budget=sc_a // 4, chunks=3)
    print("unbanded scratch", sc_a, "banded", sc_b, "q_max", sb["q_max"])
    assert np.array_equal(a, b)
    assert sc_b < sc_a


def test_banded_hot_periodic_box_replans():
    """A periodic box whose hot spot spreads: stencils grow from R = 4 to
    R ~ 12 during the run, so the reach outgrows the plan and the bands their
    slots; the bands wrap across the periodic edge."""
    _case("banded hot periodic box 96x160 40 steps")
    cfg, prim = li.smooth_periodic(3, n=96, ny=160, RT=1.0)
    y = (np.arange(160) + 0.5)[:, None]
    x = (np.arange(96) + 0.5)[None, :]
    prim["RT"] = prim["RT"] * (1.0 + 8.0 * np.exp(-((x - 48) ** 2 + (y - 150) ** 2) / 60.0))
    a, sa, sc_a = _run(cfg, prim, 40)
    b, sb, sc_b = _run(cfg, prim, 40, budget=max(sc_a // 10, 1 << 20), chunks=4)
    print("unbanded scratch", sc_a, "banded", sc_b, "q_max", sb["q_max"])
    assert np.array_equal(a, b)


@pytest.mark.parametrize("ny", [64, 1024])
def test_budget_below_a_single_tile_row_still_runs(ny):
    """A budget smaller than the records of one tile row: the smaller of one
    band of the whole domain (a short domain, where bands of one row would
    all be live at once) and bands of one tile row (a tall one)."""
    _case("tiny budget quadrants 64x%d" % ny)
    cfg, prim = li.quadrants(4, n=64, ny=ny)
    a, sa, sc_a = _run(cfg, prim, 6)
    b, sb, sc_b = _run(cfg, prim, 6, budget=4096)
    print("unbanded scratch", sc_a, "tiny budget", sc_b)
    assert np.array_equal(a, b)
    # short: one band, as unbanded; tall: bands of one row (the hot spots at
    # the quadrants' corner make the largest row several times the mean)
    assert sc_b <= sc_a if ny == 64 else sc_b < sc_a
