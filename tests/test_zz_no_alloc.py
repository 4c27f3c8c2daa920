"""The allocation-free step (lelbm_step_noalloc) against lelbm_step, through
the C ABI: the same kernels with the library's static per-GPU scratch array
instead of the context's own buffer, so the fields must agree bit for bit.
Calls in a row on one GPU, each on a smaller input than the one before (the
array keeps the previous call's contents), the first banded within the array,
on both precision paths; and a step whose bands of one tile row exceed the
array fails with ENOMEM, keeping the state."""
import numpy as np
import pytest

import lelbm_inputs as li
from helpers import gpu_moments

pytestmark = pytest.mark.gpu


def _case(name):
    print("\n[gpu case] %s" % name, flush=True)


def _pair(cfg, prim, steps, prec):
    import paper_2508_06911_amd as lb
    m = gpu_moments(cfg, prim)
    a = lb.Lelbm(cfg, m, precision=prec)
    sa = a.step(steps)
    ra = a.read_moments()
    a.close()
    b = lb.Lelbm(cfg, m, precision=prec)
    sb = b.step_noalloc(steps)
    rb = b.read_moments()
    _, scratch = b.memory()
    b.close()
    return ra, sa, rb, sb, scratch


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_step_equals_step(prec):
    _case("noalloc vs step, precision %d" % prec)
    # the first case's records exceed the static array: it runs in bands
    cases = [li.quadrants(2, n=128, ny=256), li.quadrants(4, n=72, ny=56),
             li.smooth_periodic(5, n=40, ny=24, RT=0.3)]
    for k, (cfg, prim) in enumerate(cases):
        ra, sa, rb, sb, _ = _pair(cfg, prim, 12 - 4 * k, prec)
        print("case", k, "max diff", np.abs(ra - rb).max(), "q_max", sa["q_max"], sb["q_max"])
        assert np.array_equal(ra, rb)
        assert sa["q_max"] == sb["q_max"] and sa["arrivals"] == sb["arrivals"]
        assert sa["it_mean_f"] == sb["it_mean_f"]


def test_noalloc_rejects_records_beyond_its_array():
    """Records of a hot 160 x 160 box (q ~ 3500 points per cell, ~7 GB in
    FP64; ~140 MB per tile row) do not fit the static array even in bands of
    one tile row: the step fails with ENOMEM and the state is the initial
    one; lelbm_step then runs the same context."""
    _case("noalloc ENOMEM on a hot 160x160 box")
    import paper_2508_06911_amd as lb
    cfg, prim = li.smooth_periodic(7, n=160, ny=160, RT=72.0)
    m = gpu_moments(cfg, prim)
    c = lb.Lelbm(cfg, m)
    with pytest.raises(lb.LelbmError) as e:
        c.step_noalloc(2)
    assert e.value.code == lb.ENOMEM
    node, step = c.last_failure()
    assert step == 0 and node == -1
    assert np.array_equal(c.read_moments(), m)
    c.step(1)
    assert not np.array_equal(c.read_moments(), m)
    c.close()
