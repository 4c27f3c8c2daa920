"""GPU parity: the FP64 HIP path against the CPU oracle, element by element, on
the same seeded inputs, through the C ABI.  Bar: 1e-10 relative L-infinity
after 100 steps (sizes that span several 16x16 tiles with ragged edges), the
integer statistics (stencil sizes) exactly, and conservation to rounding."""
import numpy as np
import pytest

import lelbm_inputs as li
import oracle
from helpers import gpu_moments, oracle_moments, rel_linf, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _print_case(name):
    print("\n[gpu case] %s" % name, flush=True)


def test_uniform_hotbox_is_invariant():
    _print_case("hotbox 40x24 RT=1 u=(10,10)")
    cfg, prim = li.hotbox(1.0, n=40, ny=24)
    m = gpu_moments(cfg, prim)
    out, st = run_gpu(cfg, prim, 5, mom=m)
    assert rel_linf(out, m) < 2e-11
    assert st["q_min"] == st["q_max"] == 69     # integer points within 4.5 of an integer centre


@pytest.mark.parametrize("seed", [0, 3])
def test_riemann1d_parity_100_steps(seed):
    _print_case("riemann1d seed %d n=2000 100 steps" % seed)
    cfg, prim = li.riemann1d(seed, n=2000)
    a, sa = run_gpu(cfg, prim, 100)
    b, sb = run_oracle(cfg, prim, 100)
    assert rel_linf(a, b) < TOL
    assert sa["q_min"] == sb["q_min"] and sa["q_max"] == sb["q_max"]
    assert abs(sa["q_mean"] - sb["q_mean"]) < 1e-9
    assert abs(sa["it_mean_f"] - sb["it_mean_f"]) < 0.01


@pytest.mark.parametrize("seed", [2, 4])
def test_quadrants_parity_100_steps(seed):
    _print_case("quadrants seed %d 72x56 100 steps" % seed)
    cfg, prim = li.quadrants(seed, n=72, ny=56)
    a, sa = run_gpu(cfg, prim, 100)
    b, sb = run_oracle(cfg, prim, 100)
    err = rel_linf(a, b)
    print("rel_linf", err, "q", sa["q_min"], sa["q_max"], "it", sa["it_mean_f"], sa["it_max_f"])
    assert err < TOL
    assert sa["q_min"] == sb["q_min"] and sa["q_max"] == sb["q_max"]
    assert abs(sa["it_mean_f"] - sb["it_mean_f"]) < 0.01
    assert sa["limited"] == sb["limited"]


@pytest.mark.parametrize("seed", [0, 9])
def test_hot_quadrant_seeds_parity_100_steps(seed):
    """The seeds with the hottest quadrants of the distribution (lattice RT up
    to 13.6 and 17.1: stencil radii 15 and 17, q up to ~970), where the
    limiter is active in most cells and the Newton solves take the most
    iterations."""
    _print_case("quadrants seed %d 72x56 100 steps (hot)" % seed)
    cfg, prim = li.quadrants(seed, n=72, ny=56)
    assert prim["RT"].max() > 13.0
    a, sa = run_gpu(cfg, prim, 100)
    b, sb = run_oracle(cfg, prim, 100)
    err = rel_linf(a, b)
    print("rel_linf", err, "q", sa["q_min"], sa["q_max"], "it", sa["it_mean_f"], sa["it_max_f"])
    assert err < TOL
    assert sa["q_min"] == sb["q_min"] and sa["q_max"] == sb["q_max"]
    assert sa["q_max"] > 800
    assert abs(sa["it_mean_f"] - sb["it_mean_f"]) < 0.01


def test_wide_stencils_parity_100_steps():
    """Stencil radii of 31 and more (RT ~ 70, q ~ 3500-4000): more rows than
    the reconstruction kernel's table of row spans holds, so every pass
    recomputes each row's span; the gather stages windows of ~70 x 70
    displacements in few rows per chunk."""
    _print_case("smooth periodic RT~72 24x18 100 steps (R >= 31)")
    cfg, prim = li.smooth_periodic(7, n=24, ny=18, RT=72.0)
    a, sa = run_gpu(cfg, prim, 100)
    b, sb = run_oracle(cfg, prim, 100)
    err = rel_linf(a, b)
    print("rel_linf", err, "q", sa["q_min"], sa["q_max"], "it", sa["it_mean_f"], sa["it_max_f"])
    assert err < TOL
    assert sa["q_min"] == sb["q_min"] and sa["q_max"] == sb["q_max"]
    assert sa["q_min"] > 3100          # R >= 31 in every cell: q > pi 31.5^2


@pytest.mark.parametrize("case", ["quadrants", "riemann1d", "channel"])
def test_unstaged_gather_parity(case, monkeypatch):
    """The gather's fallback for windows too wide to stage in LDS: with the
    staging capacity at its minimum (256 sources, set from the host), no
    window fits, and every destination reads its sources' descriptors from
    global memory."""
    _print_case("unstaged gather %s" % case)
    monkeypatch.setenv("LELBM_GATHER_CAP", "256")
    if case == "quadrants":
        cfg, prim = li.quadrants(4, n=72, ny=56)
        steps = 20
    elif case == "riemann1d":
        cfg, prim = li.riemann1d(0, n=600)
        steps = 30
    else:
        cfg, prim = li.hotbox(1.0, n=48, ny=40, u=(2.0 * np.sqrt(1.4), 0.0))
        cfg["bc"] = ["inflow", "outflow", "slipwall", "slipwall"]
        cfg["pad"] = 12
        cfg["in_rho"], cfg["in_u"], cfg["in_RT"] = 1.0, (2.0 * np.sqrt(1.4), 0.0), 1.0
        y = (np.arange(40) + 0.5)[:, None]
        prim["uy"] = 0.4 * np.sin(np.pi * y / 40) * np.ones((1, 48))
        steps = 20
    a, sa = run_gpu(cfg, prim, steps)
    b, sb = run_oracle(cfg, prim, steps)
    err = rel_linf(a, b)
    print("rel_linf", err)
    assert err < TOL
    assert sa["arrivals"] > 0


def test_pad_reach_error_mid_run():
    """A pad narrower than a stencil's reach toward the interior is an error
    (Sec. III): 1D gas at RT = 1.2 (R = 4) between 4-cell outflow pads, with a
    hot slug in the middle whose compression wave heats the gas at the ends
    past R = 4.  The step at which that happens fails with EREACH on the GPU
    and in the oracle alike, both keeping the state of the step before."""
    _print_case("1d pad reach error mid run")
    import paper_2508_06911_amd as lb
    cfg, prim = li.hotbox(1.2, n=80, dim=1, u=(0.0, 0.0))
    cfg["bc"] = ["outflow", "outflow", "periodic", "periodic"]
    cfg["pad"] = 4
    x = np.arange(80) + 0.5
    prim["RT"] = np.where(np.abs(x - 40) < 6, 2.4, 1.2)[None, :]
    st, ref, ostats, done = oracle.step(cfg, oracle_moments(cfg, prim), 80)
    assert st == oracle.EREACH and done > 0
    c = lb.Lelbm(cfg, gpu_moments(cfg, prim))
    with pytest.raises(lb.LelbmError) as e:
        c.step(80)
    assert e.value.code == lb.EREACH
    node, step = c.last_failure()
    assert step == done and node == ostats["fail_cell"]
    assert rel_linf(c.read_moments(), ref) < TOL
    c.close()
    # a pad that is too narrow from the start fails at creation (u_y = 0.37:
    # no integer point lies exactly on the stencil's rim, where rounding of u
    # could decide membership differently on the two sides)
    cfg2, prim2 = li.hotbox(1.0, n=36, ny=20, u=(10.0, 0.37))
    cfg2["bc"] = ["inflow", "outflow", "periodic", "periodic"]
    cfg2["pad"] = 13
    cfg2["in_rho"], cfg2["in_u"], cfg2["in_RT"] = 1.0, (10.0, 0.37), 1.0
    with pytest.raises(lb.LelbmError) as e:
        lb.Lelbm(cfg2, gpu_moments(cfg2, prim2))
    assert e.value.code == lb.EREACH
    cfg2["pad"] = 14
    a, _ = run_gpu(cfg2, prim2, 3)
    b, _ = run_oracle(cfg2, prim2, 3)
    assert rel_linf(a, b) < TOL


def test_refined_stencils_parity():
    """RT < 4/9 switches on stencil refinement (Eq. IIC9): refined tiles store
    pre-summed moment fractions."""
    _print_case("smooth periodic RT~0.3 refined 40x24 20 steps")
    cfg, prim = li.smooth_periodic(5, n=40, ny=24, RT=0.3)
    a, sa = run_gpu(cfg, prim, 20)
    b, sb = run_oracle(cfg, prim, 20)
    assert rel_linf(a, b) < TOL
    assert sa["q_max"] == sb["q_max"] and sa["q_min"] == sb["q_min"]
    assert sa["q_max"] > 25    # R = 2 base disks hold at most 21 points; refined ones more


def test_pads_and_slip_walls_parity():
    """Inflow pads (left), outflow pads (right), slip walls (top/bottom) with a
    Mach-2 stream over a density bump and a transverse velocity."""
    _print_case("channel 48x40 inflow/outflow/slip 40 steps")
    cfg, prim = li.hotbox(1.0, n=48, ny=40, u=(2.0 * np.sqrt(1.4), 0.0))
    cfg["bc"] = ["inflow", "outflow", "slipwall", "slipwall"]
    cfg["pad"] = 12
    cfg["in_rho"], cfg["in_u"], cfg["in_RT"] = 1.0, (2.0 * np.sqrt(1.4), 0.0), 1.0
    x = (np.arange(48) + 0.5)[None, :]
    y = (np.arange(40) + 0.5)[:, None]
    prim["rho"] = 1.0 + 0.3 * np.exp(-((x - 20) ** 2 + (y - 12) ** 2) / 30.0)
    prim["uy"] = 0.4 * np.sin(np.pi * y / 40) * np.ones((1, 48))
    a, sa = run_gpu(cfg, prim, 40)
    b, sb = run_oracle(cfg, prim, 40)
    assert rel_linf(a, b) < TOL
    assert sa["q_max"] == sb["q_max"]


def test_riemann1d_with_inflow_and_slip():
    _print_case("1d inflow/slipwall 300 cells 60 steps")
    cfg, prim = li.riemann1d(1, n=300)
    cfg["bc"] = ["inflow", "slipwall", "periodic", "periodic"]
    cfg["in_rho"], cfg["in_u"], cfg["in_RT"] = 0.8, (0.6, 0.0), 0.7
    a, sa = run_gpu(cfg, prim, 60)
    b, sb = run_oracle(cfg, prim, 60)
    assert rel_linf(a, b) < TOL


@pytest.mark.parametrize("shape", [(5, 3), (37, 19), (16, 16)])
def test_small_and_ragged_periodic_domains(shape):
    """Domains smaller than a stencil (populations wrap several times) and
    domains that do not fill whole tiles."""
    _print_case("smooth periodic %s" % (shape,))
    nx, ny = shape
    cfg, prim = li.smooth_periodic(6, n=nx, ny=ny)
    a, _ = run_gpu(cfg, prim, 10)
    b, _ = run_oracle(cfg, prim, 10)
    assert rel_linf(a, b) < TOL


def test_conservation_and_determinism():
    _print_case("quadrants seed 4 64x64 conservation")
    import paper_2508_06911_amd as lb
    cfg, prim = li.quadrants(4, n=64)
    m = gpu_moments(cfg, prim)
    c1 = lb.Lelbm(cfg, m)
    s0 = c1.step(0)
    tot0 = np.array(s0["sum"]) if s0 else None
    st = c1.step(30)
    a = c1.read_moments()
    c1.close()
    c2 = lb.Lelbm(cfg, m)
    c2.step(30)
    b = c2.read_moments()
    c2.close()
    assert np.array_equal(a, b)           # the gather is atomic-free: bitwise reproducible
    tot = np.array([m[0].sum(), m[1].sum(), m[2].sum(), (m[3] + m[5] + m[8]).sum()])
    new = np.array(st["sum"])
    assert abs(new[0] - tot[0]) / tot[0] < 1e-13
    assert np.all(np.abs(new[1:3] - tot[1:3]) / tot[0] < 1e-13)
    assert abs(new[3] - tot[3]) / tot[3] < 1e-13


def test_zero_steps_and_resume_are_exact():
    """Checkpoint = read moments; resume = create from them: 20 steps equal
    10 + resume + 10 bitwise."""
    _print_case("resume 48x40")
    import paper_2508_06911_amd as lb
    cfg, prim = li.quadrants(2, n=48, ny=40)
    m = gpu_moments(cfg, prim)
    c = lb.Lelbm(cfg, m)
    c.step(0)
    assert np.array_equal(c.read_moments(), m)
    c.step(20)
    full = c.read_moments()
    c.close()
    c = lb.Lelbm(cfg, m)
    c.step(10)
    half = c.read_moments()
    c.close()
    c = lb.Lelbm(cfg, half)
    c.step(10)
    assert np.array_equal(c.read_moments(), full)
    c.close()


def test_failure_is_transactional():
    """A cell with negative internal energy is not realizable: creation fails
    with LELBM_EEPR.  A Newton iteration cap too small to converge (forced from
    the host) fails the first step; the state stays at the last good step and
    the failure names step 0."""
    _print_case("failure 24x24")
    import paper_2508_06911_amd as lb
    cfg, prim = li.hotbox(1.0, n=24, ny=24, u=(0.3, 0.1))
    m = gpu_moments(cfg, prim)
    bad = m.copy()
    bad[3, 5 * 24 + 7] = -10.0
    with pytest.raises(lb.LelbmError) as e:
        lb.Lelbm(cfg, bad)
    assert e.value.code == lb.EEPR
    c2 = dict(cfg)
    c2["newton_max_it"] = 1
    c = lb.Lelbm(c2, m)
    with pytest.raises(lb.LelbmError) as e:
        c.step(3)
    assert e.value.code == lb.EEPR
    node, step = c.last_failure()
    assert step == 0 and node == 0
    assert np.array_equal(c.read_moments(), m)
    c.close()


def test_full_size_quadrants_sampled_windows():
    """Full 1024x1024 four-quadrant input in the benchmark's launch
    configuration: after two GPU steps, one more GPU step is compared on
    sampled windows with an oracle step of the same window (no sources
    outside the window; only cells farther than the maximum reach from the
    window edge are compared)."""
    _print_case("quadrants seed 0 1024x1024 sampled windows")
    import paper_2508_06911_amd as lb
    cfg, prim = li.quadrants(0, n=1024)
    m = gpu_moments(cfg, prim)
    c = lb.Lelbm(cfg, m)
    c.step(2)
    mk = c.read_moments()
    st = c.step(1)
    mk1 = c.read_moments()
    c.close()
    reach = int(np.ceil(st["colat_max"])) + 2
    W = 2 * reach + 24
    rng = np.random.default_rng(0)
    centres = [(512, 512), (0 + W // 2, 512), (512, 1023 - W // 2)] + [tuple(rng.integers(W, 1024 - W, 2)) for _ in range(2)]
    mk = mk.reshape(11, 1024, 1024)
    mk1 = mk1.reshape(11, 1024, 1024)
    for cx, cy in centres:
        x0, y0 = int(cx) - W // 2, int(cy) - W // 2
        xs = np.arange(x0, x0 + W) % 1024
        ys = np.arange(y0, y0 + W) % 1024
        win = mk[:, ys][:, :, xs].reshape(11, -1)
        wc = dict(cfg)
        wc.update(nx=W, ny=W, bc=["outflow"] * 4, pad=0)
        stt, out, _, _ = oracle.step(wc, win, 1)
        assert stt == 0
        out = out.reshape(11, W, W)[:, reach:W - reach, reach:W - reach]
        ref = mk1[:, ys[reach:W - reach]][:, :, xs[reach:W - reach]]
        err = rel_linf(ref.reshape(11, -1), out.reshape(11, -1))
        print("window", cx, cy, "rel_linf", err)
        assert err < TOL


def test_step_statistics_match_oracle():
    """The step statistics (reduced per workgroup on the GPU, then folded) equal
    the oracle's on the same input: cell and stencil counts exactly, extrema to
    rounding, Newton iteration counts to within a few cells (a residual at the
    tolerance may fall either side of it)."""
    _print_case("statistics quadrants seed 4 72x56 10 steps")
    cfg, prim = li.quadrants(4, n=72, ny=56)
    _, sa = run_gpu(cfg, prim, 10)
    _, sb = run_oracle(cfg, prim, 10)
    assert sa["cells"] == sb["cells"]
    assert round(sa["q_mean"] * sa["cells"]) == sb["q_sum"]
    assert sa["q_min"] == sb["q_min"] and sa["q_max"] == sb["q_max"]
    assert abs(sa["limited"] - sb["limited"]) <= 2
    for k in ("rt_min", "kn_max", "colat_max"):
        assert abs(sa[k] - sb[k]) <= 1e-10 * abs(sb[k]), k
    assert abs(sa["it_mean_f"] - sb["it_mean_f"]) < 1e-3 and abs(sa["it_mean_g"] - sb["it_mean_g"]) < 1e-3
    assert abs(sa["it_max_f"] - sb["it_max_f"]) <= 1 and abs(sa["it_max_g"] - sb["it_max_g"]) <= 1
