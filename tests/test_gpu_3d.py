"""The 3D step (D = 3, periodic boxes) on the HIP path: element-wise parity
with the 3D oracle in both precisions on boxes of several ragged tiles,
across step calls, exact conservation and a uniform flow at size, the
shear viscosity at a resolution the oracle would need minutes for, refined
stencils, banded records, the linearised start, stencils beyond three
refinement levels refused, and the full 96^3 box in the launch configuration
of the 3D benchmark compared on sampled windows."""
import numpy as np
import pytest

import lelbm_inputs as li
import oracle
from helpers import rel_linf

pytestmark = pytest.mark.gpu


def _case(name):
    print("\n[gpu case] %s" % name, flush=True)


def _mom(cfg, prim):
    import paper_2508_06911_amd as lb
    return lb.moments_from_primitives3(cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["uz"], prim["RT"])


def _oracle(cfg, prim, steps):
    m = oracle.moments_from_primitives3(cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["uz"], prim["RT"])
    st, out, stats, done = oracle.step(cfg, m, steps)
    assert st == 0, (st, done)
    return out, stats


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-6)])
@pytest.mark.parametrize("seed", [0, 1])
def test_parity_ragged_box(prec, tol, seed):
    import paper_2508_06911_amd as lb
    _case("3D parity seed %d precision %d, 10 x 9 x 7, 4 steps" % (seed, prec))
    cfg, prim = li.smooth_periodic3(seed, n=10, ny=9, nz=7, amp=0.08, RT=0.9)
    ref, rs = _oracle(cfg, prim, 4)
    ctx = lb.Lelbm(cfg, _mom(cfg, prim), precision=prec)
    st = ctx.step(4)
    out = ctx.read_moments()
    ctx.close()
    err = rel_linf(out, ref)
    print("rel Linf vs oracle %.3g, q mean %.1f (oracle %.1f), Newton it %.2f" % (err, st["q_mean"], rs["q_mean"],
                                                                               st["it_mean_f"]), flush=True)
    assert err < tol
    assert abs(st["q_mean"] - rs["q_mean"]) < 1e-9


def test_reach_statistic():
    """The step's colat_max is the largest |u| + R over the cells (Eq. IIC7)."""
    import paper_2508_06911_amd as lb
    _case("3D reach statistic, 10 x 9 x 7, 1 step")
    cfg, prim = li.smooth_periodic3(0, n=10, ny=9, nz=7, amp=0.08, RT=0.9)
    ctx = lb.Lelbm(cfg, _mom(cfg, prim))
    st = ctx.step(1)
    ctx.close()
    R = np.maximum(np.floor(4.0 * np.sqrt(prim["RT"]) + 0.5), 2)
    want = (np.sqrt(prim["ux"] ** 2 + prim["uy"] ** 2 + prim["uz"] ** 2) + R).max()
    print("colat_max %.15g, expected %.15g" % (st["colat_max"], want), flush=True)
    assert abs(st["colat_max"] - want) < 1e-12 * want


def test_parity_across_calls_and_hot_fast_gas():
    """A hotter, faster state (R up to 6, |u| above 2) split over two calls
    equals one call of all steps, and the oracle."""
    import paper_2508_06911_amd as lb
    _case("3D hot fast gas 8 x 8 x 8, 2 + 3 steps")
    cfg, prim = li.smooth_periodic3(2, n=8, amp=0.1, RT=2.2, u=(2.3, -1.4, 0.7))
    ref, _ = _oracle(cfg, prim, 5)
    a = lb.Lelbm(cfg, _mom(cfg, prim))
    a.step(2)
    a.step(3)
    oa = a.read_moments()
    a.close()
    b = lb.Lelbm(cfg, _mom(cfg, prim))
    b.step(5)
    ob = b.read_moments()
    b.close()
    print("rel Linf vs oracle %.3g" % rel_linf(oa, ref), flush=True)
    assert np.array_equal(oa, ob)
    assert rel_linf(oa, ref) < 1e-10


@pytest.mark.parametrize("RT,ux,what", [(2.6, 4.5, "reach ~11: 8-row gather blocks"),
                                        (5.0, 4.5, "reach ~14: unstaged gather")])
def test_parity_large_reach(RT, ux, what):
    """Fast hot gases whose reach leaves the 16-row staged gather (its source
    planes exceed the LDS): the 8-row blocks and the unstaged gather agree
    with the oracle too."""
    import paper_2508_06911_amd as lb
    _case("3D %s, RT %.1f, u_x %.1f, 8 x 7 x 6, 2 steps" % (what, RT, ux))
    cfg, prim = li.smooth_periodic3(3, n=8, ny=7, nz=6, amp=0.05, RT=RT, u=(ux, -0.8, 0.3))
    ref, _ = _oracle(cfg, prim, 2)
    ctx = lb.Lelbm(cfg, _mom(cfg, prim))
    st = ctx.step(2)
    out = ctx.read_moments()
    ctx.close()
    err = rel_linf(out, ref)
    print("rel Linf vs oracle %.3g, q max %d" % (err, st["q_max"]), flush=True)
    assert err < 1e-10


def test_conservation_and_uniform_flow_at_size():
    import paper_2508_06911_amd as lb
    _case("3D conservation 48^3, 3 steps; uniform flow 32^3")
    cfg, prim = li.smooth_periodic3(3, n=48, amp=0.1, RT=1.2)
    m = _mom(cfg, prim)
    ctx = lb.Lelbm(cfg, m)
    st = ctx.step(3)
    out = ctx.read_moments()
    ctx.close()
    E = lambda a: a[4] + a[7] + a[9] + a[13]
    for k in range(4):
        assert abs(out[k].sum() - m[k].sum()) < 1e-12 * m[0].sum()
    assert abs(E(out).sum() / E(m).sum() - 1) < 1e-12
    assert abs(st["sum"][0] / m[0].sum() - 1) < 1e-13
    cfg, prim = li.smooth_periodic3(0, n=32, amp=0.0, u=(1.3, -0.7, 0.45), RT=1.4)
    m = _mom(cfg, prim)
    ctx = lb.Lelbm(cfg, m)
    ctx.step(2)
    out = ctx.read_moments()
    ctx.close()
    assert np.abs(out - m).max() < 1e-12 * np.abs(m).max()


def test_shear_viscosity_64():
    """Transverse shear wave (Sec. IV.A) on 64 x 4 x 4 at rest: nu = RT (1/omega_f - 1/2) (Eq. C8a) within 1 %."""
    import paper_2508_06911_amd as lb
    _case("3D shear wave L = 64, RT 1, nu 0.1")
    L, nu = 64, 0.1
    cfg, prim = li.shear_wave3(L=L, ny=4, nz=4, RT=1.0, nu=nu, u0=0.0, amp=1e-4)
    k = 2 * np.pi / L
    t = int(round(1.0 / (nu * k * k)))
    ctx = lb.Lelbm(cfg, _mom(cfg, prim))
    ctx.step_nostats(t)
    out = ctx.read_moments()
    ctx.close()
    uy = (out[2] / out[0]).reshape(4, 4, L).mean(axis=(0, 1))
    x = np.arange(L) + 0.5
    amp = np.hypot((uy * np.cos(k * x)).sum(), (uy * np.sin(k * x)).sum()) * 2 / L
    nu_m = -np.log(amp / 1e-4) / (k * k * t)
    print("nu measured %.5f target %.5f" % (nu_m, nu), flush=True)
    assert abs(nu_m / nu - 1) < 0.01


def test_refinement_beyond_three_levels_is_refused():
    import paper_2508_06911_amd as lb
    _case("3D stencil beyond three refinement levels refused")
    cfg, prim = li.smooth_periodic3(4, n=4, amp=0.0, RT=0.008)
    ctx = lb.Lelbm(cfg, _mom(cfg, prim))
    with pytest.raises(lb.LelbmError) as e:
        ctx.step(1)
    ctx.close()
    assert e.value.code == lb.EREACH


@pytest.mark.parametrize("guess", ["eq", "prev"])
def test_banded_records_equal_one_band(guess):
    """Records in bands of tile layers within a small scratch budget: the
    fields equal the one-band run bit for bit (and the oracle), with a
    smaller scratch; also with the previous-step guess, whose stored
    corrections are written band by band."""
    import paper_2508_06911_amd as lb
    _case("3D banded records, 8 x 8 x 64, 3 steps, guess %s" % guess)
    g = lb.GUESS_PREV if guess == "prev" else lb.GUESS_EQ
    cfg, prim = li.smooth_periodic3(5, n=8, ny=8, nz=64, amp=0.08, RT=0.9)
    m = _mom(cfg, prim)
    a = lb.Lelbm(cfg, m, guess=g)
    a.step(3)
    whole = a.read_moments()
    _, s_whole = a.memory()
    a.close()
    b = lb.Lelbm(cfg, m, guess=g)
    b.set_scratch_budget(int(0.65 * s_whole))
    b.step(3)
    banded = b.read_moments()
    _, s_band = b.memory()
    b.close()
    ref, _ = _oracle(cfg, prim, 3)
    print("scratch one band %.1f MB, banded %.1f MB; rel Linf vs oracle %.3g" % (s_whole / 1e6, s_band / 1e6,
                                                                              rel_linf(banded, ref)), flush=True)
    assert np.array_equal(banded, whole)
    assert s_band <= 0.65 * s_whole
    assert rel_linf(banded, ref) < 1e-10


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-6)])
def test_linearised_start_matches_eq(prec, tol):
    """The linearised Newton start (Eq. IID13 plus one step with the
    continuous Maxwellian's Hessian) converges to the same multipliers in
    fewer updates."""
    import paper_2508_06911_amd as lb
    _case("3D linearised start, precision %d, 10 x 9 x 7, 4 steps" % prec)
    cfg, prim = li.smooth_periodic3(1, n=10, ny=9, nz=7, amp=0.08, RT=0.9)
    m = _mom(cfg, prim)
    outs, its = {}, {}
    for g in (lb.GUESS_EQ, lb.GUESS_LIN):
        c = lb.Lelbm(cfg, m, precision=prec, guess=g)
        st = c.step(4)
        outs[g] = c.read_moments()
        its[g] = st["it_mean_f"] + st["it_mean_g"]
        c.close()
    err = rel_linf(outs[lb.GUESS_LIN], outs[lb.GUESS_EQ])
    print("LIN vs EQ %.3g; Newton updates per cell (f + g) EQ %.2f LIN %.2f" % (err, its[lb.GUESS_EQ],
                                                                                its[lb.GUESS_LIN]), flush=True)
    assert err < tol
    assert its[lb.GUESS_LIN] < its[lb.GUESS_EQ]


@pytest.mark.parametrize("prec,tol,n,RT,amp,seed", [(0, 1e-10, 48, 0.9, 0.1, 1), (1, 1e-6, 48, 0.9, 0.1, 1),
                                                    (0, 1e-10, 10, 0.42, 0.15, 6)])
def test_previous_step_guess(prec, tol, n, RT, amp, seed):
    """The linearised start plus each cell's stored correction from the
    previous step (Sec. II.D's stored multipliers) converges to the fields of
    Eq. (IID13)'s start; its first step is the linearised path itself; on the
    smooth 48^3 box the FP64 solves need fewer Newton updates than from the
    linearised start; around RT = 0.42 refined cells keep no correction and
    start from the linearised guess."""
    import paper_2508_06911_amd as lb
    _case("3D previous-step guess, precision %d, %d^3, RT %.2f, 7 steps" % (prec, n, RT))
    cfg, prim = li.smooth_periodic3(seed, n=n, amp=amp, RT=RT)
    m = _mom(cfg, prim)
    outs, its = {}, {}
    for g in (lb.GUESS_EQ, lb.GUESS_LIN, lb.GUESS_PREV):
        c = lb.Lelbm(cfg, m, precision=prec, guess=g)
        c.step(1)
        outs[(g, 1)] = c.read_moments()
        st = c.step(6)
        outs[g] = c.read_moments()
        its[g] = st["it_mean_f"] + st["it_mean_g"]
        c.close()
    err = rel_linf(outs[lb.GUESS_PREV], outs[lb.GUESS_EQ])
    print("PREV vs EQ %.3g; Newton updates per cell (f + g) in steps 2-7: EQ %.2f LIN %.2f PREV %.2f"
          % (err, its[lb.GUESS_EQ], its[lb.GUESS_LIN], its[lb.GUESS_PREV]), flush=True)
    assert err < tol
    if prec == 0 and RT > 4.0 / 9.0:
        assert its[lb.GUESS_PREV] < its[lb.GUESS_LIN]
    assert np.array_equal(outs[(lb.GUESS_PREV, 1)], outs[(lb.GUESS_LIN, 1)])


@pytest.mark.parametrize("prec,tol,RT,amp,seed", [(0, 1e-10, 0.42, 0.15, 6), (1, 1e-6, 0.42, 0.15, 6),
                                                  (0, 1e-10, 0.03, 0.05, 8)])
def test_refined_stencils_parity(prec, tol, RT, amp, seed):
    """Cold boxes with refined stencils (Eqs. IIC9-11, 8 children per level):
    around RT = 0.42 cells on both sides of the threshold 4/9 share tiles (all
    moments per slot), at RT ~ 0.03 every cell is refined twice."""
    import paper_2508_06911_amd as lb
    _case("3D refined stencils RT %.2f precision %d, 8 x 7 x 6, 3 steps" % (RT, prec))
    cfg, prim = li.smooth_periodic3(seed, n=8, ny=7, nz=6, amp=amp, RT=RT)
    ref, rs = _oracle(cfg, prim, 3)
    ctx = lb.Lelbm(cfg, _mom(cfg, prim), precision=prec)
    st = ctx.step(3)
    out = ctx.read_moments()
    ctx.close()
    err = rel_linf(out, ref)
    print("rel Linf vs oracle %.3g; q min/mean/max %d / %.1f / %d (oracle %d / %.1f / %d)"
          % (err, st["q_min"], st["q_mean"], st["q_max"], rs["q_min"], rs["q_mean"], rs["q_max"]), flush=True)
    assert err < tol
    assert st["q_max"] == rs["q_max"] and st["q_min"] == rs["q_min"]


def _reach(m, K):
    """Largest landing displacement per axis of any cell's stencil: |u_a| + R
    + 1/2 with R = round(4 sqrt(RT)) (Eq. IIC6, r_min 2), RT the larger of the
    translational and the phonon temperature, plus one cell of margin."""
    rho = m[0]
    u = m[1:4] / rho
    rt_tr = ((m[4] + m[7] + m[9]) / rho - (u * u).sum(axis=0)) / 3
    rt = max(rt_tr.max(), (m[13] / (rho * K)).max())
    R = max(int(np.floor(4 * np.sqrt(rt) + 0.5)), 2)
    return int(np.ceil(np.abs(u).max() + R + 0.5)) + 1


@pytest.mark.parametrize("prec,guess,tol", [(1, "lin", 1e-6), (0, "eq", 1e-10)])
def test_full_size_box_sampled_windows(prec, guess, tol):
    """The 96^3 box of the 3D benchmark (seed 10, RT ~ 1, default scratch
    budget, the benchmark's precision and Newton start): after two GPU steps,
    a third is compared on sampled windows (one across the periodic corner)
    with an oracle step of the same window as an open box; cells farther
    than the reach from the window's faces only receive from inside it."""
    import paper_2508_06911_amd as lb
    _case("3D 96^3 sampled windows, precision %d, guess %s" % (prec, guess))
    n = 96
    cfg, prim = li.smooth_periodic3(10, n=n, amp=0.1, RT=1.0)
    g = lb.GUESS_LIN if guess == "lin" else lb.GUESS_EQ
    c = lb.Lelbm(cfg, _mom(cfg, prim), precision=prec, guess=g)
    c.step(2)
    mk = c.read_moments()
    c.step(1)
    mk1 = c.read_moments()
    c.close()
    reach = _reach(mk, cfg["K"])
    W = 2 * reach + 6
    rng = np.random.default_rng(1)
    corners = [(n - W // 2, n - W // 2, n - W // 2), (n // 2 - W // 2,) * 3]
    corners += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(3)]
    mk = mk.reshape(17, n, n, n)
    mk1 = mk1.reshape(17, n, n, n)
    inner = slice(reach, W - reach)
    for x0, y0, z0 in corners:
        xs, ys, zs = [np.arange(v, v + W) % n for v in (x0, y0, z0)]
        win = mk[:, zs][:, :, ys][:, :, :, xs].reshape(17, -1)
        st, out, _, _ = oracle.step(dict(cfg, nx=W, ny=W, nz=W, open=True), win, 1)
        assert st == 0
        out = out.reshape(17, W, W, W)[:, inner, inner, inner].reshape(17, -1)
        ref = mk1[:, zs[inner]][:, :, ys[inner]][:, :, :, xs[inner]].reshape(17, -1)
        err = rel_linf(ref, out)
        print("window at (%d, %d, %d), %d^3 compared: rel Linf %.3g" % (x0, y0, z0, W - 2 * reach, err), flush=True)
        assert err < tol
