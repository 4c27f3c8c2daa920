"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
independent of the oracle's own formulas: printed worked examples, direct
definitions of central moments, closed-form equilibria, a brute-force dual
minimiser, conservation, symmetry, the exact Riemann solution and measured
transport coefficients."""
import os

import numpy as np
import pytest
from scipy.optimize import minimize

import lelbm_inputs as li
import oracle
from oracle import riemann

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def prim_moments(cfg, prim):
    return oracle.moments_from_primitives(cfg["dim"], cfg["K"], prim["rho"], prim["ux"],
                                          prim["uy"], prim["RT"])


# --------------------------------------------------------------------------
# Lagrangian acoustic stencil (Sec. II.C)
# --------------------------------------------------------------------------
def test_las_worked_examples():
    rows = np.loadtxt(os.path.join(GOLDEN, "las_worked_examples.txt"))
    for RT, ux, uy, q, colat in rows:
        c, dC, d, h = oracle.las(2, (ux, uy), RT)
        assert len(dC) == int(q)
        if not np.isnan(colat):
            R = oracle.las_radius(RT)
            assert abs(np.hypot(ux, uy) + R - colat) < 0.05     # Eq. (IIC7), printed to 3 digits


def test_las_brute_force_disk():
    """Base stencil = every integer point within R + 1/2 of u, by brute force."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        RT = rng.uniform(0.5, 12.0)
        u = rng.uniform(-20, 20, size=2)
        c, dC, d, h = oracle.las(2, u, RT)
        R = max(int(np.floor(4 * np.sqrt(RT) + 0.5)), 2)
        g = np.arange(-60, 61)
        X, Y = np.meshgrid(g, g)
        inside = (X - u[0]) ** 2 + (Y - u[1]) ** 2 <= (R + 0.5) ** 2
        assert len(dC) == inside.sum()
        assert np.all(dC == 1.0) and np.all(d == c)


def test_las_1d_count_and_refinement_volume():
    # 1D: the interval |c - u| <= R + 1/2 holds 2R + 1 integers (u not half-integer)
    for RT in (0.5, 1.0, 3.7, 20.0):
        R = oracle.las_radius(RT)
        c, dC, d, h = oracle.las(1, (0.3, 0.0), RT)
        assert oracle.las_levels(RT) == 0
        assert len(dC) == 2 * R + 1
    # refinement splits velocity volume without changing it (Eq. IIC11) and
    # children of an integer parent land in the parent's cell
    for dim, u, RT in ((2, (3.7, 4.1), 0.2), (2, (-1.2, 0.4), 0.3), (1, (0.45, 0.0), 0.05), (2, (0.1, 0.2), 0.04)):
        c, dC, d, h = oracle.las(dim, u, RT)
        assert oracle.las_levels(RT) >= 1
        assert abs(dC.sum() - len(np.unique(d, axis=0))) < 1e-12
        assert np.all(np.floor(c[:, 0] + 0.5) == d[:, 0])
        if dim == 2:
            assert np.all(np.floor(c[:, 1] + 0.5) == d[:, 1])
        # each refined point sits at the centre of its own velocity cell of side h
        assert np.allclose(dC, h ** dim)


def test_las_levels_threshold():
    # N_r = [1/(3 sqrt(RT))]: refinement switches on below RT = 4/9 (Eq. IIC9)
    assert oracle.las_levels(0.45) == 0
    assert oracle.las_levels(0.44) == 1
    assert oracle.las_levels(0.05) == 1
    assert oracle.las_levels(0.049) == 2


# --------------------------------------------------------------------------
# Collision (Sec. II.B, App. D)
# --------------------------------------------------------------------------
def _random_populations(dim, rng, q=60):
    c = rng.uniform(-4, 4, size=(q, 2)) + np.array([1.3, -0.7])
    if dim == 1:
        c[:, 1] = 0.0
    f = rng.uniform(0.1, 1.0, size=q)
    g = rng.uniform(0.1, 1.0, size=q)
    return c, f, g


def _raw_moments(dim, c, f, g):
    x, y = c[:, 0], c[:, 1]
    cc = x * x + y * y
    if dim == 1:
        return np.array([f.sum(), (x * f).sum(), (x * x * f).sum(), (x ** 3 * f).sum(), g.sum(), (x * g).sum()])
    return np.array([f.sum(), (x * f).sum(), (y * f).sum(), (x * x * f).sum(), (x * y * f).sum(),
                     (y * y * f).sum(), (cc * x * f).sum(), (cc * y * f).sum(), g.sum(), (x * g).sum(),
                     (y * g).sum()])


@pytest.mark.parametrize("dim", [1, 2])
def test_noneq_central_moments_match_direct_sums(dim):
    """Eq. (IIB9) from raw moments must equal the direct central sums of
    Eq. (IIB8) (relative velocity c - u) minus the equilibrium central moments
    of Eq. (IIB7g-j)."""
    rng = np.random.default_rng(7 + dim)
    K = 3.0 if dim == 2 else 4.0
    cfg = dict(li.hotbox(1.0, n=4, dim=dim)[0])
    cfg["K"] = K
    for _ in range(5):
        c, f, g = _random_populations(dim, rng)
        mom = _raw_moments(dim, c, f, g)
        out = oracle.collide(cfg, mom)
        rho = f.sum()
        u = np.array([(c[:, 0] * f).sum(), (c[:, 1] * f).sum()]) / rho
        ct = c - u
        RT = ((ct[:, 0] ** 2 * f).sum() + (ct[:, 1] ** 2 * f).sum() + g.sum()) / rho / (dim + K)
        assert np.isclose(out["rho"], rho, rtol=1e-13)
        assert np.isclose(out["RT"], RT, rtol=1e-12)
        x, y = ct[:, 0], ct[:, 1]
        Pxx = (x * x * f).sum() - rho * RT
        assert np.isclose(out["Pxx"], Pxx, rtol=1e-10, atol=1e-12)
        Qx = ((x * x + y * y) * x * f).sum()
        assert np.isclose(out["Qx"], Qx, rtol=1e-10, atol=1e-11)
        assert np.isclose(out["g0"], g.sum() - rho * K * RT, rtol=1e-10, atol=1e-12)
        assert np.isclose(out["hx"], (x * g).sum(), rtol=1e-10, atol=1e-12)
        if dim == 2:
            assert np.isclose(out["Pxy"], (x * y * f).sum(), rtol=1e-10, atol=1e-12)
            assert np.isclose(out["Pyy"], (y * y * f).sum() - rho * RT, rtol=1e-10, atol=1e-12)
            assert np.isclose(out["Qy"], ((x * x + y * y) * y * f).sum(), rtol=1e-10, atol=1e-11)
            assert np.isclose(out["hy"], (y * g).sum(), rtol=1e-10, atol=1e-12)
        # energy identity: trace of P equals -g0 (RT is defined with G0)
        assert np.isclose(out["Pxx"] + out["Pyy"], -out["g0"], rtol=1e-9, atol=1e-11)
        # Knudsen number of Eq. (D2) from the same direct central sums: the
        # larger of the second-order ratio (all D^2 stress components and g0)
        # and the third-order ratio (heat fluxes of both species, RT^(3/2))
        P = [[Pxx, (x * y * f).sum()], [(x * y * f).sum(), (y * y * f).sum() - rho * RT]]
        Q = [Qx, ((x * x + y * y) * y * f).sum()]
        h = [(x * g).sum(), (y * g).sum()]
        g0 = g.sum() - rho * K * RT
        A = (sum(abs(P[a][b]) for a in range(dim) for b in range(dim)) + abs(g0)) / (rho * (dim + K) * RT)
        B = sum(abs(Q[a]) + abs(h[a]) for a in range(dim)) / (rho * (dim + K + 2) * RT ** 1.5)
        assert np.isclose(out["kn"], max(A, B), rtol=1e-9)


def test_targets_relaxation_and_splits():
    """Post-collision targets of Eq. (IIB16): omega = 1 gives the equilibrium
    central moments; omega = 0 keeps the input central moments; the third-order
    per-axis pieces sum to the contracted moment (Eq. IIB14)."""
    rng = np.random.default_rng(11)
    cfg = dict(li.hotbox(1.0, n=4)[0])
    cfg["kn_limiter"] = 0
    c, f, g = _random_populations(2, rng)
    mom = _raw_moments(2, c, f, g)
    for om in (1.0, 0.0):
        cfg.update(omega_f=om, omega_b=om, omega_h=om)
        out = oracle.collide(cfg, mom)
        rho, RT, K = out["rho"], out["RT"], cfg["K"]
        u = np.array([out["ux"], out["uy"]])
        ct = c - u
        x, y = ct[:, 0], ct[:, 1]
        if om == 1.0:
            assert np.allclose(out["m"], [1, 0, 0, RT, 0, RT, 0, 0, 0, 0], atol=1e-13)
            assert np.allclose(out["n"], [1, 0, 0, RT, 0, RT], atol=1e-13)
        else:
            assert np.allclose(out["m"][3:6], [(x * x * f).sum() / rho, (x * y * f).sum() / rho,
                                               (y * y * f).sum() / rho], rtol=1e-10)
            Q = np.array([((x * x + y * y) * x * f).sum(), ((x * x + y * y) * y * f).sum()])
            assert np.isclose(out["m"][6] + out["m"][8], Q[0] / rho, rtol=1e-10)
            assert np.isclose(out["m"][7] + out["m"][9], Q[1] / rho, rtol=1e-10)
            assert np.isclose(out["m"][6], 3 * out["m"][8], rtol=1e-12)
            assert np.isclose(out["n"][0], g.sum() / (rho * K * RT), rtol=1e-10)
            assert np.isclose(out["n"][1], (x * g).sum() / (rho * K * RT), rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("kn,expect", [(0.005, "w"), (10 ** -1.5, "mid"), (0.2, "one")])
def test_knudsen_limiter_branches(kn, expect):
    """App. D: unchanged below Kn = 0.01, halfway (in log10) at Kn = 10^-1.5,
    omega_H = 1 above Kn = 0.1."""
    cfg = dict(li.hotbox(1.0, n=4)[0])
    cfg.update(omega_f=1.8, omega_b=1.0, omega_h=1.6, kn_limiter=1)
    rho, RT, K = 1.3, 0.9, cfg["K"]
    mom = oracle.moments_from_primitives(2, K, [rho], [0.2], [-0.1], [RT])[:, 0]
    # pure shear non-equilibrium P_xy = eps: Kn = 2|eps| / (rho (D+K) RT)
    eps = kn * rho * (2 + K) * RT / 2
    mom = mom.copy()
    mom[4] += eps
    out = oracle.collide(cfg, mom)
    assert np.isclose(out["kn"], kn, rtol=1e-10)
    w = {"w": (1.8, 1.6), "mid": (1.4, 1.3), "one": (1.0, 1.0)}[expect]
    assert np.isclose(out["om_f"], w[0], rtol=1e-12)
    assert np.isclose(out["om_h"], w[1], rtol=1e-12)
    assert out["om_b"] == 1.0


@pytest.mark.parametrize("kn,expect", [(0.005, "w"), (10 ** -1.5, "mid"), (0.2, "one")])
@pytest.mark.parametrize("which", ["Qx", "hx", "Qy+hx"])
def test_knudsen_heat_flux_ratio_branches(kn, expect, which):
    """App. D, Eq. (D2), third-order ratio: an equilibrium cell whose only
    non-equilibrium is a heat flux of the fluon (M_Dx raises Q_x one for one)
    or of the phonon (G_x raises h_x one for one), or both on different axes
    (the ratio sums their magnitudes), normalised by rho (D+K+2) RT^(3/2).
    The limiter then takes the branch values of the text after Eq. (D3b)."""
    cfg = dict(li.hotbox(1.0, n=4)[0])
    cfg.update(omega_f=1.8, omega_b=1.2, omega_h=1.6, kn_limiter=1)
    rho, RT, K = 0.7, 2.3, cfg["K"]
    mom = oracle.moments_from_primitives(2, K, [rho], [0.4], [-0.3], [RT])[:, 0].copy()
    total = kn * rho * (2 + K + 2) * RT ** 1.5
    if which == "Qx":
        mom[6] += total                     # M_Dx
    elif which == "hx":
        mom[9] -= total                     # G_x (sign does not matter)
    else:
        mom[7] += 0.25 * total              # M_Dy -> Q_y
        mom[9] += 0.75 * total              # G_x -> h_x
    out = oracle.collide(cfg, mom)
    assert np.isclose(out["kn"], kn, rtol=1e-9)
    assert abs(out["Pxx"]) < 1e-12 and abs(out["g0"]) < 1e-12      # second-order ratio is zero
    w = {"w": (1.8, 1.2, 1.6), "mid": (1.4, 1.1, 1.3), "one": (1.0, 1.0, 1.0)}[expect]
    assert np.isclose(out["om_f"], w[0], rtol=1e-12)
    assert np.isclose(out["om_b"], w[1], rtol=1e-12)
    assert np.isclose(out["om_h"], w[2], rtol=1e-12)


# --------------------------------------------------------------------------
# Entropic population reconstruction (Sec. II.D)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("RT", [0.2, 0.5, 1.0, 4.0, 32.0])
def test_epr_equilibrium_converges_fast(RT):
    """Equilibrium targets from the guess of Eq. (IID13) converge in fewer than
    five Newton updates (Sec. II.D), to populations that reproduce them."""
    u = (0.37, -0.21)
    c, dC, d, h = oracle.las(2, u, RT)
    for nb, target in ((10, [1, 0, 0, RT, 0, RT, 0, 0, 0, 0]), (6, [1, 0, 0, RT, 0, RT])):
        st, lam, pop, it = oracle.epr(2, c, dC, u, RT, np.array(target, dtype=float))
        assert st == 0
        assert it - 1 < 5          # iterations counted here include the polishing update
        assert np.all(pop > 0)
        ct = c - np.array(u)
        T = _basis(ct, nb)
        assert np.allclose(T.T @ pop, target, atol=1e-13 * max(1, RT ** 1.5))


def _basis(ct, nb):
    x, y = ct[:, 0], ct[:, 1]
    cols = [np.ones_like(x), x, y, x * x, x * y, y * y, x ** 3, x * x * y, x * y * y, y ** 3]
    return np.stack(cols[:nb], axis=1)


def test_epr_matches_brute_force_dual_minimiser():
    """The reconstruction is the unique minimiser of the convex dual
    Phi(l) = sum_i dC_i exp(-1 - l.T_i) + l.m; an independent quasi-Newton
    minimiser of Phi must find the same multipliers."""
    rng = np.random.default_rng(5)
    for trial in range(4):
        RT = rng.uniform(0.6, 2.0)
        u = rng.uniform(-1, 1, size=2)
        c, dC, d, h = oracle.las(2, u, RT)
        ct = c - u
        T = _basis(ct, 10)
        # realizable target: moments of a perturbed Gaussian on the same stencil
        w = dC * np.exp(-(ct ** 2).sum(1) / (2 * RT)) * (1 + 0.2 * np.tanh(rng.standard_normal(len(dC))))
        w /= w.sum()
        target = T.T @ w
        st, lam, pop, it = oracle.epr(2, c, dC, u, RT, target)
        assert st == 0

        def phi(l):
            return (dC * np.exp(-1 - T @ l)).sum() + l @ target

        def grad(l):
            return -(T.T @ (dC * np.exp(-1 - T @ l))) + target

        l0 = oracle.epr_initial(2, 10, RT)
        res = minimize(phi, l0, jac=grad, method="BFGS", options={"gtol": 1e-13, "maxiter": 5000})
        assert np.allclose(res.x, lam, rtol=1e-5, atol=1e-6)
        assert np.allclose(T.T @ pop, target, atol=1e-12)
        assert np.all(pop > 0)


def test_epr_reports_unrealizable_moments():
    """A target outside the moment cone of the stencil has no positive
    reconstruction: the solve must fail loudly (status EEPR)."""
    RT = 1.0
    u = (0.0, 0.0)
    c, dC, d, h = oracle.las(2, u, RT)
    target = np.array([1, 0, 0, -0.5, 0, RT, 0, 0, 0, 0], dtype=float)   # negative variance
    st, lam, pop, it = oracle.epr(2, c, dC, u, RT, target)
    assert st == oracle.EEPR


# --------------------------------------------------------------------------
# Whole step (Sec. II.E, III.A)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("u,RT,tol", [((0.37, -0.21), 1.0, 1e-13), ((2.5, -0.5), 0.3, 1e-13),
                                      ((10.0, 10.0), 0.5, 2e-11)])
def test_uniform_state_is_invariant(u, RT, tol):
    """A uniform equilibrium is a fixed point.  At |u| = 14 the raw-to-central
    transform of Eq. (IIB9b) cancels terms of size rho |u|^3, so rounding of
    the raw moments reappears as a ~1e-12 heat flux that omega_h = 2 does not
    damp; the bound is looser there."""
    cfg, prim = li.hotbox(RT, n=6, ny=5, u=u)
    m = prim_moments(cfg, prim)
    st, out, stats, done = oracle.step(cfg, m, 3)
    assert st == 0
    assert np.max(np.abs(out - m) / np.abs(m).max(axis=1, keepdims=True)) < tol


@pytest.mark.parametrize("dim", [1, 2])
def test_conservation_periodic(dim):
    cfg, prim = li.smooth_periodic(1, n=16 if dim == 2 else 48, ny=10, dim=dim)
    m = prim_moments(cfg, prim)
    cur = m
    for _ in range(4):
        st, nxt, stats, done = oracle.step(cfg, cur, 1)
        assert st == 0
        mass = [cur[0].sum(), nxt[0].sum()]
        assert abs(mass[1] - mass[0]) / mass[0] < 1e-13
        for k in range(1, dim + 1):
            assert abs(nxt[k].sum() - cur[k].sum()) / mass[0] < 1e-13
        if dim == 2:
            e0, e1 = (cur[3] + cur[5] + cur[8]).sum(), (nxt[3] + nxt[5] + nxt[8]).sum()
        else:
            e0, e1 = (cur[2] + cur[4]).sum(), (nxt[2] + nxt[4]).sum()
        assert abs(e1 - e0) / e0 < 1e-13
        cur = nxt


def test_positivity_and_limiter_on_quadrants():
    cfg, prim = li.quadrants(4, n=24)
    m = prim_moments(cfg, prim)
    st, out, stats, done = oracle.step(cfg, m, 4)
    assert st == 0 and done == 4
    assert stats["limited"] > 0            # shocks switch the limiter on
    rho = out[0]
    assert np.all(rho > 0)


def test_integer_galilean_boost_is_exact():
    """Shifting u by an integer shifts every stencil by that integer, so the
    boosted run equals the unboosted run advected by one cell per step."""
    cfg, prim = li.smooth_periodic(2, n=12, ny=10)
    m = prim_moments(cfg, prim)
    st0, out0, *_ = oracle.step(cfg, m, 2)
    prim_b = dict(prim)
    prim_b["ux"] = prim["ux"] + 1.0
    mb = prim_moments(cfg, prim_b)
    st1, out1, *_ = oracle.step(cfg, mb, 2)
    assert st0 == 0 and st1 == 0

    def primitives(o):
        rho = o[0]
        ux, uy = o[1] / rho, o[2] / rho
        RT = ((o[3] + o[5] + o[8]) / rho - ux * ux - uy * uy) / (2 + cfg["K"])
        return np.stack([rho, ux, uy, RT])

    a = primitives(out0.reshape(11, 10, 12))
    b = primitives(out1.reshape(11, 10, 12))
    b_shift = np.roll(b, -2, axis=2)
    b_shift[1] -= 1.0
    assert np.max(np.abs(a - b_shift)) < 1e-11


def test_mirror_symmetry():
    cfg, prim = li.smooth_periodic(3, n=12, ny=8)
    m = prim_moments(cfg, prim).reshape(11, 8, 12)
    st0, out0, *_ = oracle.step(cfg, m.reshape(11, -1), 2)
    # mirror x -> -x: odd-in-x moments flip sign
    sign = np.array([1, -1, 1, 1, -1, 1, -1, 1, 1, -1, 1])[:, None, None]
    mm = (m[:, :, ::-1] * sign).reshape(11, -1)
    st1, out1, *_ = oracle.step(cfg, mm, 2)
    back = (out1.reshape(11, 8, 12)[:, :, ::-1] * sign).reshape(11, -1)
    scale = np.abs(out0).max(axis=1, keepdims=True)
    assert np.max(np.abs(back - out0) / scale) < 1e-12


def _run_riemann(cfg, prim, frac=0.4):
    m = prim_moments(cfg, prim)
    N = cfg["nx"]
    L = (prim["rho"][0, 0], prim["ux"][0, 0], prim["rho"][0, 0] * prim["RT"][0, 0])
    R = (prim["rho"][0, -1], prim["ux"][0, -1], prim["rho"][0, -1] * prim["RT"][0, -1])
    smin, smax = riemann.wave_speeds(L, R)
    steps = int(frac * (N / 2) / max(abs(smin), abs(smax)))
    st, out, stats, done = oracle.step(cfg, m, steps)
    x = np.arange(N) + 0.5
    ex = riemann.sample(L, R, (x - N / 2) / steps)
    return st, np.abs(out[0] - ex[0]).mean() / (ex[0].max() - ex[0].min()), stats


def test_riemann_solver_textbook_values():
    # Sod star state, a standard value of the exact solver: p* = 0.30313, u* = 0.92745
    ps, us = riemann.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert abs(ps - 0.30313) < 1e-5 and abs(us - 0.92745) < 1e-5


def test_sod_converges_to_exact_solution():
    """Sod's shock tube (Sec. V.A, Eq. VIA1) against the exact Riemann solution;
    L1 density error (normalised by the density range) falls with resolution."""
    errs = []
    for N in (200, 400):
        cfg, prim = li.riemann1d(n=N, states=((1.0, 0.0, 1.0), (0.125, 0.0, 0.8 * 0.125)), pad=32)
        st, e, stats = _run_riemann(cfg, prim)
        assert st == 0
        errs.append(e)
    assert errs[1] < errs[0] < 0.015


@pytest.mark.parametrize("seed", range(5))
def test_two_state_inputs_match_exact_riemann(seed):
    """The seeded two-state inputs (density and pressure U[0.1, 1]) against the
    exact solution, before any wave reaches the outflow pads."""
    errs = []
    for N in (250, 500):
        cfg, prim = li.riemann1d(seed, n=N)
        st, e, stats = _run_riemann(cfg, prim)
        assert st == 0
        errs.append(e)
    assert errs[1] < errs[0]
    assert errs[1] < 0.02


def test_lax_courant_numbers_and_accuracy():
    """Lax problem (Sec. V.B): lattice Courant numbers quoted by the paper and
    agreement with the exact solution with and without acoustic scaling."""
    rows = np.loadtxt(os.path.join(GOLDEN, "lax_courant.txt"))
    errs = []
    for scale, rtmax, colat in rows:
        cfg, prim = li.riemann1d(n=1000, states=((0.445, 0.698, 3.528), (0.5, 0.0, 0.517)),
                                 scale=scale, pad=48)
        assert abs(prim["RT"].max() - rtmax) < 0.01
        m = prim_moments(cfg, prim)
        steps = int(round(0.14 / (scale / 1000)))
        st, out, stats, done = oracle.step(cfg, m, steps)
        assert st == 0
        assert abs(stats["colat_max"] - colat) < 0.6
        L = (0.445, 0.698 * scale, 3.528 * scale ** 2)
        R = (0.5, 0.0, 0.517 * scale ** 2)
        x = np.arange(1000) + 0.5
        ex = riemann.sample(L, R, (x - 500) / steps)
        errs.append(np.abs(out[0] - ex[0]).mean() / (ex[0].max() - ex[0].min()))
    assert max(errs) < 0.02
    assert errs[1] < errs[0]          # lower lattice temperature is less diffusive


@pytest.mark.parametrize("RT", [0.5, 1.0])
def test_shear_wave_viscosity(RT):
    """Sec. IV.A: decay of a shear wave gives nu_s = RT (1/omega_f - 1/2)
    (App. C, Eq. C8a); the paper reports +-10%."""
    L, nu = 64, 0.1
    cfg, prim = li.shear_wave(L=L, ny=2, RT=RT, nu=nu)
    m = prim_moments(cfg, prim)
    k = 2 * np.pi / L
    t = int(0.5 / (nu * k * k))
    st, out, stats, done = oracle.step(cfg, m, t)
    assert st == 0
    uy = out[2] / out[0]
    nu_m = -np.log(np.abs(uy).max() / 1e-3) / (k * k * t)
    assert abs(nu_m / nu - 1) < 0.03


@pytest.mark.parametrize("RT", [0.5, 1.0])
def test_thermal_wave_diffusivity(RT):
    """Sec. IV.B: decay of an isobaric density wave gives the diffusivity
    alpha = kappa / (rho C_p) = RT (1/omega_h - 1/2) (Eq. C8c, B22b)."""
    L, a = 64, 0.1
    cfg, prim = li.shear_wave(L=L, ny=2, RT=RT, nu=a, amp=0.0)
    x = (np.arange(L) + 0.5)[None, :]
    rho = (1.0 + 0.01 * np.cos(2 * np.pi * x / L)) * np.ones((2, 1))
    prim["rho"] = rho
    prim["RT"] = RT / rho
    m = prim_moments(cfg, prim)
    k = 2 * np.pi / L
    t = int(0.5 / (a * k * k))
    st, out, stats, done = oracle.step(cfg, m, t)
    assert st == 0
    am = -np.log(np.abs(out[0] - 1.0).max() / 0.01) / (k * k * t)
    assert abs(am / a - 1) < 0.10


@pytest.mark.parametrize("RT", [0.5, 8.0])
def test_acoustic_pulse_sound_speed(RT):
    """Sec. IV.D: a small pressure pulse travels at c_s = sqrt(gamma RT)."""
    cfg, prim = li.acoustic_pulse(n=600, RT=RT, pad=40)
    m = prim_moments(cfg, prim)
    cs = np.sqrt(1.4 * RT)
    t = int(200 / cs)
    st, out, stats, done = oracle.step(cfg, m, t)
    assert st == 0
    rho = out[0]
    ux = out[1] / rho
    RTm = ((out[2] + out[4]) / rho - ux ** 2) / (1 + cfg["K"])
    p = rho * RTm
    x = np.arange(600) + 0.5
    i = np.argmax(np.where(x > 300, p, -1))
    y0, y1, y2 = p[i - 1], p[i], p[i + 1]
    xp = x[i] + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)
    assert abs((xp - 300) / t / cs - 1) < 0.01


def test_failure_is_reported_not_clamped():
    cfg, prim = li.hotbox(1.0, n=4, ny=4)
    m = prim_moments(cfg, prim)
    m[3, 5] = -10.0                     # negative energy in one cell -> RT < 0
    st, out, stats, done = oracle.step(cfg, m, 1)
    assert st == oracle.EEPR
    assert done == 0
    assert stats["fail_cell"] == 5


def _inflow_riemann(N, L, R, frac=0.8):
    """The whole tube starts in state R; the inflow face on the left holds the
    equilibrium of state L (Sec. III.A, Dirichlet).  With every wave of the
    Riemann problem (L, R) moving right, the exact solution for x > 0 is that
    problem's self-similar solution from x = 0, until its fastest wave nears
    the outflow pad.  States are physical (rho, u, p); the lattice takes
    RT_R = 0.5 by acoustic scaling."""
    s = np.sqrt(0.5 / (R[2] / R[0]))
    cfg, prim = li.riemann1d(n=N, states=(R, R), scale=s, pad=24)
    cfg["bc"] = ["inflow", "outflow", "periodic", "periodic"]
    cfg["in_rho"], cfg["in_u"], cfg["in_RT"] = L[0], (L[1] * s, 0.0), L[2] / L[0] * s * s
    Ll = (L[0], L[1] * s, L[2] * s * s)
    Rl = (R[0], R[1] * s, R[2] * s * s)
    smin, smax = riemann.wave_speeds(Ll, Rl)
    assert smin > 0                       # no wave runs back into the inflow pad
    steps = int(frac * N / smax)
    st, out, stats, done = oracle.step(cfg, prim_moments(cfg, prim), steps)
    x = np.arange(N) + 0.5
    ex = riemann.sample(Ll, Rl, x / steps)
    return st, np.abs(out[0] - ex[0]).mean() / (ex[0].max() - ex[0].min())


def test_inflow_face_drives_the_exact_riemann_solution():
    """A supersonic inflow (Mach 2.5) into gas at rest: the density behind the
    inflow face follows the exact Riemann solution, and the error falls under
    refinement.  A pad that copied the interior instead of holding the inflow
    equilibrium would leave the tube at rest."""
    L = (1.0, 2.5 * np.sqrt(1.4), 1.0)
    R = (0.4, 0.0, 0.25)
    errs = []
    for N in (200, 400):
        st, e = _inflow_riemann(N, L, R)
        assert st == 0
        errs.append(e)
    # first-order convergence (measured 1.26e-2 -> 6.5e-3 -> 3.2e-3 at N = 800)
    assert errs[1] < 1e-2 and errs[1] < 0.6 * errs[0]


@pytest.mark.parametrize("dim", [1, 2])
def test_uniform_inflow_state_is_invariant(dim):
    """A uniform state equal to the inflow state, between an inflow face and an
    outflow face, is a fixed point (both pads then hold that state)."""
    if dim == 1:
        cfg, prim = li.hotbox(0.8, n=40, u=(0.7, 0.0), dim=1)
    else:
        cfg, prim = li.hotbox(0.8, n=40, ny=24, u=(0.9, 0.3))
    cfg["bc"] = ["inflow", "outflow", "periodic", "periodic"]
    cfg["pad"] = 8
    cfg["in_rho"], cfg["in_u"], cfg["in_RT"] = 1.0, (prim["ux"][0, 0], prim["uy"][0, 0]), 0.8
    m = prim_moments(cfg, prim)
    st, out, stats, done = oracle.step(cfg, m, 4)
    assert st == 0
    assert np.abs(out - m).max() < 1e-13 * np.abs(m).max()


@pytest.mark.parametrize("xfaces,u,pad,fails", [
    ("open", (10.0, 0.37), 13, "left"),     # inflow pad: [u_x] + R = 10 + 4 = 14 > 13
    ("open", (10.0, 0.37), 14, None),
    ("periodic", (10.0, 0.4), 4, None),     # y pads: [u_y] + R = 4 <= 4 and R - [u_y] = 4 <= 4
    ("periodic", (10.0, -3.0), 6, "top"),   # top pad: R - [u_y] = 4 + 3 = 7 > 6
])
def test_pad_narrower_than_the_reach_is_rejected(xfaces, u, pad, fails):
    """Sec. III (Fig. 5): pads hold every source within reach of the interior.
    A pad narrower than the stencil's reach toward the interior is reported
    (EREACH), with the state of the last completed step left in place; the
    reach away from the interior does not count."""
    cfg, prim = li.hotbox(1.0, n=36, ny=20, u=u)
    if xfaces == "open":
        cfg["bc"] = ["inflow", "outflow", "periodic", "periodic"]
    else:
        cfg["bc"] = ["periodic", "periodic", "outflow", "outflow"]
    cfg["pad"] = pad
    cfg["in_rho"], cfg["in_u"], cfg["in_RT"] = 1.0, u, 1.0
    m = prim_moments(cfg, prim)
    st, out, stats, done = oracle.step(cfg, m, 2)
    if fails is None:
        assert st == 0 and done == 2
    else:
        assert st == oracle.EREACH and done == 0
        assert np.array_equal(out, m)
        sxn = 36 + (2 * pad if xfaces == "open" else 0)
        fx = stats["fail_cell"] % sxn - (pad if xfaces == "open" else 0)
        fy = stats["fail_cell"] // sxn - (0 if xfaces == "open" else pad)
        assert (fx < 0) if fails == "left" else (fy >= 20)


def test_pad_reach_exceeded_mid_run_keeps_the_last_state():
    """1D gas at RT = 1.2 (R = 4) between 4-cell outflow pads, with a hot slug
    in the middle: the compression wave heats the end cells past R = 4, and
    that step fails with EREACH, leaving the state after the steps before."""
    cfg, prim = li.hotbox(1.2, n=80, dim=1, u=(0.0, 0.0))
    cfg["bc"] = ["outflow", "outflow", "periodic", "periodic"]
    cfg["pad"] = 4
    x = np.arange(80) + 0.5
    prim["RT"] = np.where(np.abs(x - 40) < 6, 2.4, 1.2)[None, :]
    m = prim_moments(cfg, prim)
    st, out, stats, done = oracle.step(cfg, m, 80)
    assert st == oracle.EREACH and 0 < done < 80
    st2, out2, _, done2 = oracle.step(cfg, m, done)
    assert st2 == 0 and done2 == done
    assert np.array_equal(out, out2)
    rho, ux, _, RT = (out[0], out[1] / out[0], None, ((out[2] + out[4]) / out[0] - (out[1] / out[0]) ** 2) / 5.0)
    R = np.floor(4 * np.sqrt(RT) + 0.5)
    assert R[0] + np.floor(ux[0] + 0.5) > 4 or R[-1] - np.floor(ux[-1] + 0.5) > 4


# --------------------------------------------------------------------------
# Paths through slip walls and solid cells (Sec. III.B)
# --------------------------------------------------------------------------
def _obstacle_cfg(nx=14, ny=12, seed=0, density=0.15, bc=("periodic", "periodic", "slipwall", "slipwall")):
    cfg, _ = li.hotbox(1.0, n=nx, ny=ny)
    cfg["bc"] = list(bc)
    rng = np.random.default_rng(seed)
    cfg["solid"] = (rng.random((ny, nx)) < density).astype(np.uint8)
    return cfg


def test_walk_without_blockers_is_a_straight_path():
    cfg, _ = li.hotbox(1.0, n=9, ny=7)
    for (x, y, dx, dy) in [(0, 0, 3, -2), (8, 6, 4, 5), (4, 3, -9, 0), (2, 5, 0, -13)]:
        assert oracle.walk(cfg, x, y, dx, dy) == ((x + dx) % 9, (y + dy) % 7, 1, 1)


def test_walk_reflects_once_at_a_slip_wall_like_a_mirror():
    cfg, _ = li.hotbox(1.0, n=9, ny=7)
    cfg["bc"] = ["periodic", "periodic", "slipwall", "slipwall"]
    for y in range(7):
        for dy in range(-6, 7):
            t = y + dy
            ey, sg = (t, 1) if 0 <= t < 7 else ((-1 - t, -1) if t < 0 else (13 - t, -1))
            if 0 <= ey < 7:
                assert oracle.walk(cfg, 4, y, 2, dy) == (6, ey, 1, sg if dy else 1)


def test_walk_is_a_speed_preserving_bijection():
    """Every (cell, velocity) pair is reached by exactly one path, paths end
    in fluid cells, and reflections keep |c_x| and |c_y|: mass and energy
    are deposited exactly."""
    for seed in (0, 1, 2):
        cfg = _obstacle_cfg(seed=seed)
        sol = cfg["solid"]
        seen = set()
        n = 0
        for y in range(12):
            for x in range(14):
                if sol[y, x]:
                    continue
                for dy in range(-4, 5):
                    for dx in range(-4, 5):
                        ex, ey, sx, sy = oracle.walk(cfg, x, y, dx, dy)
                        assert 0 <= ex < 14 and 0 <= ey < 12 and not sol[ey, ex]
                        key = (ex, ey, sx * dx, sy * dy)
                        assert key not in seen
                        seen.add(key)
                        n += 1
        assert len(seen) == n


def test_gas_at_rest_around_obstacles_stays_at_rest():
    cfg = _obstacle_cfg(nx=16, ny=12, seed=3, density=0.1)
    cfg["RT"] = 0.8
    shape = (12, 16)
    prim = {"rho": np.ones(shape), "ux": np.zeros(shape), "uy": np.zeros(shape), "RT": np.full(shape, 0.8)}
    m = prim_moments(cfg, prim)
    st, out, stats, done = oracle.step(cfg, m, 3)
    assert st == 0
    fluid = cfg["solid"].ravel() == 0
    assert np.abs(out[:, ~fluid]).max() == 0.0
    err = np.abs(out[:, fluid] - m[:, fluid]).max(axis=1) / np.maximum(np.abs(m[:, fluid]).max(axis=1), 1.0)
    assert err.max() < 1e-13


def test_obstacles_conserve_mass_and_energy():
    cfg, prim = li.smooth_periodic(5, n=16, ny=12)
    rng = np.random.default_rng(7)
    cfg["solid"] = (rng.random((12, 16)) < 0.12).astype(np.uint8)
    fluid = cfg["solid"].ravel() == 0
    m = prim_moments(cfg, prim)
    m[:, ~fluid] = 0.0
    st, out, stats, done = oracle.step(cfg, m, 2)
    assert st == 0
    mass0, mass1 = m[0, fluid].sum(), out[0, fluid].sum()
    e0 = (m[3] + m[5] + m[8])[fluid].sum()
    e1 = (out[3] + out[5] + out[8])[fluid].sum()
    assert abs(mass1 - mass0) / mass0 < 1e-13
    assert abs(e1 - e0) / e0 < 1e-13
    # the obstacles exert a force: momentum changes
    assert abs(out[1, fluid].sum() - m[1, fluid].sum()) > 1e-6 * mass0


def test_flow_past_a_symmetric_obstacle_stays_symmetric():
    """A y-mirror-symmetric channel, obstacle and state stay y-symmetric
    (corner crossings are taken x first in both mirror images)."""
    nx, ny = 20, 12
    cfg, _ = li.hotbox(1.0, n=nx, ny=ny)
    cfg["bc"] = ["periodic", "periodic", "slipwall", "slipwall"]
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    X, Y = np.meshgrid(x, y)
    cfg["solid"] = (((X - 8.0) / 3.2) ** 2 + ((Y - 6.0) / 2.3) ** 2 <= 1.0).astype(np.uint8)
    assert (cfg["solid"] == cfg["solid"][::-1]).all()
    shape = (ny, nx)
    prim = {"rho": 1.0 + 0.05 * np.cos(2 * np.pi * X / nx) * np.cos(np.pi * (Y - 6.0) / 6.0),
            "ux": np.full(shape, 1.1), "uy": np.zeros(shape), "RT": np.full(shape, 0.9)}
    m = prim_moments(cfg, prim)
    st, out, *_ = oracle.step(cfg, m, 3)
    assert st == 0
    o = out.reshape(11, ny, nx)
    sign = np.array([1, 1, -1, 1, -1, 1, 1, -1, 1, 1, -1])[:, None, None]
    scale = np.abs(o).reshape(11, -1).max(axis=1)[:, None, None] + 1e-300
    assert np.max(np.abs(o[:, ::-1] * sign - o) / scale) < 1e-12


def test_solid_touching_a_pad_face_is_rejected():
    cfg, prim = li.channel(0, nx=64, ny=32, n_obstacles=1, size_scale=0.05, pad=8)
    cfg["solid"][:, 0] = 1
    st, *_ = oracle.step(cfg, prim_moments(cfg, prim), 1)
    assert st == -1


# --------------------------------------------------------------------------
# Oscillating point mass source (Sec. IV.C)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [1, 2])
def test_mass_source_adds_a_maxwellian_of_its_mass(dim):
    """Eqs. (VC6-VC8): a source of mass s adds to the post-collision central
    moments those of a Maxwellian of mass s at rest in the cell's frame at its
    temperature -- fluons s, 0, s RT delta, 0; phonons s K RT, 0,
    s K RT RT delta -- and the targets are normalised by rho + s (Eq. IIB18).
    Checked as the difference of the un-normalised targets with and without
    the source, on random non-equilibrium cells."""
    rng = np.random.default_rng(31 + dim)
    cfg = dict(li.hotbox(1.0, n=4, dim=dim)[0])
    cfg["omega_f"], cfg["omega_b"], cfg["omega_h"], cfg["kn_limiter"] = 1.3, 0.9, 1.6, 0
    K = cfg["K"]
    for s in (0.3, -0.05, 1e-6):
        c, f, g = _random_populations(dim, rng)
        mom = _raw_moments(dim, c, f, g)
        a = oracle.collide(cfg, mom)
        b = oracle.collide(cfg, mom, src=s)
        assert a["status"] == 0 and b["status"] == 0
        rho, RT = a["rho"], a["RT"]
        assert b["rho"] == rho and b["RT"] == RT
        dm = (rho + s) * b["m"] - rho * a["m"]
        dn = (rho + s) * K * RT * b["n"] - rho * K * RT * a["n"]
        if dim == 1:
            em, en = [s, 0, s * RT, 0], [s * K * RT, 0, s * K * RT * RT]
        else:
            em = [s, 0, 0, s * RT, 0, s * RT, 0, 0, 0, 0]
            en = [s * K * RT, 0, 0, s * K * RT * RT, 0, s * K * RT * RT]
        scale = rho * max(1.0, RT) ** 2
        assert np.allclose(dm, em, rtol=0, atol=1e-12 * scale)
        assert np.allclose(dn, en, rtol=0, atol=1e-12 * scale * K)


@pytest.mark.parametrize("dim", [1, 2])
def test_mass_source_exact_balances(dim):
    """Each step adds exactly the source's mass s_k = rate sin(omega t_k) with
    t_k = t0 + k (Eq. VC1 at the step's collision, Delta t = 1), the momentum
    s_k u and the energy trace s_k (|u|^2 + (D + K) RT) of the source cell at
    the step's start (a Maxwellian in its frame); everything else moves
    conservatively."""
    cfg, prim = li.smooth_periodic(2, n=16 if dim == 2 else 48, ny=10, dim=dim)
    sx, sy = (5, 3) if dim == 2 else (17, 0)
    rate, omega, t0 = 2e-3, 0.7, 3.0
    cfg["source"] = {"x": sx, "y": sy, "rate": rate, "omega": omega, "t0": t0}
    nx = cfg["nx"]
    cur = prim_moments(cfg, prim)
    K, D = cfg["K"], dim
    for k in range(5):
        c2 = dict(cfg)
        c2["source"] = dict(cfg["source"], t0=t0 + k)
        st, nxt, stats, done = oracle.step(c2, cur, 1)
        assert st == 0
        s = rate * np.sin(omega * (t0 + k))
        i = sy * nx + sx
        rho = cur[0, i]
        u = np.array([cur[1, i], cur[2, i] if dim == 2 else 0.0]) / rho
        if dim == 2:
            tr = cur[3] + cur[5] + cur[8]
            trn = nxt[3] + nxt[5] + nxt[8]
        else:
            tr = cur[2] + cur[4]
            trn = nxt[2] + nxt[4]
        RT = (tr[i] / rho - u @ u) / (D + K)
        assert abs((nxt[0].sum() - cur[0].sum()) - s) < 1e-11
        for a in range(dim):
            assert abs((nxt[1 + a].sum() - cur[1 + a].sum()) - s * u[a]) < 1e-11
        assert abs((trn.sum() - tr.sum()) - s * (u @ u + (D + K) * RT)) < 1e-10


def _source_pressure_amplitude(cfg, prim, t_fit0, t_fit1):
    """Runs the source case and fits a sin + cos + constant of the source's
    frequency to the pressure history of every cell over [t_fit0, t_fit1)."""
    m = prim_moments(cfg, prim)
    st, cur, _, _ = oracle.step(cfg, m, t_fit0)
    assert st == 0
    hist = []
    for k in range(t_fit0, t_fit1):
        c2 = dict(cfg)
        c2["source"] = dict(cfg["source"], t0=float(k))
        st, cur, _, _ = oracle.step(c2, cur, 1)
        assert st == 0
        rho = cur[0]
        ux = cur[1] / rho
        RT = ((cur[2] + cur[4]) / rho - ux ** 2) / (1 + cfg["K"])
        hist.append(rho * RT)
    t = np.arange(t_fit0, t_fit1) + 1.0
    w = cfg["source"]["omega"]
    A = np.stack([np.sin(w * t), np.cos(w * t), np.ones_like(t)], 1)
    coef = np.linalg.lstsq(A, np.array(hist), rcond=None)[0]
    return np.hypot(coef[0], coef[1])


def test_acoustic_source_bulk_viscosity_and_amplitude():
    """Sec. IV.C: a 1D oscillating point mass source radiates plane waves whose
    amplitude decays as exp(-alpha_x x) with alpha_x of Eq. (VC3); Eq. (VC4)
    then gives the bulk viscosity, to compare with RT (2/D - 2/(D+K))
    (1/omega_b - 1/2) (Eq. C8b); the paper's bar is +-10 %.  The source adds
    mass at the local temperature, a pressure source RT rate, so the
    linearised equations fix the radiated amplitude at RT rate / (2 c_s) on
    each side (before absorption)."""
    cfg, prim = li.acoustic_source(n=1200, RT=1.0, rate=1e-6, period=64.0, nu_b=0.8, nu=1e-3)
    amp = _source_pressure_amplitude(cfg, prim, 320, 448)
    cs = np.sqrt(1.4)
    w = cfg["source"]["omega"]
    xs = cfg["source"]["x"]
    d1, d2 = 40, 200
    for side in (1, -1):
        ax = -np.log(amp[xs + side * d2] / amp[xs + side * d1]) / (d2 - d1)
        nu_b = 2 * cs ** 3 / w ** 2 * ax - 0.4 * cfg["nu"]
        assert abs(nu_b / cfg["nu_b"] - 1) < 0.03
        a0 = amp[xs + side * d1] * np.exp(ax * d1)
        assert abs(a0 / (1.0 * 1e-6 / (2 * cs)) - 1) < 0.03


# --------------------------------------------------------------------------
# Oblique shock (Sec. V.F)
# --------------------------------------------------------------------------
def test_oblique_shock_relations_match_the_printed_table():
    """The textbook theta-beta-Mach relation and normal-shock jumps
    (oracle/oblique.py) reproduce the analytical rows of Table II to the
    printed precision (golden file)."""
    from oracle import oblique
    rows = np.loadtxt(os.path.join(GOLDEN, "oblique_shock_table2.txt"))
    for M, th, beta, m2, r, t in rows:
        b = oblique.weak_beta(M, np.deg2rad(th))
        m2c, rc, tc, _ = oblique.jumps(M, b, np.deg2rad(th))
        assert abs(np.rad2deg(b) - beta) < 6e-4
        assert abs(m2c - m2) < 6e-4 and abs(rc - r) < 6e-4 and abs(tc - t) < 6e-4


def test_oblique_shock_angle_and_jumps():
    """Sec. V.F: Mach-2 inflow turned by 5 degrees by a slip wall (RT 0.5,
    gamma 1.4): the shock angle within 0.1 degree of theta-beta-Mach and the
    post-shock density, temperature and Mach number within 0.3 % of the
    oblique-shock jumps."""
    from helpers import oblique_shock_measure
    cfg, prim = li.oblique_shock(mach=2.0, theta_deg=5.0, nx=160, ny=100)
    st, out, stats, done = oracle.step(cfg, prim_moments(cfg, prim), 200)
    assert st == 0
    meas, exact = oblique_shock_measure(out, cfg)
    assert abs(meas[0] - exact[0]) < 0.1
    for k in (1, 2, 3):
        assert abs(meas[k] / exact[k] - 1) < 3e-3


# --------------------------------------------------------------------------
# No-slip walls: extended bounce-back (Sec. III.B)
# --------------------------------------------------------------------------
def test_gas_at_rest_between_no_slip_walls_stays_at_rest():
    """Static no-slip walls: the image velocity equals the gas velocity (0), so
    the image populations leaving a wall mirror the absorbed ones and a gas
    at rest stays at rest."""
    cfg, prim = li.couette(ny=20, nx=6, RT=0.8, U=0.0)
    m = prim_moments(cfg, prim)
    st, out, stats, done = oracle.step(cfg, m, 5)
    assert st == 0
    assert np.abs(out - m).max() < 1e-13 * np.abs(m).max()


@pytest.mark.parametrize("u0", [(0.3, 0.2), (0.2, -1.5)])
def test_no_slip_walls_conserve_mass_and_phonon_energy(u0):
    """Eq. (IIIB15) rescales the image populations to the absorbed mass, so
    mass is exact at every step; momentum is not (the walls exert a force).
    The phonons are rescaled by their own ratio, so streaming keeps their
    zeroth moment too: exact over a first step from equilibrium, where the
    collision changes nothing (later collisions exchange energy between
    fluons and phonons).  The second case flows toward the bottom wall at 1.5
    cells per step with RT = 0.5: cells 2-4 rows above it absorb populations
    but no image population reaches back across the wall, so the absorbed
    ones are reflected specularly there."""
    cfg, prim = li.couette(ny=24, nx=8, RT=0.5, U=0.07, u0=u0)
    y = (np.arange(24) + 0.5)[:, None]
    prim["rho"] = 1.0 + 0.05 * np.sin(2 * np.pi * y / 24) * np.ones((1, 8))
    cur = prim_moments(cfg, prim)
    p0 = cur[1:3].sum(axis=1)
    nsteps = 3 if u0[1] > -1 else 1      # the fast case expands the top cell into the refined range
    for k in range(nsteps):
        st, nxt, stats, done = oracle.step(cfg, cur, 1)
        assert st == 0
        assert abs(nxt[0].sum() / cur[0].sum() - 1) < 1e-13
        if k == 0:
            assert abs(nxt[8].sum() / cur[8].sum() - 1) < 1e-13
        cur = nxt
    assert np.abs(cur[1:3].sum(axis=1) - p0).max() > 1e-3 * np.abs(p0).max()   # the walls exert a force


def test_couette_flow_profile():
    """Sec. III.B with a moving wall: between a static bottom wall and a top
    wall moving at U the steady profile is linear (uniform shear stress) and,
    by the symmetry of the set-up, antisymmetric about the mid-plane:
    u(y) + u(H - y) = U, with no normal flow.  The paper fixes no effective
    wall position for this scheme; the no-slip condition holds within one
    cell of the wall faces (the line through the profile reaches 0 and U
    there)."""
    U, ny = 0.1, 8
    cfg, prim = li.couette(ny=ny, nx=4, RT=0.5, U=U, nu=0.05)
    st, out, stats, done = oracle.step(cfg, prim_moments(cfg, prim), 3000)
    assert st == 0
    ux = (out[1] / out[0]).reshape(ny, 4).mean(axis=1)
    uy = (out[2] / out[0]).reshape(ny, 4)
    y = np.arange(ny) + 0.5                   # distance of the cell centres from the bottom wall face
    b, a = np.polyfit(y, ux, 1)
    assert np.abs(ux - (a + b * y)).max() < 5e-3 * U
    assert np.abs(ux + ux[::-1] - U).max() < 1e-4 * U
    assert np.abs(uy).max() < 1e-4 * U
    assert abs(-a / b) < 1.0 and abs((U - a) / b - ny) < 1.0
