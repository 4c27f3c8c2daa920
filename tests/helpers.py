"""Shared test helpers: run the same seeded input through the oracle and through
the GPU library (via its C ABI binding) and compare."""
import numpy as np

import oracle


def oracle_moments(cfg, prim):
    return oracle.moments_from_primitives(cfg["dim"], cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])


def gpu_moments(cfg, prim):
    import paper_2508_06911_amd as lb
    return lb.moments_from_primitives(cfg["dim"], cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])


def run_oracle(cfg, prim, steps, mom=None):
    m = oracle_moments(cfg, prim) if mom is None else mom
    st, out, stats, done = oracle.step(cfg, m, steps)
    assert st == 0, "oracle failed with %d at step %d cell %d" % (st, done, stats["fail_cell"])
    return out, stats


def run_gpu(cfg, prim, steps, precision=0, guess=0, mom=None):
    import paper_2508_06911_amd as lb
    m = gpu_moments(cfg, prim) if mom is None else mom
    ctx = lb.Lelbm(cfg, m, precision=precision, guess=guess)
    stats = ctx.step(steps) if steps > 0 else None
    out = ctx.read_moments()
    ctx.close()
    return out, stats


def rel_linf(a, b):
    """max over moments of max |a - b| / max(max |b_k|, max |b_0|)."""
    scale = np.maximum(np.abs(b).max(axis=1), np.abs(b[0]).max())
    return float((np.abs(a - b).max(axis=1) / scale).max())


def primitives(mom, dim, K):
    rho = mom[0]
    if dim == 1:
        ux = mom[1] / rho
        RT = ((mom[2] + mom[4]) / rho - ux * ux) / (1 + K)
        return rho, ux, np.zeros_like(ux), RT
    ux, uy = mom[1] / rho, mom[2] / rho
    RT = ((mom[3] + mom[5] + mom[8]) / rho - ux * ux - uy * uy) / (2 + K)
    return rho, ux, uy, RT


def oblique_shock_measure(mom, cfg, x0f=0.5, x1f=0.9):
    """Shock angle and post-shock state of an oblique-shock run (Sec. V.F).
    Per column in [x0f, x1f) of the width, the shock is where the density,
    scanned down from the top, first reaches the mid value between the
    inflow and the exact post-shock density; a line fitted through these
    points gives the shock's angle to the wall, plus theta the angle to the
    inflow.  Density, temperature and Mach number are averaged between the
    wall and the shock (3 cells above the wall to 8 below the shock).
    Returns (beta_deg, rho2/rho1, T2/T1, M2) measured and the exact values."""
    from oracle import oblique
    nx, ny, K = cfg["nx"], cfg["ny"], cfg["K"]
    rho = mom[0].reshape(ny, nx)
    ux = mom[1].reshape(ny, nx) / rho
    uy = mom[2].reshape(ny, nx) / rho
    RT = ((mom[3] + mom[5] + mom[8]).reshape(ny, nx) / rho - ux ** 2 - uy ** 2) / (2 + K)
    M, th = cfg["mach"], np.deg2rad(cfg["theta_deg"])
    beta = oblique.weak_beta(M, th)
    m2, r2, t2, _ = oblique.jumps(M, beta, th)
    half = 0.5 * (cfg["in_rho"] + r2 * cfg["in_rho"])
    xs, ys = [], []
    for x in range(int(x0f * nx), int(x1f * nx)):
        col = rho[:, x]
        for y in range(ny - 2, 0, -1):
            if col[y] < half <= col[y - 1]:
                ys.append(y - 1 + (col[y - 1] - half) / (col[y - 1] - col[y]) + 0.5)
                xs.append(x + 0.5)
                break
    b, a = np.polyfit(np.array(xs), np.array(ys), 1)
    beta_m = np.arctan(b) + th
    cells = [(y, x) for x in range(int(x0f * nx), int(x1f * nx)) for y in range(3, int(a + b * (x + 0.5) - 8))]
    yy, xx = np.array(cells).T
    r = rho[yy, xx].mean() / cfg["in_rho"]
    T = RT[yy, xx].mean()
    m2m = np.hypot(ux[yy, xx], uy[yy, xx]).mean() / np.sqrt(cfg["gamma"] * T)
    return (np.rad2deg(beta_m), r, T / cfg["in_RT"], m2m), (np.rad2deg(beta), r2, t2, m2)
