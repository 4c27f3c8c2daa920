"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the
CPU oracle.

This module holds data generation only: primitive fields (density, velocity,
temperature RT in lattice units) and run parameters.  It contains none of the
method's arithmetic -- each side converts primitives to raw moments with its
own code.  Boundary kinds are returned as strings so neither side depends on
the other's enum values.

Random numbers come from ``numpy.random.Generator(PCG64(seed))`` with a fixed
draw order per workload.

Workloads (lattice units, dx = dt = 1):
  * ``riemann1d``  -- 1D two-state problem split at the midpoint, zero-gradient
    outflow pads at both ends (the paper's shock tubes, Sec. V.A-B).
  * ``quadrants``  -- 2D periodic four-quadrant piecewise-constant states with a
    1% smooth Fourier density perturbation (structure of the paper's 2D Riemann
    problem, Sec. V.D; the published reference solutions are not used).
  * ``hotbox``     -- uniform periodic advection (Sec. IV.E).
  * ``channel``    -- supersonic inflow past seeded elliptical obstacles in a
    channel with slip walls (structure of the paper's blunt-body cases,
    Sec. V.E; no external reference data is used).
  * ``shear_wave`` / ``acoustic_pulse`` / ``acoustic_source`` -- the paper's
    verification problems (Sec. IV.A, IV.D, IV.C).
  * ``couette`` -- gas between no-slip walls on the y faces, the top wall
    moving along x (Sec. III.B).
  * ``smooth_periodic3`` / ``shear_wave3`` -- 3D periodic boxes (smooth
    random fields; the transverse shear wave of Sec. IV.A in 3D).
  * ``oblique_shock`` -- uniform supersonic flow turned by a slip wall
    (Sec. V.F): the flow enters through the left and top faces inclined by
    theta toward the bottom slip wall, which deflects it along the wall.

Physical states are mapped to lattice units by acoustic scaling (Sec. V.B):
RT_lat = s^2 RT_phys and u_lat = s u_phys with s^2 = RT_floor / min RT_phys.
"""
import numpy as np

GAMMA = 1.4
# internal degrees of freedom for gamma = 1.4: gamma = (D + K + 2)/(D + K)
K_1D = 4.0
K_2D = 3.0
K_3D = 2.0

RT_FLOOR = 0.5


def _base_cfg(dim, nx, ny, K):
    return {
        "dim": dim, "nx": nx, "ny": ny, "K": K, "gamma": GAMMA,
        # inviscid shock runs: tau = 0 for shear and heat flux, omega_b = 1
        "omega_f": 2.0, "omega_b": 1.0, "omega_h": 2.0,
        "n_conf": 4.0, "r_min": 2,
        "newton_tol": 1e-12, "newton_max_it": 50,
        "kn_limiter": 1, "kn_lo": -2.0, "kn_hi": -1.0, "omega_H": 1.0,
        "bc": ["periodic"] * 4, "pad": 0,
        "in_rho": 1.0, "in_u": (0.0, 0.0), "in_RT": 1.0,
    }


def riemann1d(seed=None, n=2000, states=None, pad=48, rt_floor=RT_FLOOR, scale=None):
    """1D two-state problem.  With ``states=None`` draws rho_L, p_L, rho_R, p_R
    ~ U[0.1, 1.0] in that order (zero velocity); otherwise ``states`` is
    ((rho_L, u_L, p_L), (rho_R, u_R, p_R)) in physical units.  Returns
    (cfg, prim) with prim fields of shape (1, n)."""
    if states is None:
        g = np.random.Generator(np.random.PCG64(seed))
        rl, pl, rr, pr = g.uniform(0.1, 1.0, size=4)
        states = ((rl, 0.0, pl), (rr, 0.0, pr))
    (rl, ul, pl), (rr, ur, pr) = states
    rtl, rtr = pl / rl, pr / rr
    s = np.sqrt(rt_floor / min(rtl, rtr)) if scale is None else scale
    cfg = _base_cfg(1, n, 1, K_1D)
    cfg["bc"] = ["outflow", "outflow", "periodic", "periodic"]
    cfg["pad"] = pad
    cfg["scale"] = float(s)
    cfg["states_phys"] = states
    i = np.arange(n)
    left = i < n // 2
    rho = np.where(left, rl, rr).astype(np.float64)
    ux = np.where(left, ul, ur) * s
    RT = np.where(left, rtl, rtr) * s * s
    prim = {"rho": rho[None, :], "ux": ux[None, :].astype(np.float64),
            "uy": np.zeros((1, n)), "RT": RT[None, :].astype(np.float64)}
    return cfg, prim


def quadrants(seed, n=1024, ny=None, rt_floor=RT_FLOOR, perturb=0.01):
    """2D periodic four-quadrant states (SW, SE, NW, NE; split at the middle).
    Per quadrant, in that order: rho ~ U[0.1, 1.5], p ~ U[0.03, 1.5], then
    u_x, u_y ~ U[-1.2, 1.2] times the local sound speed sqrt(gamma p / rho).
    Density is perturbed by ``perturb`` times a smooth Fourier field
    phi = sum_{kx,ky=1..4} a sin(2 pi (kx x + ky y)/L + theta), a ~ N(0,1),
    theta ~ U[0, 2 pi), normalised to max |phi| = 1, at fixed pressure."""
    ny = n if ny is None else ny
    g = np.random.Generator(np.random.PCG64(seed))
    quads = []
    for _ in range(4):
        rho = g.uniform(0.1, 1.5)
        p = g.uniform(0.03, 1.5)
        cs = np.sqrt(GAMMA * p / rho)
        ux = g.uniform(-1.2, 1.2) * cs
        uy = g.uniform(-1.2, 1.2) * cs
        quads.append((rho, ux, uy, p))
    amps = g.standard_normal((4, 4))
    phases = g.uniform(0.0, 2.0 * np.pi, size=(4, 4))
    x = (np.arange(n) + 0.5)[None, :]
    y = (np.arange(ny) + 0.5)[:, None]
    phi = np.zeros((ny, n))
    for a in range(4):
        for b in range(4):
            phi += amps[a, b] * np.sin(2 * np.pi * ((a + 1) * x / n + (b + 1) * y / ny) + phases[a, b])
    phi /= np.abs(phi).max()
    east = np.broadcast_to(x >= n / 2, (ny, n))
    north = np.broadcast_to(y >= ny / 2, (ny, n))
    idx = east.astype(int) + 2 * north.astype(int)
    table = np.array(quads)
    rho0 = table[idx, 0]
    ux = table[idx, 1]
    uy = table[idx, 2]
    p = table[idx, 3]
    rho = rho0 * (1.0 + perturb * phi)
    rt_phys = p / rho
    s = np.sqrt(rt_floor / rt_phys.min())
    cfg = _base_cfg(2, n, ny, K_2D)
    cfg["scale"] = float(s)
    cfg["quadrants_phys"] = quads
    prim = {"rho": rho, "ux": ux * s, "uy": uy * s, "RT": rt_phys * s * s}
    return cfg, prim


def channel(seed, nx=4096, ny=2048, n_obstacles=None, mach=None, size_scale=1.0, pad=24, start="rest"):
    """Channel with uniform supersonic inflow past 1-4 elliptical obstacles.

    Draw order: Mach ~ U[2, 6] (unless given), obstacle count ~ U{1..4}
    (unless given), then per obstacle semi-axes a, b ~ U[20, 120] * size_scale,
    rotation ~ U[0, pi), centre x ~ U[0.15, 0.7] nx, y ~ U[0.2, 0.8] ny,
    rejected (and redrawn) while it overlaps an earlier obstacle's bounding
    circle or comes closer than 10 cells to a wall.  Lattice inflow state
    rho = 1, RT = 1, u = (Ma sqrt(gamma), 0); the initial field is the inflow
    state with zero velocity (start="rest": the inflow enters through the left
    face; at these Mach numbers every population of the inflow stencil moves
    downstream, so an initial field moving at the inflow velocity would leave
    vacuum cells in the lee of each obstacle after one step), or the inflow
    state itself (start="inflow").  A cell is solid iff its centre lies inside
    an ellipse.
    Faces: inflow left, zero-gradient outflow right, slip walls top and
    bottom.  Returns (cfg, prim) with cfg["solid"] a uint8 [ny][nx] mask."""
    g = np.random.Generator(np.random.PCG64(seed))
    ma = g.uniform(2.0, 6.0) if mach is None else float(mach)
    nob = int(g.integers(1, 5)) if n_obstacles is None else int(n_obstacles)
    obs = []
    tries = 0
    while len(obs) < nob:
        tries += 1
        if tries > 10000:
            raise RuntimeError("could not place the obstacles")
        a = g.uniform(20.0, 120.0) * size_scale
        b = g.uniform(20.0, 120.0) * size_scale
        th = g.uniform(0.0, np.pi)
        cx = g.uniform(0.15, 0.7) * nx
        cy = g.uniform(0.2, 0.8) * ny
        r = max(a, b)
        if cy - r < 10 or cy + r > ny - 10 or cx - r < 10 or cx + r > nx - 10:
            continue
        if any(np.hypot(cx - o[3], cy - o[4]) < r + max(o[0], o[1]) for o in obs):
            continue
        obs.append((a, b, th, cx, cy))
    x = (np.arange(nx) + 0.5)[None, :]
    y = (np.arange(ny) + 0.5)[:, None]
    solid = np.zeros((ny, nx), dtype=bool)
    for a, b, th, cx, cy in obs:
        c, sn = np.cos(th), np.sin(th)
        xr = (x - cx) * c + (y - cy) * sn
        yr = -(x - cx) * sn + (y - cy) * c
        solid |= (xr / a) ** 2 + (yr / b) ** 2 <= 1.0
    u_in = ma * np.sqrt(GAMMA)
    cfg = _base_cfg(2, nx, ny, K_2D)
    cfg["bc"] = ["inflow", "outflow", "slipwall", "slipwall"]
    cfg["pad"] = pad
    cfg["in_rho"], cfg["in_u"], cfg["in_RT"] = 1.0, (float(u_in), 0.0), 1.0
    cfg["solid"] = solid.astype(np.uint8)
    cfg["mach"] = float(ma)
    cfg["obstacles"] = obs
    shape = (ny, nx)
    ux0 = np.full(shape, u_in) if start == "inflow" else np.zeros(shape)
    prim = {"rho": np.ones(shape), "ux": ux0, "uy": np.zeros(shape), "RT": np.ones(shape)}
    return cfg, prim


def hotbox(RT, n=256, ny=None, u=(10.0, 10.0), dim=2):
    """Uniform periodic advection: rho = 1, u = (10, 10) by default."""
    ny = (n if ny is None else ny) if dim == 2 else 1
    cfg = _base_cfg(dim, n, ny, K_2D if dim == 2 else K_1D)
    shape = (ny, n)
    prim = {"rho": np.ones(shape), "ux": np.full(shape, float(u[0])),
            "uy": np.full(shape, float(u[1]) if dim == 2 else 0.0), "RT": np.full(shape, float(RT))}
    return cfg, prim


def shear_wave(L=64, ny=4, RT=0.5, u0=0.5, amp=1e-3, nu=0.05, K=K_2D):
    """Decaying transverse shear wave u_y = amp cos(2 pi x / L) on a uniform
    flow u_x = u0 (Sec. IV.A).  Shear frequency from nu = RT (1/omega - 1/2)."""
    cfg = _base_cfg(2, L, ny, K)
    omega = 1.0 / (nu / RT + 0.5)
    cfg.update({"omega_f": omega, "omega_b": 1.0, "omega_h": omega, "kn_limiter": 0, "nu": nu})
    x = (np.arange(L) + 0.5)[None, :]
    shape = (ny, L)
    prim = {"rho": np.ones(shape), "ux": np.full(shape, u0),
            "uy": np.broadcast_to(amp * np.cos(2 * np.pi * x / L), shape).copy(),
            "RT": np.full(shape, RT)}
    return cfg, prim


def acoustic_pulse(n=400, RT=1.0, drho=1e-4, width=4.0, K=K_1D, pad=32):
    """Quiescent 1D gas with a small Gaussian density bump at the centre at
    constant temperature (Sec. IV.D uses a point bump)."""
    cfg = _base_cfg(1, n, 1, K)
    cfg.update({"omega_f": 1.0, "omega_b": 1.0, "omega_h": 1.0, "kn_limiter": 0})
    cfg["bc"] = ["outflow", "outflow", "periodic", "periodic"]
    cfg["pad"] = pad
    x = np.arange(n) + 0.5
    rho = 1.0 + drho * np.exp(-0.5 * ((x - n / 2) / width) ** 2)
    prim = {"rho": rho[None, :], "ux": np.zeros((1, n)), "uy": np.zeros((1, n)), "RT": np.full((1, n), RT)}
    return cfg, prim


def acoustic_source(n=1200, RT=1.0, rate=1e-6, period=64.0, nu_b=0.8, nu=1e-3, K=K_1D):
    """Quiescent periodic 1D gas with an oscillating point mass source of
    rate * sin(2 pi t / period) in the centre cell (Sec. IV.C).  Collision
    frequencies from the targets: shear and heat flux from nu = RT (1/omega -
    1/2), bulk from nu_b = RT (2/D - 2/(D + K)) (1/omega_b - 1/2) (Eqs.
    C8a-c with D = 1)."""
    cfg = _base_cfg(1, n, 1, K)
    om = 1.0 / (nu / RT + 0.5)
    om_b = 1.0 / (nu_b / (RT * (2.0 - 2.0 / (1.0 + K))) + 0.5)
    cfg.update({"omega_f": om, "omega_b": om_b, "omega_h": om, "kn_limiter": 0,
                "source": {"x": n // 2, "y": 0, "rate": rate, "omega": 2 * np.pi / period, "t0": 0.0},
                "nu": nu, "nu_b": nu_b})
    shape = (1, n)
    prim = {"rho": np.ones(shape), "ux": np.zeros(shape), "uy": np.zeros(shape), "RT": np.full(shape, RT)}
    return cfg, prim


def couette(ny=16, nx=4, RT=1.0, U=0.1, nu=0.2, K=K_2D, u0=(0.0, 0.0)):
    """Gas at rest (or at velocity u0) between no-slip walls on the y faces,
    periodic in x; the top wall moves at U along x.  Shear and heat-flux
    frequencies from nu = RT (1/omega - 1/2)."""
    cfg = _base_cfg(2, nx, ny, K)
    om = 1.0 / (nu / RT + 0.5)
    cfg.update({"omega_f": om, "omega_b": 1.0, "omega_h": om, "kn_limiter": 0,
                "bc": ["periodic", "periodic", "wall", "wall"], "wall_u": (0.0, 0.0, 0.0, U), "nu": nu})
    shape = (ny, nx)
    prim = {"rho": np.ones(shape), "ux": np.full(shape, float(u0[0])), "uy": np.full(shape, float(u0[1])),
            "RT": np.full(shape, RT)}
    return cfg, prim


def oblique_shock(mach=2.0, theta_deg=5.0, nx=512, ny=320, RT=0.5, pad=8):
    """Sec. V.F: inflow at Mach `mach` (rho 1, RT) inclined by theta toward
    the bottom slip wall through the left and top faces, outflow on the right.
    The wall turns the flow by theta, which makes an oblique shock from the
    bottom-left corner; the whole domain starts in the inflow state.
    Inviscid shock settings (reading 11) with the Knudsen limiter."""
    cfg = _base_cfg(2, nx, ny, K_2D)
    th = np.deg2rad(theta_deg)
    u = mach * np.sqrt(GAMMA * RT)
    uin = (u * np.cos(th), -u * np.sin(th))
    cfg["bc"] = ["inflow", "outflow", "slipwall", "inflow"]
    cfg["pad"] = pad
    cfg.update({"in_rho": 1.0, "in_u": uin, "in_RT": RT, "mach": mach, "theta_deg": theta_deg})
    shape = (ny, nx)
    prim = {"rho": np.ones(shape), "ux": np.full(shape, uin[0]), "uy": np.full(shape, uin[1]),
            "RT": np.full(shape, RT)}
    return cfg, prim


def smooth_periodic(seed, n=16, ny=12, dim=2, amp=0.05, RT=0.8):
    """Small smooth random periodic state (a few Fourier modes in each field)
    for conservation and parity checks."""
    g = np.random.Generator(np.random.PCG64(seed))
    ny = ny if dim == 2 else 1
    x = (np.arange(n) + 0.5)[None, :] / n
    y = (np.arange(ny) + 0.5)[:, None] / ny
    fields = []
    for _ in range(4):
        f = np.zeros((ny, n))
        for a in range(1, 3):
            for b in range(0, 3 if dim == 2 else 1):
                f += g.standard_normal() * np.sin(2 * np.pi * (a * x + b * y) + g.uniform(0, 2 * np.pi))
        fields.append(f / max(np.abs(f).max(), 1e-30))
    cfg = _base_cfg(dim, n, ny, K_2D if dim == 2 else K_1D)
    prim = {"rho": 1.0 + amp * fields[0], "ux": 0.3 + 0.5 * amp * 10 * fields[1],
            "uy": (-0.2 + 0.5 * amp * 10 * fields[2]) if dim == 2 else np.zeros((ny, n)),
            "RT": RT * (1.0 + amp * fields[3])}
    return cfg, prim


BC_NAMES = ("periodic", "outflow", "inflow", "slipwall")


def _base_cfg3(nx, ny, nz, K=K_3D):
    cfg = _base_cfg(3, nx, ny, K)
    cfg["nz"] = nz
    cfg["bc"] = ["periodic"] * 6
    return cfg


def smooth_periodic3(seed, n=12, ny=None, nz=None, amp=0.05, RT=1.0, u=(0.3, -0.2, 0.1)):
    """3D periodic box with a few smooth random Fourier modes in each of rho,
    u_x, u_y, u_z and RT (fields [nz][ny][nx])."""
    g = np.random.Generator(np.random.PCG64(seed))
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny, (np.arange(n) + 0.5) / n,
                          indexing="ij")
    fields = []
    for _ in range(5):
        f = np.zeros((nz, ny, n))
        for a in range(1, 3):
            for b in range(0, 2):
                for c in range(0, 2):
                    f += g.standard_normal() * np.sin(2 * np.pi * (a * x + b * y + c * z) + g.uniform(0, 2 * np.pi))
        fields.append(f / max(np.abs(f).max(), 1e-30))
    cfg = _base_cfg3(n, ny, nz)
    prim = {"rho": 1.0 + amp * fields[0], "ux": u[0] + 5 * amp * fields[1], "uy": u[1] + 5 * amp * fields[2],
            "uz": u[2] + 5 * amp * fields[3], "RT": RT * (1.0 + amp * fields[4])}
    return cfg, prim


def shear_wave3(L=16, ny=1, nz=1, RT=1.0, u0=0.5, amp=1e-3, nu=0.05, K=K_3D):
    """3D transverse shear wave u_y = amp cos(2 pi x / L) on a uniform flow
    u_x = u0 (Sec. IV.A); uniform along y and z.  Shear frequency from
    nu = RT (1/omega - 1/2)."""
    cfg = _base_cfg3(L, ny, nz, K)
    om = 1.0 / (nu / RT + 0.5)
    cfg.update({"omega_f": om, "omega_b": 1.0, "omega_h": om, "kn_limiter": 0, "nu": nu})
    x = (np.arange(L) + 0.5)[None, None, :] * np.ones((nz, ny, 1))
    prim = {"rho": np.ones((nz, ny, L)), "ux": np.full((nz, ny, L), u0),
            "uy": amp * np.cos(2 * np.pi * x / L), "uz": np.zeros((nz, ny, L)), "RT": np.full((nz, ny, L), RT)}
    return cfg, prim
