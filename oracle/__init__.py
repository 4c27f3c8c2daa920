"""Plain FP64 CPU oracle of the LELBM time step -- TEST INFRASTRUCTURE ONLY.

The oracle is the slow, obviously-correct reference the GPU library is checked
against.  It shares no code with the GPU library and the library never imports
it.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it.

``lelbm_oracle.c`` holds the method itself in 1D and 2D and
``lelbm_oracle3.c`` in 3D (see their headers for the paper passages each
stage follows); this module only builds them and marshals arguments through
ctypes.  ``riemann.py`` is the textbook exact Riemann solver
and ``mlp_ref.py`` the FP64 reference of the warm-start network.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lelbm_oracle.c")
_SRC3 = os.path.join(_HERE, "lelbm_oracle3.c")
_LIB = os.path.join(_HERE, "liblelbm_oracle.so")

BC_PERIODIC, BC_OUTFLOW, BC_INFLOW, BC_SLIPWALL, BC_WALL = 0, 1, 2, 3, 4
OK, EINVAL, ENOMEM, EEPR, ENONFINITE, EREACH = 0, -1, -2, -4, -5, -6


def build(force=False):
    """Compile the oracle with gcc (FP64, no contraction, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= max(os.path.getmtime(_SRC),
                                                                             os.path.getmtime(_SRC3)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=gnu99", "-o", tmp, _SRC, _SRC3, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("K", ctypes.c_double),
        ("omega_f", ctypes.c_double), ("omega_b", ctypes.c_double), ("omega_h", ctypes.c_double),
        ("n_conf", ctypes.c_double), ("r_min", ctypes.c_int),
        ("newton_tol", ctypes.c_double), ("newton_max_it", ctypes.c_int),
        ("kn_limiter", ctypes.c_int),
        ("kn_lo", ctypes.c_double), ("kn_hi", ctypes.c_double), ("omega_H", ctypes.c_double),
        ("bc", ctypes.c_int * 4), ("pad", ctypes.c_int),
        ("in_rho", ctypes.c_double), ("in_u", ctypes.c_double * 2), ("in_RT", ctypes.c_double),
        ("solid", ctypes.c_void_p),
        ("src_x", ctypes.c_int), ("src_y", ctypes.c_int),
        ("src_rate", ctypes.c_double), ("src_omega", ctypes.c_double), ("src_t", ctypes.c_double),
        ("wall_u", ctypes.c_double * 4),
    ]


class Params3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("K", ctypes.c_double),
        ("omega_f", ctypes.c_double), ("omega_b", ctypes.c_double), ("omega_h", ctypes.c_double),
        ("n_conf", ctypes.c_double), ("r_min", ctypes.c_int),
        ("newton_tol", ctypes.c_double), ("newton_max_it", ctypes.c_int),
        ("kn_limiter", ctypes.c_int),
        ("kn_lo", ctypes.c_double), ("kn_hi", ctypes.c_double), ("omega_H", ctypes.c_double),
        ("open", ctypes.c_int),
    ]


class Stats3(ctypes.Structure):
    _fields_ = [
        ("cells", ctypes.c_long), ("it_sum_f", ctypes.c_long), ("it_sum_g", ctypes.c_long),
        ("it_max_f", ctypes.c_int), ("it_max_g", ctypes.c_int),
        ("q_sum", ctypes.c_long), ("q_min", ctypes.c_int), ("q_max", ctypes.c_int),
        ("limited", ctypes.c_long),
        ("rt_min", ctypes.c_double), ("kn_max", ctypes.c_double),
        ("fail_cell", ctypes.c_long), ("fail_code", ctypes.c_int),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        c = max(self.cells, 1)
        d["it_mean_f"] = self.it_sum_f / c
        d["it_mean_g"] = self.it_sum_g / c
        d["q_mean"] = self.q_sum / c
        return d


class Stats(ctypes.Structure):
    _fields_ = [
        ("cells", ctypes.c_long), ("it_sum_f", ctypes.c_long), ("it_sum_g", ctypes.c_long),
        ("it_max_f", ctypes.c_int), ("it_max_g", ctypes.c_int),
        ("q_sum", ctypes.c_long), ("q_min", ctypes.c_int), ("q_max", ctypes.c_int),
        ("limited", ctypes.c_long),
        ("rt_min", ctypes.c_double), ("kn_max", ctypes.c_double), ("colat_max", ctypes.c_double),
        ("fail_cell", ctypes.c_long), ("fail_code", ctypes.c_int),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        c = max(self.cells, 1)
        d["it_mean_f"] = self.it_sum_f / c
        d["it_mean_g"] = self.it_sum_g / c
        d["q_mean"] = self.q_sum / c
        return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_num_moments.argtypes = [ctypes.c_int]
        L.orc_moments_from_primitives.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_long,
                                                  dp, dp, dp, dp, dp]
        L.orc_collide_flat.argtypes = [ctypes.POINTER(Params), dp, dp]
        L.orc_collide_src_flat.argtypes = [ctypes.POINTER(Params), dp, ctypes.c_double, dp]
        L.orc_las.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                              ctypes.c_int, dp, dp, ip, dp]
        L.orc_las_radius.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_las_levels.argtypes = [ctypes.c_double]
        L.orc_epr.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_double,
                              dp, ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, dp, ip]
        L.orc_epr_initial.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        L.orc_step.argtypes = [ctypes.POINTER(Params), dp, dp, ctypes.POINTER(Stats)]
        L.orc_run.argtypes = [ctypes.POINTER(Params), dp, dp, ctypes.c_int, ctypes.POINTER(Stats), ip]
        L.orc_walk.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip]
        L.orc_walk.restype = None
        P3 = ctypes.POINTER(Params3)
        L.orc3_moments_from_primitives.argtypes = [ctypes.c_double, ctypes.c_long, dp, dp, dp, dp, dp, dp]
        L.orc3_collide_flat.argtypes = [P3, dp, dp]
        L.orc3_las_radius.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc3_las_levels.argtypes = [ctypes.c_double]
        L.orc3_las.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp, ip]
        L.orc3_epr_initial.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.orc3_epr.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_double, dp, ctypes.c_int, dp,
                               ctypes.c_double, ctypes.c_int, dp, ip]
        L.orc3_run.argtypes = [P3, dp, dp, ctypes.c_int, ctypes.POINTER(Stats3), ip]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def num_moments(dim):
    return {1: 6, 2: 11, 3: 17}[dim]


def make_params(cfg):
    """Oracle parameter struct from a configuration dict (see lelbm_inputs)."""
    p = Params()
    p.dim = cfg["dim"]
    p.nx = cfg["nx"]
    p.ny = cfg.get("ny", 1)
    p.K = cfg["K"]
    p.omega_f, p.omega_b, p.omega_h = cfg["omega_f"], cfg["omega_b"], cfg["omega_h"]
    p.n_conf = cfg.get("n_conf", 4.0)
    p.r_min = cfg.get("r_min", 2)
    p.newton_tol = cfg.get("newton_tol", 1e-12)
    p.newton_max_it = cfg.get("newton_max_it", 50)
    p.kn_limiter = cfg.get("kn_limiter", 1)
    p.kn_lo, p.kn_hi, p.omega_H = cfg.get("kn_lo", -2.0), cfg.get("kn_hi", -1.0), cfg.get("omega_H", 1.0)
    names = {"periodic": BC_PERIODIC, "outflow": BC_OUTFLOW, "inflow": BC_INFLOW, "slipwall": BC_SLIPWALL,
             "wall": BC_WALL}
    for i, b in enumerate(cfg.get("bc", ["periodic"] * 4)):
        p.bc[i] = names[b] if isinstance(b, str) else int(b)
    p.pad = cfg.get("pad", 0)
    p.in_rho = cfg.get("in_rho", 1.0)
    iu = cfg.get("in_u", (0.0, 0.0))
    p.in_u[0], p.in_u[1] = iu[0], iu[1]
    p.in_RT = cfg.get("in_RT", 1.0)
    solid = cfg.get("solid")
    if solid is None:
        p.solid = None
    else:
        m = np.ascontiguousarray(solid, dtype=np.uint8).reshape(p.ny, p.nx)
        p._solid_ref = m                     # keep the mask alive with the struct
        p.solid = m.ctypes.data_as(ctypes.c_void_p)
    src = cfg.get("source")
    if src is not None:
        p.src_x, p.src_y = src["x"], src.get("y", 0)
        p.src_rate, p.src_omega, p.src_t = src["rate"], src["omega"], src.get("t0", 0.0)
    for i, v in enumerate(cfg.get("wall_u", (0.0, 0.0, 0.0, 0.0))):
        p.wall_u[i] = v
    return p


def moments_from_primitives(dim, K, rho, ux, uy, RT):
    """Equilibrium raw moments (SoA [nmom][n]) of primitive fields."""
    rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
    n = rho.size
    ux = np.ascontiguousarray(ux, dtype=np.float64).ravel()
    uy = np.ascontiguousarray(uy if uy is not None else np.zeros(n), dtype=np.float64).ravel()
    RT = np.ascontiguousarray(RT, dtype=np.float64).ravel()
    out = np.zeros((num_moments(dim), n))
    st = lib().orc_moments_from_primitives(dim, K, n, _dp(rho), _dp(ux), _dp(uy), _dp(RT), _dp(out))
    assert st == OK
    return out


_COLLIDE_KEYS = ["rho", "ux", "uy", "RT", "kn", "om_f", "om_b", "om_h", "limited",
                 "Pxx", "Pxy", "Pyy", "Qx", "Qy", "g0", "hx", "hy"]


def collide(cfg, mom, src=None):
    """Collision stage of one cell: dict of macroscopic variables, non-equilibrium
    central moments, effective frequencies and the normalised targets m, n
    (with src: a mass source of src in the cell, Eqs. VC6-VC8)."""
    p = make_params(cfg)
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    out = np.zeros(len(_COLLIDE_KEYS) + 16)
    if src is None:
        st = lib().orc_collide_flat(ctypes.byref(p), _dp(mom), _dp(out))
    else:
        st = lib().orc_collide_src_flat(ctypes.byref(p), _dp(mom), ctypes.c_double(src), _dp(out))
    d = dict(zip(_COLLIDE_KEYS, out[:len(_COLLIDE_KEYS)]))
    k = len(_COLLIDE_KEYS)
    nf, ng = (4, 3) if cfg["dim"] == 1 else (10, 6)
    d["m"] = out[k:k + nf].copy()
    d["n"] = out[k + 10:k + 10 + ng].copy()
    d["status"] = st
    return d


def las(dim, u, RT, n_conf=4.0, r_min=2):
    """Stencil of one cell: (c [q,2], dC [q], d [q,2] landing displacement, h [q] spacing)."""
    u = np.ascontiguousarray([u[0], u[1] if dim == 2 else 0.0], dtype=np.float64)
    cap = 256
    while True:
        c = np.zeros((cap, 2)); dC = np.zeros(cap); d = np.zeros((cap, 2), dtype=np.int32); h = np.zeros(cap)
        q = lib().orc_las(dim, _dp(u), RT, n_conf, r_min, cap, _dp(c), _dp(dC), _ip(d), _dp(h))
        if q >= 0:
            return c[:q].copy(), dC[:q].copy(), d[:q].copy(), h[:q].copy()
        cap = -q


def las_radius(RT, n_conf=4.0, r_min=2):
    return lib().orc_las_radius(RT, n_conf, r_min)


def las_levels(RT):
    return lib().orc_las_levels(RT)


def epr_initial(dim, nb, RT):
    lam = np.zeros(nb)
    lib().orc_epr_initial(dim, nb, RT, _dp(lam))
    return lam


def epr(dim, c, dC, u, RT, target, lam0=None, tol=1e-12, maxit=50):
    """Entropic reconstruction on a given stencil.  Returns (status, lambda, populations, iterations)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    dC = np.ascontiguousarray(dC, dtype=np.float64)
    q = dC.size
    target = np.ascontiguousarray(target, dtype=np.float64)
    nb = target.size
    u = np.ascontiguousarray([u[0], u[1] if dim == 2 else 0.0], dtype=np.float64)
    lam = np.zeros(nb) if lam0 is None else np.ascontiguousarray(lam0, dtype=np.float64).copy()
    pop = np.zeros(q)
    it = np.zeros(1, dtype=np.int32)
    st = lib().orc_epr(dim, nb, q, _dp(c), _dp(dC), _dp(u), RT, _dp(target), 0 if lam0 is None else 1,
                       _dp(lam), tol, maxit, _dp(pop), _ip(it))
    return st, lam, pop, int(it[0])


def make_params3(cfg):
    """3D oracle parameter struct from a configuration dict (a periodic box,
    or with ``open`` true a window with no sources outside it whose outgoing
    populations are dropped)."""
    p = Params3()
    p.nx, p.ny, p.nz = cfg["nx"], cfg["ny"], cfg["nz"]
    p.K = cfg["K"]
    p.omega_f, p.omega_b, p.omega_h = cfg["omega_f"], cfg["omega_b"], cfg["omega_h"]
    p.n_conf = cfg.get("n_conf", 4.0)
    p.r_min = cfg.get("r_min", 2)
    p.newton_tol = cfg.get("newton_tol", 1e-12)
    p.newton_max_it = cfg.get("newton_max_it", 50)
    p.kn_limiter = cfg.get("kn_limiter", 1)
    p.kn_lo, p.kn_hi, p.omega_H = cfg.get("kn_lo", -2.0), cfg.get("kn_hi", -1.0), cfg.get("omega_H", 1.0)
    p.open = 1 if cfg.get("open") else 0
    return p


def moments_from_primitives3(K, rho, ux, uy, uz, RT):
    """3D equilibrium raw moments (SoA [17][n]) of primitive fields."""
    f = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (rho, ux, uy, uz, RT)]
    n = f[0].size
    out = np.zeros((17, n))
    st = lib().orc3_moments_from_primitives(K, n, *[_dp(a) for a in f], _dp(out))
    assert st == OK
    return out


_COLLIDE3_KEYS = ["rho", "ux", "uy", "uz", "RT", "kn", "om_f", "om_b", "om_h", "limited"]


def collide3(cfg, mom):
    """3D collision stage of one cell: macroscopic variables, the non-equilibrium
    central moments P (3x3), Q, g0, h, the frequencies and the targets m (19), n (10)."""
    p = make_params3(cfg)
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    out = np.zeros(10 + 9 + 3 + 1 + 3 + 19 + 10)
    st = lib().orc3_collide_flat(ctypes.byref(p), _dp(mom), _dp(out))
    d = dict(zip(_COLLIDE3_KEYS, out[:10]))
    d["P"] = out[10:19].reshape(3, 3).copy()
    d["Q"] = out[19:22].copy()
    d["g0"] = out[22]
    d["h"] = out[23:26].copy()
    d["m"] = out[26:45].copy()
    d["n"] = out[45:55].copy()
    d["status"] = st
    return d


def las3(u, RT, n_conf=4.0, r_min=2, full=False):
    """3D stencil of one cell: the landing displacements d [q, 3] (base points
    z-major, then y, x; refined children follow their parent), with full=True
    (c [q, 3] velocities, dC [q] volumes, d), or the status if refused."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    cap = 1024
    while True:
        c = np.zeros((cap, 3)); dC = np.zeros(cap); d = np.zeros((cap, 3), dtype=np.int32)
        q = lib().orc3_las(_dp(u), RT, n_conf, r_min, cap, _dp(c), _dp(dC), _ip(d))
        if q == EREACH:
            return q
        if q >= 0:
            return (c[:q].copy(), dC[:q].copy(), d[:q].copy()) if full else d[:q].copy()
        cap = -q


def epr3(d, u, RT, target, lam0=None, tol=1e-12, maxit=50, dC=None):
    """3D entropic reconstruction on the points d (velocities, [q, 3]; volumes
    dC, default 1).  Returns (status, lambda, populations, iterations)."""
    c = np.ascontiguousarray(d, dtype=np.float64)
    q = c.shape[0]
    dC = np.ones(q) if dC is None else np.ascontiguousarray(dC, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float64)
    nb = target.size
    u = np.ascontiguousarray(u, dtype=np.float64)
    lam = np.zeros(nb) if lam0 is None else np.ascontiguousarray(lam0, dtype=np.float64).copy()
    pop = np.zeros(q)
    it = np.zeros(1, dtype=np.int32)
    st = lib().orc3_epr(nb, q, _dp(c), _dp(dC), _dp(u), RT, _dp(target), 0 if lam0 is None else 1, _dp(lam), tol,
                        maxit, _dp(pop), _ip(it))
    return st, lam, pop, int(it[0])


def epr3_initial(nb, RT):
    lam = np.zeros(nb)
    lib().orc3_epr_initial(nb, RT, _dp(lam))
    return lam


def step(cfg, mom, nsteps=1):
    """Advance SoA moments [nmom][cells] by nsteps.  Returns (status, moments, stats dict, steps_done)."""
    if cfg["dim"] == 3:
        p3 = make_params3(cfg)
        mom = np.ascontiguousarray(mom, dtype=np.float64)
        out = np.zeros_like(mom)
        st3 = Stats3()
        done = np.zeros(1, dtype=np.int32)
        status = lib().orc3_run(ctypes.byref(p3), _dp(mom), _dp(out), nsteps, ctypes.byref(st3), _ip(done))
        return status, out, st3.as_dict(), int(done[0])
    p = make_params(cfg)
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    out = np.zeros_like(mom)
    st = Stats()
    done = np.zeros(1, dtype=np.int32)
    status = lib().orc_run(ctypes.byref(p), _dp(mom), _dp(out), nsteps, ctypes.byref(st), _ip(done))
    return status, out, st.as_dict(), int(done[0])


def walk(cfg, x, y, dx, dy):
    """Path of one population (Sec. III.B): (final x, final y, sign x, sign y)."""
    p = make_params(cfg)
    out = np.zeros(4, dtype=np.int32)
    lib().orc_walk(ctypes.byref(p), x, y, dx, dy, _ip(out))
    return tuple(int(v) for v in out)


def num_threads():
    return lib().orc_num_threads()
