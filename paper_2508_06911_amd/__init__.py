"""Python binding of the MI355X LELBM library (``liblelbm.so``, C ABI in
``include/lelbm.h``).

Argument marshalling only: every stage of the time step runs in the library's
HIP kernels.  PyTorch supplies the HIP stream (and device buffers for the
``*_device`` calls).  If the library has not been built, importing works but
every call raises; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblelbm.so")

OK, EINVAL, ENOMEM, EDEVICE, EEPR, ENONFINITE, EREACH = 0, -1, -2, -3, -4, -5, -6
BC = {"periodic": 0, "outflow": 1, "inflow": 2, "slipwall": 3, "wall": 4}
FP64, MIXED = 0, 1
GUESS_EQ, GUESS_MLP, GUESS_LIN, GUESS_PREV, GUESS_MLP_PREV = 0, 1, 2, 3, 4


class LelbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("K", ctypes.c_double),
        ("omega_f", ctypes.c_double), ("omega_b", ctypes.c_double), ("omega_h", ctypes.c_double),
        ("n_conf", ctypes.c_double), ("r_min", ctypes.c_int),
        ("newton_tol", ctypes.c_double), ("newton_max_it", ctypes.c_int),
        ("kn_limiter", ctypes.c_int),
        ("kn_lo", ctypes.c_double), ("kn_hi", ctypes.c_double), ("omega_H", ctypes.c_double),
        ("precision", ctypes.c_int), ("guess", ctypes.c_int),
        ("bc", ctypes.c_int * 4), ("pad", ctypes.c_int),
        ("in_rho", ctypes.c_double), ("in_u", ctypes.c_double * 2), ("in_RT", ctypes.c_double),
        ("solid", ctypes.c_void_p),
        ("src_x", ctypes.c_int), ("src_y", ctypes.c_int),
        ("src_rate", ctypes.c_double), ("src_omega", ctypes.c_double), ("src_t0", ctypes.c_double),
        ("wall_u", ctypes.c_double * 4),
        ("nz", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("it_mean_f", ctypes.c_double), ("it_mean_g", ctypes.c_double),
        ("it_max_f", ctypes.c_int), ("it_max_g", ctypes.c_int),
        ("fallbacks", ctypes.c_long), ("limited", ctypes.c_long),
        ("q_min", ctypes.c_long), ("q_max", ctypes.c_long), ("q_mean", ctypes.c_double),
        ("rt_min", ctypes.c_double), ("kn_max", ctypes.c_double), ("colat_max", ctypes.c_double),
        ("sum", ctypes.c_double * 4), ("cells", ctypes.c_long),
        ("point_passes", ctypes.c_long), ("arrivals", ctypes.c_long),
        ("point_passes_refined", ctypes.c_long), ("wave_point_passes", ctypes.c_long),
        ("row_passes", ctypes.c_long),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["sum"] = list(self.sum)
        return d


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime with the same soname as the system
        # one; loading torch first makes the library bind to that runtime, so
        # torch streams and device pointers are valid in the library.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblelbm.so is not built (run python -m paper_2508_06911_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.lelbm_num_moments.argtypes = [ctypes.c_int]
        L.lelbm_moments_from_primitives.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_long,
                                                    dp, dp, dp, dp, dp]
        L.lelbm_moments_from_primitives3.argtypes = [ctypes.c_double, ctypes.c_long, dp, dp, dp, dp, dp, dp]
        L.lelbm_create.argtypes = [ctypes.POINTER(Params), dp, vp, ctypes.POINTER(vp)]
        L.lelbm_create_device.argtypes = [ctypes.POINTER(Params), vp, ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.lelbm_step.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Stats)]
        L.lelbm_step_noalloc.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Stats)]
        L.lelbm_read_moments.argtypes = [vp, dp]
        L.lelbm_read_moments_device.argtypes = [vp, vp]
        L.lelbm_last_failure.argtypes = [vp, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_int)]
        L.lelbm_last_failure_detail.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_double)]
        L.lelbm_set_timing.argtypes = [vp, ctypes.c_int]
        L.lelbm_kernel_times.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_long), ctypes.c_int]
        L.lelbm_memory.argtypes = [vp, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]
        L.lelbm_set_scratch_budget.argtypes = [vp, ctypes.c_longlong]
        L.lelbm_strerror.argtypes = [ctypes.c_int]
        L.lelbm_strerror.restype = ctypes.c_char_p
        L.lelbm_destroy.argtypes = [vp]
        L.lelbm_destroy.restype = None
        fp = ctypes.POINTER(ctypes.c_float)
        ll = ctypes.c_longlong
        L.lelbm_mlp_create.argtypes = [fp, ctypes.c_ulonglong, vp, ctypes.POINTER(vp)]
        L.lelbm_mlp_get_params.argtypes = [vp, fp]
        L.lelbm_mlp_forward.argtypes = [vp, vp, ll, ll, vp]
        L.lelbm_mlp_gradient.argtypes = [vp, vp, ll, fp, ctypes.POINTER(ctypes.c_double)]
        L.lelbm_mlp_train.argtypes = [vp, vp, ll, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_ulonglong,
                                      ctypes.POINTER(ctypes.c_double)]
        L.lelbm_mlp_fit_normalization.argtypes = [vp, vp, ll]
        L.lelbm_mlp_get_norm.argtypes = [vp, fp]
        L.lelbm_mlp_set_norm.argtypes = [vp, fp]
        L.lelbm_mlp_destroy.argtypes = [vp]
        L.lelbm_mlp_destroy.restype = None
        L.lelbm_set_mlp.argtypes = [vp, vp]
        L.lelbm_harvest.argtypes = [vp, vp, ll, ctypes.c_int]
        L.lelbm_harvest_count.argtypes = [vp, ctypes.POINTER(ll)]
        _lib = L
    return _lib


def _check(code):
    if code != OK:
        raise LelbmError(code, lib().lelbm_strerror(code).decode())
    return code


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_moments(dim):
    return lib().lelbm_num_moments(dim)


def moments_from_primitives(dim, K, rho, ux, uy, RT):
    rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
    n = rho.size
    ux = np.ascontiguousarray(ux, dtype=np.float64).ravel()
    uy = np.ascontiguousarray(uy if uy is not None else np.zeros(n), dtype=np.float64).ravel()
    RT = np.ascontiguousarray(RT, dtype=np.float64).ravel()
    out = np.zeros((num_moments(dim), n))
    _check(lib().lelbm_moments_from_primitives(dim, K, n, _dp(rho), _dp(ux), _dp(uy), _dp(RT), _dp(out)))
    return out


def moments_from_primitives3(K, rho, ux, uy, uz, RT):
    """3D equilibrium raw moments (SoA [17][n]) of primitive fields."""
    f = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (rho, ux, uy, uz, RT)]
    out = np.zeros((17, f[0].size))
    _check(lib().lelbm_moments_from_primitives3(K, f[0].size, *[_dp(a) for a in f], _dp(out)))
    return out


def make_params(cfg, precision=FP64, guess=GUESS_EQ):
    p = Params()
    p.dim, p.nx, p.ny = cfg["dim"], cfg["nx"], cfg.get("ny", 1)
    p.K = cfg["K"]
    p.omega_f, p.omega_b, p.omega_h = cfg["omega_f"], cfg["omega_b"], cfg["omega_h"]
    p.n_conf = cfg.get("n_conf", 4.0)
    p.r_min = cfg.get("r_min", 2)
    p.newton_tol = cfg.get("newton_tol", 1e-12)
    p.newton_max_it = cfg.get("newton_max_it", 50)
    p.kn_limiter = cfg.get("kn_limiter", 1)
    p.kn_lo, p.kn_hi, p.omega_H = cfg.get("kn_lo", -2.0), cfg.get("kn_hi", -1.0), cfg.get("omega_H", 1.0)
    p.precision = precision
    p.guess = guess
    for i, b in enumerate(cfg.get("bc", ["periodic"] * 4)[:4]):
        p.bc[i] = BC[b] if isinstance(b, str) else int(b)
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
        p._solid_ref = m                     # kept alive with the struct; the library copies it
        p.solid = m.ctypes.data_as(ctypes.c_void_p)
    src = cfg.get("source")
    if src is not None:
        p.src_x, p.src_y = src["x"], src.get("y", 0)
        p.src_rate, p.src_omega, p.src_t0 = src["rate"], src["omega"], src.get("t0", 0.0)
    for i, v in enumerate(cfg.get("wall_u", (0.0, 0.0, 0.0, 0.0))):
        p.wall_u[i] = v
    p.nz = cfg.get("nz", 0)
    return p


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Lelbm:
    """One simulation context (``lelbm_ctx``)."""

    def __init__(self, cfg, moments, precision=FP64, guess=GUESS_EQ, stream=None):
        self.cfg = cfg
        self.params = make_params(cfg, precision, guess)
        self.nmom = num_moments(cfg["dim"])
        self.shape = (self.nmom, (cfg.get("nz", 1) if cfg["dim"] == 3 else 1) * cfg.get("ny", 1) * cfg["nx"])
        self._h = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        if hasattr(moments, "data_ptr"):           # torch tensor on the device
            is32 = 1 if str(moments.dtype) == "torch.float32" else 0
            _check(lib().lelbm_create_device(ctypes.byref(self.params), ctypes.c_void_p(moments.data_ptr()),
                                             is32, self._stream, ctypes.byref(self._h)))
        else:
            m = np.ascontiguousarray(moments, dtype=np.float64).reshape(self.shape)
            _check(lib().lelbm_create(ctypes.byref(self.params), _dp(m), self._stream, ctypes.byref(self._h)))

    def step(self, n=1):
        st = Stats()
        code = lib().lelbm_step(self._h, n, ctypes.byref(st))
        if code != OK:
            node, stp = self.last_failure()
            why, sp, res = self.last_failure_detail()
            raise LelbmError(code, "%s at cell %d, step %d (reason %d, species %d, residual %.3e)"
                             % (lib().lelbm_strerror(code).decode(), node, stp, why, sp, res))
        return st.as_dict()

    def step_noalloc(self, n=1):
        """lelbm_step_noalloc: the same steps with the library's static scratch
        array and no allocation."""
        st = Stats()
        code = lib().lelbm_step_noalloc(self._h, n, ctypes.byref(st))
        if code != OK:
            node, stp = self.last_failure()
            raise LelbmError(code, "%s at cell %d, step %d" % (lib().lelbm_strerror(code).decode(), node, stp))
        return st.as_dict()

    def last_failure_detail(self):
        why, sp, res = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        lib().lelbm_last_failure_detail(self._h, ctypes.byref(why), ctypes.byref(sp), ctypes.byref(res))
        return why.value, sp.value, res.value

    def step_nostats(self, n=1):
        _check(lib().lelbm_step(self._h, n, None))

    def read_moments(self):
        out = np.zeros(self.shape)
        _check(lib().lelbm_read_moments(self._h, _dp(out)))
        return out

    def read_moments_device(self, tensor):
        _check(lib().lelbm_read_moments_device(self._h, ctypes.c_void_p(tensor.data_ptr())))

    def last_failure(self):
        node, stp = ctypes.c_long(), ctypes.c_int()
        lib().lelbm_last_failure(self._h, ctypes.byref(node), ctypes.byref(stp))
        return node.value, stp.value

    def set_timing(self, on):
        _check(lib().lelbm_set_timing(self._h, 1 if on else 0))

    def kernel_times(self):
        ms = (ctypes.c_double * 8)()
        ln = (ctypes.c_long * 8)()
        _check(lib().lelbm_kernel_times(self._h, ms, ln, 8))
        names = ["fill_pads", "prepare", "scan", "epr", "gather", "totals", "walls", "epr_ref"]
        return {n: (ms[i], ln[i]) for i, n in enumerate(names)}

    def memory(self):
        a, b = ctypes.c_long(), ctypes.c_long()
        _check(lib().lelbm_memory(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_scratch_budget(self, nbytes):
        _check(lib().lelbm_set_scratch_budget(self._h, int(nbytes)))

    def set_mlp(self, mlp):
        _check(lib().lelbm_set_mlp(self._h, mlp._h))

    def harvest(self, tensor, stride):
        """Record (features, multipliers) pairs into a torch float32 tensor of
        shape (capacity, 32) on the device; tensor=None stops."""
        if tensor is None:
            _check(lib().lelbm_harvest(self._h, None, 0, 1))
            self._harvest_ref = None
            return
        assert tensor.dtype == __import__("torch").float32 and tensor.shape[1] == 32 and tensor.is_contiguous()
        self._harvest_ref = tensor
        _check(lib().lelbm_harvest(self._h, ctypes.c_void_p(tensor.data_ptr()), tensor.shape[0], stride))

    def harvest_count(self):
        n = ctypes.c_longlong()
        _check(lib().lelbm_harvest_count(self._h, ctypes.byref(n)))
        return n.value

    def close(self):
        if self._h:
            lib().lelbm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create(cfg, moments, precision=FP64, guess=GUESS_EQ, stream=None):
    return Lelbm(cfg, moments, precision, guess, stream)


MLP_NPARAM = 6288


class Mlp:
    """Warm-start network (``lelbm_mlp``): training and inference run in the
    library's BF16-MFMA kernels; torch tensors supply device buffers."""

    def __init__(self, params=None, seed=0, stream=None):
        self._h = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        fp = ctypes.POINTER(ctypes.c_float)
        if params is not None:
            p = np.ascontiguousarray(params, dtype=np.float32)
            assert p.size == MLP_NPARAM
            _check(lib().lelbm_mlp_create(p.ctypes.data_as(fp), seed, self._stream, ctypes.byref(self._h)))
        else:
            _check(lib().lelbm_mlp_create(None, seed, self._stream, ctypes.byref(self._h)))

    def params(self):
        out = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check(lib().lelbm_mlp_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def fit_normalization(self, pairs):
        _check(lib().lelbm_mlp_fit_normalization(self._h, ctypes.c_void_p(pairs.data_ptr()), pairs.shape[0]))

    def norm(self):
        out = np.zeros(64, dtype=np.float32)
        _check(lib().lelbm_mlp_get_norm(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def set_norm(self, nm):
        nm = np.ascontiguousarray(nm, dtype=np.float32)
        _check(lib().lelbm_mlp_set_norm(self._h, nm.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def forward(self, x):
        """x: torch float32 (n, >=16) on the device -> (n, 16) outputs."""
        import torch
        n = x.shape[0]
        y = torch.empty((n, 16), dtype=torch.float32, device=x.device)
        _check(lib().lelbm_mlp_forward(self._h, ctypes.c_void_p(x.data_ptr()), x.stride(0), n,
                                       ctypes.c_void_p(y.data_ptr())))
        return y

    def gradient(self, pairs):
        """pairs: torch float32 (n, 32) on the device -> (gradient, loss)."""
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        loss = ctypes.c_double()
        _check(lib().lelbm_mlp_gradient(self._h, ctypes.c_void_p(pairs.data_ptr()), pairs.shape[0],
                                        g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss)))
        return g, loss.value

    def train(self, pairs, steps, batch=4096, lr=1e-3, seed=0):
        loss = ctypes.c_double()
        _check(lib().lelbm_mlp_train(self._h, ctypes.c_void_p(pairs.data_ptr()), pairs.shape[0], steps, batch,
                                     lr, seed, ctypes.byref(loss)))
        return loss.value

    def close(self):
        if self._h:
            lib().lelbm_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
