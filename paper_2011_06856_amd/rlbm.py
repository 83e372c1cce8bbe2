"""Python binding of librlbm.so (include/rlbm.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels.  PyTorch supplies
device memory (the workspace tensor) and the stream.  If the shared library is
missing the import of this module fails; there is no fallback.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "librlbm.so")

RLBM_OK, RLBM_EINVAL, RLBM_ENOMEM, RLBM_EDEVICE, RLBM_ENONPHYS, RLBM_ESTATE = 0, -1, -2, -3, -4, -5
RLBM_F64, RLBM_F32, RLBM_BF16DEV, RLBM_F32DEV, RLBM_F64DEV = 0, 1, 2, 3, 4
RLBM_BC_PERIODIC, RLBM_BC_CLAMP = 0, 1
PRECISIONS = {"f64": RLBM_F64, "f32": RLBM_F32, "bf16dev": RLBM_BF16DEV, "f32dev": RLBM_F32DEV,
              "f64dev": RLBM_F64DEV}
ELEM_BYTES = {RLBM_F64: 8, RLBM_F32: 4, RLBM_BF16DEV: 2, RLBM_F32DEV: 4, RLBM_F64DEV: 8}
DEVIATION = (RLBM_BF16DEV, RLBM_F32DEV, RLBM_F64DEV)

_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_L = None

# (name, restype, argtypes) of every exported entry point of include/rlbm.h
SIGNATURES = [
    ("rlbm_init_quadrature", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    ("rlbm_nvel", ctypes.c_int, [_vp]),
    ("rlbm_get_quadrature", ctypes.c_int, [_vp, _dp, _dp, _dp]),
    ("rlbm_workspace_bytes", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    ("rlbm_init_fields", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    ("rlbm_step", ctypes.c_int, [_vp, ctypes.c_int]),
    ("rlbm_step_timed", ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    ("rlbm_moments", ctypes.c_int, [_vp, _dp, _dp, _dp, _dp, _dp]),
    ("rlbm_moments_device", ctypes.c_int, [_vp, _vp, _vp]),
    ("rlbm_populations_bytes", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    ("rlbm_get_populations", ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    ("rlbm_set_populations", ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    ("rlbm_set_waves", ctypes.c_int, [_vp, ctypes.c_int]),
    ("rlbm_get_waves", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    ("rlbm_set_kernel", ctypes.c_int, [_vp, ctypes.c_int]),
    ("rlbm_get_kernel", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    ("rlbm_set_statistics", ctypes.c_int, [_vp, ctypes.c_int]),
    ("rlbm_host_feq", ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]),
    ("rlbm_host_landau", ctypes.c_int, [_dp, _dp]),
    ("rlbm_device_landau", ctypes.c_int, [ctypes.c_int, _dp, _dp]),
    ("rlbm_batch_create", ctypes.c_int, [ctypes.POINTER(_vp), _vp, ctypes.c_int, ctypes.c_int, _vp]),
    ("rlbm_batch_count", ctypes.c_int, [_vp]),
    ("rlbm_batch_problem", ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_vp)]),
    ("rlbm_batch_step", ctypes.c_int, [_vp, ctypes.c_int]),
    ("rlbm_batch_step_eager", ctypes.c_int, [_vp, ctypes.c_int]),
    ("rlbm_batch_step_timed", ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    ("rlbm_batch_set_waves", ctypes.c_int, [_vp, ctypes.c_int]),
    ("rlbm_batch_get_waves", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    ("rlbm_batch_set_push_bands", ctypes.c_int, [_vp, ctypes.c_int]),
    ("rlbm_batch_get_push_bands", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    ("rlbm_batch_set_mode", ctypes.c_int, [_vp, ctypes.c_int]),
    ("rlbm_batch_get_mode", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    ("rlbm_batch_autotune", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int), _dp]),
    ("rlbm_mlp_create", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, _vp]),
    ("rlbm_mlp_nparams", ctypes.c_long, [_vp]),
    ("rlbm_mlp_set_params", ctypes.c_int, [_vp, _vp]),
    ("rlbm_mlp_get_params", ctypes.c_int, [_vp, _vp]),
    ("rlbm_mlp_get_grad", ctypes.c_int, [_vp, _vp]),
    ("rlbm_mlp_set_norm", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    ("rlbm_mlp_forward", ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp]),
    ("rlbm_mlp_grad", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _dp]),
    ("rlbm_mlp_adam_step", ctypes.c_int, [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    ("rlbm_site_stats", ctypes.c_int, [_vp, _vp]),
    ("rlbm_mlp_features", ctypes.c_int, [_vp, _vp, _vp]),
    ("rlbm_mlp_correct", ctypes.c_int, [_vp, _vp, ctypes.c_float, ctypes.c_int]),
    ("rlbm_mlp_readout", ctypes.c_int, [_vp, _vp, ctypes.c_float, _dp, _dp, _dp, _dp]),
    ("rlbm_mlp_set_extra", ctypes.c_int, [_vp, ctypes.c_float]),
    ("rlbm_add_stress", ctypes.c_int, [_vp, _vp, ctypes.c_float]),
    ("rlbm_resample", ctypes.c_int, [_vp, _vp]),
    ("rlbm_mlp_last_error", ctypes.c_char_p, [_vp]),
    ("rlbm_mlp_destroy", ctypes.c_int, [_vp]),
    ("rlbm_batch_info", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    ("rlbm_batch_last_error", ctypes.c_char_p, [_vp]),
    ("rlbm_batch_destroy", ctypes.c_int, [_vp]),
    ("rlbm_last_error", ctypes.c_char_p, [_vp]),
    ("rlbm_destroy", ctypes.c_int, [_vp]),
]


class RlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("rlbm error %d: %s" % (code, msg))
        self.code = code


class NonPhysicalState(RlbmError):
    pass


def lib():
    """Load librlbm.so (built in-tree by paper_2011_06856_amd.build)."""
    global _L
    if _L is None:
        # torch ships its own libamdhip64.so.7; load it (and initialise it)
        # first so that librlbm.so binds to the same HIP runtime by soname.
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:
            pass
        if not os.path.exists(SO_PATH):
            raise ImportError("librlbm.so is not built: run `python -m paper_2011_06856_amd.build` "
                              "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(SO_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        _L = L
    return _L


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _arr(a, shape):
    if a is None:
        return None
    return np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))


def host_landau(mom9):
    """Landau frame of nine moments with the library's host code (no GPU):
    (n, eps, U^x, U^y, T, U^0), ok."""
    m = np.ascontiguousarray(mom9, dtype=np.float64)
    out = np.zeros(6)
    rc = lib().rlbm_host_landau(_p(m), _p(out))
    return out, rc == RLBM_OK


def device_landau(moms):
    """Landau frames of moment sets (count, 9) on the GPU: (count, 7) with
    columns n, eps, U^x, U^y, T, U^0, ok."""
    m = np.ascontiguousarray(moms, dtype=np.float64).reshape(-1, 9)
    out = np.zeros((m.shape[0], 7))
    rc = lib().rlbm_device_landau(m.shape[0], _p(m), _p(out))
    if rc != RLBM_OK:
        raise RlbmError(rc, "device_landau failed")
    return out


class RlbmProblem(ctypes.Structure):
    """rlbm_problem of include/rlbm.h."""
    _fields_ = [("n_radial", ctypes.c_int), ("n_angle", ctypes.c_int), ("order", ctypes.c_int),
                ("rotate", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("n", _dp), ("T", _dp), ("ux", _dp), ("uy", _dp),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double), ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int)]


class Solver:
    """One simulation context (rlbm_ctx)."""

    @classmethod
    def view(cls, handle, Np, K, N, nx, ny, precision):
        """Non-owning view of a context owned by a batch."""
        s = cls.__new__(cls)
        s._h, s._owned = handle, False
        s.Np, s.K, s.N = Np, K, N
        s.nvel = lib().rlbm_nvel(handle)
        s.nx, s.ny, s.precision = nx, ny, precision
        s.workspace = None
        return s

    def __init__(self, n_radial, n_angle, order=None, rotate=True):
        self._owned = True
        order = n_radial - 1 if order is None else order
        h = _vp()
        rc = lib().rlbm_init_quadrature(ctypes.byref(h), int(n_radial), int(n_angle), int(order), 1 if rotate else 0)
        if rc != RLBM_OK:
            raise RlbmError(rc, "invalid quadrature (Np=%d, K=%d, N=%d)" % (n_radial, n_angle, order))
        self._h = h
        self.Np, self.K, self.N = int(n_radial), int(n_angle), int(order)
        self.nvel = lib().rlbm_nvel(h)
        self.workspace = None
        self.nx = self.ny = 0
        self.precision = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and getattr(self, "_owned", True) and _L is not None:
            _L.rlbm_destroy(h)
        self._h = None

    def _check(self, rc):
        if rc == RLBM_OK:
            return
        msg = lib().rlbm_last_error(self._h).decode()
        if rc == RLBM_ENONPHYS:
            raise NonPhysicalState(rc, msg)
        raise RlbmError(rc, msg)

    def quadrature(self):
        p, th, w = (np.zeros(self.nvel) for _ in range(3))
        self._check(lib().rlbm_get_quadrature(self._h, _p(p), _p(th), _p(w)))
        return p, th, w

    def host_feq(self, n, T, ux=0.0, uy=0.0):
        out = np.zeros(self.nvel)
        self._check(lib().rlbm_host_feq(self._h, n, T, ux, uy, _p(out)))
        return out

    def workspace_bytes(self, nx, ny, precision="f32"):
        b = ctypes.c_size_t()
        self._check(lib().rlbm_workspace_bytes(self._h, nx, ny, PRECISIONS[precision], ctypes.byref(b)))
        return b.value

    def init_fields(self, nx, ny, n, T, ux=None, uy=None, tau=math.inf, dt=1.0, bcx=0, bcy=0,
                    precision="f32", device=None, stream=None, workspace=None):
        """Fields are (ny, nx) host arrays.  The workspace is a torch uint8
        tensor on the GPU unless given."""
        import torch
        prec = PRECISIONS[precision]
        shape = (ny, nx)
        n, T, ux, uy = _arr(n, shape), _arr(T, shape), _arr(ux, shape), _arr(uy, shape)
        if workspace is None:
            nbytes = self.workspace_bytes(nx, ny, precision)
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")
        if stream is None:
            stream = torch.cuda.current_stream(workspace.device)
        rc = lib().rlbm_init_fields(self._h, nx, ny, _p(n), _p(T), _p(ux), _p(uy), float(tau), float(dt),
                                    int(bcx), int(bcy), prec, _vp(workspace.data_ptr()), _vp(stream.cuda_stream))
        # the context refers to the new workspace only after a successful
        # call; after a failed one it holds no fields and uses no workspace
        if rc == RLBM_OK:
            self.workspace, self.stream = workspace, stream
            self.nx, self.ny, self.precision = nx, ny, prec
        self._check(rc)
        return self

    def step(self, nsteps=1):
        self._check(lib().rlbm_step(self._h, int(nsteps)))

    def step_timed(self, nsteps):
        ms = ctypes.c_double()
        self._check(lib().rlbm_step_timed(self._h, int(nsteps), ctypes.byref(ms)))
        return ms.value

    def moments(self, raise_nonphysical=True):
        """n, eps, U^x, U^y as (ny, nx) arrays and the four global charges."""
        shape = (self.ny, self.nx)
        n, eps, ux, uy = (np.empty(shape) for _ in range(4))
        ch = np.zeros(4)
        rc = lib().rlbm_moments(self._h, _p(n), _p(eps), _p(ux), _p(uy), _p(ch))
        if rc != RLBM_ENONPHYS or raise_nonphysical:
            self._check(rc)
        return n, eps, ux, uy, ch

    def moments_device(self, fields=None, charges=None):
        """rlbm_moments_device: fields (torch float64 tensor of 4 * ny * nx
        elements on the context's device, or None) and charges (4 elements,
        or None) are written asynchronously on the context's stream."""
        import torch
        for t, n in ((fields, 4 * self.nx * self.ny), (charges, 4)):
            if t is not None and (t.dtype != torch.float64 or t.numel() != n or not t.is_contiguous()):
                raise ValueError("moments_device: need a contiguous float64 tensor of %d elements" % n)
        self._check(lib().rlbm_moments_device(self._h, None if fields is None else _vp(fields.data_ptr()),
                                              None if charges is None else _vp(charges.data_ptr())))

    def populations_bytes(self):
        b = ctypes.c_size_t()
        self._check(lib().rlbm_populations_bytes(self._h, ctypes.byref(b)))
        return b.value

    def get_populations(self):
        """Plain storage: f as (nvel, ny, nx).  Deviation storage: the raw
        checkpoint bytes (deviations, then equilibrium coefficients)."""
        if self.precision in DEVIATION:
            buf = np.empty(self.populations_bytes(), dtype=np.uint8)
            self._check(lib().rlbm_get_populations(self._h, _vp(buf.ctypes.data), buf.nbytes))
            return buf
        dt = {RLBM_F64: np.float64, RLBM_F32: np.float32}[self.precision]
        buf = np.empty(self.populations_bytes() // np.dtype(dt).itemsize, dtype=dt)
        self._check(lib().rlbm_get_populations(self._h, _vp(buf.ctypes.data), buf.nbytes))
        return buf.reshape(self.nvel, self.ny, self.nx)

    def set_populations(self, f):
        f = np.ascontiguousarray(f)
        self._check(lib().rlbm_set_populations(self._h, _vp(f.ctypes.data), f.nbytes))

    def set_waves(self, waves):
        self._check(lib().rlbm_set_waves(self._h, int(waves)))

    def get_waves(self):
        w = ctypes.c_int()
        self._check(lib().rlbm_get_waves(self._h, ctypes.byref(w)))
        return w.value

    STATISTICS = {"mj": 0, "fd": 1, "be": 2}

    def set_statistics(self, name):
        """Equilibrium statistics for the next init_fields (and host_feq):
        "mj" Maxwell-Juttner, "fd" Fermi-Dirac, "be" Bose-Einstein."""
        self._check(lib().rlbm_set_statistics(self._h, self.STATISTICS[name]))
        return self

    KERNELS = {"auto": 0, "tile": 1, "push": 2}

    def set_kernel(self, kind):
        """Step kernel: "auto", "tile" or "push" (same step, two schedules)."""
        self._check(lib().rlbm_set_kernel(self._h, self.KERNELS[kind]))
        return self

    def get_kernel(self):
        k = ctypes.c_int()
        self._check(lib().rlbm_get_kernel(self._h, ctypes.byref(k)))
        return {v: n for n, v in self.KERNELS.items()}[k.value]


class Batch:
    """A batch of independent problems advanced together (rlbm_batch).

    problems: list of dicts with keys Np, K, N, nx, ny, fields=(n, T, ux, uy),
    tau, dt and optional bcx, bcy, rotate.
    """

    def __init__(self, problems, precision="f32", stream=None):
        import torch
        torch.cuda.init()
        prec = PRECISIONS[precision]
        arr = (RlbmProblem * len(problems))()
        self._keep = []
        for i, p in enumerate(problems):
            shape = (p["ny"], p["nx"])
            fl = [_arr(a, shape) if a is not None else None for a in p["fields"]]
            self._keep.append(fl)
            arr[i] = RlbmProblem(p["Np"], p["K"], p.get("N", p["Np"] - 1), 1 if p.get("rotate", True) else 0,
                                 p["nx"], p["ny"], _p(fl[0]), _p(fl[1]), _p(fl[2]), _p(fl[3]),
                                 float(p["tau"]), float(p["dt"]), int(p.get("bcx", 0)), int(p.get("bcy", 0)))
        self.stream = stream   # None: the library creates and owns a stream
        h = _vp()
        rc = lib().rlbm_batch_create(ctypes.byref(h), ctypes.cast(arr, _vp), len(problems), prec,
                                     _vp(stream.cuda_stream) if stream is not None else None)
        if rc != RLBM_OK:
            raise RlbmError(rc, "rlbm_batch_create failed")
        self._h = h
        self.problems = problems
        self.precision = prec
        self.views = []
        for i, p in enumerate(problems):
            c = _vp()
            self._check(lib().rlbm_batch_problem(h, i, ctypes.byref(c)))
            self.views.append(Solver.view(c, p["Np"], p["K"], p.get("N", p["Np"] - 1), p["nx"], p["ny"], prec))
        self.nsv = sum(v.nvel * p["nx"] * p["ny"] for v, p in zip(self.views, problems))

    def __del__(self):
        h = getattr(self, "_h", None)
        self.views = []
        if h and _L is not None:
            _L.rlbm_batch_destroy(h)
        self._h = None

    def _check(self, rc):
        if rc != RLBM_OK:
            raise RlbmError(rc, lib().rlbm_batch_last_error(self._h).decode())

    def __len__(self):
        return len(self.views)

    def problem(self, i):
        return self.views[i]

    def step(self, nsteps=1):
        self._check(lib().rlbm_batch_step(self._h, int(nsteps)))

    def step_eager(self, nsteps=1):
        self._check(lib().rlbm_batch_step_eager(self._h, int(nsteps)))

    def step_timed(self, nsteps):
        ms = ctypes.c_double()
        self._check(lib().rlbm_batch_step_timed(self._h, int(nsteps), ctypes.byref(ms)))
        return ms.value

    def set_waves(self, waves):
        self._check(lib().rlbm_batch_set_waves(self._h, int(waves)))

    def info(self):
        """(resident work-groups of the persistent launch, work items per step)"""
        g, it = ctypes.c_int(), ctypes.c_int()
        self._check(lib().rlbm_batch_info(self._h, ctypes.byref(g), ctypes.byref(it)))
        return g.value, it.value

    def get_waves(self):
        w = ctypes.c_int()
        self._check(lib().rlbm_batch_get_waves(self._h, ctypes.byref(w)))
        return w.value

    MODES = {"persistent": 0, "flat": 1}

    def set_mode(self, mode):
        """Launch mode of a step: "persistent" (work queues) or "flat"."""
        self._check(lib().rlbm_batch_set_mode(self._h, self.MODES[mode]))

    def get_mode(self):
        m = ctypes.c_int()
        self._check(lib().rlbm_batch_get_mode(self._h, ctypes.byref(m)))
        return {v: k for k, v in self.MODES.items()}[m.value]

    def set_push_bands(self, bands):
        """Work-group order of the push-kernel problems: bands of 4 rows per
        group (0: the built-in choice); results do not depend on it."""
        self._check(lib().rlbm_batch_set_push_bands(self._h, int(bands)))

    def get_push_bands(self):
        v = ctypes.c_int()
        self._check(lib().rlbm_batch_get_push_bands(self._h, ctypes.byref(v)))
        return v.value

    def autotune(self, candidates=(2, 3, 4, 6, 8), steps=6, cache=None, key=None):
        """Pick the fastest work-group shape and launch mode, then the push
        part's band grouping; with `cache` (a JSON file path) and `key`,
        reuse a stored choice or store the new one."""
        import json
        if cache and key and os.path.exists(cache):
            try:
                d = json.load(open(cache))
                if key in d:
                    self.set_waves(d[key]["waves"])
                    self.set_mode(d[key].get("mode", "persistent"))
                    self.set_push_bands(d[key].get("push_bands", 0))
                    return d[key]["waves"], d[key]["ms"]
            except (ValueError, KeyError):
                pass
        c = (ctypes.c_int * len(candidates))(*candidates)
        bw, bms = ctypes.c_int(), ctypes.c_double()
        self._check(lib().rlbm_batch_autotune(self._h, c, len(candidates), int(steps), ctypes.byref(bw),
                                              ctypes.byref(bms)))
        if cache and key:
            d = {}
            if os.path.exists(cache):
                try:
                    d = json.load(open(cache))
                except ValueError:
                    d = {}
            d[key] = {"waves": bw.value, "mode": self.get_mode(), "push_bands": self.get_push_bands(),
                      "ms": bms.value}
            json.dump(d, open(cache, "w"), indent=1)
        return bw.value, bms.value


def _fptr(t):
    """Device pointer of a contiguous float32 torch tensor."""
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    return _vp(t.data_ptr())


def site_stats(solver):
    """(S, 8) device tensor: n, eps, U^x, U^y, pi^xx, pi^xy, pi^yy, 0 per site."""
    import torch
    out = torch.empty((solver.nx * solver.ny, 8), dtype=torch.float32, device="cuda")
    rc = lib().rlbm_site_stats(solver._h, _fptr(out))
    if rc != RLBM_OK:
        raise RlbmError(rc, "rlbm_site_stats failed")
    return out


def add_stress(solver, dstress, scale=1.0):
    """Add a change of the traceless stress (device (S, 3) tensor: dT^xx,
    dT^xy, dT^yy) to the populations, leaving N^mu and T^0mu unchanged."""
    rc = lib().rlbm_add_stress(solver._h, _fptr(dstress), float(scale))
    if rc != RLBM_OK:
        raise RlbmError(rc, "rlbm_add_stress failed")


def resample(src, dst):
    """Resample src's populations onto dst's angle set (same grid and shells)."""
    rc = lib().rlbm_resample(src._h, dst._h)
    if rc != RLBM_OK:
        raise RlbmError(rc, "rlbm_resample failed")


class MLP:
    """The learned correction network (rlbm_mlp): in_dim -> hidden^n_hidden -> out_dim."""

    def __init__(self, in_dim=64, hidden=128, n_hidden=3, out_dim=3, max_batch=65536, stream=None):
        h = _vp()
        rc = lib().rlbm_mlp_create(ctypes.byref(h), in_dim, hidden, n_hidden, out_dim, max_batch,
                                   _vp(stream.cuda_stream) if stream is not None else None)
        if rc != RLBM_OK:
            raise RlbmError(rc, "rlbm_mlp_create failed")
        self._h = h
        self.in_dim, self.hidden, self.n_hidden, self.out_dim, self.max_batch = in_dim, hidden, n_hidden, out_dim, max_batch
        self.nparams = int(lib().rlbm_mlp_nparams(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _L is not None:
            _L.rlbm_mlp_destroy(h)
        self._h = None

    def _check(self, rc):
        if rc != RLBM_OK:
            raise RlbmError(rc, lib().rlbm_mlp_last_error(self._h).decode())

    def layer_shapes(self):
        dims = [self.in_dim] + [self.hidden] * self.n_hidden + [self.out_dim]
        return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]

    def init_params(self, seed=0):
        """He-style uniform initialisation from the counter-based generator."""
        import workloads as W
        out, k = [], 0
        for (o, i) in self.layer_shapes():
            u = W.uniform(seed, k + np.arange(o * i))
            k += o * i
            lim = np.sqrt(6.0 / i) if o != self.out_dim else np.sqrt(1.0 / i)
            out.append(((2 * u - 1) * lim).astype(np.float32))
            out.append(np.zeros(o, dtype=np.float32))
        p = np.concatenate(out)
        self.set_params(p)
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparams
        self._check(lib().rlbm_mlp_set_params(self._h, _vp(p.ctypes.data)))

    def get_params(self):
        p = np.empty(self.nparams, dtype=np.float32)
        self._check(lib().rlbm_mlp_get_params(self._h, _vp(p.ctypes.data)))
        return p

    def get_grad(self):
        g = np.empty(self.nparams, dtype=np.float32)
        self._check(lib().rlbm_mlp_get_grad(self._h, _vp(g.ctypes.data)))
        return g

    def set_norm(self, in_mu, in_sig, out_mu, out_sig):
        a = [np.ascontiguousarray(x, dtype=np.float32) for x in (in_mu, in_sig, out_mu, out_sig)]
        self._keep_norm = a
        self._check(lib().rlbm_mlp_set_norm(self._h, *[_vp(x.ctypes.data) for x in a]))

    def forward(self, X):
        import torch
        Y = torch.empty((X.shape[0], self.out_dim), dtype=torch.float32, device="cuda")
        self._check(lib().rlbm_mlp_forward(self._h, _fptr(X), int(X.shape[0]), _fptr(Y)))
        return Y

    def grad(self, X, T):
        loss = ctypes.c_double()
        self._check(lib().rlbm_mlp_grad(self._h, _fptr(X), _fptr(T), int(X.shape[0]), ctypes.byref(loss)))
        return loss.value

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self._check(lib().rlbm_mlp_adam_step(self._h, lr, b1, b2, eps))

    def features(self, solver):
        import torch
        X = torch.empty((solver.nx * solver.ny, self.in_dim), dtype=torch.float32, device="cuda")
        self._check(lib().rlbm_mlp_features(solver._h, self._h, _fptr(X)))
        return X

    def set_extra(self, extra):
        """The per-run input in column 63 of the features (e.g. log10 Kn)."""
        self._check(lib().rlbm_mlp_set_extra(self._h, float(extra)))

    def readout(self, solver, extra):
        """Readout-corrected fields n, eps, U^x, U^y ([ny][nx] each) of the
        solver's current populations (a network with out_dim = 4)."""
        out = [np.empty((solver.ny, solver.nx)) for _ in range(4)]
        rc = lib().rlbm_mlp_readout(solver._h, self._h, float(extra), *[_p(a) for a in out])
        if rc == RLBM_ENONPHYS:
            solver._check(rc)
        self._check(rc)
        return out

    def correct(self, solver, scale=1.0, relax=False):
        self._check(lib().rlbm_mlp_correct(solver._h, self._h, float(scale), int(bool(relax))))
