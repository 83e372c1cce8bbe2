"""ctypes binding of the FP64 CPU oracle (``rlbm_oracle.c``).

Test infrastructure only (see the package docstring).  The shared library is
compiled with gcc by :func:`build`; :func:`_lib` builds it on first use when it
is missing.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rlbm_oracle.c")
_SO = os.path.join(_HERE, "librlbm_oracle.so")
_L = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force=True):
    """Compile the oracle with gcc (OpenMP, -O2, strict IEEE: no -ffast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _L
    if _L is None:
        build(force=False)
        L = ctypes.CDLL(_SO)
        L.orc_quad_new.restype = ctypes.c_void_p
        L.orc_quad_new.argtypes = [ctypes.c_int] * 4
        L.orc_quad_free.argtypes = [ctypes.c_void_p]
        L.orc_quad_nvel.argtypes = [ctypes.c_void_p]
        L.orc_quad_nbasis.argtypes = [ctypes.c_void_p]
        L.orc_quad_get.argtypes = [ctypes.c_void_p] + [_dp] * 5
        L.orc_quad_basis.argtypes = [ctypes.c_void_p, _dp, _ip]
        L.orc_mj_moment.restype = ctypes.c_double
        L.orc_mj_moment.argtypes = [ctypes.c_int, _ip] + [ctypes.c_double] * 4
        L.orc_feq.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 4 + [_dp]
        L.orc_eq_coeffs.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 4 + [_dp]
        L.orc_moments.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_landau.argtypes = [_dp, _dp]
        L.orc_sim_new.restype = ctypes.c_void_p
        L.orc_sim_new.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_feq_qs.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 4 + [ctypes.c_int, _dp]
        L.orc_qs_G.restype = ctypes.c_double
        L.orc_qs_G.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.orc_qs_landau.argtypes = [_dp, ctypes.c_int, _dp]
        L.orc_sim_free.argtypes = [ctypes.c_void_p]
        L.orc_sim_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_sim_stream.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_sim_fields.restype = ctypes.c_long
        L.orc_sim_fields.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        L.orc_sim_moments.argtypes = [ctypes.c_void_p, _dp]
        L.orc_sim_charges.argtypes = [ctypes.c_void_p, _dp]
        L.orc_sim_get_f.argtypes = [ctypes.c_void_p, _dp]
        L.orc_sim_set_f.argtypes = [ctypes.c_void_p, _dp]
        L.orc_sim_nonphys.restype = ctypes.c_long
        L.orc_sim_nonphys.argtypes = [ctypes.c_void_p]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _L = L
    return _L


def _ptr(a):
    return a.ctypes.data_as(_dp)


def num_threads():
    """OpenMP threads the oracle uses."""
    return int(_lib().orc_num_threads())


def set_threads(n):
    """Use n OpenMP threads from now on."""
    _lib().orc_set_threads(int(n))


class Quadrature:
    """Product quadrature and orthonormal basis (Sec. 2.3, Eq. off-lattice-quad).

    Np radial shells (roots of L_Np), K angles per shell, expansion order N,
    ``rotate`` toggles the per-shell angular offset i/Np.
    """

    def __init__(self, Np, K, N, rotate=True):
        self.Np, self.K, self.N, self.rotate = Np, K, N, bool(rotate)
        self._h = _lib().orc_quad_new(Np, K, N, 1 if rotate else 0)
        if not self._h:
            raise ValueError("invalid quadrature (Np=%d K=%d N=%d)" % (Np, K, N))
        self.nvel = _lib().orc_quad_nvel(self._h)
        self.nb = _lib().orc_quad_nbasis(self._h)
        arrs = [np.zeros(self.nvel) for _ in range(5)]
        _lib().orc_quad_get(self._h, *[_ptr(a) for a in arrs])
        self.p, self.theta, self.w, self.cth, self.sth = arrs

    def __del__(self):
        if getattr(self, "_h", None):
            _lib().orc_quad_free(self._h)
            self._h = None

    def basis(self):
        """J[b][v] at the nodes and the monomial exponents (a, b, c) of each b."""
        J = np.zeros((self.nb, self.nvel))
        ex = np.zeros((self.nb, 3), dtype=np.int32)
        _lib().orc_quad_basis(self._h, _ptr(J), ex.ctypes.data_as(_ip))
        return J, ex

    def feq(self, n, T, ux=0.0, uy=0.0, stat=0):
        """Discrete truncated equilibrium f_eq_v (Eq. mj-feq-expansion-truncated)
        of the statistics stat (0 Maxwell-Juttner, 1 Fermi-Dirac, 2
        Bose-Einstein; Eq. feq_dist)."""
        out = np.zeros(self.nvel)
        if stat == 0:
            _lib().orc_feq(self._h, n, T, ux, uy, _ptr(out))
        elif _lib().orc_feq_qs(self._h, n, T, ux, uy, int(stat), _ptr(out)):
            raise ValueError("no equilibrium of statistics %d at n=%g, T=%g" % (stat, n, T))
        return out

    def eq_coeffs(self, n, T, ux=0.0, uy=0.0):
        out = np.zeros(self.nb)
        _lib().orc_eq_coeffs(self._h, n, T, ux, uy, _ptr(out))
        return out

    def moments(self, f):
        """(N^0, N^x, N^y, T^00, T^0x, T^0y, T^xx, T^xy, T^yy) of one site."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(9)
        _lib().orc_moments(self._h, _ptr(f), _ptr(out))
        return out


def mj_moment(idx, n, T, ux=0.0, uy=0.0):
    """Closed-form rank-k moment of the Maxwell-Juttner equilibrium; idx in {0,1,2}^k."""
    a = np.ascontiguousarray(idx, dtype=np.int32)
    return _lib().orc_mj_moment(len(a), a.ctypes.data_as(_ip), n, T, ux, uy)


def landau(mom):
    """Landau-frame solve of nine moments -> (n, eps, U^x, U^y, T, U^0), ok flag."""
    m = np.ascontiguousarray(mom, dtype=np.float64)
    out = np.zeros(6)
    bad = _lib().orc_landau(_ptr(m), _ptr(out))
    return out, bad == 0


STATISTICS = {"mj": 0, "fd": 1, "be": 2}


def qs_G(k, z, stat):
    """Radial integral G_k(z) of the statistics (z, -Li_{k+1}(-z), Li_{k+1}(z))."""
    return _lib().orc_qs_G(int(k), float(z), int(stat))


def qs_landau(mom, stat):
    """Landau frame and statistics -> (n, eps, U^x, U^y, T, U^0, z, phi_2), ok."""
    m = np.ascontiguousarray(mom, dtype=np.float64)
    out = np.zeros(8)
    bad = _lib().orc_qs_landau(_ptr(m), int(stat), _ptr(out))
    return out, bad == 0


def site_stats(mom):
    """(n, eps, U^x, U^y, pi^xx, pi^xy, pi^yy) of one site from its nine
    moments: Landau frame, then the shear stress of the Landau-Lifshitz
    decomposition T^ij = (eps + P) U^i U^j + P delta^ij + pi^ij with the
    massless equation of state P = eps / 2 (Sec. 2)."""
    fr, ok = landau(mom)
    if not ok:
        return None
    n, eps, ux, uy = fr[0], fr[1], fr[2], fr[3]
    P, w = 0.5 * eps, 1.5 * eps
    return np.array([n, eps, ux, uy, mom[6] - w * ux * ux - P, mom[7] - w * ux * uy, mom[8] - w * uy * uy - P])


class Sim:
    """Lattice evolution on an nx x ny grid (Eq. discrete-rbe).

    Fields are host arrays of shape (ny, nx); u = spatial part U^i of the
    four-velocity.  bc: 0 periodic, 1 clamp (zero gradient), per axis.
    """

    def __init__(self, quad, nx, ny, n, T, ux=None, uy=None, tau=np.inf, dt=1.0, bcx=0, bcy=0, stat=0):
        self.q, self.nx, self.ny = quad, nx, ny
        S = nx * ny
        fld = [np.ascontiguousarray(np.broadcast_to(a, (ny, nx)), dtype=np.float64).reshape(S)
               for a in (n, T, 0.0 if ux is None else ux, 0.0 if uy is None else uy)]
        self._keep = fld
        self._h = _lib().orc_sim_new(quad._h, nx, ny, *[_ptr(a) for a in fld],
                                     float(tau), float(dt), int(bcx), int(bcy), int(stat))
        if not self._h:
            raise ValueError("invalid simulation arguments")

    def __del__(self):
        if getattr(self, "_h", None):
            _lib().orc_sim_free(self._h)
            self._h = None

    def step(self, nsteps=1):
        _lib().orc_sim_step(self._h, int(nsteps))

    def stream(self, nsteps=1):
        _lib().orc_sim_stream(self._h, int(nsteps))

    def fields(self):
        """n, eps, U^x, U^y of the stored populations, each (ny, nx)."""
        S = self.nx * self.ny
        out = [np.zeros(S) for _ in range(4)]
        _lib().orc_sim_fields(self._h, *[_ptr(a) for a in out])
        return [a.reshape(self.ny, self.nx) for a in out]

    def moments(self):
        out = np.zeros((9, self.ny, self.nx))
        _lib().orc_sim_moments(self._h, _ptr(out))
        return out

    def charges(self):
        out = np.zeros(4)
        _lib().orc_sim_charges(self._h, _ptr(out))
        return out

    def get_f(self):
        out = np.zeros((self.q.nvel, self.ny, self.nx))
        _lib().orc_sim_get_f(self._h, _ptr(out))
        return out

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.size == self.q.nvel * self.nx * self.ny
        _lib().orc_sim_set_f(self._h, _ptr(f))

    def nonphys(self):
        return int(_lib().orc_sim_nonphys(self._h))
