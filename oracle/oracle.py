"""ctypes wrapper of the C oracle (test infrastructure only)."""
import ctypes as C
import os

import numpy as np

from .build import OUT as lib_path, OUT_OMP as lib_path_omp, build as _build

_lib = None
_lib_omp = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def build(force=True):
    global _lib, _lib_omp
    _lib = None
    _lib_omp = None
    return _build(force=force)


def _load(threaded=False):
    """the serial oracle, or (threaded=True) its -fopenmp build"""
    global _lib, _lib_omp
    if threaded and _lib_omp is not None:
        return _lib_omp
    if not threaded and _lib is not None:
        return _lib
    _build(force=False)
    lib = C.CDLL(lib_path_omp if threaded else lib_path)
    vp = C.c_void_p
    sig = {
        "or_create": (vp, [_ip, _dp, _dp]),
        "or_destroy": (None, [vp]),
        "or_set_state": (None, [vp, _dp]),
        "or_get_state": (None, [vp, _dp]),
        "or_rhs": (None, [vp, _dp, _dp]),
        "or_cn_old": (None, [vp, _dp, C.c_double, _dp]),
        "or_residual": (None, [vp, _dp, _dp, C.c_double, _dp]),
        "or_time_step": (None, [vp, _dp, _dp]),
        "or_set_scales": (None, [vp, _dp]),
        "or_jv": (None, [vp, _dp, _dp, C.c_double, _dp, _dp]),
        "or_jv_eps": (None, [vp, _dp, _dp, C.c_double, _dp, C.c_double, _dp]),
        "or_precond": (None, [vp, _dp, C.c_double, _dp, _dp]),
        "or_newton_solve": (C.c_int, [vp, C.c_double, _dp]),
        "or_newton_history": (C.c_int, [vp, _dp, _dp, _dp, C.c_int]),
        "or_ew_forcing": (C.c_double, [C.c_double] * 5),
        "or_extrap_info": (None, [vp, _dp]),
        "or_implicit_step": (C.c_int, [vp, _dp]),
        "or_get_sources": (None, [vp, _dp]),
        "or_set_scalars": (None, [vp, C.c_int, C.c_int, _dp]),
        "or_get_scalars": (None, [vp, _dp]),
        "or_scalar_rhs": (None, [vp, _dp, _dp, _dp]),
        "or_scalar_its": (C.c_int, [vp, _ip]),
        "or_threads": (C.c_int, []),
        "or_tridiag": (None, [C.c_int, _dp, _dp, _dp, _dp, _dp, C.c_int]),
        "or_gmres_dense": (None, [C.c_long, _dp, _dp, _dp, _dp, C.c_int, C.c_int, C.c_double, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if threaded:
        _lib_omp = lib
    else:
        _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _arr(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


STAT_KEYS = ("t", "dt", "cfl_hydro", "cfl_adv", "cfl_rad", "rel_res", "max_rel_corr",
             "mass_drift", "energy_drift", "newton_its", "gmres_its", "rejections",
             "status", "f0", "f", "newton_exit")


class Oracle:
    """One problem held by the oracle: desc/opts dicts as built by workloads."""

    def __init__(self, desc, opts, u0, threaded=False):
        """threaded=True: the -fopenmp build (same results bit for bit, used
        to time the oracle on all host cores)"""
        lib = _load(threaded)
        self._lib = lib
        self.desc, self.opts = dict(desc), dict(opts)
        n = desc["n"]
        self.N = n[0] * n[1] * n[2]
        self.nvec = (2 + desc["ndim"]) * self.N
        ip = np.array([desc["ndim"], n[0], n[1], n[2], desc["bc"][0], desc["bc"][1],
                       desc["bc"][2], desc["heat_balance"], opts["newton_max"],
                       opts["gmres_restart"], opts["gmres_max_cycles"], opts["pc"],
                       opts["max_halvings"], opts["pc_solver"], opts["mg_nu1"], opts["mg_nu2"],
                       opts["mg_nuc"], opts["mg_cycles"], desc.get("energy_form", 0),
                       desc.get("geometry", 0), opts.get("mg_light_cells", 0),
                       opts.get("newton_target", 0), opts.get("scalar_converge", 1),
                       opts.get("gmres_forcing", 0), opts.get("newton_extrapolate", 0)], dtype=np.int32)
        dp = np.array(list(desc["lo"]) + list(desc["hi"]) + [desc["gamma"]] + list(desc["g"]) +
                      [desc["chi0"], opts["newton_rtol"], opts["newton_atol"], opts["gmres_eta"],
                       opts["cfl_hydro"], opts["cfl_adv_max"], opts["cfl_rad_max"], opts["dt_max"],
                       opts["newton_corr_tol"], opts.get("dt_grow", 0.0)],
                      dtype=np.float64)
        u0 = _arr(u0, self.nvec)
        self._h = lib.or_create(ip.ctypes.data_as(_ip), _d(dp), _d(u0))
        if not self._h:
            raise RuntimeError("or_create failed")

    def __del__(self):
        if getattr(self, "_h", None) and getattr(self, "_lib", None) is not None:
            self._lib.or_destroy(self._h)
            self._h = None

    # state
    def set_state(self, u):
        u = _arr(u, self.nvec)
        self._lib.or_set_state(self._h, _d(u))

    def get_state(self):
        u = np.empty(self.nvec)
        self._lib.or_get_state(self._h, _d(u))
        return u

    # kernels
    def rhs(self, u):
        u = _arr(u, self.nvec)
        R = np.empty(self.nvec)
        self._lib.or_rhs(self._h, _d(u), _d(R))
        return R

    def cn_old(self, un, dt):
        un = _arr(un, self.nvec)
        b = np.empty(self.nvec)
        self._lib.or_cn_old(self._h, _d(un), float(dt), _d(b))
        return b

    def residual(self, u, b, dt):
        u, b = _arr(u, self.nvec), _arr(b, self.nvec)
        F = np.empty(self.nvec)
        self._lib.or_residual(self._h, _d(u), _d(b), float(dt), _d(F))
        return F

    def time_step(self, u):
        """dt, max (|u|+c)/dx, max |u|/dx, max D/dx^2, scales[5] (sets scales)."""
        u = _arr(u, self.nvec)
        out = np.empty(9)
        self._lib.or_time_step(self._h, _d(u), _d(out))
        return dict(dt=out[0], hyd=out[1], adv=out[2], rad=out[3], scales=out[4:9].copy())

    def set_scales(self, s):
        s = _arr(list(s) + [1.0] * (5 - len(s)), 5)
        self._lib.or_set_scales(self._h, _d(s))

    def jv(self, u, b, dt, v):
        u, b, v = _arr(u, self.nvec), _arr(b, self.nvec), _arr(v, self.nvec)
        w = np.empty(self.nvec)
        self._lib.or_jv(self._h, _d(u), _d(b), float(dt), _d(v), _d(w))
        return w

    def jv_eps(self, u, b, dt, v, eps):
        """Jv at a given difference step eps > 0"""
        u, b, v = _arr(u, self.nvec), _arr(b, self.nvec), _arr(v, self.nvec)
        w = np.empty(self.nvec)
        self._lib.or_jv_eps(self._h, _d(u), _d(b), float(dt), _d(v), float(eps), _d(w))
        return w

    def precond(self, u, dt, v):
        u, v = _arr(u, self.nvec), _arr(v, self.nvec)
        z = np.empty(self.nvec)
        self._lib.or_precond(self._h, _d(u), float(dt), _d(v), _d(z))
        return z

    def sources(self):
        s = np.empty(self.N)
        self._lib.or_get_sources(self._h, _d(s))
        return s

    # passive scalars (partial densities s_k = c_k rho, nscal * N values)
    def set_scalars(self, s, nscal, renormalize=True):
        s = _arr(s, nscal * self.N)
        self.nscal = int(nscal)
        self._lib.or_set_scalars(self._h, self.nscal, 1 if renormalize else 0, _d(s))

    def get_scalars(self):
        out = np.empty(self.nscal * self.N)
        self._lib.or_get_scalars(self._h, _d(out))
        return out

    def scalar_rhs(self, u, s):
        u = _arr(u, self.nvec)
        s = _arr(s)
        out = np.empty(s.size)
        self._lib.or_scalar_rhs(self._h, _d(u), _d(s), _d(out))
        return out

    def scalar_its(self):
        out = (C.c_int * 2)()
        self._lib.or_scalar_its(self._h, out)
        return int(out[0]), int(out[1])

    # solver
    def newton_solve(self, dt):
        st = np.empty(len(STAT_KEYS))
        rc = self._lib.or_newton_solve(self._h, float(dt), _d(st))
        return rc, dict(zip(STAT_KEYS, st.tolist()))

    def implicit_step(self):
        st = np.empty(len(STAT_KEYS))
        rc = self._lib.or_implicit_step(self._h, _d(st))
        return rc, dict(zip(STAT_KEYS, st.tolist()))

    def newton_history(self):
        """the last Newton solve: residual norms |S^-1 F(u_k)|, and per
        iteration the linear tolerance and the GMRES solve's final relative
        residual"""
        f, eta, lin = np.empty(64), np.empty(64), np.empty(64)
        n = self._lib.or_newton_history(self._h, _d(f), _d(eta), _d(lin), 64)
        return f[:n].copy(), eta[:n - 1].copy(), lin[:n - 1].copy()

    def extrap_info(self):
        """the last solve's extrapolated first iterate: its residual norm
        (-1 when none was tried) and whether the solve started from it"""
        return _extrap_info(self._lib, self._h)


def _extrap_info(lib, h):
    out = np.empty(2)
    lib.or_extrap_info(h, _d(out))
    return float(out[0]), bool(out[1])


def ew_forcing(f, f_prev, eta_prev, eta_max, tol):
    """the oracle's Eisenstat-Walker forcing term of a Newton iteration"""
    return float(_load().or_ew_forcing(float(f), float(f_prev), float(eta_prev), float(eta_max), float(tol)))


def threads(threaded=False):
    """host threads the serial or the -fopenmp oracle runs on"""
    return int(_load(threaded).or_threads())


def tridiag(a, b, c, d, periodic=False):
    lib = _load()
    a, b, c, d = (_arr(v) for v in (a, b, c, d))
    x = np.empty_like(d)
    lib.or_tridiag(int(d.size), _d(a), _d(b), _d(c), _d(d), _d(x), int(bool(periodic)))
    return x


def gmres_dense(A, b, m, max_cycles, eta, M=None):
    lib = _load()
    A = _arr(A)
    b = _arr(b)
    n = b.size
    Mp = _d(_arr(M)) if M is not None else None
    x = np.zeros(n)
    info = np.zeros(5)
    lib.or_gmres_dense(n, _d(A), Mp, _d(b), _d(x), int(m), int(max_cycles), float(eta), _d(info))
    return x, dict(its=int(info[0]), cycles=int(info[1]), converged=bool(info[2]),
                   res=info[3], beta0=info[4])
