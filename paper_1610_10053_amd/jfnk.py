"""Python binding of the implicit-step C-ABI (include/jfnk.h).

Argument marshalling only: every step of the solve runs in the HIP library
libjfnk.so.  Host inputs are numpy arrays; device inputs are torch CUDA
tensors (float64, contiguous), passed by pointer with on_device = 1.  Work is
enqueued on torch's current stream of the problem's device unless another
stream handle is given.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjfnk.so")

BC_PERIODIC, BC_WALL = 0, 1
PC_NONE, PC_ACOUSTIC, PC_ACOUSTIC_DIFFUSION = 0, 1, 2
PCS_MULTIGRID, PCS_ADI = 0, 1
FP64, MIXED = 0, 1


class ProblemDesc(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("bc", C.c_int * 3), ("gamma", C.c_double), ("g", C.c_double * 3), ("chi0", C.c_double),
                ("heat_balance", C.c_int), ("energy_form", C.c_int), ("geometry", C.c_int)]


class SolverOpts(C.Structure):
    _fields_ = [("newton_rtol", C.c_double), ("newton_atol", C.c_double), ("newton_corr_tol", C.c_double),
                ("newton_max", C.c_int), ("gmres_restart", C.c_int), ("gmres_max_cycles", C.c_int),
                ("gmres_eta", C.c_double), ("pc", C.c_int), ("pc_solver", C.c_int), ("mg_nu1", C.c_int),
                ("mg_nu2", C.c_int), ("mg_nuc", C.c_int), ("mg_cycles", C.c_int), ("prec", C.c_int),
                ("cfl_hydro", C.c_double), ("cfl_adv_max", C.c_double), ("cfl_rad_max", C.c_double),
                ("dt_max", C.c_double), ("max_halvings", C.c_int), ("mg_light_cells", C.c_int),
                ("newton_target", C.c_int), ("dt_grow", C.c_double), ("scalar_converge", C.c_int),
                ("gmres_forcing", C.c_int), ("newton_extrapolate", C.c_int)]


class StepStats(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("cfl_hydro", C.c_double), ("cfl_adv", C.c_double),
                ("cfl_rad", C.c_double), ("rel_res", C.c_double), ("max_rel_corr", C.c_double),
                ("mass_drift", C.c_double), ("energy_drift", C.c_double), ("f0", C.c_double),
                ("f", C.c_double), ("newton_its", C.c_int), ("gmres_its", C.c_int),
                ("rejections", C.c_int), ("status", C.c_int), ("wall_ms", C.c_double),
                ("scalar_newton_its", C.c_int), ("scalar_gmres_its", C.c_int), ("newton_exit", C.c_int),
                ("extrapolated", C.c_int), ("f_extrap", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Diagnostics(C.Structure):
    _fields_ = [("kinetic", C.c_double), ("mass", C.c_double), ("energy", C.c_double), ("max_mach", C.c_double),
                ("mix_width", C.c_double), ("mix_width_scalars", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RequestStats(C.Structure):
    _fields_ = [("status", C.c_int), ("steps_done", C.c_int), ("newton_its", C.c_int), ("gmres_its", C.c_int),
                ("rejections", C.c_int), ("pad", C.c_int), ("cells", C.c_double), ("t_submit_ms", C.c_double),
                ("t_admit_ms", C.c_double), ("t_done_ms", C.c_double), ("sim_time", C.c_double),
                ("footprint_bytes", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


EXPORTS = ("jfnk_default_opts", "jfnk_footprint_bytes", "jfnk_create_problem", "jfnk_destroy_problem",
           "jfnk_set_state", "jfnk_get_state", "jfnk_set_time", "jfnk_set_opts", "jfnk_set_scalars",
           "jfnk_get_scalars", "jfnk_implicit_step",
           "jfnk_newton_solve", "jfnk_eval_rhs", "jfnk_eval_cn_old", "jfnk_eval_residual",
           "jfnk_eval_time_step", "jfnk_eval_diagnostics", "jfnk_velocity_error", "jfnk_velocity_error_noalloc", "jfnk_set_scales", "jfnk_apply_jv", "jfnk_apply_jv_eps", "jfnk_apply_precond",
           "jfnk_profile_enable", "jfnk_profile_sample", "jfnk_profile_read", "jfnk_profile_class_name", "jfnk_server_create",
           "jfnk_server_submit", "jfnk_server_poll", "jfnk_server_wait", "jfnk_server_destroy",
           "jfnk_last_error")

_lib = None


class JfnkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("jfnk error %d: %s" % (code, msg))
        self.code = code


def load():
    """Load libjfnk.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libjfnk.so is not built (run __graft_entry__.build() or "
                          "python paper_1610_10053_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_int
    P = C.POINTER
    sig = {
        "jfnk_default_opts": (None, [P(SolverOpts)]),
        "jfnk_footprint_bytes": (ip, [P(ProblemDesc), P(SolverOpts), P(C.c_size_t)]),
        "jfnk_create_problem": (ip, [P(ProblemDesc), P(SolverOpts), vp, ip, vp, P(vp)]),
        "jfnk_destroy_problem": (ip, [vp]),
        "jfnk_set_state": (ip, [vp, vp, ip]),
        "jfnk_get_state": (ip, [vp, vp, ip]),
        "jfnk_set_time": (ip, [vp, C.c_double]),
        "jfnk_set_scalars": (ip, [vp, ip, ip, vp, ip]),
        "jfnk_get_scalars": (ip, [vp, vp, ip]),
        "jfnk_set_opts": (ip, [vp, P(SolverOpts)]),
        "jfnk_implicit_step": (ip, [vp, P(StepStats)]),
        "jfnk_newton_solve": (ip, [vp, C.c_double, P(StepStats)]),
        "jfnk_eval_rhs": (ip, [vp, vp, vp, ip]),
        "jfnk_eval_cn_old": (ip, [vp, vp, C.c_double, vp, ip]),
        "jfnk_eval_residual": (ip, [vp, vp, vp, C.c_double, vp, ip]),
        "jfnk_eval_time_step": (ip, [vp, vp, dp, ip]),
        "jfnk_eval_diagnostics": (ip, [vp, vp, ip, C.c_double, C.c_double, ip, P(Diagnostics)]),
        "jfnk_velocity_error": (ip, [vp, vp, vp, ip, ip, ip, P(C.c_double)]),
        "jfnk_velocity_error_noalloc": (ip, [vp, vp, vp, ip, ip, P(C.c_double)]),
        "jfnk_set_scales": (ip, [vp, dp]),
        "jfnk_apply_jv": (ip, [vp, vp, vp, C.c_double, vp, vp, ip]),
        "jfnk_apply_jv_eps": (ip, [vp, vp, vp, C.c_double, vp, C.c_double, vp, ip]),
        "jfnk_apply_precond": (ip, [vp, vp, C.c_double, vp, vp, ip]),
        "jfnk_profile_enable": (ip, [vp, C.c_uint]),
        "jfnk_profile_sample": (ip, [vp, ip, ip]),
        "jfnk_profile_read": (ip, [vp, dp, C.POINTER(C.c_longlong), dp, ip]),
        "jfnk_profile_class_name": (C.c_char_p, [ip]),
        "jfnk_server_create": (ip, [C.c_size_t, ip, P(vp)]),
        "jfnk_server_submit": (ip, [vp, P(ProblemDesc), P(SolverOpts), vp, ip, P(C.c_longlong)]),
        "jfnk_server_poll": (ip, [vp, C.c_longlong]),
        "jfnk_server_wait": (ip, [vp, C.c_longlong, vp, P(RequestStats), dp, ip, P(ip)]),
        "jfnk_server_destroy": (ip, [vp]),
        "jfnk_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error():
    return load().jfnk_last_error().decode()


def _check(rc):
    if rc < 0:
        raise JfnkError(rc, last_error())
    return rc


def default_opts():
    o = SolverOpts()
    load().jfnk_default_opts(C.byref(o))
    return o


def make_desc(d):
    """ProblemDesc from a dict with keys ndim, n, lo, hi, bc, gamma, g, chi0, heat_balance
    (and optionally energy_form, geometry)."""
    pd = ProblemDesc()
    pd.ndim = d["ndim"]
    for a in range(3):
        pd.n[a] = d["n"][a]
        pd.lo[a] = d["lo"][a]
        pd.hi[a] = d["hi"][a]
        pd.bc[a] = d["bc"][a]
        pd.g[a] = d["g"][a]
    pd.gamma = d["gamma"]
    pd.chi0 = d["chi0"]
    pd.heat_balance = d["heat_balance"]
    pd.energy_form = d.get("energy_form", 0)
    pd.geometry = d.get("geometry", 0)
    return pd


def make_opts(o):
    """SolverOpts from a dict (keys as in the header; newton_corr_tol etc.)."""
    so = default_opts()
    for k, _ in SolverOpts._fields_:
        if k in o:
            setattr(so, k, o[k])
    return so


def _ptr(a):
    """(pointer, on_device, keepalive) for a numpy array or torch tensor."""
    if isinstance(a, np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.float64)
        return a.ctypes.data, 0, a
    # torch tensor
    if a.dtype.is_floating_point and a.element_size() != 8:
        raise TypeError("device buffers must be float64")
    if not a.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return a.data_ptr(), 1 if a.is_cuda else 0, a


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class Problem:
    """One simulation: state, Krylov workspace and solver options on the device."""

    def __init__(self, desc, opts, u0, stream=None):
        lib = load()
        self.desc = dict(desc)
        self._pd = make_desc(desc)
        self._po = make_opts(opts)
        n = desc["n"]
        self.N = n[0] * n[1] * n[2]
        self.nvec = (2 + desc["ndim"]) * self.N
        p, on_dev, keep = _ptr(u0)
        self._check_size(keep)
        h = C.c_void_p()
        if stream is None:
            stream = _current_stream()
        _check(lib.jfnk_create_problem(C.byref(self._pd), C.byref(self._po), p, on_dev, stream, C.byref(h)))
        self._h = h

    def _check_size(self, a):
        size = a.size if isinstance(a, np.ndarray) else a.numel()
        if size != self.nvec:
            raise ValueError("expected %d values, got %d" % (self.nvec, size))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.jfnk_destroy_problem(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _out(self, like):
        if isinstance(like, np.ndarray):
            return np.empty(self.nvec)
        import torch
        return torch.empty(self.nvec, dtype=torch.float64, device=like.device)

    # ---- state
    def set_state(self, u):
        p, d, keep = _ptr(u)
        self._check_size(keep)
        _check(_lib.jfnk_set_state(self._h, p, d))

    def get_state(self, out=None):
        out = np.empty(self.nvec) if out is None else out
        p, d, keep = _ptr(out)
        self._check_size(keep)
        _check(_lib.jfnk_get_state(self._h, p, d))
        return out

    def set_scalars(self, s, nscal, renormalize=True):
        """attach nscal passive scalars (partial densities c_k rho, nscal * N values)"""
        p, d, keep = _ptr(s)
        size = keep.size if isinstance(keep, np.ndarray) else keep.numel()
        if size != nscal * self.N:
            raise ValueError("expected %d values, got %d" % (nscal * self.N, size))
        _check(_lib.jfnk_set_scalars(self._h, int(nscal), 1 if renormalize else 0, p, d))
        self.nscal = int(nscal)

    def get_scalars(self, out=None):
        out = np.empty(self.nscal * self.N) if out is None else out
        p, d, keep = _ptr(out)
        _check(_lib.jfnk_get_scalars(self._h, p, d))
        return out

    def set_time(self, t):
        _check(_lib.jfnk_set_time(self._h, float(t)))

    def set_opts(self, opts):
        self._po = make_opts(opts)
        _check(_lib.jfnk_set_opts(self._h, C.byref(self._po)))

    # ---- stepping
    def implicit_step(self):
        st = StepStats()
        rc = _check(_lib.jfnk_implicit_step(self._h, C.byref(st)))
        return rc, st.as_dict()

    def newton_solve(self, dt):
        st = StepStats()
        rc = _check(_lib.jfnk_newton_solve(self._h, float(dt), C.byref(st)))
        return rc, st.as_dict()

    # ---- components
    def eval_rhs(self, u):
        out = self._out(u)
        pu, d, k1 = _ptr(u)
        po, _, k2 = _ptr(out)
        _check(_lib.jfnk_eval_rhs(self._h, pu, po, d))
        return out

    def eval_cn_old(self, un, dt):
        out = self._out(un)
        pu, d, k1 = _ptr(un)
        po, _, k2 = _ptr(out)
        _check(_lib.jfnk_eval_cn_old(self._h, pu, float(dt), po, d))
        return out

    def eval_residual(self, u, b, dt):
        out = self._out(u)
        pu, d, k1 = _ptr(u)
        pb, _, k2 = _ptr(b)
        po, _, k3 = _ptr(out)
        _check(_lib.jfnk_eval_residual(self._h, pu, pb, float(dt), po, d))
        return out

    def eval_time_step(self, u):
        out = np.empty(9)
        pu, d, k1 = _ptr(u)
        _check(_lib.jfnk_eval_time_step(self._h, pu, out.ctypes.data_as(C.POINTER(C.c_double)), d))
        return dict(dt=out[0], hyd=out[1], adv=out[2], rad=out[3], scales=out[4:9].copy())

    def eval_diagnostics(self, u=None, rho_light=0.0, rho_heavy=1.0, mix_axis=-1):
        """kinetic energy, mass, energy, max Mach and mixing width (dict)"""
        out = Diagnostics()
        if u is None:
            _check(_lib.jfnk_eval_diagnostics(self._h, None, 0, float(rho_light), float(rho_heavy), int(mix_axis),
                                              C.byref(out)))
        else:
            pu, d, k1 = _ptr(u)
            self._check_size(k1)
            _check(_lib.jfnk_eval_diagnostics(self._h, pu, d, float(rho_light), float(rho_heavy), int(mix_axis),
                                              C.byref(out)))
        return out.as_dict()

    def velocity_error(self, u_high, ratio, axis, u_low=None):
        """eq. (17) error of velocity component `axis` against u_high, a
        state on the grid `ratio` times finer (u_low: None for the current
        state); both arrays host, or both device"""
        out = C.c_double()
        ph, d, k1 = _ptr(u_high)
        size = k1.size if isinstance(k1, np.ndarray) else k1.numel()
        if size != self.nvec * int(ratio) ** self.desc["ndim"]:
            raise ValueError("u_high has the wrong size for ratio %d" % ratio)
        pl, k2 = None, None
        if u_low is not None:
            pl, d2, k2 = _ptr(u_low)
            self._check_size(k2)
            if d2 != d:
                raise ValueError("u_low and u_high must both be host or both device arrays")
        _check(_lib.jfnk_velocity_error(self._h, pl, ph, d, int(ratio), int(axis), C.byref(out)))
        return out.value

    def velocity_error_noalloc(self, u_high, ratio, axis, u_low=None):
        """the allocation-free form of velocity_error: u_high (and u_low, or
        None for the current state) must be device tensors"""
        out = C.c_double()
        ph, d, k1 = _ptr(u_high)
        if d != 1:
            raise ValueError("velocity_error_noalloc takes device tensors")
        if k1.numel() != self.nvec * int(ratio) ** self.desc["ndim"]:
            raise ValueError("u_high has the wrong size for ratio %d" % ratio)
        pl, k2 = None, None
        if u_low is not None:
            pl, d2, k2 = _ptr(u_low)
            self._check_size(k2)
            if d2 != 1:
                raise ValueError("velocity_error_noalloc takes device tensors")
        _check(_lib.jfnk_velocity_error_noalloc(self._h, pl, ph, int(ratio), int(axis), C.byref(out)))
        return out.value

    def set_scales(self, s):
        s = np.ascontiguousarray(list(s) + [1.0] * (5 - len(s)), dtype=np.float64)
        _check(_lib.jfnk_set_scales(self._h, s.ctypes.data_as(C.POINTER(C.c_double))))

    def apply_jv(self, u, b, dt, v):
        out = self._out(u)
        pu, d, k1 = _ptr(u)
        pb, _, k2 = _ptr(b)
        pv, _, k3 = _ptr(v)
        po, _, k4 = _ptr(out)
        _check(_lib.jfnk_apply_jv(self._h, pu, pb, float(dt), pv, po, d))
        return out

    def apply_jv_eps(self, u, b, dt, v, eps):
        """the Jacobian-free product with a given difference step eps"""
        out = self._out(u)
        pu, d, k1 = _ptr(u)
        pb, _, k2 = _ptr(b)
        pv, _, k3 = _ptr(v)
        po, _, k4 = _ptr(out)
        _check(_lib.jfnk_apply_jv_eps(self._h, pu, pb, float(dt), pv, float(eps), po, d))
        return out

    def profile_enable(self, classes):
        """classes: iterable of class names or indices; empty disables."""
        mask = 0
        names = profile_class_names()
        for c in classes:
            mask |= 1 << (names.index(c) if isinstance(c, str) else int(c))
        _check(_lib.jfnk_profile_enable(self._h, mask))

    def profile_sample(self, period, burst=1):
        """burst 1: time one launch in every `period` of each enabled class;
        burst > 1: events on every launch in the first `burst` of each
        `period` launches, enabled classes counted after a window's first"""
        _check(_lib.jfnk_profile_sample(self._h, int(period), int(burst)))

    def profile_read(self):
        """{class name: (milliseconds, launches, compulsory bytes)} since enable / last read."""
        names = profile_class_names()
        ms = np.zeros(len(names))
        by = np.zeros(len(names))
        cnt = (C.c_longlong * len(names))()
        dpp = C.POINTER(C.c_double)
        _check(_lib.jfnk_profile_read(self._h, ms.ctypes.data_as(dpp), cnt, by.ctypes.data_as(dpp), len(names)))
        return {names[i]: (float(ms[i]), int(cnt[i]), float(by[i])) for i in range(len(names)) if cnt[i]}

    def apply_precond(self, u, dt, v):
        out = self._out(u)
        pu, d, k1 = _ptr(u)
        pv, _, k2 = _ptr(v)
        po, _, k3 = _ptr(out)
        _check(_lib.jfnk_apply_precond(self._h, pu, float(dt), pv, po, d))
        return out


def profile_class_names():
    lib = load()
    out = []
    for c in range(64):
        s = lib.jfnk_profile_class_name(c).decode()
        if not s:
            break
        out.append(s)
    return out


def footprint_bytes(desc, opts):
    lib = load()
    out = C.c_size_t()
    _check(lib.jfnk_footprint_bytes(C.byref(make_desc(desc)), C.byref(make_opts(opts)), C.byref(out)))
    return out.value


# C-ABI names
def create_problem(desc, opts, u0, stream=None):
    return Problem(desc, opts, u0, stream)


def implicit_step(problem):
    return problem.implicit_step()


def newton_solve(problem, dt):
    return problem.newton_solve(dt)


def get_state(problem, out=None):
    return problem.get_state(out)


def set_state(problem, u):
    return problem.set_state(u)


def destroy_problem(problem):
    problem.close()


class Server:
    """Continuous-batching request loop on one device (jfnk_server_*).

    submit() queues a simulation (host initial state, number of implicit
    steps) and returns its id at once; the library's worker threads admit
    waiting requests by device-memory footprint as workers and memory free
    up.  wait(id) blocks (without the GIL) until the request is finished and
    returns (final state, request statistics, per-step wall milliseconds)."""

    def __init__(self, hbm_bytes, max_active):
        lib = load()
        h = C.c_void_p()
        _check(lib.jfnk_server_create(int(hbm_bytes), int(max_active), C.byref(h)))
        self._h = h
        self._nvec = {}

    def submit(self, desc, opts, u0, nsteps):
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        n = desc["n"]
        nvec = (2 + desc["ndim"]) * n[0] * n[1] * n[2]
        if u0.size != nvec:
            raise ValueError("expected %d values, got %d" % (nvec, u0.size))
        rid = C.c_longlong()
        _check(_lib.jfnk_server_submit(self._h, C.byref(make_desc(desc)), C.byref(make_opts(opts)),
                                       u0.ctypes.data, int(nsteps), C.byref(rid)))
        self._nvec[rid.value] = (nvec, int(nsteps))
        return rid.value

    def poll(self, rid):
        return _lib.jfnk_server_poll(self._h, rid)

    def wait(self, rid):
        nvec, nsteps = self._nvec.pop(rid)
        u = np.empty(nvec)
        st = RequestStats()
        ms = np.empty(max(nsteps, 1))
        cnt = C.c_int()
        _check(_lib.jfnk_server_wait(self._h, rid, u.ctypes.data, C.byref(st),
                                     ms.ctypes.data_as(C.POINTER(C.c_double)), len(ms), C.byref(cnt)))
        return u, st.as_dict(), ms[:cnt.value].copy()

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.jfnk_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def server_create(hbm_bytes, max_active):
    return Server(hbm_bytes, max_active)
