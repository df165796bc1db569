"""ctypes binding of libbfal (include/bfal.h): argument marshalling only.

Every entry point of the C-ABI is exposed under its own name; the small
Context / Problem classes only pack numpy arrays (host memory) or torch
tensors (device memory) into pointers and raise on error statuses.  All of
the Newton step runs in the library's HIP kernels; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfal.so")

BF_OK = 0
BF_WARN_PCG_MAXITER = 1
STATUS = {0: "OK", 1: "WARN_PCG_MAXITER", -1: "ERR_INVALID_ARG", -2: "ERR_OOM", -3: "ERR_HIP",
          -4: "ERR_INVERTED_ELEMENT", -5: "ERR_DEGENERATE_CONSTRAINT", -6: "ERR_NOT_SPD", -7: "ERR_BUDGET",
          -8: "ERR_STATE"}
BF_MEM_HOST, BF_MEM_DEVICE = 0, 1
BF_PREC_FP32, BF_PREC_BF16_REFINE = 0, 1


class bf_mesh_desc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_tets", C.c_int32), ("tets", C.c_void_p), ("rest", C.c_void_p),
                ("E", C.c_void_p), ("nu", C.c_void_p), ("rho", C.c_void_p), ("fixed", C.c_void_p),
                ("material", C.c_void_p)]


class bf_constraint_desc(C.Structure):
    _fields_ = [("n_pt", C.c_int32), ("n_ee", C.c_int32), ("pt", C.c_void_p), ("ee", C.c_void_p),
                ("lambda_", C.c_void_p), ("gamma", C.c_void_p), ("kappa", C.c_double), ("delta", C.c_double)]


class bf_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("refine_tol", C.c_double), ("poll_every", C.c_int32), ("check_every", C.c_int32),
                ("time_spmv", C.c_int32), ("max_sweeps", C.c_int32)]


class bf_step_stats(C.Structure):
    _fields_ = [("pcg_iters", C.c_int32), ("refine_sweeps", C.c_int32), ("rel_residual", C.c_double),
                ("newton_inf_over_h", C.c_double), ("max_violation", C.c_double), ("nnzb", C.c_int64),
                ("ms_lin", C.c_double), ("ms_pattern", C.c_double), ("ms_assemble", C.c_double),
                ("ms_pcg", C.c_double), ("spmv_timed", C.c_int32), ("ms_spmv_avg", C.c_double),
                ("sweep_rel_residual", C.c_double * 16)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["sweep_rel_residual"] = [float(v) for v in self.sweep_rel_residual][: self.refine_sweeps + 1]
        return d


class BfalError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class bf_subproblem_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("pcg_iters", C.c_int32), ("energy_evals", C.c_int32),
                ("energy_initial", C.c_double), ("energy_final", C.c_double), ("last_step", C.c_double),
                ("max_violation", C.c_double), ("active", C.c_int32), ("decayed", C.c_int32),
                ("ms_total", C.c_double), ("truncated", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bf_ccd_stats(C.Structure):
    _fields_ = [("candidates_pt", C.c_int64), ("candidates_ee", C.c_int64), ("colliding_pt", C.c_int32),
                ("colliding_ee", C.c_int32), ("new_pt", C.c_int32), ("new_ee", C.c_int32), ("added_pt", C.c_int32),
                ("added_ee", C.c_int32), ("removed", C.c_int32), ("n_pt", C.c_int32), ("n_ee", C.c_int32),
                ("alpha_ccd", C.c_double), ("alpha_inversion", C.c_double), ("ms_tree", C.c_double),
                ("ms_query", C.c_double), ("ms_update", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bf_time_step_opts(C.Structure):
    _fields_ = [("solve", bf_solve_opts), ("k_min", C.c_int32), ("eps", C.c_double), ("max_outer", C.c_int32),
                ("max_newton", C.c_int32), ("decay", C.c_double), ("sep", C.c_double), ("mu_init_c", C.c_double),
                ("mu_f", C.c_double), ("eps_v", C.c_double)]


class bf_time_step_stats(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("newton_iters", C.c_int32), ("pcg_iters", C.c_int32),
                ("truncated", C.c_int32), ("beta", C.c_double), ("alpha_min", C.c_double),
                ("alpha_last", C.c_double), ("n_pt", C.c_int32), ("n_ee", C.c_int32), ("mu_doublings", C.c_int32),
                ("kappa", C.c_double), ("delta", C.c_double), ("ms_subproblem", C.c_double),
                ("ms_ccd", C.c_double), ("ms_total", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bf_server_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_active", C.c_int32), ("iters_per_round", C.c_int32),
                ("admit_threads", C.c_int32)]


class bf_stall_rule(C.Structure):
    _fields_ = [("alpha_min", C.c_double), ("window", C.c_int32), ("count", C.c_int32)]


class bf_request_times(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


_lib = None

# (name, restype, argtypes) of every exported entry point
_PROTOS = [
    ("bf_context_create", C.c_int, [C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("bf_context_destroy", None, [C.c_void_p]),
    ("bf_last_error", C.c_char_p, [C.c_void_p]),
    ("bf_problem_create", C.c_int, [C.c_void_p, C.POINTER(bf_mesh_desc), C.c_int32, C.POINTER(C.c_void_p)]),
    ("bf_problem_destroy", None, [C.c_void_p]),
    ("bf_set_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32]),
    ("bf_set_constraints", C.c_int, [C.c_void_p, C.POINTER(bf_constraint_desc), C.c_int32]),
    ("bf_newton_step", C.c_int, [C.c_void_p, C.POINTER(bf_solve_opts), C.c_void_p, C.c_int32,
                                 C.POINTER(bf_step_stats)]),
    ("bf_get_gradient", C.c_int, [C.c_void_p, C.c_void_p]),
    ("bf_get_nnzb", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("bf_get_pattern", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("bf_get_blocks", C.c_int, [C.c_void_p, C.c_void_p]),
    ("bf_footprint_bytes", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    ("bf_solve_subproblem", C.c_int, [C.c_void_p, C.POINTER(bf_solve_opts), C.c_int32, C.c_double, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(bf_subproblem_stats)]),
    ("bf_energy", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    ("bf_energy_noalloc", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    ("bf_mu_init", C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_double)]),
    ("bf_set_friction", C.c_int, [C.c_void_p, C.c_double, C.c_double]),
    ("bf_update_active_set", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.POINTER(bf_ccd_stats)]),
    ("bf_max_step_size", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double),
                                   C.POINTER(bf_ccd_stats)]),
    ("bf_time_step", C.c_int, [C.c_void_p, C.POINTER(bf_time_step_opts), C.c_void_p, C.c_void_p, C.c_int32,
                               C.POINTER(bf_time_step_stats)]),
    ("bf_get_collisions", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("bf_get_constraint_counts", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("bf_get_constraints", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("bf_clock_now", C.c_double, []),
    ("bf_server_create", C.c_int, [C.c_int32, C.POINTER(bf_server_opts), C.POINTER(C.c_void_p)]),
    ("bf_server_submit", C.c_int, [C.c_void_p, C.c_int64, C.POINTER(bf_mesh_desc), C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_double, C.POINTER(bf_constraint_desc),
                                   C.POINTER(bf_solve_opts)]),
    ("bf_server_poll", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)]),
    ("bf_server_result", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.POINTER(bf_step_stats),
                                   C.POINTER(bf_request_times), C.POINTER(C.c_int32)]),
    ("bf_server_stats", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_size_t)]),
    ("bf_server_destroy", None, [C.c_void_p]),
    # host rules (include/bfal_host.h): no device needed
    ("bf_check_mesh", C.c_int, [C.POINTER(bf_mesh_desc), C.c_char_p, C.c_int32]),
    ("bf_check_state", C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_char_p, C.c_int32]),
    ("bf_check_constraints", C.c_int, [C.c_int32, C.POINTER(bf_constraint_desc), C.c_char_p, C.c_int32]),
    ("bf_check_solve_opts", C.c_int, [C.POINTER(bf_solve_opts), C.c_char_p, C.c_int32]),
    ("bf_stall_step", C.c_int32, [C.POINTER(bf_stall_rule), C.c_double, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]),
    ("bf_admission_create", C.c_int, [C.c_uint64, C.c_int32, C.POINTER(C.c_void_p)]),
    ("bf_admission_destroy", None, [C.c_void_p]),
    ("bf_admission_push", C.c_int, [C.c_void_p, C.c_int64, C.c_uint64]),
    ("bf_admission_next", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    ("bf_admission_release", C.c_int, [C.c_void_p, C.c_int32, C.c_uint64]),
    ("bf_admission_used", C.c_uint64, [C.c_void_p]),
    ("bf_admission_waiting", C.c_int32, [C.c_void_p]),
    ("bf_admission_active", C.c_int32, [C.c_void_p]),
    ("bf_slice_plan", C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
]

EXPORTED = [p[0] for p in _PROTOS]


def lib():
    """Load libbfal.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime; importing it first makes libbfal bind
        # to that same runtime (one HIP runtime per process, shared streams and
        # device memory).  Without torch, libbfal uses the system ROCm runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _PROTOS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    """Pointer of a numpy array (host) or a torch tensor (device); None stays NULL."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    return a.data_ptr()


def _mem(a):
    return BF_MEM_HOST if isinstance(a, np.ndarray) else BF_MEM_DEVICE


class Context:
    """A device plus the HIP stream all work of its problems is ordered on."""

    def __init__(self, device: int = 0, stream=None):
        self.h = C.c_void_p()
        st = lib().bf_context_create(int(device), stream, C.byref(self.h))
        if st != BF_OK:
            raise BfalError(st, "bf_context_create failed")

    def check(self, st):
        if st < 0:
            raise BfalError(st, lib().bf_last_error(self.h).decode())
        return st

    def close(self):
        if self.h:
            lib().bf_context_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Problem:
    """One mesh on one context: state, constraints, Newton steps, introspection."""

    def __init__(self, ctx: Context, tets, rest, E, nu, rho, fixed=None, material=None):
        """material: per-tet codes, 0 Neo-Hookean, 1 stable Neo-Hookean, 2 corotated linear (None: all 0)."""
        self.ctx = ctx
        dev = not isinstance(tets, np.ndarray)
        if not dev:
            tets, rest = _host(tets, np.int32), _host(rest, np.float64)
            E, nu, rho = _host(E, np.float64), _host(nu, np.float64), _host(rho, np.float64)
            fixed = None if fixed is None else _host(fixed, np.uint8)
            material = None if material is None else _host(material, np.int32)
        elif any(isinstance(a, np.ndarray) for a in (rest, E, nu, rho, fixed, material)):
            raise TypeError("device meshes take every array on the device")
        self.N, self.T = int(rest.shape[0]), int(tets.shape[0])
        d = bf_mesh_desc(self.N, self.T, _ptr(tets), _ptr(rest), _ptr(E), _ptr(nu), _ptr(rho), _ptr(fixed),
                         _ptr(material))
        self.h = C.c_void_p()
        ctx.check(lib().bf_problem_create(ctx.h, C.byref(d), BF_MEM_DEVICE if dev else BF_MEM_HOST, C.byref(self.h)))
        self.n_c = 0

    @classmethod
    def from_scene(cls, ctx, sc):
        pb = cls(ctx, sc["tets"], sc["rest"], sc["E"], sc["nu"], sc["rho"], sc["fixed"], sc.get("material"))
        pb.set_state(sc["x"], sc["x_hat"], sc["x_tilde"], sc["dt"])
        pb.set_constraints(sc["pt"], sc["ee"], sc["lam"], sc["gamma"], sc["kappa"], sc["delta"])
        return pb

    def set_state(self, x, x_hat, x_tilde, dt):
        if isinstance(x, np.ndarray):
            x, x_hat, x_tilde = (_host(a, np.float64) for a in (x, x_hat, x_tilde))
        self._keep_state = (x, x_hat, x_tilde)
        self.dt = float(dt)
        self.ctx.check(lib().bf_set_state(self.h, _ptr(x), _ptr(x_hat), _ptr(x_tilde), self.dt, _mem(x)))

    def set_constraints(self, pt, ee, lam, gamma, kappa, delta):
        if isinstance(lam, np.ndarray):
            pt, ee = _host(pt, np.int32).reshape(-1, 4), _host(ee, np.int32).reshape(-1, 4)
            lam = _host(lam, np.float64)
            gamma = None if gamma is None else _host(gamma, np.float64)
        d = bf_constraint_desc(int(pt.shape[0]), int(ee.shape[0]), _ptr(pt) if pt.shape[0] else None,
                               _ptr(ee) if ee.shape[0] else None, _ptr(lam) if lam.shape[0] else None,
                               _ptr(gamma) if gamma is not None and gamma.shape[0] else None,
                               float(kappa), float(delta))
        self.ctx.check(lib().bf_set_constraints(self.h, C.byref(d), _mem(lam)))
        self.n_c = int(pt.shape[0] + ee.shape[0])

    def newton_step(self, tol=1e-5, max_iter=20000, precision=BF_PREC_FP32, refine_tol=1e-6, poll_every=16,
                    check_every=1, time_spmv=0, max_sweeps=0, out=None):
        """Returns (p [N,3] (numpy, or `out` when a device tensor is passed), stats dict, status)."""
        o = bf_solve_opts(float(tol), int(max_iter), int(precision), float(refine_tol), int(poll_every),
                          int(check_every), int(time_spmv), int(max_sweeps))
        p = np.empty((self.N, 3), dtype=np.float64) if out is None else out
        s = bf_step_stats()
        st = self.ctx.check(lib().bf_newton_step(self.h, C.byref(o), _ptr(p), _mem(p), C.byref(s)))
        return p, s.as_dict(), st

    def solve_subproblem(self, tol=1e-5, max_iter=20000, max_newton=50, decay=0.9, poll_every=16, check_every=1):
        """Algorithm 2 from the current x_hat: returns (x_hat, lambda, gamma, stats dict, status)."""
        o = bf_solve_opts(float(tol), int(max_iter), BF_PREC_FP32, 1e-6, int(poll_every), int(check_every), 0, 0)
        xh = np.empty((self.N, 3), np.float64)
        lam = np.empty(max(self.n_c, 1), np.float64)
        gam = np.empty(max(self.n_c, 1), np.float64)
        s = bf_subproblem_stats()
        st = self.ctx.check(lib().bf_solve_subproblem(self.h, C.byref(o), int(max_newton), float(decay),
                                                      xh.ctypes.data, lam.ctypes.data, gam.ctypes.data,
                                                      BF_MEM_HOST, C.byref(s)))
        return xh, lam[: self.n_c], gam[: self.n_c], s.as_dict(), st

    def energy(self):
        """(L at the current x_hat in FP64, inverted flag)."""
        e, inv = C.c_double(), C.c_int32()
        self.ctx.check(lib().bf_energy(self.h, C.byref(e), C.byref(inv)))
        return float(e.value), bool(inv.value)

    def energy_noalloc(self):
        """bf_energy_noalloc: (L at the current x_hat, inverted flag) with no device allocation."""
        e, inv = C.c_double(), C.c_int32()
        self.ctx.check(lib().bf_energy_noalloc(self.h, C.byref(e), C.byref(inv)))
        return float(e.value), bool(inv.value)

    def update_active_set(self, x_hat=None, sep=0.1):
        """Algorithm 3 along x -> x_hat (None: the problem's x_hat); returns the stats."""
        st = bf_ccd_stats()
        xp = None if x_hat is None else _ptr(x_hat)
        mem = BF_MEM_HOST if x_hat is None else _mem(x_hat)
        self.ctx.check(lib().bf_update_active_set(self.h, xp, mem, sep, C.byref(st)))
        return st.as_dict()

    def max_step_size(self, x_hat=None, sep=0.1):
        """MaxStepSize along x -> x_hat; returns (alpha, stats)."""
        st = bf_ccd_stats()
        a = C.c_double()
        xp = None if x_hat is None else _ptr(x_hat)
        mem = BF_MEM_HOST if x_hat is None else _mem(x_hat)
        self.ctx.check(lib().bf_max_step_size(self.h, xp, mem, sep, C.byref(a), C.byref(st)))
        return float(a.value), st.as_dict()

    def time_step(self, tol=1e-7, max_iter=50000, k_min=2, eps=1e-3, max_outer=200, max_newton=20, decay=0.9,
                  sep=0.1, mu_init_c=0.0, poll_every=16, mu_f=0.0, eps_v=1e-3):
        """Algorithm 1 from the current state; returns (x, v, stats, status) on the host."""
        o = bf_time_step_opts()
        o.solve = bf_solve_opts(tol, max_iter, BF_PREC_FP32, 1e-6, poll_every, 1, 0, 0)
        o.k_min, o.eps, o.max_outer, o.max_newton = k_min, eps, max_outer, max_newton
        o.decay, o.sep, o.mu_init_c = decay, sep, mu_init_c
        o.mu_f, o.eps_v = mu_f, eps_v
        x = np.empty((self.N, 3))
        v = np.empty((self.N, 3))
        st = bf_time_step_stats()
        status = self.ctx.check(lib().bf_time_step(self.h, C.byref(o), x.ctypes.data, v.ctypes.data, BF_MEM_HOST,
                                                   C.byref(st)))
        return x, v, st.as_dict(), status

    def collisions(self, stats):
        """The colliding pairs of the last collision call: (pt rows, pt times, ee rows, ee times)."""
        npt, nee = stats["colliding_pt"], stats["colliding_ee"]
        pt = np.empty((npt, 4), dtype=np.int32)
        ee = np.empty((nee, 4), dtype=np.int32)
        tp = np.empty(npt)
        te = np.empty(nee)
        self.ctx.check(lib().bf_get_collisions(self.h, pt.ctypes.data, tp.ctypes.data, ee.ctypes.data,
                                               te.ctypes.data))
        return pt, tp, ee, te

    def constraints(self):
        """The active set: (pt [n_pt,4], ee [n_ee,4], lambda, gamma) on the host."""
        npt, nee = C.c_int32(), C.c_int32()
        self.ctx.check(lib().bf_get_constraint_counts(self.h, C.byref(npt), C.byref(nee)))
        pt = np.empty((npt.value, 4), dtype=np.int32)
        ee = np.empty((nee.value, 4), dtype=np.int32)
        lam = np.empty(npt.value + nee.value)
        gam = np.empty(npt.value + nee.value)
        self.ctx.check(lib().bf_get_constraints(self.h, pt.ctypes.data, ee.ctypes.data, lam.ctypes.data,
                                                gam.ctypes.data, BF_MEM_HOST))
        return pt, ee, lam, gam

    def set_friction(self, mu_f, eps_v=1e-3):
        """Appendix A: capture the friction set from the current constraints at x (mu_f = 0 clears it)."""
        self.ctx.check(lib().bf_set_friction(self.h, float(mu_f), float(eps_v)))

    def mu_init(self, C_=0.1):
        """C max_i (grad^2 E)_ii at the start-of-step state x (Section 5.2)."""
        m = C.c_double()
        self.ctx.check(lib().bf_mu_init(self.h, C_, C.byref(m)))
        return float(m.value)

    def gradient(self):
        g = np.empty((self.N, 3), dtype=np.float64)
        self.ctx.check(lib().bf_get_gradient(self.h, g.ctypes.data))
        return g

    def nnzb(self):
        n = C.c_int64()
        self.ctx.check(lib().bf_get_nnzb(self.h, C.byref(n)))
        return int(n.value)

    def pattern(self):
        nnzb = self.nnzb()
        row_ptr = np.empty(self.N + 1, np.int32)
        col = np.empty(nnzb, np.int32)
        emap = np.empty((self.T, 10), np.int32)
        cmap = np.empty((max(self.n_c, 1), 10), np.int32)
        diag = np.empty(self.N, np.int32)
        self.ctx.check(lib().bf_get_pattern(self.h, row_ptr.ctypes.data, col.ctypes.data, emap.ctypes.data,
                                            cmap.ctypes.data, diag.ctypes.data))
        return row_ptr, col, emap, cmap[: self.n_c], diag

    def blocks(self):
        v = np.empty((self.nnzb(), 3, 3), np.float64)
        self.ctx.check(lib().bf_get_blocks(self.h, v.ctypes.data))
        return v

    def close(self):
        if self.h:
            lib().bf_problem_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint_bytes(n_nodes, n_tets, n_constraints):
    out = C.c_size_t()
    st = lib().bf_footprint_bytes(int(n_nodes), int(n_tets), int(n_constraints), C.byref(out))
    if st != BF_OK:
        raise BfalError(st, "bf_footprint_bytes failed")
    return int(out.value)


# ------------------------------------------------ host rules (bfal_host.h)

def _checked(fn, *args):
    msg = C.create_string_buffer(256)
    st = fn(*args, msg, len(msg))
    return int(st), msg.value.decode()


def check_mesh(tets, rest, E, nu, rho, fixed=None, material=None):
    """bf_check_mesh on host arrays: (status, message)."""
    tets, rest = _host(tets, np.int32).reshape(-1, 4), _host(rest, np.float64).reshape(-1, 3)
    E, nu, rho = _host(E, np.float64), _host(nu, np.float64), _host(rho, np.float64)
    fixed = None if fixed is None else _host(fixed, np.uint8)
    material = None if material is None else _host(material, np.int32)
    d = bf_mesh_desc(len(rest), len(tets), _ptr(tets), _ptr(rest), _ptr(E), _ptr(nu), _ptr(rho), _ptr(fixed),
                     _ptr(material))
    return _checked(lib().bf_check_mesh, C.byref(d))


def check_state(n_nodes, x, x_hat, x_tilde, dt):
    """bf_check_state on host arrays: (status, message)."""
    x, xh, xt = (None if a is None else _host(a, np.float64) for a in (x, x_hat, x_tilde))
    return _checked(lib().bf_check_state, int(n_nodes), _ptr(x), _ptr(xh), _ptr(xt), float(dt))


def check_constraints(n_nodes, pt, ee, lam, gamma, kappa, delta):
    """bf_check_constraints on host arrays: (status, message)."""
    pt, ee = _host(pt, np.int32).reshape(-1, 4), _host(ee, np.int32).reshape(-1, 4)
    lam = _host(lam, np.float64)
    gamma = None if gamma is None else _host(gamma, np.float64)
    d = bf_constraint_desc(len(pt), len(ee), _ptr(pt) if len(pt) else None, _ptr(ee) if len(ee) else None,
                           _ptr(lam) if len(lam) else None, _ptr(gamma) if gamma is not None and len(gamma) else None,
                           float(kappa), float(delta))
    return _checked(lib().bf_check_constraints, int(n_nodes), C.byref(d))


def check_solve_opts(tol=1e-5, max_iter=20000, precision=BF_PREC_FP32, refine_tol=1e-6):
    """bf_check_solve_opts: (status, message)."""
    o = bf_solve_opts(float(tol), int(max_iter), int(precision), float(refine_tol), 16, 1, 0, 0)
    return _checked(lib().bf_check_solve_opts, C.byref(o))


class StallRule:
    """Section 5.2's stall rule (bf_stall_step)."""

    def __init__(self, alpha_min=1e-4, window=50):
        self.r = bf_stall_rule(float(alpha_min), int(window), 0)

    def step(self, alpha, kappa, delta):
        """Returns (fired, kappa, delta) after one outer iteration's alpha."""
        k, d = C.c_double(kappa), C.c_double(delta)
        fired = lib().bf_stall_step(C.byref(self.r), float(alpha), C.byref(k), C.byref(d))
        if fired < 0:
            raise BfalError(-1, "bf_stall_step: bad argument")
        return bool(fired), k.value, d.value


def slice_plan(slot_u, slot_l, pairs, nparts):
    """bf_slice_plan: (status, wave_ptr [nparts + 1], wave_slices [nslices]) for
    the slot offsets slot_u, slot_l ([nslices + 1] each)."""
    su = np.ascontiguousarray(slot_u, dtype=np.int32)
    sl = np.ascontiguousarray(slot_l, dtype=np.int32)
    n = len(su) - 1
    ptr = np.full(max(int(nparts), 0) + 1, -7, np.int32)
    out = np.full(max(n, 0), -7, np.int32)
    st = lib().bf_slice_plan(int(n), su.ctypes.data, sl.ctypes.data, int(pairs), int(nparts), ptr.ctypes.data,
                             out.ctypes.data)
    return int(st), ptr, out


class Admission:
    """The serving engine's admission policy (bf_admission_*)."""

    def __init__(self, hbm_budget, slots):
        self.h = C.c_void_p()
        st = lib().bf_admission_create(int(hbm_budget), int(slots), C.byref(self.h))
        if st != BF_OK:
            raise BfalError(st, "bf_admission_create failed")

    def push(self, req_id, footprint):
        st = lib().bf_admission_push(self.h, int(req_id), int(footprint))
        if st != BF_OK:
            raise BfalError(st, "bf_admission_push failed")

    def next(self):
        """(+1, id, slot) admitted, (-1, id, -1) rejected as never fitting, (0, None, None) wait."""
        i, s = C.c_int64(), C.c_int32()
        d = lib().bf_admission_next(self.h, C.byref(i), C.byref(s))
        return (int(d), int(i.value), int(s.value)) if d else (0, None, None)

    def release(self, slot, footprint):
        return int(lib().bf_admission_release(self.h, int(slot), int(footprint)))

    def used(self):
        return int(lib().bf_admission_used(self.h))

    def waiting(self):
        return int(lib().bf_admission_waiting(self.h))

    def active(self):
        return int(lib().bf_admission_active(self.h))

    def close(self):
        if self.h:
            lib().bf_admission_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def clock_now():
    """The library's monotonic clock (seconds), the one request times use."""
    return float(lib().bf_clock_now())


class Server:
    """Continuous-batching server (bf_server_*): submit host-memory requests,
    poll for finished ids, take results.  Arguments are marshalled only."""

    def __init__(self, device=0, hbm_budget=8 << 30, max_active=64, iters_per_round=8, admit_threads=0):
        o = bf_server_opts(int(hbm_budget), int(max_active), int(iters_per_round), int(admit_threads))
        self.h = C.c_void_p()
        st = lib().bf_server_create(int(device), C.byref(o), C.byref(self.h))
        if st != BF_OK:
            raise BfalError(st, "bf_server_create failed")
        self._n = {}

    def submit(self, req_id, sc, tol=1e-5, max_iter=20000, check_every=1):
        """Queue the scene dict `sc` (the scenes module's layout) as request req_id."""
        tets, rest = _host(sc["tets"], np.int32), _host(sc["rest"], np.float64)
        E, nu, rho = (_host(sc[k], np.float64) for k in ("E", "nu", "rho"))
        fixed = None if sc.get("fixed") is None else _host(sc["fixed"], np.uint8)
        x, xh, xt = (_host(sc[k], np.float64) for k in ("x", "x_hat", "x_tilde"))
        pt, ee = _host(sc["pt"], np.int32).reshape(-1, 4), _host(sc["ee"], np.int32).reshape(-1, 4)
        lam = _host(sc["lam"], np.float64)
        gamma = None if sc.get("gamma") is None else _host(sc["gamma"], np.float64)
        material = None if sc.get("material") is None else _host(sc["material"], np.int32)
        m = bf_mesh_desc(len(rest), len(tets), _ptr(tets), _ptr(rest), _ptr(E), _ptr(nu), _ptr(rho), _ptr(fixed),
                         _ptr(material))
        d = bf_constraint_desc(len(pt), len(ee), _ptr(pt) if len(pt) else None, _ptr(ee) if len(ee) else None,
                               _ptr(lam) if len(lam) else None,
                               _ptr(gamma) if gamma is not None and len(gamma) else None,
                               float(sc["kappa"]), float(sc["delta"]))
        o = bf_solve_opts(float(tol), int(max_iter), BF_PREC_FP32, 1e-6, 16, int(check_every), 0, 0)
        st = lib().bf_server_submit(self.h, int(req_id), C.byref(m), _ptr(x), _ptr(xh), _ptr(xt),
                                    float(sc["dt"]), C.byref(d), C.byref(o))
        if st != BF_OK:
            raise BfalError(st, "bf_server_submit failed")
        self._n[int(req_id)] = len(rest)

    def poll(self, cap=1024):
        ids = (C.c_int64 * cap)()
        n = C.c_int32()
        st = lib().bf_server_poll(self.h, ids, int(cap), C.byref(n))
        if st != BF_OK:
            raise BfalError(st, "bf_server_poll failed")
        return [int(ids[i]) for i in range(n.value)]

    def result(self, req_id):
        """(p [N,3], stats dict, times dict, status) of a finished request."""
        n = self._n.pop(int(req_id))
        p = np.empty((n, 3), np.float64)
        s, t, rs = bf_step_stats(), bf_request_times(), C.c_int32()
        st = lib().bf_server_result(self.h, int(req_id), p.ctypes.data, C.byref(s), C.byref(t), C.byref(rs))
        if st != BF_OK:
            raise BfalError(st, "bf_server_result failed")
        times = {"t_submit": t.t_submit, "t_admit": t.t_admit, "t_done": t.t_done}
        return p, s.as_dict(), times, int(rs.value)

    def stats(self):
        a, b, u = C.c_int32(), C.c_int32(), C.c_size_t()
        lib().bf_server_stats(self.h, C.byref(a), C.byref(b), C.byref(u))
        return {"pending": a.value, "active": b.value, "used_bytes": u.value}

    def close(self):
        if self.h:
            lib().bf_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
