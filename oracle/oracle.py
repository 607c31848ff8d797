"""ctypes binding of the CPU oracle (liboracle_sharp.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke entry point
and the benchmark's CPU-baseline leg.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_sharp.so")
SRC = os.path.join(_HERE, "sharp_oracle.c")


def build(force=True):
    """Compile the oracle with gcc (plain C11, FP64, no fast-math, no FMA)."""
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("n", C.c_int * 3), ("lo", C.c_double * 3), ("h", C.c_double),
        ("bc", C.c_int * 3), ("gamma", C.c_double * 2), ("pinf", C.c_double * 2),
        ("cfl", C.c_double), ("rk", C.c_int), ("n_thr", C.c_double), ("alpha_mix", C.c_double),
        ("ls_band", C.c_double), ("ext_band", C.c_double), ("mix_band", C.c_double),
        ("ext_iters", C.c_int), ("reinit_iters", C.c_int), ("weno_eps", C.c_double),
        ("force_cycle", C.c_int), ("no_correction", C.c_int),
        ("dt_replay", C.c_void_p), ("n_dt_replay", C.c_long),
        ("log_levelset", C.c_int), ("ls_replay", C.c_void_p), ("n_ls_replay", C.c_long),
        ("sigma", C.c_double),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("cycles", C.c_long), ("steps", C.c_long * 2), ("cell_updates", C.c_long * 2),
        ("t", C.c_double), ("last_n", C.c_double), ("last_dt", C.c_double * 2),
        ("bflux", (C.c_double * 5) * 2),
    ]

    def as_dict(self):
        return dict(cycles=self.cycles, steps=list(self.steps), cell_updates=list(self.cell_updates),
                    t=self.t, last_n=self.last_n, last_dt=list(self.last_dt),
                    bflux=np.array([list(r) for r in self.bflux]))


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build_at(src, out, defines=()):
    """Compile an oracle source file to a shared library at `out` (the tests
    also build deliberately broken copies of the oracle this way, to show
    that a pin catches the mistake)."""
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off"]
                          + ["-D" + d for d in defines] + ["-o", out, src, "-lm"])
    return out


def load(path):
    """ctypes handle of an oracle library with every entry point typed."""
    L = C.CDLL(path)
    L.or_default_params.argtypes = [C.POINTER(Params)]
    L.or_create.argtypes = [C.POINTER(Params)]
    L.or_create.restype = C.c_void_p
    L.or_destroy.argtypes = [C.c_void_p]
    L.or_set_state.argtypes = [C.c_void_p, _dp, _dp]
    L.or_advance.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_long, C.POINTER(Stats)]
    L.or_schedule.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_long]
    L.or_schedule.restype = C.c_long
    L.or_levelset_log.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_long]
    L.or_levelset_log.restype = C.c_long
    L.or_get_state.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.or_totals.argtypes = [C.c_void_p, _dp]
    L.or_last_error.restype = C.c_char_p
    L.or_prim2cons.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp]
    L.or_cons2prim.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp]
    L.or_weno5.argtypes = [C.c_double] * 6
    L.or_weno5.restype = C.c_double
    L.or_riemann.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double, _dp]
    L.or_riemann_jump.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, _dp]
    L.or_riemann_sample.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_double, _dp]
    L.or_clip_area.argtypes = [_dp]
    L.or_clip_area.restype = C.c_double
    L.or_face_flux_1d.argtypes = [_dp, C.c_double, C.c_double, C.c_double, _dp]
    L.or_geometry.argtypes = [C.c_void_p, _dp, _dp]
    L.or_face_count.argtypes = [C.c_void_p]
    L.or_face_count.restype = C.c_long
    L.or_plan_cycle.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.or_substep.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                             C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.or_substep.restype = C.c_double
    L.or_ls_transport.argtypes = [C.POINTER(Params), _dp, _dp, C.c_double, C.c_int]
    L.or_reinit_run.argtypes = [C.POINTER(Params), _dp]
    L.or_extend_v_run.argtypes = [C.POINTER(Params), _dp, _dp]
    L.or_extend_w_run.argtypes = [C.POINTER(Params), _dp, _dp]
    L.or_curvature_run.argtypes = [C.POINTER(Params), _dp, _dp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load(LIB_PATH)
    return _lib


def default_params(L=None):
    p = Params()
    (L or lib()).or_default_params(C.byref(p))
    return p


def params_from_case(case, L=None, **over):
    p = default_params(L)
    p.ndim = case["ndim"]
    for d in range(3):
        p.n[d] = case["n"][d]
        p.lo[d] = case["lo"][d]
        p.bc[d] = case["bc"][d]
    p.h = case["h"]
    p.gamma[0], p.gamma[1] = case["gamma"]
    p.pinf[0], p.pinf[1] = case["pinf"]
    p.sigma = float(case.get("sigma", 0.0))
    _apply(p, over)
    return p


def _apply(p, over):
    """set parameter fields; the replayed arrays are kept on the returned
    object until or_create has copied them"""
    for k, v in over.items():
        if k in ("dt_replay", "ls_replay"):
            a = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1))
            setattr(p, "_%s_keep" % k, a)
            setattr(p, k, a.ctypes.data if a.size else None)
            setattr(p, "n_" + k, int(a.size))
            continue
        setattr(p, k, v)


class OracleSim:
    """Plain CPU reference of the whole method (test infrastructure)."""

    def __init__(self, case, L=None, **over):
        self.case = case
        self.L = L or lib()
        self.p = params_from_case(case, self.L, **over)
        self.D = case["ndim"]
        self.NV = self.D + 2
        self.nc = int(np.prod(case["n"]))
        self.h = self.L.or_create(C.byref(self.p))
        if not self.h:
            raise RuntimeError(self.L.or_last_error().decode())
        self.set_state(case["phi"], case["prim"])

    def __del__(self):
        if getattr(self, "h", None):
            self.L.or_destroy(self.h)
            self.h = None

    def set_state(self, phi, prim):
        rc = self.L.or_set_state(self.h, np.ascontiguousarray(phi, dtype=np.float64).reshape(-1),
                                np.ascontiguousarray(prim, dtype=np.float64).reshape(-1))
        if rc:
            raise RuntimeError(self.L.or_last_error().decode())

    def schedule(self):
        """the CFL steps taken since creation (or_schedule's order)"""
        n = self.L.or_schedule(self.h, None, 0)
        out = np.zeros(n)
        if n:
            self.L.or_schedule(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), n)
        return out

    def levelset_log(self):
        """the level sets of every single-dt stage (log_levelset), [stages, cells]"""
        n = self.L.or_levelset_log(self.h, None, 0)
        out = np.zeros(n)
        if n:
            self.L.or_levelset_log(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), n)
        return out.reshape(-1, self.nc)

    def advance(self, t_end, mode=0, max_cycles=0):
        st = Stats()
        rc = self.L.or_advance(self.h, float(t_end), int(mode), int(max_cycles), C.byref(st))
        if rc:
            raise RuntimeError("oracle advance failed (%d): %s" % (rc, self.L.or_last_error().decode()))
        return st.as_dict()

    def state(self):
        phi = np.empty(self.nc)
        cons = np.empty(2 * self.NV * self.nc)
        alpha = np.empty(self.nc)
        self.L.or_get_state(self.h, phi, cons, alpha)
        return phi, cons.reshape(2, self.NV, self.nc), alpha

    def totals(self):
        out = np.empty(10)
        self.L.or_totals(self.h, out)
        return out.reshape(2, 5)

    def geometry(self):
        nf = self.L.or_face_count(self.h)
        alpha = np.empty(self.nc)
        ap = np.empty(3 * nf)
        self.L.or_geometry(self.h, alpha, ap)
        return alpha, ap.reshape(3, nf)


def weno5(v, eps=1e-6):
    return lib().or_weno5(*[float(x) for x in v], float(eps))


def riemann(WL, WR, gL, piL, gR, piR):
    out = np.empty(5)
    lib().or_riemann(np.asarray(WL, dtype=np.float64), np.asarray(WR, dtype=np.float64),
                     gL, piL, gR, piR, out)
    return out


def riemann_jump(WL, WR, gL, piL, gR, piR, jump):
    """Riemann problem with the contact pressure jump p_L - p_R = jump:
    {p*_L, u*, rho*_L, rho*_R, iterations}"""
    out = np.empty(5)
    lib().or_riemann_jump(np.asarray(WL, dtype=np.float64), np.asarray(WR, dtype=np.float64),
                          gL, piL, gR, piR, float(jump), out)
    return out


def riemann_sample(WL, WR, gL, piL, gR, piR, xi):
    out = np.empty(4)
    lib().or_riemann_sample(np.asarray(WL, dtype=np.float64), np.asarray(WR, dtype=np.float64),
                            gL, piL, gR, piR, float(xi), out)
    return out


def clip_area(v):
    return lib().or_clip_area(np.asarray(v, dtype=np.float64))


def prim2cons(D, g, pi, W):
    U = np.empty(D + 2)
    lib().or_prim2cons(D, g, pi, np.asarray(W, dtype=np.float64), U)
    return U


def cons2prim(D, g, pi, U):
    W = np.empty(D + 2)
    rc = lib().or_cons2prim(D, g, pi, np.asarray(U, dtype=np.float64), W)
    return W, rc


def face_flux_1d(W6, g, pi, eps=1e-6):
    F = np.empty(3)
    lib().or_face_flux_1d(np.asarray(W6, dtype=np.float64).reshape(-1), g, pi, eps, F)
    return F


def plan_cycle(dt_slow, dt_fast, remaining, thr=0.7):
    out = C.c_double()
    single = C.c_int()
    lib().or_plan_cycle(dt_slow, dt_fast, remaining, thr, C.byref(out), C.byref(single))
    return out.value, bool(single.value)


def substep(tau, t1, dt_fast, rk, half_done):
    hh = C.c_int()
    fin = C.c_int()
    d = lib().or_substep(tau, t1, dt_fast, rk, half_done, C.byref(hh), C.byref(fin))
    return d, bool(hh.value), bool(fin.value)


def exact_tube(case, x, t):
    """Exact solution (rho, u, p, fluid) of a 1-D two-fluid Riemann problem at
    time t, by sampling the exact stiffened-gas Riemann solution."""
    xi = case["x_interface"]
    WL = np.array([case["prim"][0, 0, 0], case["prim"][0, 1, 0], case["prim"][0, 2, 0]])
    WR = np.array([case["prim"][1, 0, -1], case["prim"][1, 1, -1], case["prim"][1, 2, -1]])
    g, pi = case["gamma"], case["pinf"]
    out = np.empty((len(x), 4))
    for i, xx in enumerate(x):
        out[i] = riemann_sample(WL, WR, g[0], pi[0], g[1], pi[1], (xx - xi) / t)
    return out


def _grid_params(L, ndim, n, bc, **over):
    """parameters of a unit run on [0, 1]^ndim with n cells per direction"""
    p = default_params(L)
    p.ndim = ndim
    for d in range(3):
        p.n[d] = n if d < ndim else 1
        p.lo[d] = 0.0
        p.bc[d] = bc if d < ndim else 0
    p.h = 1.0 / n
    _apply(p, over)
    return p


def ls_transport(phi, vel, dt, nsteps, ndim, n, bc=1, L=None, **over):
    """level-set transport by the fixed velocity field vel[D][cells]"""
    L = L or lib()
    p = _grid_params(L, ndim, n, bc, **over)
    out = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1).copy()
    v = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1)
    if L.or_ls_transport(C.byref(p), out, v, float(dt), int(nsteps)):
        raise RuntimeError("or_ls_transport failed")
    return out


def reinit_run(phi, ndim, n, bc=0, L=None, **over):
    L = L or lib()
    p = _grid_params(L, ndim, n, bc, **over)
    out = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1).copy()
    if L.or_reinit_run(C.byref(p), out):
        raise RuntimeError("or_reinit_run failed")
    return out


def extend_v_run(phi, v, ndim, n, bc=0, L=None, **over):
    L = L or lib()
    p = _grid_params(L, ndim, n, bc, **over)
    out = np.ascontiguousarray(v, dtype=np.float64).reshape(-1).copy()
    if L.or_extend_v_run(C.byref(p), np.ascontiguousarray(phi, dtype=np.float64).reshape(-1), out):
        raise RuntimeError("or_extend_v_run failed")
    return out.reshape(ndim, -1)


def extend_w_run(phi, W, ndim, n, bc=0, L=None, **over):
    L = L or lib()
    p = _grid_params(L, ndim, n, bc, **over)
    out = np.ascontiguousarray(W, dtype=np.float64).reshape(-1).copy()
    if L.or_extend_w_run(C.byref(p), np.ascontiguousarray(phi, dtype=np.float64).reshape(-1), out):
        raise RuntimeError("or_extend_w_run failed")
    return out.reshape(2, ndim + 2, -1)


def curvature_run(phi, ndim, n, bc=0, L=None, **over):
    """curvature of the level set at the interface point nearest each cell
    centre (the one the Laplace jump takes)"""
    L = L or lib()
    p = _grid_params(L, ndim, n, bc, **over)
    out = np.empty(int(n) ** ndim)
    if L.or_curvature_run(C.byref(p), np.ascontiguousarray(phi, dtype=np.float64).reshape(-1), out):
        raise RuntimeError("or_curvature_run failed")
    return out
