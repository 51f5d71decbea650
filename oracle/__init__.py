"""CPU ORACLE for the coupled pseudopotential / improved-thermal LB step.

Test infrastructure only: the test-suite, the smoke check and the CPU baseline
leg of the benchmark may import this package; the GPU product never does.

It wraps ``liblbpo.so`` (plain single-threaded FP64 C, built from ``lbpo.c``
with ``-O2 -ffp-contract=off``) through ctypes and adds the Maxwell
equal-area construction for the Peng-Robinson EOS of Eq. (56), which fixes the
coexistence densities the flat-interface pin compares against.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbpo.so")
SRC_PATH = os.path.join(HERE, "lbpo.c")

BC_PERIODIC, BC_WALL, BC_OPEN = 0, 1, 2
LAMBDA_CONST, LAMBDA_RHO_CV_CHI = 0, 1
THERMAL_IMPROVED, THERMAL_COMPROMISED, THERMAL_GONG_CHENG = 0, 1, 2
THERMAL_IMPROVED_BGK = 3
FLAG_FREEZE_FLOW = 1
FLAG_FREEZE_THERMAL = 2
FIELDS = {"rho": 0, "T": 1, "ux": 2, "uy": 3, "psi": 4, "Fx": 5, "Fy": 6,
          "phi_prev": 7, "jx": 8, "jy": 9}
ERR_NUMERIC = -5


class Config(ctypes.Structure):
    """Mirror of ``lbpo_config`` (oracle/lbpo.h)."""
    _fields_ = [
        ("a", ctypes.c_double), ("b", ctypes.c_double),
        ("R", ctypes.c_double), ("omega", ctypes.c_double),
        ("cv", ctypes.c_double), ("lambda0", ctypes.c_double),
        ("chi", ctypes.c_double),
        ("s_f", ctypes.c_double * 9), ("s_g", ctypes.c_double * 9),
        ("G", ctypes.c_double), ("sigma", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("T_bc", ctypes.c_double * 4), ("T_hot", ctypes.c_double),
        ("rho_ref", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("rho_v", ctypes.c_double), ("rho_l", ctypes.c_double),
        ("wet_amp", ctypes.c_double), ("wet_shift", ctypes.c_double),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 4),
        ("hot_x0", ctypes.c_int32), ("hot_x1", ctypes.c_int32),
        ("lambda_mode", ctypes.c_int32), ("thermal_model", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("sum_T", ctypes.c_double),
        ("sum_rhocvT", ctypes.c_double), ("liquid_area", ctypes.c_double),
        ("radius", ctypes.c_double), ("radius_count", ctypes.c_double),
        ("max_speed", ctypes.c_double), ("sum_S0", ctypes.c_double),
        ("sum_Fx", ctypes.c_double), ("sum_Fy", ctypes.c_double),
        ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile liblbpo.so (plain C, FP64, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH) or (
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH)):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
             "-D_DEFAULT_SOURCE", "-Wall", "-Wextra", "-fPIC", "-shared",
             "-o", tmp, SRC_PATH, "-lm"], cwd=HERE)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    """The loaded oracle library.  LBPO_LIB in the environment names another
    build of the oracle's source to load instead (the planted-slip test
    loads scratch copies with a deliberate mistake this way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("LBPO_LIB")
        if not path:
            build()
            path = LIB_PATH
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.lbpo_create.argtypes = [ctypes.POINTER(Config),
                                  ctypes.POINTER(ctypes.c_void_p)]
        L.lbpo_destroy.argtypes = [ctypes.c_void_p]
        L.lbpo_destroy.restype = None
        L.lbpo_init_fields.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.lbpo_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.lbpo_get_rho_u_T.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.lbpo_get_field.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        L.lbpo_get_diag.argtypes = [ctypes.c_void_p, ctypes.POINTER(Diag)]
        L.lbpo_get_state.argtypes = [
            ctypes.c_void_p, dp, dp, dp, ctypes.POINTER(ctypes.c_int32), dp,
            ctypes.POINTER(ctypes.c_int64)]
        L.lbpo_set_state.argtypes = [ctypes.c_void_p, dp, dp, dp,
                                     ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_int64]
        L.lbpo_get_tv_prev.argtypes = [ctypes.c_void_p, dp]
        L.lbpo_set_tv_prev.argtypes = [ctypes.c_void_p, dp]
        L.lbpo_matrix_M.argtypes = [dp]
        L.lbpo_matrix_M.restype = None
        L.lbpo_matrix_Minv.argtypes = [dp]
        L.lbpo_matrix_Minv.restype = None
        for nm in ("lbpo_flow_meq", "lbpo_thermal_meq", "lbpo_gc_geq",
                   "lbpo_lin_geq"):
            fn = getattr(L, nm)
            fn.argtypes = [ctypes.c_double] * 3 + [dp]
            fn.restype = None
        L.lbpo_Tc.argtypes = [ctypes.c_double] * 3
        L.lbpo_Tc.restype = ctypes.c_double
        for nm in ("lbpo_p_eos", "lbpo_dpdT"):
            fn = getattr(L, nm)
            fn.argtypes = [ctypes.POINTER(Config), ctypes.c_double,
                           ctypes.c_double]
            fn.restype = ctypes.c_double
        L.lbpo_iso_grad_lap.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp,
                                        dp, dp]
        L.lbpo_iso_grad_lap.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_config(d: dict) -> Config:
    c = Config()
    for name, ctype in Config._fields_:
        if name not in d:
            continue
        v = d[name]
        if hasattr(ctype, "_length_"):
            arr = getattr(c, name)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(c, name, v)
    return c


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what} failed with status {status}")
        self.status = status


class Oracle:
    """One simulation held by the C oracle."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.c = make_config(cfg)
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        h = ctypes.c_void_p()
        st = lib().lbpo_create(ctypes.byref(self.c), ctypes.byref(h))
        if st != 0:
            raise OracleError(st, "lbpo_create")
        self.h = h

    def close(self):
        if self.h:
            lib().lbpo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            raise OracleError(st, what)

    def init_fields(self, rho, ux, uy, T):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(
            self.ny, self.nx) for a in (rho, ux, uy, T)]
        self._check(lib().lbpo_init_fields(self.h, *map(_dp, arrs)),
                    "lbpo_init_fields")

    def step(self, n=1):
        self._check(lib().lbpo_step(self.h, int(n)), "lbpo_step")

    def rho_u_T(self):
        out = [np.empty((self.ny, self.nx)) for _ in range(4)]
        self._check(lib().lbpo_get_rho_u_T(self.h, *map(_dp, out)),
                    "lbpo_get_rho_u_T")
        return tuple(out)

    def field(self, name):
        out = np.empty((self.ny, self.nx))
        self._check(lib().lbpo_get_field(self.h, FIELDS[name], _dp(out)),
                    "lbpo_get_field")
        return out

    def diag(self) -> dict:
        d = Diag()
        self._check(lib().lbpo_get_diag(self.h, ctypes.byref(d)),
                    "lbpo_get_diag")
        return {n: getattr(d, n) for n, _ in Diag._fields_ if n != "pad"}

    def get_state(self):
        n = self.nx * self.ny
        f = np.empty((9, self.ny, self.nx))
        g = np.empty((9, self.ny, self.nx))
        ph = np.empty((self.ny, self.nx))
        pv = ctypes.c_int32()
        ra = ctypes.c_double()
        stp = ctypes.c_int64()
        self._check(lib().lbpo_get_state(
            self.h, _dp(f), _dp(g), _dp(ph), ctypes.byref(pv),
            ctypes.byref(ra), ctypes.byref(stp)), "lbpo_get_state")
        assert f.size == 9 * n
        tv = np.empty((2, self.ny, self.nx))
        self._check(lib().lbpo_get_tv_prev(self.h, _dp(tv)),
                    "lbpo_get_tv_prev")
        return {"f": f, "g": g, "phi_prev": ph, "phi_valid": pv.value,
                "rho_ave": ra.value, "step": stp.value, "tv_prev": tv}

    def set_state(self, st):
        f = np.ascontiguousarray(st["f"], dtype=np.float64)
        g = np.ascontiguousarray(st["g"], dtype=np.float64)
        ph = np.ascontiguousarray(st["phi_prev"], dtype=np.float64)
        self._check(lib().lbpo_set_state(
            self.h, _dp(f), _dp(g), _dp(ph), int(st["phi_valid"]),
            float(st["rho_ave"]), int(st["step"])), "lbpo_set_state")
        if "tv_prev" in st:
            tv = np.ascontiguousarray(st["tv_prev"], dtype=np.float64)
            self._check(lib().lbpo_set_tv_prev(self.h, _dp(tv)),
                        "lbpo_set_tv_prev")


# ---------------------------------------------------------------- pieces --

def matrix_M():
    out = np.empty(81)
    lib().lbpo_matrix_M(_dp(out))
    return out.reshape(9, 9)


def matrix_Minv():
    out = np.empty(81)
    lib().lbpo_matrix_Minv(_dp(out))
    return out.reshape(9, 9)


def flow_meq(rho, vx, vy):
    out = np.empty(9)
    lib().lbpo_flow_meq(rho, vx, vy, _dp(out))
    return out


def thermal_meq(T, vx, vy):
    out = np.empty(9)
    lib().lbpo_thermal_meq(T, vx, vy, _dp(out))
    return out


def gc_geq(T, vx, vy):
    """Per-direction equilibrium of the Gong-Cheng model, Eq. (14)."""
    out = np.zeros(9)
    lib().lbpo_gc_geq(T, vx, vy, _dp(out))
    return out


def lin_geq(T, vx, vy):
    """Per-direction equilibrium linear in v, Eq. (29)."""
    out = np.zeros(9)
    lib().lbpo_lin_geq(T, vx, vy, _dp(out))
    return out


def Tc(a, b, R):
    return lib().lbpo_Tc(a, b, R)


def p_eos(cfg: dict, rho, T):
    c = make_config(cfg)
    return lib().lbpo_p_eos(ctypes.byref(c), float(rho), float(T))


def dpdT(cfg: dict, rho, T):
    c = make_config(cfg)
    return lib().lbpo_dpdT(ctypes.byref(c), float(rho), float(T))


def iso_grad_lap(X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    ny, nx = X.shape
    dx, dy, lap = np.empty_like(X), np.empty_like(X), np.empty_like(X)
    lib().lbpo_iso_grad_lap(nx, ny, _dp(X), _dp(dx), _dp(dy), _dp(lap))
    return dx, dy, lap


def maxwell(cfg: dict, T: float):
    """Maxwell equal-area coexistence densities (rho_v, rho_l) of the EOS of
    Eq. (56) at temperature T: equal pressure and equal area in the p-V plane,
    int_{V_l}^{V_v} p dV = p_s (V_v - V_l), with V = 1/rho."""
    from scipy import integrate, optimize

    def p(r):
        return p_eos(cfg, r, T)

    def dp_drho(r):
        h = 1e-6 * r
        return (p(r + h) - p(r - h)) / (2 * h)

    # spinodal points bracket the two branches
    grid = np.linspace(0.05, 0.98 / cfg["b"], 4000)
    der = np.array([dp_drho(r) for r in grid])
    neg = np.where(der < 0)[0]
    if len(neg) == 0:
        raise ValueError("T is supercritical: no coexistence")
    r_s1 = optimize.brentq(dp_drho, grid[neg[0] - 1], grid[neg[0]])
    r_s2 = optimize.brentq(dp_drho, grid[neg[-1]], grid[neg[-1] + 1])

    def branch(ps, lo, hi):
        return optimize.brentq(lambda r: p(r) - ps, lo, hi, xtol=1e-300,
                               rtol=1e-15, maxiter=500)

    def area(ps):
        rv = branch(ps, 1e-300, r_s1)
        rl = branch(ps, r_s2, 0.999 / cfg["b"])
        val, _ = integrate.quad(lambda r: p(r) / (r * r), rv, rl,
                                epsabs=1e-14, epsrel=1e-13, limit=400)
        return val - ps * (1.0 / rv - 1.0 / rl)

    p_lo = max(p(r_s2), 1e-9 * p(r_s1))
    p_hi = p(r_s1)
    ps = optimize.brentq(area, p_lo * (1 + 1e-12), p_hi * (1 - 1e-12),
                         xtol=1e-16, rtol=1e-15, maxiter=500)
    rv = branch(ps, 1e-300, r_s1)
    rl = branch(ps, r_s2, 0.999 / cfg["b"])
    return rv, rl, ps
