"""ctypes binding of the plain FP64 CPU oracle (``mmfv_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to check the HIP library.  The product never imports
it.  ``build()`` compiles the C source with gcc (no fast-math, no FP
contraction, so every operation is rounded once as written).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mmfv_oracle.c")
_DUAL = os.path.join(_HERE, "or_dual.h")
_LIB = os.path.join(_HERE, "libmmfv_oracle.so")
_LIB_T = os.path.join(_HERE, "libmmfv_oracle_tangent.so")
MAXM = 8
N_DIAG_HEAD = 9


def _stale(lib, srcs):
    return not os.path.exists(lib) or \
        any(os.path.getmtime(lib) < os.path.getmtime(x) for x in srcs)


def build(force=True):
    """Compile the oracle into ``oracle/libmmfv_oracle.so`` (C, double) and
    its tangent build ``oracle/libmmfv_oracle_tangent.so`` (the same source
    compiled as C++ with a value+derivative scalar)."""
    flags = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]
    if force or _stale(_LIB, [_SRC]):
        subprocess.check_call(["gcc", *flags, "-o", _LIB + ".tmp", _SRC, "-lm"])
        os.replace(_LIB + ".tmp", _LIB)
    if force or _stale(_LIB_T, [_SRC, _DUAL]):
        subprocess.check_call(["g++", "-std=c++17", "-DOR_TANGENT", *flags, "-o",
                               _LIB_T + ".tmp", "-x", "c++", _SRC, "-lm"])
        os.replace(_LIB_T + ".tmp", _LIB_T)
    return _LIB


class Config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("n_mat", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double),
                ("y1", C.c_double),
                ("gamma", C.c_double * MAXM), ("pinf", C.c_double * MAXM),
                ("bc", C.c_int32 * 4), ("inflow_W", C.c_double * 4),
                ("inflow_mat", C.c_int32), ("rk_order", C.c_int32),
                ("cfl", C.c_double), ("alpha_mix", C.c_double),
                ("k_ext", C.c_int32), ("band_ls", C.c_int32),
                ("eos", C.c_int32 * MAXM), ("rho0", C.c_double * MAXM),
                ("tait_B", C.c_double * MAXM), ("p0", C.c_double * MAXM),
                ("flux", C.c_int32), ("scale_sep", C.c_int32),
                ("coord", C.c_int32), ("fs_on", C.c_int32), ("fs_mat", C.c_int32),
                ("fs_p", C.c_double * 5), ("reinit", C.c_int32)]


def make_config(cfg):
    c = Config()
    for k in ("dim", "nx", "ny", "n_mat", "inflow_mat", "rk_order", "k_ext",
              "band_ls"):
        setattr(c, k, int(cfg[k]))
    for k in ("x0", "x1", "y0", "y1", "cfl", "alpha_mix"):
        setattr(c, k, float(cfg[k]))
    for m in range(cfg["n_mat"]):
        c.gamma[m] = float(cfg["gamma"][m])
        c.pinf[m] = float(cfg["pinf"][m])
        c.eos[m] = int(cfg.get("eos", [0] * cfg["n_mat"])[m])
        c.rho0[m] = float(cfg.get("rho0", [0.0] * cfg["n_mat"])[m])
        c.tait_B[m] = float(cfg.get("tait_B", [0.0] * cfg["n_mat"])[m])
        c.p0[m] = float(cfg.get("p0", [0.0] * cfg["n_mat"])[m])
    c.flux = int(cfg.get("flux", 0))
    c.scale_sep = int(cfg.get("scale_sep", 0))
    c.coord = int(cfg.get("coord", 0))
    c.fs_on = int(cfg.get("fs_on", 0))
    c.fs_mat = int(cfg.get("fs_mat", 0))
    for q, v in enumerate(cfg.get("fs_p", [0.0] * 5)):
        c.fs_p[q] = float(v)
    c.reinit = int(cfg.get("reinit", 0))
    for q in range(4):
        c.bc[q] = int(cfg["bc"][q])
        c.inflow_W[q] = float(cfg["inflow_W"][q])
    return c


_libs = {}


def lib(tangent=False):
    path = _LIB_T if tangent else _LIB
    if path not in _libs:
        if _stale(_LIB, [_SRC]) or _stale(_LIB_T, [_SRC, _DUAL]):
            build(force=False)
        L = C.CDLL(path)
        vp = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.or_create.restype = vp
        L.or_create.argtypes = [C.POINTER(Config)]
        L.or_destroy.argtypes = [vp]
        L.or_init.argtypes = [vp, dp, ip, dp]
        L.or_step.argtypes = [vp, C.c_int]
        L.or_get.argtypes = [vp, vp, vp, vp, vp]
        L.or_get_apertures.argtypes = [vp, vp, vp]
        L.or_get_closure.argtypes = [vp, vp, vp]
        L.or_diag.argtypes = [vp, dp]
        L.or_set_dt.argtypes = [vp, C.c_double]
        L.or_set_state.argtypes = [vp, dp, dp, ip]
        L.or_err_cell.restype = C.c_long
        L.or_err_cell.argtypes = [vp]
        d = C.c_double
        L.or_t_weno5.restype = d
        L.or_t_weno5.argtypes = [d, d, d, d, d]
        L.or_t_hllc.argtypes = [vp, C.c_int, dp, dp, dp]
        L.or_t_roe.argtypes = [vp, C.c_int, dp, dp, dp]
        L.or_t_char_weno.argtypes = [vp, C.c_int, dp, dp, dp]
        L.or_t_iface.argtypes = [vp, C.c_int, dp, C.c_int, dp, dp]
        L.or_t_reinit.argtypes = [vp]
        up = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        L.or_t_mixing.argtypes = [vp, dp, dp, dp, ip, dp]
        L.or_t_extension.argtypes = [vp, dp, ip, dp, up, dp, up]
        L.or_t_ls_velocity.argtypes = [vp, dp, ip, dp, up, dp, up, dp]
        if tangent:
            L.or_init_tangent.argtypes = [vp, dp, ip, dp, dp]
            L.or_set_inflow_tangent.argtypes = [vp, dp]
            L.or_seed_state.argtypes = [vp, dp, dp]
            L.or_get_tangent.argtypes = [vp, vp, vp, vp]
        _libs[path] = L
    return _libs[path]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Oracle:
    """One solver instance.  ``cfg`` is a plain dict (see ``workloads``).
    With ``tangent=True`` the instance is the tangent build: every value is
    the same, and each quantity also carries one directional derivative
    (seeded by ``init_tangent``, ``set_inflow_tangent`` or ``seed_state``,
    read by ``get_tangent``); the step size is held fixed under
    differentiation."""

    def __init__(self, cfg, tangent=False):
        self.cfg = dict(cfg)
        self.tangent = bool(tangent)
        self._L = lib(self.tangent)
        self._c = make_config(cfg)
        self._h = self._L.or_create(C.byref(self._c))
        if not self._h:
            raise ValueError("oracle: invalid configuration")
        self.ny, self.nx = int(cfg["ny"]), int(cfg["nx"])
        self.M, self.nv = int(cfg["n_mat"]), int(cfg["dim"]) + 2

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.or_destroy(h)
            self._h = None

    def init(self, phi, chi, W):
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.ny, self.nx)
        chi = np.ascontiguousarray(chi, dtype=np.int32).reshape(self.ny, self.nx)
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(
            self.M, self.nv, self.ny, self.nx)
        return self._L.or_init(self._h, phi, chi, W)

    def step(self, n=1):
        return self._L.or_step(self._h, int(n))

    def set_dt(self, dt):
        self._L.or_set_dt(self._h, float(dt))

    def hllc(self, m, WL, WR):
        F = np.zeros(4)
        self._L.or_t_hllc(self._h, int(m), np.ascontiguousarray(WL, float),
                        np.ascontiguousarray(WR, float), F)
        return F

    def roe(self, m, WL, WR):
        F = np.zeros(4)
        self._L.or_t_roe(self._h, int(m), np.ascontiguousarray(WL, float),
                         np.ascontiguousarray(WR, float), F)
        return F

    def char_weno(self, m, Wc):
        """Characteristic-wise WENO5 face states from the six stencil states
        (rows: cells i-2 .. i+3; columns rho, u_n, u_t, p)."""
        WL, WR = np.zeros(4), np.zeros(4)
        self._L.or_t_char_weno(self._h, int(m), np.ascontiguousarray(Wc, float).ravel(), WL, WR)
        return WL, WR

    def reinit(self):
        """Redistance the current level set (the step's final pass) and
        evaluate the geometry again."""
        self._L.or_t_reinit(self._h)

    def iface(self, mL, WL, mR, WR):
        out = np.zeros(4)
        self._L.or_t_iface(self._h, int(mL), np.ascontiguousarray(WL, float),
                         int(mR), np.ascontiguousarray(WR, float), out)
        return dict(SL=out[0], SR=out[1], SM=out[2], pstar=out[3])

    # -- single operators, for the oracle's own unit pins ---------------------
    def _plane(self, a, dtype=np.float64, lead=()):
        return np.ascontiguousarray(a, dtype=dtype).reshape(lead + (self.ny, self.nx))

    def mix(self, Qt, alpha, phi, chi):
        """Mixing alone: the state ``Qt`` after the stage update, volume
        fractions ``alpha`` and level set (phi, chi) of the new stage; returns
        the mixed state."""
        Qt = self._plane(Qt, lead=(self.M, self.nv))
        al = self._plane(alpha, lead=(self.M,))
        out = np.zeros((self.M, self.nv, self.ny, self.nx))
        rc = self._L.or_t_mixing(self._h, Qt, al, self._plane(phi),
                                 self._plane(chi, np.int32), out)
        if rc:
            raise ValueError(f"or_t_mixing: {rc}")
        return out

    def extend(self, phi, chi, W, valid):
        """Ghost-state extension alone: W [n_mat][4] (rho, u, v, p) and its
        validity before; returns (W, valid) after."""
        W = self._plane(W, lead=(self.M, 4))
        v = self._plane(valid, np.uint8, lead=(self.M,))
        Wo = np.zeros_like(W)
        vo = np.zeros_like(v)
        rc = self._L.or_t_extension(self._h, self._plane(phi), self._plane(chi, np.int32),
                                    W, v, Wo, vo)
        if rc:
            raise ValueError(f"or_t_extension: {rc}")
        return Wo, vo

    def ls_velocity(self, phi, chi, vel, vok, W, valid):
        """Level-set advection velocity alone: the velocities ``vel`` [2]
        already set where ``vok``, material states W [n_mat][4] with their
        validity; returns the velocity field [2][ny][nx]."""
        out = np.zeros((2, self.ny, self.nx))
        rc = self._L.or_t_ls_velocity(
            self._h, self._plane(phi), self._plane(chi, np.int32),
            self._plane(vel, lead=(2,)), self._plane(vok, np.uint8),
            self._plane(W, lead=(self.M, 4)), self._plane(valid, np.uint8, lead=(self.M,)), out)
        if rc:
            raise ValueError(f"or_t_ls_velocity: {rc}")
        return out

    def err_cell(self):
        return self._L.or_err_cell(self._h)

    def get(self):
        Q = np.zeros((self.M, self.nv, self.ny, self.nx))
        al = np.zeros((self.M, self.ny, self.nx))
        phi = np.zeros((self.ny, self.nx))
        chi = np.zeros((self.ny, self.nx), dtype=np.int32)
        self._L.or_get(self._h, _ptr(Q), _ptr(al), _ptr(phi), _ptr(chi))
        return dict(Q=Q, alpha=al, phi=phi, chi=chi)

    def apertures(self):
        Ax = np.zeros((self.M, self.ny, self.nx + 1))
        Ay = np.zeros((self.M, self.ny + 1, self.nx)) if self.cfg["dim"] == 2 \
            else None
        self._L.or_get_apertures(self._h, _ptr(Ax), _ptr(Ay))
        return Ax, Ay

    def closure(self):
        cx = np.zeros((self.M, self.ny, self.nx))
        cy = np.zeros((self.M, self.ny, self.nx))
        self._L.or_get_closure(self._h, _ptr(cx), _ptr(cy))
        return cx, cy

    def diag(self):
        out = np.zeros(N_DIAG_HEAD + 3 * self.M * 4 + 3)
        self._L.or_diag(self._h, out)
        M = self.M
        head = out[:N_DIAG_HEAD]
        return dict(t=head[0], dt=head[1], steps=int(head[2]),
                    n_posfix=int(head[3]), n_fluxskip=int(head[4]),
                    n_ifskip=int(head[5]), n_stranded=int(head[6]),
                    n_mixsrc=int(head[7]), n_updates=int(head[8]),
                    bnd=out[9:9 + 4 * M].reshape(M, 4),
                    xsum=out[9 + 4 * M:9 + 8 * M].reshape(M, 4),
                    n_absorb=int(out[9 + 8 * M]), n_relabel=int(out[10 + 8 * M]),
                    n_oddball=int(out[11 + 8 * M]),
                    xfer=out[12 + 8 * M:12 + 12 * M].reshape(M, 4))

    def set_state(self, Q, phi, chi):
        """Replace (Q, phi, chi); the geometry is rebuilt from the level set
        with the current partial densities as correction masses."""
        Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(self.M, self.nv, self.ny, self.nx)
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.ny, self.nx)
        chi = np.ascontiguousarray(chi, dtype=np.int32).reshape(self.ny, self.nx)
        return self._L.or_set_state(self._h, Q, phi, chi)

    # -- tangent build only ------------------------------------------------
    def init_tangent(self, phi, chi, W, dW):
        """Initial state with derivative dW of the primitive input field."""
        assert self.tangent
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.ny, self.nx)
        chi = np.ascontiguousarray(chi, dtype=np.int32).reshape(self.ny, self.nx)
        shp = (self.M, self.nv, self.ny, self.nx)
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(shp)
        dW = np.ascontiguousarray(dW, dtype=np.float64).reshape(shp)
        return self._L.or_init_tangent(self._h, phi, chi, W, dW)

    def set_inflow_tangent(self, d):
        assert self.tangent
        self._L.or_set_inflow_tangent(self._h, np.ascontiguousarray(d, dtype=np.float64))

    def seed_state(self, dQ, dphi):
        """Set the derivative of the current state (Q, phi)."""
        assert self.tangent
        dQ = np.ascontiguousarray(dQ, dtype=np.float64).reshape(self.M, self.nv, self.ny, self.nx)
        dphi = np.ascontiguousarray(dphi, dtype=np.float64).reshape(self.ny, self.nx)
        self._L.or_seed_state(self._h, dQ, dphi)

    def get_tangent(self):
        assert self.tangent
        dQ = np.zeros((self.M, self.nv, self.ny, self.nx))
        da = np.zeros((self.M, self.ny, self.nx))
        dphi = np.zeros((self.ny, self.nx))
        self._L.or_get_tangent(self._h, _ptr(dQ), _ptr(da), _ptr(dphi))
        return dict(Q=dQ, alpha=da, phi=dphi)


def weno5(v1, v2, v3, v4, v5):
    return lib().or_t_weno5(float(v1), float(v2), float(v3), float(v4), float(v5))


def run(workload, steps=None):
    """Initialise an oracle from a workload dict and advance it."""
    o = Oracle(workload["cfg"])
    rc = o.init(workload["phi"], workload["chi"], workload["W"])
    if rc:
        raise RuntimeError(f"oracle init failed: {rc}")
    n = workload["steps"] if steps is None else steps
    if n:
        rc = o.step(n)
        if rc:
            raise RuntimeError(f"oracle step failed: {rc} at cell {o.err_cell()}")
    return o
