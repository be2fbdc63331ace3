"""ctypes binding of the C ABI in ``include/mmfv.h`` (argument marshalling
only: every step of the method runs in the HIP kernels of ``libmmfv.so``).

Arrays may be numpy arrays (host memory) or torch tensors on the GPU
(device memory, passed by ``data_ptr()``).  Torch is used for device memory
and the HIP stream, nothing else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmmfv.so")

MM_OK, MM_EINVAL, MM_ENOMEM, MM_EDEVICE, MM_ENONPHYS, MM_ESTATE, MM_ENOTIMPL = range(7)
MM_HOST, MM_DEVICE = 0, 1
MAX_MAT = 8
STATUS = {0: "MM_OK", 1: "MM_EINVAL", 2: "MM_ENOMEM", 3: "MM_EDEVICE",
          4: "MM_ENONPHYS", 5: "MM_ESTATE", 6: "MM_ENOTIMPL"}

EXPORTS = ("mm_create", "mm_init_state", "mm_step", "mm_get_conserved",
           "mm_get_diagnostics", "mm_set_dt", "mm_set_dt_schedule", "mm_set_guard",
           "mm_adjoint_step", "mm_adjoint_inflow",
           "mm_tape_info", "mm_destroy",
           "mm_last_error", "mm_set_profiling", "mm_get_profile", "mm_mr_analyse",
           "mm_batch_create", "mm_batch_init_state", "mm_batch_step",
           "mm_batch_get_conserved", "mm_batch_get_diagnostics",
           "mm_batch_set_threads", "mm_batch_get_threads", "mm_batch_destroy",
           "mm_batch_last_error", "mm_batch_run_noalloc")


class MMConfig(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("n_mat", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double),
                ("y1", C.c_double),
                ("gamma", C.c_double * MAX_MAT), ("pinf", C.c_double * MAX_MAT),
                ("bc", C.c_int32 * 4), ("inflow_W", C.c_double * 4),
                ("inflow_mat", C.c_int32), ("rk_order", C.c_int32),
                ("cfl", C.c_double), ("alpha_mix", C.c_double),
                ("k_ext", C.c_int32), ("band_ls", C.c_int32),
                ("eos", C.c_int32 * MAX_MAT), ("rho0", C.c_double * MAX_MAT),
                ("tait_B", C.c_double * MAX_MAT), ("p0", C.c_double * MAX_MAT),
                ("flux", C.c_int32), ("scale_sep", C.c_int32),
                ("coord", C.c_int32), ("fs_on", C.c_int32), ("fs_mat", C.c_int32),
                ("fs_p", C.c_double * 5), ("reinit", C.c_int32)]


class MMDiag(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("steps", C.c_int64),
                ("n_posfix", C.c_int64), ("n_fluxskip", C.c_int64),
                ("n_ifskip", C.c_int64), ("n_stranded", C.c_int64),
                ("n_mixsrc", C.c_int64), ("n_updates", C.c_int64),
                ("err_cell", C.c_int64),
                ("sum_Q", (C.c_double * 4) * 8), ("bnd_in", (C.c_double * 4) * 8),
                ("exch", (C.c_double * 4) * 8),
                ("n_band", C.c_int64), ("n_ghost", C.c_int64), ("n_tiles", C.c_int64),
                ("err_step", C.c_int64), ("n_absorb", C.c_int64),
                ("n_relabel", C.c_int64), ("n_oddball", C.c_int64)]


_DIAG_ARRAYS = ("sum_Q", "bnd_in", "exch")


def _diag_dict(d, n_mat):
    out = {}
    for k, _ in MMDiag._fields_:
        v = getattr(d, k)
        out[k] = np.array([[v[r][c] for c in range(4)] for r in range(n_mat)]) \
            if k in _DIAG_ARRAYS else v
    return out


class MMProfile(C.Structure):
    _fields_ = [("bulk_ms", C.c_double), ("bulk_launches", C.c_int64),
                ("bulk_updates", C.c_int64), ("bulk_bytes", C.c_double)]


MR_MAXL = 10


class MMMrParams(C.Structure):
    _fields_ = [("block", C.c_int32), ("levels", C.c_int32), ("eps", C.c_double),
                ("band", C.c_double)]


class MMMrResult(C.Structure):
    _fields_ = [("exist", C.c_int64 * (MR_MAXL + 1)), ("leaf", C.c_int64 * (MR_MAXL + 1)),
                ("compression", C.c_double), ("scale", C.c_double * 2)]


class MMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load ``libmmfv.so``; raise if it has not been built (there is no
    fallback implementation)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "paper_1704_00519_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        L.mm_create.argtypes = [C.POINTER(MMConfig), vp, C.POINTER(vp)]
        L.mm_init_state.argtypes = [vp, vp, vp, vp, i32]
        L.mm_step.argtypes = [vp, i32, i32, C.POINTER(dbl)]
        L.mm_get_conserved.argtypes = [vp, vp, vp, vp, vp, i32]
        L.mm_get_diagnostics.argtypes = [vp, C.POINTER(MMDiag)]
        L.mm_set_dt.argtypes = [vp, dbl]
        L.mm_set_dt_schedule.argtypes = [vp, vp, i32]
        L.mm_set_guard.argtypes = [vp, i32]
        L.mm_adjoint_step.argtypes = [vp, vp, vp, vp, vp, vp, i32]
        L.mm_adjoint_inflow.argtypes = [vp, vp]
        L.mm_tape_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp]
        L.mm_destroy.argtypes = [vp]
        L.mm_set_profiling.argtypes = [vp, i32]
        L.mm_get_profile.argtypes = [vp, C.POINTER(MMProfile)]
        L.mm_mr_analyse.argtypes = [vp, C.POINTER(MMMrParams), vp, vp, C.POINTER(MMMrResult), i32]
        L.mm_batch_create.argtypes = [vp, i32, vp, C.POINTER(vp)]
        L.mm_batch_init_state.argtypes = [vp, vp, vp, vp, i32]
        L.mm_batch_step.argtypes = [vp, i32]
        L.mm_batch_get_conserved.argtypes = [vp, vp, vp, vp, vp, i32]
        L.mm_batch_get_diagnostics.argtypes = [vp, vp]
        L.mm_batch_set_threads.argtypes = [vp, i32]
        L.mm_batch_get_threads.argtypes = [vp, C.POINTER(i32), vp]
        L.mm_batch_destroy.argtypes = [vp]
        L.mm_batch_last_error.argtypes = [vp]
        L.mm_batch_last_error.restype = C.c_char_p
        for name in ("mm_batch_create", "mm_batch_init_state", "mm_batch_step",
                     "mm_batch_get_conserved", "mm_batch_get_diagnostics",
                     "mm_batch_set_threads", "mm_batch_get_threads",
                     "mm_batch_destroy"):
            getattr(L, name).restype = i32
        L.mm_batch_run_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp]
        L.mm_batch_run_noalloc.restype = i32
        L.mm_last_error.argtypes = [vp]
        L.mm_last_error.restype = C.c_char_p
        for name in ("mm_create", "mm_init_state", "mm_step", "mm_get_conserved",
                     "mm_get_diagnostics", "mm_set_dt", "mm_set_dt_schedule",
                     "mm_set_guard", "mm_adjoint_step",
                     "mm_adjoint_inflow", "mm_tape_info",
                     "mm_destroy", "mm_set_profiling", "mm_get_profile", "mm_mr_analyse"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def make_config(cfg):
    c = MMConfig()
    for k in ("dim", "nx", "ny", "n_mat", "inflow_mat", "rk_order", "k_ext",
              "band_ls"):
        setattr(c, k, int(cfg[k]))
    for k in ("x0", "x1", "y0", "y1", "cfl", "alpha_mix"):
        setattr(c, k, float(cfg[k]))
    M = int(cfg["n_mat"])
    for m in range(M):
        c.gamma[m] = float(cfg["gamma"][m])
        c.pinf[m] = float(cfg["pinf"][m])
        c.eos[m] = int(cfg.get("eos", [0] * M)[m])
        c.rho0[m] = float(cfg.get("rho0", [0.0] * M)[m])
        c.tait_B[m] = float(cfg.get("tait_B", [0.0] * M)[m])
        c.p0[m] = float(cfg.get("p0", [0.0] * M)[m])
    c.flux = int(cfg.get("flux", 0))
    c.scale_sep = int(cfg.get("scale_sep", 0))
    c.coord = int(cfg.get("coord", 0))
    c.fs_on = int(cfg.get("fs_on", 0))
    c.fs_mat = int(cfg.get("fs_mat", 0))
    for q, x in enumerate(cfg.get("fs_p", [0.0] * 5)):
        c.fs_p[q] = float(x)
    c.reinit = int(cfg.get("reinit", 0))
    for q in range(4):
        c.bc[q] = int(cfg["bc"][q])
        c.inflow_W[q] = float(cfg["inflow_W"][q])
    return c


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _device_arg(a, dtype, numel, name):
    """Device pointer of a torch tensor after checking that it lives on
    the GPU, has the expected dtype, is contiguous and has numel elements."""
    if not (_is_torch(a) and getattr(a, "is_cuda", False)):
        raise TypeError(f"{name}: expected a CUDA tensor")
    if str(a.dtype) != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {a.dtype}")
    if not a.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if a.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {a.numel()}")
    return C.c_void_p(a.data_ptr())


class Solver:
    """One context of the HIP library.  ``cfg``: dict with the fields of
    ``mm_config``; ``stream``: a hipStream_t handle (int) or None."""

    def __init__(self, cfg, stream=None):
        L = load()
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        h = C.c_void_p()
        st = L.mm_create(C.byref(self._c), C.c_void_p(stream or 0), C.byref(h))
        if st != MM_OK:
            raise MMError(st, L.mm_last_error(None).decode())
        self._h = h
        self.ny, self.nx = int(cfg["ny"]), int(cfg["nx"])
        self.M, self.nv = int(cfg["n_mat"]), int(cfg["dim"]) + 2

    def _check(self, st):
        if st != MM_OK:
            raise MMError(st, load().mm_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            load().mm_destroy(self._h)
            self._h = None

    __del__ = close

    def init(self, phi, chi, W):
        if _is_torch(phi) or _is_torch(chi) or _is_torch(W):
            n = self.nx * self.ny
            st = load().mm_init_state(
                self._h, _device_arg(phi, "torch.float64", n, "phi"),
                _device_arg(chi, "torch.int32", n, "chi"),
                _device_arg(W, "torch.float64", self.M * self.nv * n, "W"), MM_DEVICE)
        else:
            phi = np.ascontiguousarray(phi, np.float64)
            chi = np.ascontiguousarray(chi, np.int32)
            W = np.ascontiguousarray(W, np.float64)
            assert phi.size == self.nx * self.ny and chi.size == phi.size
            assert W.size == self.M * self.nv * phi.size
            st = load().mm_init_state(self._h, phi.ctypes.data, chi.ctypes.data,
                                      W.ctypes.data, MM_HOST)
        self._check(st)

    def step(self, n=1, record=0):
        """Advance n steps; record = K > 0 keeps the adjoint tape with a
        checkpoint every K steps."""
        t = C.c_double()
        self._check(load().mm_step(self._h, int(n), int(record), C.byref(t)))
        return t.value

    def adjoint_step(self, lamQ=None, lamPhi=None, lamAlpha=None, out=True):
        """Reverse the last recorded step.  Inputs (numpy, interior layout)
        replace the carried adjoint; None continues from it.  Returns
        (lamQ, lamPhi) of the state before the step, or None with out=False."""
        def inp(a, shape):
            if a is None:
                return None, None
            a = np.ascontiguousarray(a, np.float64).reshape(shape)
            return a, a.ctypes.data
        qa, qp = inp(lamQ, (self.M, self.nv, self.ny, self.nx))
        pa, pp = inp(lamPhi, (self.ny, self.nx))
        aa, ap = inp(lamAlpha, (self.M, self.ny, self.nx))
        oq = op = None
        if out:
            oq = np.zeros((self.M, self.nv, self.ny, self.nx))
            op = np.zeros((self.ny, self.nx))
        self._check(load().mm_adjoint_step(
            self._h, qp, pp, ap, oq.ctypes.data if out else None,
            op.ctypes.data if out else None, MM_HOST))
        del qa, pa, aa
        return (oq, op) if out else None

    def adjoint_inflow(self):
        out = np.zeros(4)
        self._check(load().mm_adjoint_inflow(self._h, out.ctypes.data))
        return out

    def tape(self):
        """(recorded steps, steps left to reverse, recorded step sizes)."""
        n, rem = C.c_int64(), C.c_int64()
        self._check(load().mm_tape_info(self._h, C.byref(n), C.byref(rem), None))
        dt = np.zeros(max(n.value, 1))
        if n.value:
            self._check(load().mm_tape_info(self._h, None, None, dt.ctypes.data))
        return n.value, rem.value, dt[:n.value]

    def set_dt(self, dt):
        self._check(load().mm_set_dt(self._h, float(dt)))

    def set_dt_schedule(self, dts):
        """The next len(dts) steps use these step sizes, one per step."""
        a = np.ascontiguousarray(dts, np.float64).ravel()
        self._check(load().mm_set_dt_schedule(self._h, a.ctypes.data if a.size else None,
                                              int(a.size)))

    def set_guard(self, on=True):
        """Keep the state of the last completed step when a step fails."""
        self._check(load().mm_set_guard(self._h, 1 if on else 0))

    def get(self):
        Q = np.zeros((self.M, self.nv, self.ny, self.nx))
        al = np.zeros((self.M, self.ny, self.nx))
        phi = np.zeros((self.ny, self.nx))
        chi = np.zeros((self.ny, self.nx), np.int32)
        self._check(load().mm_get_conserved(self._h, Q.ctypes.data, al.ctypes.data,
                                            phi.ctypes.data, chi.ctypes.data,
                                            MM_HOST))
        return dict(Q=Q, alpha=al, phi=phi, chi=chi)

    def get_device(self, Q, alpha=None, phi=None, chi=None):
        """Write the state into torch tensors on the device (no host copy)."""
        n = self.nx * self.ny
        args = (_device_arg(Q, "torch.float64", self.M * self.nv * n, "Q"),
                None if alpha is None else _device_arg(alpha, "torch.float64", self.M * n, "alpha"),
                None if phi is None else _device_arg(phi, "torch.float64", n, "phi"),
                None if chi is None else _device_arg(chi, "torch.int32", n, "chi"))
        self._check(load().mm_get_conserved(self._h, *args, MM_DEVICE))

    def set_profiling(self, on=True):
        self._check(load().mm_set_profiling(self._h, 1 if on else 0))

    def mr_analyse(self, block=16, levels=3, eps=1e-3, band=None, flags=True):
        """Multiresolution analysis of the current state (2D): the leaf level
        of every block of the grid, per level the detail flags (levels
        0..L-1) and interface identifiers (0..L), the counts of existing and
        leaf blocks, the compression and the fields' largest magnitudes.
        band defaults to the level set's band width."""
        if band is None:
            band = self.cfg["band_ls"] * min((self.cfg["x1"] - self.cfg["x0"]) / self.nx,
                                             (self.cfg["y1"] - self.cfg["y0"]) / self.ny)
        nbx, nby = self.nx // block, self.ny // block
        leaf = np.zeros((nby, nbx), np.int32)
        shapes = [(nby >> (levels - l), nbx >> (levels - l)) for l in range(levels + 1)]
        nfl = sum(a * b for a, b in shapes[:levels]) + sum(a * b for a, b in shapes)
        fl = np.zeros(nfl, np.uint8)
        p = MMMrParams(int(block), int(levels), float(eps), float(band))
        r = MMMrResult()
        self._check(load().mm_mr_analyse(self._h, C.byref(p), leaf.ctypes.data,
                                         fl.ctypes.data if flags else None, C.byref(r),
                                         MM_HOST))
        out = dict(leaf=leaf, counts=[(int(r.exist[l]), int(r.leaf[l])) for l in range(levels + 1)],
                   compression=r.compression, scale=[r.scale[0], r.scale[1]])
        if flags:
            det, ifc, o = [], [], 0
            for l in range(levels):
                n = shapes[l][0] * shapes[l][1]
                det.append(fl[o:o + n].reshape(shapes[l]).astype(bool))
                o += n
            for l in range(levels + 1):
                n = shapes[l][0] * shapes[l][1]
                ifc.append(fl[o:o + n].reshape(shapes[l]).astype(bool))
                o += n
            out.update(detail=det, iface=ifc)
        return out

    def profile(self):
        p = MMProfile()
        self._check(load().mm_get_profile(self._h, C.byref(p)))
        return {k: getattr(p, k) for k, _ in MMProfile._fields_}

    def diag(self):
        d = MMDiag()
        self._check(load().mm_get_diagnostics(self._h, C.byref(d)))
        return _diag_dict(d, self.M)


class Batch:
    """Many ragged 1D instances advanced by one persistent launch.
    ``instances``: list of workload dicts (cfg, phi, chi, W) with the same
    n_mat and rk_order."""

    def __init__(self, instances, stream=None):
        L = load()
        self.n = len(instances)
        cfgs = (MMConfig * self.n)(*[make_config(w["cfg"]) for w in instances])
        self._cfgs = cfgs
        h = C.c_void_p()
        st = L.mm_batch_create(cfgs, self.n, C.c_void_p(stream or 0), C.byref(h))
        if st != MM_OK:
            raise MMError(st, L.mm_batch_last_error(None).decode())
        self._h = h
        self.nx = [int(w["cfg"]["nx"]) for w in instances]
        self.M = int(instances[0]["cfg"]["n_mat"])
        self.off = np.concatenate([[0], np.cumsum(self.nx)]).astype(np.int64)

    def _check(self, st):
        if st != MM_OK:
            raise MMError(st, load().mm_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            load().mm_batch_destroy(self._h)
            self._h = None

    __del__ = close

    def init(self, instances):
        phi = np.concatenate([np.asarray(w["phi"], np.float64).ravel() for w in instances])
        chi = np.concatenate([np.asarray(w["chi"], np.int32).ravel() for w in instances])
        W = np.concatenate([np.asarray(w["W"], np.float64).ravel() for w in instances])
        self._check(load().mm_batch_init_state(self._h, phi.ctypes.data, chi.ctypes.data,
                                               W.ctypes.data, MM_HOST))

    def step(self, n=1):
        self._check(load().mm_batch_step(self._h, int(n)))

    def set_threads(self, t):
        self._check(load().mm_batch_set_threads(self._h, int(t)))

    def threads(self):
        t = C.c_int32()
        ms = (C.c_float * 5)()
        self._check(load().mm_batch_get_threads(self._h, C.byref(t), ms))
        return t.value, list(ms)

    def get(self):
        """List of per-instance dicts (Q [M][3][1][nx], alpha, phi, chi)."""
        N = int(self.off[-1])
        Q = np.zeros(self.M * 3 * N)
        al = np.zeros(self.M * N)
        phi = np.zeros(N)
        chi = np.zeros(N, np.int32)
        self._check(load().mm_batch_get_conserved(self._h, Q.ctypes.data, al.ctypes.data,
                                                  phi.ctypes.data, chi.ctypes.data, MM_HOST))
        out = []
        for q, nx in enumerate(self.nx):
            o = int(self.off[q])
            out.append(dict(
                Q=Q[self.M * 3 * o:self.M * 3 * (o + nx)].reshape(self.M, 3, 1, nx),
                alpha=al[self.M * o:self.M * (o + nx)].reshape(self.M, 1, nx),
                phi=phi[o:o + nx].reshape(1, nx), chi=chi[o:o + nx].reshape(1, nx)))
        return out

    def diag(self):
        arr = (MMDiag * self.n)()
        self._check(load().mm_batch_get_diagnostics(self._h, arr))
        return [_diag_dict(d, self.M) for d in arr]


def batch_run_noalloc(cfgs, phi, chi, W, n_steps, threads, Q, alpha=None, phi_out=None,
                      chi_out=None, stream=None):
    """mm_batch_run_noalloc: initialise and advance 1D instances with no
    device allocation.  ``cfgs``: list of config dicts; phi, chi, W and the
    outputs are torch tensors on the current GPU in mm_batch_init_state /
    mm_batch_get_conserved's packed layouts (float64, int32 for chi)."""
    L = load()
    n = len(cfgs)
    arr = (MMConfig * n)(*[make_config(c) for c in cfgs])
    ncell = sum(int(c["nx"]) for c in cfgs)
    M = int(cfgs[0]["n_mat"])

    def dev(a, dtype, numel, name):
        return None if a is None else _device_arg(a, dtype, numel, name)

    args = (dev(phi, "torch.float64", ncell, "phi"), dev(chi, "torch.int32", ncell, "chi"),
            dev(W, "torch.float64", M * 3 * ncell, "W"))
    outs = (dev(Q, "torch.float64", M * 3 * ncell, "Q"),
            dev(alpha, "torch.float64", M * ncell, "alpha"),
            dev(phi_out, "torch.float64", ncell, "phi_out"),
            dev(chi_out, "torch.int32", ncell, "chi_out"))
    st = L.mm_batch_run_noalloc(arr, n, C.c_void_p(stream or 0), *args, int(n_steps),
                                int(threads), *outs)
    if st != MM_OK:
        raise MMError(st, L.mm_last_error(None).decode())
