"""ctypes binding of liblbpc.so (include/lbpc.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch supplies the device workspace and the HIP stream.
The module-level functions carry the C names; :class:`Simulation` bundles one
handle with its workspace.  Loading fails loudly when the library is absent.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbpc.so")

OK, ERR_ARG, ERR_HIP, ERR_OOM, ERR_STATE, ERR_NUMERIC, ERR_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)
FP64, FP32, FP32_SHIFTED, FP16_SHIFTED, FP16_LOCAL = 0, 1, 2, 3, 4

# every entry point declared in include/lbpc.h
EXPORTS = (
    "lbpc_workspace_bytes", "lbpc_create", "lbpc_init_fields", "lbpc_step",
    "lbpc_get_rho_u_T", "lbpc_get_diag", "lbpc_get_diag_noalloc",
    "lbpc_step_diag", "lbpc_state_bytes",
    "lbpc_save_state", "lbpc_load_state", "lbpc_destroy", "lbpc_last_error",
    "lbpc_set_tiles", "lbpc_get_tiles", "lbpc_autotune", "lbpc_memory_probe",
    "lbpc_steps_per_launch",
    "lbpc_batch_workspace_bytes", "lbpc_batch_create",
    "lbpc_batch_init_fields", "lbpc_batch_set_tiles", "lbpc_batch_autotune",
    "lbpc_batch_step", "lbpc_batch_step_diag", "lbpc_batch_get_rho_u_T",
    "lbpc_batch_get_diag",
    "lbpc_batch_nodes", "lbpc_batch_destroy", "lbpc_batch_last_error",
)


class Config(ctypes.Structure):
    """Mirror of ``lbpc_config``."""
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
    """Mirror of ``lbpc_diag``."""
    _fields_ = [
        ("mass", ctypes.c_double), ("sum_T", ctypes.c_double),
        ("sum_rhocvT", ctypes.c_double), ("liquid_area", ctypes.c_double),
        ("radius", ctypes.c_double), ("radius_count", ctypes.c_double),
        ("max_speed", ctypes.c_double), ("sum_S0", ctypes.c_double),
        ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


class LbpcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbpc status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1709_04400_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.lbpc_workspace_bytes.argtypes = [ctypes.POINTER(Config),
                                           ctypes.POINTER(ctypes.c_size_t)]
        L.lbpc_create.argtypes = [ctypes.POINTER(Config), vp, ctypes.c_size_t,
                                  vp, ctypes.POINTER(vp)]
        L.lbpc_init_fields.argtypes = [vp, dp, dp, dp, dp]
        L.lbpc_step.argtypes = [vp, ctypes.c_int64]
        L.lbpc_get_rho_u_T.argtypes = [vp, dp, dp, dp, dp]
        L.lbpc_get_diag.argtypes = [vp, ctypes.POINTER(Diag)]
        L.lbpc_step_diag.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(Diag)]
        L.lbpc_get_diag_noalloc.argtypes = [vp, ctypes.POINTER(Diag)]
        L.lbpc_state_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.lbpc_save_state.argtypes = [vp, vp, ctypes.c_size_t]
        L.lbpc_load_state.argtypes = [vp, vp, ctypes.c_size_t]
        L.lbpc_destroy.argtypes = [vp]
        L.lbpc_destroy.restype = None
        L.lbpc_last_error.argtypes = [vp]
        L.lbpc_last_error.restype = ctypes.c_char_p
        i32, i64p = ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
        L.lbpc_set_tiles.argtypes = [vp, i32, i32]
        L.lbpc_get_tiles.argtypes = [vp, ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.lbpc_autotune.argtypes = [vp, i32, ctypes.POINTER(i32),
                                    ctypes.POINTER(i32), dp]
        L.lbpc_memory_probe.argtypes = [vp, i32, dp]
        L.lbpc_steps_per_launch.argtypes = [vp, ctypes.POINTER(i32)]
        L.lbpc_batch_workspace_bytes.argtypes = [
            ctypes.POINTER(Config), i32, ctypes.POINTER(ctypes.c_size_t)]
        L.lbpc_batch_create.argtypes = [ctypes.POINTER(Config), i32, vp,
                                        ctypes.c_size_t, vp,
                                        ctypes.POINTER(vp)]
        L.lbpc_batch_init_fields.argtypes = [vp, i32, dp, dp, dp, dp]
        L.lbpc_batch_set_tiles.argtypes = [vp, i32, i32]
        L.lbpc_batch_autotune.argtypes = [vp, i32, ctypes.POINTER(i32),
                                          ctypes.POINTER(i32), dp]
        L.lbpc_batch_step.argtypes = [vp, ctypes.c_int64]
        L.lbpc_batch_step_diag.argtypes = [vp, ctypes.c_int64,
                                           ctypes.POINTER(Diag)]
        L.lbpc_batch_get_rho_u_T.argtypes = [vp, i32, dp, dp, dp, dp]
        L.lbpc_batch_get_diag.argtypes = [vp, i32, ctypes.POINTER(Diag)]
        L.lbpc_batch_nodes.argtypes = [vp, i64p]
        L.lbpc_batch_destroy.argtypes = [vp]
        L.lbpc_batch_destroy.restype = None
        L.lbpc_batch_last_error.argtypes = [vp]
        L.lbpc_batch_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("lbpc_destroy", "lbpc_last_error",
                            "lbpc_batch_destroy", "lbpc_batch_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


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


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(st, h=None):
    if st != OK:
        msg = lib().lbpc_last_error(h)
        raise LbpcError(st, msg.decode() if msg else "")


# ------------------------------------------------ the C entry points ---

def lbpc_workspace_bytes(cfg: dict) -> int:
    c = make_config(cfg)
    out = ctypes.c_size_t()
    _check(lib().lbpc_workspace_bytes(ctypes.byref(c), ctypes.byref(out)))
    return out.value


def lbpc_create(cfg: dict, workspace_ptr: int, workspace_bytes: int,
                stream_ptr: int):
    c = make_config(cfg)
    h = ctypes.c_void_p()
    _check(lib().lbpc_create(ctypes.byref(c), ctypes.c_void_p(workspace_ptr),
                             workspace_bytes, ctypes.c_void_p(stream_ptr),
                             ctypes.byref(h)))
    return h


def lbpc_init_fields(h, rho, ux, uy, T):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy, T)]
    _check(lib().lbpc_init_fields(h, *map(_dp, arrs)), h)


def lbpc_step(h, n: int):
    _check(lib().lbpc_step(h, int(n)), h)


def lbpc_get_rho_u_T(h, shape):
    out = [np.empty(shape, dtype=np.float64) for _ in range(4)]
    _check(lib().lbpc_get_rho_u_T(h, *map(_dp, out)), h)
    return tuple(out)


def _diag_dict(d) -> dict:
    return {n: getattr(d, n) for n, _ in Diag._fields_ if n != "pad"}


def lbpc_get_diag(h) -> dict:
    d = Diag()
    _check(lib().lbpc_get_diag(h, ctypes.byref(d)), h)
    return _diag_dict(d)


def lbpc_get_diag_noalloc(h) -> dict:
    d = Diag()
    _check(lib().lbpc_get_diag_noalloc(h, ctypes.byref(d)), h)
    return _diag_dict(d)


def lbpc_step_diag(h, n: int) -> dict:
    d = Diag()
    _check(lib().lbpc_step_diag(h, int(n), ctypes.byref(d)), h)
    return _diag_dict(d)


def lbpc_save_state(h) -> np.ndarray:
    nb = ctypes.c_size_t()
    _check(lib().lbpc_state_bytes(h, ctypes.byref(nb)), h)
    buf = np.empty(nb.value, dtype=np.uint8)
    _check(lib().lbpc_save_state(h, buf.ctypes.data_as(ctypes.c_void_p),
                                 nb.value), h)
    return buf


def lbpc_load_state(h, buf: np.ndarray):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(lib().lbpc_load_state(h, buf.ctypes.data_as(ctypes.c_void_p),
                                 buf.nbytes), h)


def lbpc_get_tiles(h) -> dict:
    bw, rows, re = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lbpc_get_tiles(h, ctypes.byref(bw), ctypes.byref(rows),
                                ctypes.byref(re)), h)
    return {"block_width": bw.value, "rows": rows.value,
            "rows_edge": re.value}


def lbpc_destroy(h):
    lib().lbpc_destroy(h)


# ------------------------------------------------------------- wrapper ---

def _log_records(log, records):
    """Appends records as JSON lines to `log` (a path or a text file)."""
    if log is None:
        return
    if isinstance(log, (str, os.PathLike)):
        with open(log, "a") as fh:
            for r in records:
                fh.write(json.dumps(r) + "\n")
    else:
        for r in records:
            log.write(json.dumps(r) + "\n")
        log.flush()


class Simulation:
    """One lattice on one GPU: workspace from torch, library handle.

    Uses its own (default-priority) torch stream unless one is given (a
    capturable stream, for the optional hipGraph replay of steady steps)."""

    def __init__(self, cfg: dict, device: str = "cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lbpc library needs one")
        self.cfg = dict(cfg)
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        self.device = torch.device(device)
        nbytes = lbpc_workspace_bytes(cfg)
        with self._on():
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8,
                                  device=self.device)
            ptr = self.ws.data_ptr()
            ptr = (ptr + 255) // 256 * 256
            self.stream = stream if stream is not None else \
                torch.cuda.Stream(self.device)
            self.h = lbpc_create(cfg, ptr, nbytes, self.stream.cuda_stream)

    def _on(self):
        """Every library call on the handle runs with its device current."""
        import torch
        return torch.cuda.device(self.device)

    def init_fields(self, rho, ux, uy, T):
        with self._on():
            lbpc_init_fields(self.h, rho, ux, uy, T)

    def step(self, n: int = 1):
        with self._on():
            lbpc_step(self.h, n)

    def rho_u_T(self):
        with self._on():
            return lbpc_get_rho_u_T(self.h, (self.ny, self.nx))

    def set_tiles(self, block_width, rows):
        _check(lib().lbpc_set_tiles(self.h, int(block_width), int(rows)),
               self.h)

    def tiles(self) -> dict:
        return lbpc_get_tiles(self.h)

    def steps_per_launch(self) -> int:
        v = ctypes.c_int32()
        _check(lib().lbpc_steps_per_launch(self.h, ctypes.byref(v)), self.h)
        return v.value

    def autotune(self, steps=3):
        bw, rows = ctypes.c_int32(), ctypes.c_int32()
        ms = ctypes.c_double()
        with self._on():
            _check(lib().lbpc_autotune(self.h, int(steps), ctypes.byref(bw),
                                       ctypes.byref(rows), ctypes.byref(ms)),
                   self.h)
        return {"block_width": bw.value, "rows": rows.value,
                "ms_per_step": ms.value}

    def memory_probe(self, launches=20) -> float:
        """lbpc_memory_probe: ms per launch of the step's memory schedule
        without its arithmetic (state unchanged)."""
        ms = ctypes.c_double()
        with self._on():
            _check(lib().lbpc_memory_probe(self.h, int(launches),
                                           ctypes.byref(ms)), self.h)
        return ms.value

    def diag(self) -> dict:
        with self._on():
            return lbpc_get_diag(self.h)

    def diag_noalloc(self) -> dict:
        """lbpc_get_diag_noalloc: the same values, with the library's static
        scratch instead of the workspace."""
        with self._on():
            return lbpc_get_diag_noalloc(self.h)

    def step_diag(self, n: int = 1) -> dict:
        """n steps; the diagnostics of the level they start from, reduced
        inside the first of them."""
        with self._on():
            return lbpc_step_diag(self.h, n)

    def run(self, steps: int, every: int, log=None) -> list:
        """Advances `steps` steps, taking the FP64 diagnostics after every
        `every` steps (and after the last); returns the records and appends
        each as one JSON line to `log` (a path or text file) if given.  The
        records of the levels a later step starts from are reduced inside
        that step; the last level's by a no-store pass."""
        out = []
        done = min(every, steps)
        self.step(done)
        while done < steps:
            k = min(every, steps - done)
            out.append(self.step_diag(k))
            done += k
        out.append(self.diag())
        _log_records(log, out)
        return out

    def save_state(self) -> np.ndarray:
        with self._on():
            return lbpc_save_state(self.h)

    def load_state(self, buf):
        with self._on():
            lbpc_load_state(self.h, buf)

    def close(self):
        if getattr(self, "h", None):
            with self._on():
                lbpc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- batches ---

def _bcheck(st, b=None):
    if st != OK:
        msg = lib().lbpc_batch_last_error(b)
        raise LbpcError(st, msg.decode() if msg else "")


def _config_array(cfgs):
    arr = (Config * len(cfgs))()
    for i, d in enumerate(cfgs):
        arr[i] = make_config(d)
    return arr


def lbpc_batch_workspace_bytes(cfgs) -> int:
    arr = _config_array(cfgs)
    out = ctypes.c_size_t()
    _bcheck(lib().lbpc_batch_workspace_bytes(arr, len(cfgs),
                                             ctypes.byref(out)))
    return out.value


class Batch:
    """Many independent lattices stepped by one persistent launch per step.

    Uses its own (default-priority) torch stream (a capturable stream, for
    the optional hipGraph replay of steady steps)."""

    def __init__(self, cfgs, device: str = "cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lbpc library needs one")
        self.cfgs = [dict(c) for c in cfgs]
        self.device = torch.device(device)
        arr = _config_array(self.cfgs)
        nbytes = lbpc_batch_workspace_bytes(self.cfgs)
        h = ctypes.c_void_p()
        with self._on():
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8,
                                  device=self.device)
            ptr = (self.ws.data_ptr() + 255) // 256 * 256
            self.stream = stream if stream is not None else \
                torch.cuda.Stream(self.device)
            _bcheck(lib().lbpc_batch_create(arr, len(self.cfgs),
                                            ctypes.c_void_p(ptr), nbytes,
                                            ctypes.c_void_p(
                                                self.stream.cuda_stream),
                                            ctypes.byref(h)))
        self.h = h

    def _on(self):
        """Every library call on the batch runs with its device current."""
        import torch
        return torch.cuda.device(self.device)

    def __len__(self):
        return len(self.cfgs)

    def init_fields(self, c, rho, ux, uy, T):
        arrs = [np.ascontiguousarray(a, dtype=np.float64)
                for a in (rho, ux, uy, T)]
        with self._on():
            _bcheck(lib().lbpc_batch_init_fields(self.h, int(c),
                                                 *map(_dp, arrs)), self.h)

    def set_tiles(self, block_width, rows):
        _bcheck(lib().lbpc_batch_set_tiles(self.h, int(block_width),
                                           int(rows)), self.h)

    def autotune(self, steps=3):
        bw, rows = ctypes.c_int32(), ctypes.c_int32()
        ms = ctypes.c_double()
        with self._on():
            _bcheck(lib().lbpc_batch_autotune(self.h, int(steps),
                                              ctypes.byref(bw),
                                              ctypes.byref(rows),
                                              ctypes.byref(ms)), self.h)
        return {"block_width": bw.value, "rows": rows.value,
                "ms_per_step": ms.value}

    def step(self, n=1):
        with self._on():
            _bcheck(lib().lbpc_batch_step(self.h, int(n)), self.h)

    def rho_u_T(self, c):
        cfg = self.cfgs[c]
        out = [np.empty((cfg["ny"], cfg["nx"])) for _ in range(4)]
        with self._on():
            _bcheck(lib().lbpc_batch_get_rho_u_T(self.h, int(c),
                                                 *map(_dp, out)), self.h)
        return tuple(out)

    def diag(self, c) -> dict:
        d = Diag()
        with self._on():
            _bcheck(lib().lbpc_batch_get_diag(self.h, int(c),
                                              ctypes.byref(d)), self.h)
        return _diag_dict(d)

    def step_diag(self, n: int = 1) -> list:
        """n steps of every lattice; each lattice's diagnostics of the level
        they start from, reduced inside the first of them."""
        arr = (Diag * len(self.cfgs))()
        with self._on():
            _bcheck(lib().lbpc_batch_step_diag(self.h, int(n), arr), self.h)
        return [_diag_dict(d) for d in arr]

    def run(self, steps: int, every: int, log=None) -> list:
        """Advances every lattice `steps` steps, taking each lattice's FP64
        diagnostics after every `every` steps (and after the last); returns
        the records (each with its lattice index) and appends them as JSON
        lines to `log` if given."""
        out = []
        done = min(every, steps)
        self.step(done)
        while done < steps:
            k = min(every, steps - done)
            out += [dict(d, lattice=c)
                    for c, d in enumerate(self.step_diag(k))]
            done += k
        out += [dict(self.diag(c), lattice=c) for c in range(len(self.cfgs))]
        _log_records(log, out)
        return out

    def nodes(self) -> int:
        v = ctypes.c_int64()
        _bcheck(lib().lbpc_batch_nodes(self.h, ctypes.byref(v)), self.h)
        return v.value

    def close(self):
        if getattr(self, "h", None):
            with self._on():
                lib().lbpc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
