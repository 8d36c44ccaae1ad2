"""Python binding of libjfnk (include/jfnk.h): argument marshalling only.

Every step of the solve runs in the HIP library; this module converts torch
device tensors and numpy host arrays into the C structs of the ABI.  It
raises if the built library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; JFNK_LIB names another build of the same sources
LIB_PATH = os.environ.get("JFNK_LIB", os.path.join(HERE, "libjfnk.so"))

JFNK_OK, JFNK_NOT_CONVERGED = 0, 1
JFNK_EINVAL, JFNK_ENOMEM, JFNK_EHIP, JFNK_ECAPACITY, JFNK_EMODEL = -1, -2, -3, -4, -5
BC_DIRICHLET, BC_ZERO_FLUX = 0, 1
GUESS_PREV, GUESS_EXTRAP, GUESS_LEARNED = 0, 1, 2
PREC_FP64, PREC_FP32 = 0, 1
PRECK_BLOCK, PRECK_SCHUR, PRECK_NONE, PRECK_SCHUR_MG = 0, 1, 2, 3
SCHED_PLAIN, SCHED_BATCHED = 0, 1
COL_CONVERGED, COL_MAX_NEWTON, COL_NONFINITE, COL_LINESEARCH, COL_BAD_INPUT = 0, 1, 2, 3, 4

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class jfnk_config(C.Structure):
    _fields_ = [("max_cols", C.c_int32), ("max_total_cells", C.c_int64),
                ("max_cells_per_col", C.c_int32), ("gmres_restart", C.c_int32),
                ("max_restarts", C.c_int32), ("max_newton", C.c_int32),
                ("max_backtracks", C.c_int32), ("tol_f", C.c_double), ("tol_x", C.c_double),
                ("gamma", C.c_double), ("ls_theta", C.c_double), ("chord_tol", C.c_double),
                ("prec_precision", C.c_int32), ("guess", C.c_int32), ("schedule", C.c_int32),
                ("threads_override", C.c_int32), ("prec_kind", C.c_int32), ("mg_tol", C.c_double),
                ("mg_blocks", C.c_int32), ("mg_transfer", C.c_int32)]


class jfnk_table(C.Structure):
    _fields_ = [("nc", C.c_int32), ("nx", C.c_int32), ("c_min", C.c_double), ("c_max", C.c_double),
                ("x_min", C.c_double), ("x_max", C.c_double), ("mu", C.c_void_p), ("diff", C.c_void_p)]


class jfnk_problem(C.Structure):
    _fields_ = [("ncols", C.c_int32), ("col_offset", _lp), ("length", _dp), ("dt", _dp),
                ("phi_left", _dp), ("phi_right", _dp), ("eps_over_e", _dp),
                ("bc_left", _ip), ("bc_right", _ip), ("ne_left", _dp), ("ne_right", _dp),
                ("mu", C.c_void_p), ("diff", C.c_void_p), ("src", C.c_void_p),
                ("k_loss", C.c_void_p), ("q_ion", C.c_void_p), ("u_face", C.c_void_p),
                ("temp", C.c_void_p), ("table", C.POINTER(jfnk_table)), ("prog", C.c_void_p),
                ("gas_n", C.c_void_p)]


class jfnk_misdc(C.Structure):
    _fields_ = [("k_max", C.c_int32), ("electron_sdc", C.c_int32), ("cfl", C.c_double), ("t", _dp),
                ("ac_amp", _dp), ("ac_freq", _dp), ("mu_ion", C.c_void_p), ("k_rec", C.c_void_p),
                ("n_ion", C.c_void_p), ("dt_used", _dp)]


class jfnk_state(C.Structure):
    _fields_ = [("ne", C.c_void_p), ("phi", C.c_void_p), ("ne_prev", C.c_void_p),
                ("phi_prev", C.c_void_p), ("ne_out", C.c_void_p), ("phi_out", C.c_void_p)]


class jfnk_net_config(C.Structure):
    _fields_ = [("max_cols", C.c_int32), ("max_total_cells", C.c_int64),
                ("out_scale_ne", C.c_float), ("out_scale_phi", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("adam_eps", C.c_float)]


class jfnk_stats(C.Structure):
    _fields_ = [("status", _ip), ("newton_iters", _ip), ("gmres_iters", _ip),
                ("backtracks", _ip), ("guess_used", _ip), ("res_scaled", _dp), ("chord_steps", _ip),
                ("phase_counts", _ip), ("mg_cycles", _ip)]


_LIB = None


def lib():
    """The loaded libjfnk.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libjfnk.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.jfnk_config_default.argtypes = [C.POINTER(jfnk_config)]
        L.jfnk_config_default.restype = None
        L.jfnk_create.argtypes = [C.POINTER(jfnk_config), C.POINTER(C.c_void_p)]
        L.jfnk_create.restype = C.c_int
        L.jfnk_step.argtypes = [C.c_void_p, C.POINTER(jfnk_problem), C.POINTER(jfnk_state),
                                C.POINTER(jfnk_stats), C.c_void_p]
        L.jfnk_step.restype = C.c_int
        L.jfnk_step_async.argtypes = [C.c_void_p, C.POINTER(jfnk_problem), C.POINTER(jfnk_state),
                                      C.POINTER(jfnk_stats), C.POINTER(C.c_int32), C.c_void_p]
        L.jfnk_step_async.restype = C.c_int
        L.jfnk_step_finish.argtypes = [C.c_void_p, C.POINTER(jfnk_stats)]
        L.jfnk_step_finish.restype = C.c_int
        L.jfnk_destroy.argtypes = [C.c_void_p]
        L.jfnk_destroy.restype = None
        L.jfnk_last_error.argtypes = [C.c_void_p]
        L.jfnk_last_error.restype = C.c_char_p
        L.jfnk_last_timing.argtypes = [C.c_void_p, _dp, _ip]
        L.jfnk_last_timing.restype = C.c_int
        L.jfnk_last_kernel_times.argtypes = [C.c_void_p, _dp]
        L.jfnk_last_kernel_times.restype = C.c_int
        L.jfnk_eval_residual.argtypes = [C.c_void_p, C.POINTER(jfnk_problem), C.POINTER(jfnk_state),
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, _dp, C.c_void_p]
        L.jfnk_eval_residual.restype = C.c_int
        L.jfnk_eval_jv.argtypes = [C.c_void_p, C.POINTER(jfnk_problem), C.POINTER(jfnk_state),
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p]
        L.jfnk_eval_jv.restype = C.c_int
        L.jfnk_block_solve.argtypes = [C.c_void_p, C.POINTER(jfnk_problem), C.POINTER(jfnk_state),
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p]
        L.jfnk_block_solve.restype = C.c_int
        _fp = C.POINTER(C.c_float)
        P, S = C.POINTER(jfnk_problem), C.POINTER(jfnk_state)
        L.jfnk_net_config_default.argtypes = [C.POINTER(jfnk_net_config)]
        L.jfnk_net_config_default.restype = None
        L.jfnk_net_param_count.argtypes = []
        L.jfnk_net_param_count.restype = C.c_int64
        L.jfnk_net_create.argtypes = [C.POINTER(jfnk_net_config), C.POINTER(C.c_void_p)]
        L.jfnk_net_create.restype = C.c_int
        L.jfnk_net_destroy.argtypes = [C.c_void_p]
        L.jfnk_net_destroy.restype = None
        L.jfnk_net_last_error.argtypes = [C.c_void_p]
        L.jfnk_net_last_error.restype = C.c_char_p
        L.jfnk_net_set_params.argtypes = [C.c_void_p, _fp, C.c_int64]
        L.jfnk_net_set_params.restype = C.c_int
        L.jfnk_net_get_params.argtypes = [C.c_void_p, _fp, C.c_int64]
        L.jfnk_net_get_params.restype = C.c_int
        L.jfnk_net_predict.argtypes = [C.c_void_p, P, S, C.c_void_p, C.c_void_p, C.c_void_p]
        L.jfnk_net_predict.restype = C.c_int
        L.jfnk_net_grad.argtypes = [C.c_void_p, P, S, C.c_void_p, C.c_void_p, _fp, _dp, C.c_void_p]
        L.jfnk_net_grad.restype = C.c_int
        L.jfnk_net_train_step.argtypes = [C.c_void_p, P, S, C.c_void_p, C.c_void_p, C.c_float, _dp,
                                          C.c_void_p]
        L.jfnk_net_train_step.restype = C.c_int
        L.jfnk_autotune.argtypes = [C.c_void_p, C.POINTER(jfnk_problem), C.POINTER(jfnk_state), C.c_int32,
                                    _ip, _dp, C.c_void_p]
        L.jfnk_autotune.restype = C.c_int
        L.jfnk_autotune_save.argtypes = [C.c_void_p, C.c_char_p]
        L.jfnk_autotune_save.restype = C.c_int
        L.jfnk_autotune_load.argtypes = [C.c_void_p, C.c_char_p, _ip]
        L.jfnk_autotune_load.restype = C.c_int
        L.jfnk_schedule_threads.argtypes = [C.c_void_p, C.POINTER(jfnk_problem), _ip]
        L.jfnk_schedule_threads.restype = C.c_int
        L.jfnk_set_model.argtypes = [C.c_void_p, C.c_void_p]
        L.jfnk_set_model.restype = C.c_int
        L.jfnk_step_noalloc.argtypes = [C.POINTER(jfnk_config), C.POINTER(jfnk_problem), C.POINTER(jfnk_state),
                                        C.POINTER(jfnk_stats), C.c_void_p, C.c_char_p, C.c_size_t]
        L.jfnk_step_noalloc.restype = C.c_int
        L.jfnk_misdc_step.argtypes = [C.c_void_p, C.POINTER(jfnk_problem), C.POINTER(jfnk_misdc),
                                      C.POINTER(jfnk_state), C.POINTER(jfnk_stats), C.c_void_p]
        L.jfnk_misdc_step.restype = C.c_int
        _LIB = L
    return _LIB


EXPORTED_SYMBOLS = ("jfnk_config_default", "jfnk_create", "jfnk_step", "jfnk_step_async", "jfnk_step_finish",
                    "jfnk_destroy",
                    "jfnk_last_error", "jfnk_last_timing", "jfnk_last_kernel_times", "jfnk_eval_residual", "jfnk_eval_jv",
                    "jfnk_block_solve", "jfnk_net_config_default", "jfnk_net_param_count",
                    "jfnk_net_create", "jfnk_net_destroy", "jfnk_net_last_error",
                    "jfnk_net_set_params", "jfnk_net_get_params", "jfnk_net_predict",
                    "jfnk_net_grad", "jfnk_net_train_step", "jfnk_set_model", "jfnk_autotune",
                    "jfnk_step_noalloc", "jfnk_misdc_step", "jfnk_autotune_save", "jfnk_autotune_load",
                    "jfnk_schedule_threads")

NOALLOC_BYTES = 64 << 20      # JFNK_NOALLOC_BYTES
NOALLOC_MAX_COLS = 64         # JFNK_NOALLOC_MAX_COLS


class JfnkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"jfnk error {code}: {msg}")
        self.code = code


def default_config(**kw) -> jfnk_config:
    cfg = jfnk_config()
    lib().jfnk_config_default(C.byref(cfg))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise AttributeError(k)
        setattr(cfg, k, v)
    return cfg


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return t.data_ptr()


@dataclass
class DeviceProblem:
    """Host per-column arrays + device per-cell tensors of one batch."""
    ncols: int
    col_offset: np.ndarray
    length: np.ndarray
    dt: np.ndarray
    phi_left: np.ndarray
    phi_right: np.ndarray
    eps_over_e: np.ndarray
    bc_left: np.ndarray
    bc_right: np.ndarray
    ne_left: np.ndarray
    ne_right: np.ndarray
    mu: object
    diff: object
    src: object
    kloss: object
    q: object
    temp: object
    uface: object = None
    table: object = None      # DeviceTable or None
    prog: object = None
    gas_n: object = None

    def __setattr__(self, name, value):
        # a field bound to another object invalidates the cached argument
        # struct (an in-place update, x *= 2, rebinds the same object)
        if self.__dict__.get(name, self) is not value:
            object.__setattr__(self, "_cached", None)
        object.__setattr__(self, name, value)

    def cstruct(self) -> jfnk_problem:
        """The C argument struct.  It is cached while no field is reassigned
        and every host array is already contiguous in the C type (it then
        points at the arrays themselves, so in-place updates reach the
        library); otherwise it is rebuilt from converted copies each call."""
        cached = self.__dict__.get("_cached")
        if cached is not None:
            return cached
        p = jfnk_problem()
        p.ncols = self.ncols
        keep = [np.ascontiguousarray(self.col_offset, dtype=np.int64)]
        direct = keep[0] is self.col_offset
        p.col_offset = keep[0].ctypes.data_as(_lp)
        for name in ("length", "dt", "phi_left", "phi_right", "eps_over_e", "ne_left", "ne_right"):
            a = np.ascontiguousarray(getattr(self, name), dtype=np.float64)
            direct = direct and a is getattr(self, name)
            keep.append(a)
            setattr(p, name, a.ctypes.data_as(_dp))
        for name in ("bc_left", "bc_right"):
            a = np.ascontiguousarray(getattr(self, name), dtype=np.int32)
            direct = direct and a is getattr(self, name)
            keep.append(a)
            setattr(p, name, a.ctypes.data_as(_ip))
        p.mu, p.diff, p.src = _ptr(self.mu), _ptr(self.diff), _ptr(self.src)
        p.k_loss, p.q_ion = _ptr(self.kloss), _ptr(self.q)
        p.u_face, p.temp = _ptr(self.uface), _ptr(self.temp)
        p.prog, p.gas_n = _ptr(self.prog), _ptr(self.gas_n)
        if self.table is not None:
            t = self.table.cstruct()
            keep.append(t)
            p.table = C.pointer(t)
        object.__setattr__(self, "_keep", keep)
        object.__setattr__(self, "_cached", p if direct else None)
        return p


@dataclass
class DeviceTable:
    """A transport table (workloads.TransportTable) with its arrays on the GPU."""
    c_min: float
    c_max: float
    x_min: float
    x_max: float
    mu: object
    diff: object

    def cstruct(self) -> jfnk_table:
        return jfnk_table(int(self.mu.shape[0]), int(self.mu.shape[1]), self.c_min, self.c_max, self.x_min,
                          self.x_max, _ptr(self.mu), _ptr(self.diff))


@dataclass
class DeviceIons:
    """Ion species and chemistry of a batch for the MISDC step: per-cell
    mobility, recombination coefficient and density on the GPU, per-column AC
    amplitude and frequency of the right electrode on the host."""
    mu_ion: object
    k_rec: object
    n_ion: object
    ac_amp: Optional[np.ndarray] = None
    ac_freq: Optional[np.ndarray] = None

    def cstruct(self, t, k_max: int, ncols: int, electron_sdc: bool = False, cfl: float = 0.0,
                dt_out: Optional[np.ndarray] = None) -> jfnk_misdc:
        """t: the start time of every column (a scalar) or per column;
        dt_out: float64 [ncols] receiving the step each column took."""
        m = jfnk_misdc()
        m.k_max = int(k_max)
        m.electron_sdc = 1 if electron_sdc else 0
        m.cfl = float(cfl)
        if dt_out is not None:
            assert dt_out.dtype == np.float64 and dt_out.flags.c_contiguous and dt_out.shape == (ncols,)
            m.dt_used = dt_out.ctypes.data_as(_dp)
        keep = [np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), (ncols,)))]
        m.t = keep[0].ctypes.data_as(_dp)
        for name in ("ac_amp", "ac_freq"):
            v = getattr(self, name)
            if v is not None:
                keep.append(np.ascontiguousarray(v, dtype=np.float64))
                setattr(m, name, keep[-1].ctypes.data_as(_dp))
        object.__setattr__(self, "_keep", keep)
        m.mu_ion, m.k_rec, m.n_ion = _ptr(self.mu_ion), _ptr(self.k_rec), _ptr(self.n_ion)
        return m


def device_ions(mu_ion, k_rec, n_ion, ac_amp=None, ac_freq=None, device="cuda") -> DeviceIons:
    import torch

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)

    return DeviceIons(dev(mu_ion), dev(k_rec), dev(n_ion), ac_amp, ac_freq)


def device_problem(packed, device="cuda") -> tuple:
    """(DeviceProblem, ne, phi, ne_prev, phi_prev) on the GPU from a workloads.Packed."""
    import torch

    def dev(a):
        return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)

    dp = DeviceProblem(packed.ncols, packed.col_offset, packed.length, packed.dt, packed.phi_left,
                       packed.phi_right, packed.eps_over_e, packed.bc_left, packed.bc_right,
                       packed.ne_left, packed.ne_right, dev(packed.mu), dev(packed.diff),
                       dev(packed.src), dev(packed.kloss), dev(packed.q), dev(packed.temp))
    if getattr(packed, "uface", None) is not None:
        dp.uface = dev(packed.uface)
    tab = getattr(packed, "table", None)
    if tab is not None:
        dp.table = DeviceTable(tab.c_min, tab.c_max, tab.x_min, tab.x_max, dev(tab.mu).contiguous(),
                               dev(tab.diff).contiguous())
        dp.prog, dp.gas_n = dev(packed.prog), dev(packed.gas_n)
    return dp, dev(packed.ne), dev(packed.phi), dev(packed.ne_prev), dev(packed.phi_prev)


class Stats:
    def __init__(self, n):
        self.status = np.zeros(n, np.int32)
        self.newton_iters = np.zeros(n, np.int32)
        self.gmres_iters = np.zeros(n, np.int32)
        self.backtracks = np.zeros(n, np.int32)
        self.guess_used = np.zeros(n, np.int32)
        self.res_scaled = np.zeros(n, np.float64)
        self.chord_steps = np.zeros(n, np.int32)
        self.phase_counts = np.zeros((n, 8), np.int32)
        self.mg_cycles = np.zeros(n, np.int32)

    def __setattr__(self, name, value):
        # an array bound to another object invalidates the cached argument struct
        if self.__dict__.get(name, self) is not value:
            object.__setattr__(self, "_cached", None)
        object.__setattr__(self, name, value)

    def cstruct(self) -> jfnk_stats:
        cached = self.__dict__.get("_cached")
        if cached is not None:
            return cached
        s = jfnk_stats()
        for name in ("status", "newton_iters", "gmres_iters", "backtracks", "guess_used", "chord_steps",
                     "phase_counts", "mg_cycles"):
            a = getattr(self, name)
            assert a.dtype == np.int32 and a.flags.c_contiguous
            setattr(s, name, a.ctypes.data_as(_ip))
        assert self.res_scaled.dtype == np.float64 and self.res_scaled.flags.c_contiguous
        s.res_scaled = self.res_scaled.ctypes.data_as(_dp)
        object.__setattr__(self, "_cached", s)
        return s


def _stream_ptr(stream):
    """hipStream_t of a torch stream (None: torch's current stream)."""
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


class Solver:
    """Owns one jfnk_ctx."""

    def __init__(self, config: jfnk_config):
        self.config = config
        h = C.c_void_p()
        rc = lib().jfnk_create(C.byref(config), C.byref(h))
        if rc != JFNK_OK:
            raise JfnkError(rc, "jfnk_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().jfnk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().jfnk_last_error(self.h).decode()

    def last_timing(self):
        """(solve ms, launches) of the last step, from HIP events."""
        ms = C.c_double()
        n = C.c_int32()
        self._check(lib().jfnk_last_timing(self.h, C.byref(ms), C.byref(n)), (JFNK_OK,))
        return ms.value, n.value

    def last_kernel_times(self):
        """(gather, solve, write-back) ms of the last batched step (-1 each otherwise)."""
        out = (C.c_double * 3)()
        self._check(lib().jfnk_last_kernel_times(self.h, out), (JFNK_OK,))
        return tuple(out)

    def _check(self, rc, allow=(JFNK_OK, JFNK_NOT_CONVERGED)):
        if rc not in allow:
            raise JfnkError(rc, self.last_error())
        return rc

    @staticmethod
    def _state(ne, phi, ne_prev=None, phi_prev=None, ne_out=None, phi_out=None) -> jfnk_state:
        s = jfnk_state()
        s.ne, s.phi = _ptr(ne), _ptr(phi)
        s.ne_prev, s.phi_prev = _ptr(ne_prev), _ptr(phi_prev)
        s.ne_out, s.phi_out = _ptr(ne_out), _ptr(phi_out)
        return s

    def step(self, prob: DeviceProblem, ne, phi, ne_prev=None, phi_prev=None, stream=None,
             stats: Optional[Stats] = None, raw: bool = False, ne_out=None, phi_out=None):
        """One backward-Euler step of all columns: in place on ne/phi, or into
        ne_out/phi_out (which may be ne_prev/phi_prev) when given."""
        p = prob.cstruct()
        s = self._state(ne, phi, ne_prev, phi_prev, ne_out, phi_out)
        st = stats if stats is not None else Stats(prob.ncols)
        rc = lib().jfnk_step(self.h, C.byref(p), C.byref(s), C.byref(st.cstruct()), _stream_ptr(stream))
        if raw:
            return rc, st
        self._check(rc)
        return rc, st

    def misdc_step(self, prob: DeviceProblem, ions: "DeviceIons", t, k_max: int, ne, phi, ne_prev=None,
                   phi_prev=None, stream=None, stats: Optional[Stats] = None, raw: bool = False, ne_out=None,
                   phi_out=None, electron_sdc: bool = False, cfl: float = 0.0, dt_out=None):
        """One MISDC step t -> t + dt of all columns (jfnk_misdc_step): X in
        place on ne/phi (or into ne_out/phi_out), the ions in place on
        ions.n_ion.  The problem's kloss must be None; its q is not read.
        cfl > 0: the step at that ion-drift CFL number (capped by the
        problem's dt), reported in dt_out when given."""
        p = prob.cstruct()
        m = ions.cstruct(t, k_max, prob.ncols, electron_sdc, cfl, dt_out)
        s = self._state(ne, phi, ne_prev, phi_prev, ne_out, phi_out)
        st = stats if stats is not None else Stats(prob.ncols)
        rc = lib().jfnk_misdc_step(self.h, C.byref(p), C.byref(m), C.byref(s), C.byref(st.cstruct()),
                                   _stream_ptr(stream))
        if raw:
            return rc, st
        self._check(rc)
        return rc, st

    def step_async(self, prob: DeviceProblem, ne, phi, ne_prev=None, phi_prev=None, stream=None,
                   prev_stats: Optional[Stats] = None, ne_out=None, phi_out=None):
        """Queue one step and return; if a step was in flight, wait for it and
        return (its return code, its stats), else (None, None).  The tensors of
        the queued step must stay alive until it is reported."""
        p = prob.cstruct()
        s = self._state(ne, phi, ne_prev, phi_prev, ne_out, phi_out)
        st = prev_stats if prev_stats is not None else Stats(prob.ncols)
        prc = C.c_int32(-1)
        # the tensors of the queued step stay referenced until it is reported
        self._inflight = (p, s, ne, phi, ne_prev, phi_prev, ne_out, phi_out)
        rc = lib().jfnk_step_async(self.h, C.byref(p), C.byref(s), C.byref(st.cstruct()), C.byref(prc),
                                   _stream_ptr(stream))
        self._check(rc)
        if prc.value < 0:
            return None, None
        return prc.value, st

    def step_finish(self, stats: Optional[Stats] = None, ncols: Optional[int] = None):
        """Wait for the step in flight; (its return code, its stats)."""
        st = stats if stats is not None else Stats(ncols)
        rc = lib().jfnk_step_finish(self.h, C.byref(st.cstruct()))
        self._check(rc)
        self._inflight = None
        return rc, st

    def autotune(self, prob: DeviceProblem, ne, phi, ne_prev=None, phi_prev=None, steps: int = 3,
                 stream=None):
        """Pick the workgroup size per column for this layout by timing
        `steps` steps per candidate; returns (chosen, {T: ms})."""
        p = prob.cstruct()
        s = self._state(ne, phi, ne_prev, phi_prev)
        ch = C.c_int32()
        t = np.zeros(4)
        self._check(lib().jfnk_autotune(self.h, C.byref(p), C.byref(s), int(steps), C.byref(ch),
                                        t.ctypes.data_as(_dp), _stream_ptr(stream)), (JFNK_OK,))
        return ch.value, {T: float(v) for T, v in zip((64, 128, 256, 512), t) if v >= 0}

    def autotune_save(self, path: str):
        """Append this context's tuned layouts to the text file at path."""
        self._check(lib().jfnk_autotune_save(self.h, os.fsencode(path)), (JFNK_OK,))

    def autotune_load(self, path: str) -> int:
        """Read tuned layouts from path (those of this device, precision and
        preconditioner kind); returns how many were kept."""
        n = C.c_int32()
        self._check(lib().jfnk_autotune_load(self.h, os.fsencode(path), C.byref(n)), (JFNK_OK,))
        return n.value

    def schedule_threads(self, prob: DeviceProblem) -> int:
        """Workgroup size per column the next step takes for prob's layout."""
        p = prob.cstruct()
        t = C.c_int32()
        self._check(lib().jfnk_schedule_threads(self.h, C.byref(p), C.byref(t)), (JFNK_OK,))
        return t.value

    def set_model(self, net: Optional["Net"]):
        """Attach a learned-guess network (None detaches)."""
        self._model = net
        self._check(lib().jfnk_set_model(self.h, net.h if net is not None else None), (JFNK_OK,))

    def eval_residual(self, prob: DeviceProblem, ne_old, phi_old, x_ne, x_phi, stream=None):
        import torch
        fe = torch.empty_like(x_ne)
        fp = torch.empty_like(x_phi)
        scal = np.zeros(4 * prob.ncols)
        p = prob.cstruct()
        s = self._state(ne_old, phi_old)
        rc = lib().jfnk_eval_residual(self.h, C.byref(p), C.byref(s), _ptr(x_ne), _ptr(x_phi),
                                      _ptr(fe), _ptr(fp), scal.ctypes.data_as(_dp), _stream_ptr(stream))
        self._check(rc, (JFNK_OK,))
        return fe, fp, scal.reshape(-1, 4)

    def eval_jv(self, prob, ne_old, phi_old, x_ne, x_phi, v_ne, v_phi, stream=None):
        import torch
        w_ne = torch.empty_like(x_ne)
        w_phi = torch.empty_like(x_phi)
        p = prob.cstruct()
        s = self._state(ne_old, phi_old)
        rc = lib().jfnk_eval_jv(self.h, C.byref(p), C.byref(s), _ptr(x_ne), _ptr(x_phi), _ptr(v_ne),
                                _ptr(v_phi), _ptr(w_ne), _ptr(w_phi), _stream_ptr(stream))
        self._check(rc, (JFNK_OK,))
        return w_ne, w_phi

    def block_solve(self, prob, ne_old, phi_old, x_ne, x_phi, r_ne, r_phi, stream=None):
        import torch
        z_ne = torch.empty_like(x_ne)
        z_phi = torch.empty_like(x_phi)
        p = prob.cstruct()
        s = self._state(ne_old, phi_old)
        rc = lib().jfnk_block_solve(self.h, C.byref(p), C.byref(s), _ptr(x_ne), _ptr(x_phi),
                                    _ptr(r_ne), _ptr(r_phi), _ptr(z_ne), _ptr(z_phi),
                                    _stream_ptr(stream))
        self._check(rc, (JFNK_OK,))
        return z_ne, z_phi


def step_noalloc(config: jfnk_config, prob: DeviceProblem, ne, phi, ne_prev=None, phi_prev=None, stream=None,
                 stats: Optional[Stats] = None, ne_out=None, phi_out=None):
    """One batched step without a context (jfnk_step_noalloc: the workspace
    is the library's static device array).  Returns (rc, stats, message)."""
    p = prob.cstruct()
    s = Solver._state(ne, phi, ne_prev, phi_prev, ne_out, phi_out)
    st = stats if stats is not None else Stats(prob.ncols)
    msg = C.create_string_buffer(256)
    rc = lib().jfnk_step_noalloc(C.byref(config), C.byref(p), C.byref(s), C.byref(st.cstruct()),
                                 _stream_ptr(stream), msg, len(msg))
    return rc, st, msg.value.decode()


def config_for(packed, **kw) -> jfnk_config:
    """Config with capacity sized for a packed batch."""
    ns = np.diff(packed.col_offset)
    base = dict(max_cols=int(packed.ncols), max_total_cells=int(packed.col_offset[-1]),
                max_cells_per_col=int(ns.max()))
    base.update(kw)
    return default_config(**base)


def config_for_dims(ncols: int, total_cells: int, max_cells: int, **kw) -> jfnk_config:
    """Config with the given capacity."""
    base = dict(max_cols=int(ncols), max_total_cells=int(total_cells), max_cells_per_col=int(max_cells))
    base.update(kw)
    return default_config(**base)


def net_param_count() -> int:
    return int(lib().jfnk_net_param_count())


def net_default_config(**kw) -> jfnk_net_config:
    cfg = jfnk_net_config()
    lib().jfnk_net_config_default(C.byref(cfg))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise AttributeError(k)
        setattr(cfg, k, v)
    return cfg


class Net:
    """Owns one jfnk_net (learned Newton initial guess)."""

    def __init__(self, config: Optional[jfnk_net_config] = None, **kw):
        self.config = config if config is not None else net_default_config(**kw)
        h = C.c_void_p()
        rc = lib().jfnk_net_create(C.byref(self.config), C.byref(h))
        if rc != JFNK_OK:
            raise JfnkError(rc, "jfnk_net_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().jfnk_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().jfnk_net_last_error(self.h).decode()

    def _check(self, rc):
        if rc != JFNK_OK:
            raise JfnkError(rc, self.last_error())

    def set_params(self, params: np.ndarray):
        a = np.ascontiguousarray(params, dtype=np.float32)
        self._check(lib().jfnk_net_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))

    def get_params(self) -> np.ndarray:
        a = np.zeros(net_param_count(), np.float32)
        self._check(lib().jfnk_net_get_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    def predict(self, prob: DeviceProblem, ne, phi, ne_prev=None, phi_prev=None, stream=None):
        import torch
        ne_out = torch.empty_like(ne)
        phi_out = torch.empty_like(phi)
        p = prob.cstruct()
        s = Solver._state(ne, phi, ne_prev, phi_prev)
        self._check(lib().jfnk_net_predict(self.h, C.byref(p), C.byref(s), _ptr(ne_out), _ptr(phi_out),
                                           _stream_ptr(stream)))
        return ne_out, phi_out

    def grad(self, prob: DeviceProblem, ne, phi, ne_prev, phi_prev, ne_next, phi_next, stream=None):
        """(loss, gradient) of one batch."""
        g = np.zeros(net_param_count(), np.float32)
        loss = C.c_double()
        p = prob.cstruct()
        s = Solver._state(ne, phi, ne_prev, phi_prev)
        self._check(lib().jfnk_net_grad(self.h, C.byref(p), C.byref(s), _ptr(ne_next), _ptr(phi_next),
                                        g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss),
                                        _stream_ptr(stream)))
        return loss.value, g

    def train_step(self, prob: DeviceProblem, ne, phi, ne_prev, phi_prev, ne_next, phi_next, lr: float,
                   want_loss: bool = False, stream=None):
        loss = C.c_double()
        p = prob.cstruct()
        s = Solver._state(ne, phi, ne_prev, phi_prev)
        self._check(lib().jfnk_net_train_step(self.h, C.byref(p), C.byref(s), _ptr(ne_next), _ptr(phi_next),
                                              float(lr), C.byref(loss) if want_loss else None,
                                              _stream_ptr(stream)))
        return loss.value if want_loss else None
