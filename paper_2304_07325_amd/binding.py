"""Thin Python binding of libsymba's C ABI (include/symba.h).

Argument marshalling only: every step of the kick/encounter path runs in the
HIP kernels of libsymba.so.  PyTorch provides device memory and streams.
The library must be built (paper_2304_07325_amd.build); importing this module
raises if it is not -- there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsymba.so")

SYMBA_OK, SYMBA_EINVAL, SYMBA_ENOMEM, SYMBA_EDEVICE, SYMBA_ETOOBIG = 0, 1, 2, 3, 4
STATUS_CAPACITY, STATUS_NONFINITE, STATUS_ENC_SKIPPED = 1, 2, 4
ENC_MAX_PAIRS, ENC_MAX_GROUP_PAIRS = 8192, 255
FIELD_SEG_ROWS = 192   # massive rows per field task
OPT_TILE_ROWS, OPT_FIELD_ROWS, OPT_SCREEN, OPT_TIMING, OPT_BIN, OPT_ACC, OPT_SPLIT = 1, 2, 4, 5, 6, 7, 8
OPT_ENC_FUSE = 9
OPT_ENC_REGS = 10
SCREEN_AUTO, SCREEN_FP32, SCREEN_FP64 = 0, 1, 2
ACC_INTERACTION, ACC_HELIO = 0, 1

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double


class symba_state(ctypes.Structure):
    _fields_ = [(k, _P) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "rh")]


class symba_out(ctypes.Structure):
    _fields_ = [("ax", _P), ("ay", _P), ("az", _P), ("pair_i", _P), ("pair_j", _P),
                ("pair_cap", _I64), ("n_pairs", _P), ("group_id", _P), ("n_groups", _P),
                ("status", _P)]


class symba_mstate(ctypes.Structure):
    _fields_ = [(k, _P) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "rh")]


class symba_step_problem(ctypes.Structure):
    _fields_ = [("state", symba_mstate), ("n", _I64), ("n_m", _I64), ("h", _D), ("rcrit_factor", _D),
                ("out", symba_out)]


class symba_problem(ctypes.Structure):
    _fields_ = [("state", symba_state), ("n", _I64), ("n_m", _I64), ("dt", _D),
                ("rcrit_factor", _D), ("out", symba_out)]


EXPORTS = ("symba_ctx_create", "symba_ctx_destroy", "symba_set_option", "symba_kick_encounter",
           "symba_kick_encounter_batch", "symba_strerror", "symba_plan_tasks", "symba_read_timing",
           "symba_scratch_bytes", "symba_autotune", "symba_read_stats", "symba_step", "symba_step_batch",
           "symba_step_enc", "symba_enc_prepare",
           "symba_plan_for", "symba_kick_encounter_noalloc")
NOALLOC_MAX_N, NOALLOC_MAX_PAIRS = 8192, 65536


class SymbaError(RuntimeError):
    pass


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run paper_2304_07325_amd.build.build() "
                          "(the kick/encounter path has no other implementation)")
    lib = ctypes.CDLL(path)
    lib.symba_ctx_create.restype = ctypes.c_int
    lib.symba_ctx_create.argtypes = [ctypes.POINTER(_P), ctypes.c_int, _I64, _I64, ctypes.c_uint32]
    lib.symba_ctx_destroy.restype = ctypes.c_int
    lib.symba_ctx_destroy.argtypes = [_P]
    lib.symba_set_option.restype = ctypes.c_int
    lib.symba_set_option.argtypes = [_P, ctypes.c_int, ctypes.c_int]
    lib.symba_kick_encounter.restype = ctypes.c_int
    lib.symba_kick_encounter.argtypes = [_P, ctypes.POINTER(symba_state), _I64, _I64, _D, _D,
                                         ctypes.POINTER(symba_out), _P]
    lib.symba_kick_encounter_noalloc.restype = ctypes.c_int
    lib.symba_kick_encounter_noalloc.argtypes = [ctypes.POINTER(symba_state), _I64, _I64, _D, _D,
                                                 ctypes.POINTER(symba_out), _P]
    lib.symba_step.restype = ctypes.c_int
    lib.symba_step.argtypes = [_P, ctypes.POINTER(symba_mstate), _I64, _I64, _D, _D, ctypes.POINTER(symba_out), _P]
    for name in ("symba_step_enc", "symba_enc_prepare"):
        getattr(lib, name).restype = ctypes.c_int
        getattr(lib, name).argtypes = [_P, ctypes.POINTER(symba_mstate), _I64, _I64, _D, _D,
                                       ctypes.POINTER(symba_out), _P]
    lib.symba_step_batch.restype = ctypes.c_int
    lib.symba_step_batch.argtypes = [_P, ctypes.POINTER(symba_step_problem), ctypes.c_int32, _P]
    lib.symba_kick_encounter_batch.restype = ctypes.c_int
    lib.symba_kick_encounter_batch.argtypes = [_P, ctypes.POINTER(symba_problem), ctypes.c_int32, _P]
    lib.symba_strerror.restype = ctypes.c_char_p
    lib.symba_strerror.argtypes = [ctypes.c_int]
    lib.symba_read_timing.restype = ctypes.c_int
    lib.symba_read_timing.argtypes = [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_I64)]
    lib.symba_read_stats.restype = ctypes.c_int
    lib.symba_read_stats.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]
    lib.symba_autotune.restype = ctypes.c_int
    lib.symba_autotune.argtypes = [_P, ctypes.POINTER(symba_state), _I64, _I64, _D, _D,
                                   ctypes.POINTER(symba_out), _P, ctypes.POINTER(ctypes.c_int32)]
    lib.symba_scratch_bytes.restype = _I64
    lib.symba_scratch_bytes.argtypes = [_P, _I64, _I64, _I64]
    lib.symba_plan_for.restype = ctypes.c_int
    lib.symba_plan_for.argtypes = [_P, _I64, _I64, _P, _P]
    lib.symba_plan_tasks.restype = _I64
    lib.symba_plan_tasks.argtypes = [_I64, _I64, ctypes.c_int32, ctypes.c_int32, _P, _I64]
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(rc: int, what: str):
    if rc != SYMBA_OK:
        raise SymbaError(f"{what}: {lib().symba_strerror(rc).decode()} (code {rc})")


STATE_KEYS = ("x", "y", "z", "vx", "vy", "vz", "m", "rh")


def to_device_state(state: dict, device="cuda") -> dict:
    """Host numpy (or torch) SoA arrays -> contiguous float64 device tensors."""
    return {k: torch.as_tensor(state[k], dtype=torch.float64).contiguous().to(device) for k in STATE_KEYS}


class Outputs:
    """Caller-owned device outputs of one evaluation (see symba_out)."""

    def __init__(self, n: int, pair_cap: int, device="cuda"):
        self.n = n
        self.pair_cap = pair_cap
        self.acc = torch.empty((3, n), dtype=torch.float64, device=device)
        self.pair_i = torch.empty(max(pair_cap, 1), dtype=torch.int32, device=device)
        self.pair_j = torch.empty(max(pair_cap, 1), dtype=torch.int32, device=device)
        self.group_id = torch.empty(n, dtype=torch.int32, device=device)
        self.scalars64 = torch.zeros(1, dtype=torch.int64, device=device)
        self.scalars32 = torch.zeros(2, dtype=torch.int32, device=device)

    def c_struct(self) -> symba_out:
        a = self.acc
        s32 = self.scalars32.data_ptr()
        return symba_out(a[0].data_ptr(), a[1].data_ptr(), a[2].data_ptr(), self.pair_i.data_ptr(),
                         self.pair_j.data_ptr(), self.pair_cap, self.scalars64.data_ptr(),
                         self.group_id.data_ptr(), s32, s32 + 4)

    def to_host(self) -> dict:
        """Synchronising copy of everything to numpy (acc as [N, 3])."""
        n_pairs = int(self.scalars64.item())
        n_groups, status = (int(v) for v in self.scalars32.tolist())
        out = dict(acc=self.acc.t().cpu().numpy(), n_pairs=n_pairs, n_groups=n_groups, status=status,
                   group_id=self.group_id.cpu().numpy())
        k = n_pairs if (status & STATUS_CAPACITY) == 0 else 0
        out["pair_i"] = self.pair_i[:k].cpu().numpy()
        out["pair_j"] = self.pair_j[:k].cpu().numpy()
        return out


def _state_struct(st: dict, out: "Outputs | None" = None) -> symba_state:
    """Checks a state (and the outputs it is written to) before its pointers
    reach the library, which takes every array to hold n = len(x) bodies."""
    n = st["x"].numel()
    for k in STATE_KEYS:
        if st[k].numel() != n:
            raise ValueError(f"state[{k!r}] has {st[k].numel()} elements, state['x'] has {n}")
    if out is not None and out.n < n:
        raise ValueError(f"the outputs hold {out.n} bodies, the state has {n}")
    for k in STATE_KEYS:
        t = st[k]
        if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"state[{k!r}] must be a contiguous float64 device tensor")
    return symba_state(*(st[k].data_ptr() for k in STATE_KEYS))


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Context:
    """symba_ctx: device scratch for problems of up to max_n bodies."""

    def __init__(self, max_n: int, max_pairs: int = 0, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        h = _P()
        _check(lib().symba_ctx_create(ctypes.byref(h), device, max_n, max_pairs, 0), "symba_ctx_create")
        self._h = h
        self.max_n = max_n
        self.max_pairs = max_pairs if max_pairs else max(4 * max_n, 4096)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().symba_ctx_destroy(self._h), "symba_ctx_destroy")
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option: int, value: int):
        _check(lib().symba_set_option(self._h, option, value), "symba_set_option")

    def read_timing(self):
        """symba_read_timing: (tile-kernel ms, finalize ms, calls) since the last read."""
        t, fz, n = _D(), _D(), _I64()
        _check(lib().symba_read_timing(self._h, ctypes.byref(t), ctypes.byref(fz), ctypes.byref(n)),
               "symba_read_timing")
        return t.value, fz.value, n.value

    def read_stats(self):
        """symba_read_stats: (screen candidates, flagged pairs, problems) since the last read."""
        a, b, c = _I64(), _I64(), _I64()
        _check(lib().symba_read_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "symba_read_stats")
        return a.value, b.value, c.value

    def scratch_bytes(self, n: int, n_m: int, pair_cap: int) -> int:
        """symba_scratch_bytes: device scratch one problem takes in a call."""
        v = lib().symba_scratch_bytes(self._h, int(n), int(n_m), int(pair_cap))
        if v < 0:
            raise SymbaError("symba_scratch_bytes: invalid arguments")
        return int(v)

    def plan_for(self, n: int, n_m: int):
        """symba_plan_for: (bodies per lane, split diagonals) a call on a problem
        of this size would use now."""
        r, d = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().symba_plan_for(self._h, int(n), int(n_m), ctypes.byref(r), ctypes.byref(d)), "symba_plan_for")
        return int(r.value), int(d.value)

    def kick_encounter(self, state: dict, n_m: int, dt: float, rcrit_factor: float,
                       out: Outputs | None = None, stream=None) -> Outputs:
        """Enqueue one evaluation (symba_kick_encounter); returns the outputs."""
        n = int(state["x"].numel())
        if out is None:
            out = Outputs(n, min(self.max_pairs, max(4 * n, 4096)), device=state["x"].device)
        st = _state_struct(state, out)
        o = out.c_struct()
        rc = lib().symba_kick_encounter(self._h, ctypes.byref(st), n, int(n_m), float(dt),
                                        float(rcrit_factor), ctypes.byref(o), _stream_handle(stream))
        _check(rc, "symba_kick_encounter")
        return out

    def step(self, state: dict, n_m: int, h: float, rcrit_factor: float, out: Outputs, stream=None) -> Outputs:
        """symba_step: one step of length h in place on the device state; out holds
        the accelerations at the current positions on entry and the new
        evaluation on return."""
        n = int(state["x"].numel())
        _state_struct(state, out)  # the same checks as an evaluation's state
        st = symba_mstate(*(state[k].data_ptr() for k in STATE_KEYS))
        o = out.c_struct()
        rc = lib().symba_step(self._h, ctypes.byref(st), n, int(n_m), float(h), float(rcrit_factor),
                              ctypes.byref(o), _stream_handle(stream))
        _check(rc, "symba_step")
        return out

    def _enc_call(self, name, state, n_m, h, rcrit_factor, out, stream):
        n = int(state["x"].numel())
        _state_struct(state, out)
        st = symba_mstate(*(state[k].data_ptr() for k in STATE_KEYS))
        o = out.c_struct()
        rc = getattr(lib(), name)(self._h, ctypes.byref(st), n, int(n_m), float(h), float(rcrit_factor),
                                  ctypes.byref(o), _stream_handle(stream))
        _check(rc, name)
        return out

    def enc_prepare(self, state: dict, n_m: int, h: float, rcrit_factor: float, out: Outputs,
                    stream=None) -> Outputs:
        """symba_enc_prepare: out := the evaluation at state with the flagged
        pairs inside the critical radius reweighted to level 0 (the input of
        step_enc)."""
        return self._enc_call("symba_enc_prepare", state, n_m, h, rcrit_factor, out, stream)

    def step_enc(self, state: dict, n_m: int, h: float, rcrit_factor: float, out: Outputs,
                 stream=None) -> Outputs:
        """symba_step_enc: one step with the encounter groups integrated through
        the shells, in place on the device state; out holds the level-0
        evaluation of the current state on entry and of the new one on return."""
        return self._enc_call("symba_step_enc", state, n_m, h, rcrit_factor, out, stream)

    def step_batch(self, problems, stream=None):
        """symba_step_batch: problems = list of (device state, n_m, h, rcrit_factor, Outputs)."""
        arr = (symba_step_problem * len(problems))()
        for k, (state, n_m, h, f, out) in enumerate(problems):
            _state_struct(state, out)
            arr[k].state = symba_mstate(*(state[key].data_ptr() for key in STATE_KEYS))
            arr[k].n = int(state["x"].numel())
            arr[k].n_m = int(n_m)
            arr[k].h = float(h)
            arr[k].rcrit_factor = float(f)
            arr[k].out = out.c_struct()
        _check(lib().symba_step_batch(self._h, arr, len(problems), _stream_handle(stream)), "symba_step_batch")
        return [p[4] for p in problems]

    def autotune(self, state: dict, n_m: int, dt: float, rcrit_factor: float, out: Outputs | None = None,
                 stream=None) -> int:
        """symba_autotune: times every tile size on this problem, keeps the
        fastest for its size class; returns the chosen bodies per lane."""
        n = int(state["x"].numel())
        if out is None:
            out = Outputs(n, min(self.max_pairs, max(4 * n, 4096)), device=state["x"].device)
        st = _state_struct(state, out)
        o = out.c_struct()
        rows = ctypes.c_int32(0)
        rc = lib().symba_autotune(self._h, ctypes.byref(st), n, int(n_m), float(dt), float(rcrit_factor),
                                  ctypes.byref(o), _stream_handle(stream), ctypes.byref(rows))
        _check(rc, "symba_autotune")
        return int(rows.value)

    def kick_encounter_batch(self, problems, stream=None):
        """problems: list of (state, n_m, dt, rcrit_factor, Outputs)."""
        arr = (symba_problem * len(problems))(*(problem_struct(*p) for p in problems))
        self.kick_encounter_batch_structs(arr, stream)
        return [p[4] for p in problems]

    def kick_encounter_batch_structs(self, arr, stream=None):
        """symba_kick_encounter_batch on a ctypes array of symba_problem built by
        problem_struct (for callers that keep the structs of resident problems)."""
        rc = lib().symba_kick_encounter_batch(self._h, arr, len(arr), _stream_handle(stream))
        _check(rc, "symba_kick_encounter_batch")

    def step_batch_structs(self, arr, stream=None):
        """symba_step_batch on a ctypes array of symba_step_problem built by
        step_problem_struct."""
        _check(lib().symba_step_batch(self._h, arr, len(arr), _stream_handle(stream)), "symba_step_batch")


def problem_struct(state: dict, n_m: int, dt: float, rcrit_factor: float, out: Outputs) -> symba_problem:
    """The symba_problem of one batch entry (pointers into state and out, which
    must outlive every call that uses it)."""
    p = symba_problem()
    p.state = _state_struct(state, out)
    p.n = int(state["x"].numel())
    p.n_m = int(n_m)
    p.dt = float(dt)
    p.rcrit_factor = float(rcrit_factor)
    p.out = out.c_struct()
    return p


def step_problem_struct(state: dict, n_m: int, h: float, rcrit_factor: float, out: Outputs) -> symba_step_problem:
    """The symba_step_problem of one step-batch entry (pointers as problem_struct)."""
    p = symba_step_problem()
    _state_struct(state, out)
    p.state = symba_mstate(*(state[key].data_ptr() for key in STATE_KEYS))
    p.n = int(state["x"].numel())
    p.n_m = int(n_m)
    p.h = float(h)
    p.rcrit_factor = float(rcrit_factor)
    p.out = out.c_struct()
    return p


def kick_encounter_noalloc(state: dict, n_m: int, dt: float, rcrit_factor: float, out: Outputs,
                           stream=None) -> Outputs:
    """symba_kick_encounter_noalloc: one evaluation without a context, in the
    library's fixed scratch of the current device (n <= NOALLOC_MAX_N; calls
    overlapping on one device race)."""
    n = int(state["x"].numel())
    st = _state_struct(state, out)
    o = out.c_struct()
    rc = lib().symba_kick_encounter_noalloc(ctypes.byref(st), n, int(n_m), float(dt), float(rcrit_factor),
                                            ctypes.byref(o), _stream_handle(stream))
    _check(rc, "symba_kick_encounter_noalloc")
    return out


def plan_tasks(n: int, n_m: int, rows: int, field_rows: int = 1):
    """symba_plan_tasks: the folded task list as an [T, 3] int64 array (host only)."""
    import numpy as np
    total = lib().symba_plan_tasks(n, n_m, rows, field_rows, None, 0)
    if total < 0:
        raise SymbaError("symba_plan_tasks: invalid arguments")
    buf = np.zeros((max(total, 1), 3), np.int64)
    got = lib().symba_plan_tasks(n, n_m, rows, field_rows, buf.ctypes.data, total)
    assert got == total
    return buf[:total]
