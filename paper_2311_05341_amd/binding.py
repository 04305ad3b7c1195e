"""Python binding of the dedispersion C ABI (include/dd.h).

Argument marshalling only: every step of the transform runs in the HIP library
``libdd.so``.  PyTorch supplies device memory and streams.  If the library is
missing the import fails; there is no other execution path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libdd.so is not built: run `python -m paper_2311_05341_amd._build` "
                      "(or __graft_entry__.build()) first")

_lib = ctypes.CDLL(LIB_PATH)

DD_U8, DD_U4, DD_F32, DD_U16 = 1, 2, 3, 4
_DTYPES = {"u8": DD_U8, "u4": DD_U4, "f32": DD_F32, "u16": DD_U16}
# torch element type and bytes per element of an input row, per dtype
_IN_TORCH = {"u8": (torch.uint8, 1), "u4": (torch.uint8, 1), "u16": (torch.uint16, 2), "f32": (torch.float32, 4)}
STATUS = {0: "DD_OK", -1: "DD_ERR_ARG", -2: "DD_ERR_TOO_SHORT", -3: "DD_ERR_RANGE", -4: "DD_ERR_ALIGN",
          -5: "DD_ERR_DTYPE", -6: "DD_ERR_NOT_BOUND", -7: "DD_ERR_HIP", -8: "DD_ERR_NOMEM"}


class PlanDesc(ctypes.Structure):
    _fields_ = [("n_chan", ctypes.c_int32), ("n_samp", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("f_high_mhz", ctypes.c_double), ("chan_bw_mhz", ctypes.c_double),
                ("chan_freq_mhz", ctypes.POINTER(ctypes.c_double)), ("t_samp_s", ctypes.c_double),
                ("dm_start", ctypes.c_double), ("dm_step", ctypes.c_double), ("n_dm", ctypes.c_int32),
                ("in_pitch_bytes", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_out", ctypes.c_int64), ("max_shift", ctypes.c_int32), ("n_dm", ctypes.c_int32),
                ("n_chan", ctypes.c_int32), ("in_pitch_bytes", ctypes.c_int64),
                ("dev_table_bytes", ctypes.c_size_t), ("host_shift", ctypes.POINTER(ctypes.c_int32)),
                ("kernel_ns", ctypes.c_int32), ("kernel_dm_per_wave", ctypes.c_int32),
                ("kernel_waves", ctypes.c_int32), ("kernel_chan_block", ctypes.c_int32),
                ("kernel_order", ctypes.c_int32), ("tune_ws_bytes", ctypes.c_size_t)]


class Tiles(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("order", ctypes.c_int32), ("ns", ctypes.c_int32),
                ("per_wave", ctypes.c_int32), ("waves", ctypes.c_int32), ("row_block", ctypes.c_int32),
                ("segs", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class TuneReport(ctypes.Structure):
    _fields_ = [("n_tried", ctypes.c_int32), ("best", Tiles), ("best_ms", ctypes.c_double),
                ("default_ms", ctypes.c_double), ("timed_out_samples", ctypes.c_int64)]


_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_lib.dd_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(_vp)]
_lib.dd_plan_create.restype = _i32
_lib.dd_plan_destroy.argtypes = [_vp]
_lib.dd_plan_destroy.restype = None
_lib.dd_plan_query.argtypes = [_vp, ctypes.POINTER(PlanInfo)]
_lib.dd_plan_query.restype = _i32
_lib.dd_plan_bind.argtypes = [_vp, _vp, _sz, _vp]
_lib.dd_plan_bind.restype = _i32
_lib.dd_execute.argtypes = [_vp, _vp, _vp, _i64, _vp]
_lib.dd_execute.restype = _i32
_lib.dd_execute_noalloc.argtypes = [_vp, _vp, _vp, _i64, _vp]
_lib.dd_execute_noalloc.restype = _i32
_lib.dd_execute_adjoint.argtypes = [_vp, _vp, _i64, _vp, _vp]
_lib.dd_execute_adjoint.restype = _i32
_lib.dd_plan_shape_count.argtypes = [_vp, ctypes.POINTER(_i32)]
_lib.dd_plan_shape_count.restype = _i32
_lib.dd_plan_get_tiles.argtypes = [_vp, _i32, ctypes.POINTER(Tiles)]
_lib.dd_plan_get_tiles.restype = _i32
_lib.dd_plan_set_tiles.argtypes = [_vp, _i32, _i32, _i32]
_lib.dd_plan_set_tiles.restype = _i32
_lib.dd_plan_autotune.argtypes = [_vp, _i32, _vp, _vp, _i64, _vp, _sz, _vp, ctypes.POINTER(TuneReport)]
_lib.dd_plan_autotune.restype = _i32
_lib.dd_batch_create.argtypes = [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp)]
_lib.dd_batch_create.restype = _i32
_lib.dd_batch_workspace_bytes.argtypes = [_vp, ctypes.POINTER(_sz)]
_lib.dd_batch_workspace_bytes.restype = _i32
_lib.dd_batch_bind.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i64), _vp, _sz, _vp]
_lib.dd_batch_bind.restype = _i32
_lib.dd_execute_batched.argtypes = [_vp, _vp]
_lib.dd_execute_batched.restype = _i32
_lib.dd_batch_get_tiles.argtypes = [_vp, ctypes.POINTER(Tiles)]
_lib.dd_batch_get_tiles.restype = _i32
_lib.dd_batch_get_beam_tiles.argtypes = [_vp, _i32, ctypes.POINTER(Tiles)]
_lib.dd_batch_get_beam_tiles.restype = _i32
_lib.dd_batch_set_tiles.argtypes = [_vp, _i32]
_lib.dd_batch_set_tiles.restype = _i32
_lib.dd_batch_autotune.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i64), _vp, _sz, _vp,
                                   ctypes.POINTER(TuneReport)]
_lib.dd_batch_autotune.restype = _i32
_lib.dd_batch_destroy.argtypes = [_vp]
_lib.dd_batch_destroy.restype = None
_lib.dd_bin_time.argtypes = [_i32, _vp, _i64, _i32, _i64, _i32, _vp, _i64, _vp]
_lib.dd_bin_time.restype = _i32
_lib.dd_bin_out_dtype.argtypes = [_i32]
_lib.dd_bin_out_dtype.restype = _i32


class Range(ctypes.Structure):
    _fields_ = [("dm_start", ctypes.c_double), ("dm_step", ctypes.c_double), ("n_dm", ctypes.c_int32),
                ("bin", ctypes.c_int32)]


_lib.dd_corner_turn.argtypes = [_i32, _vp, _i64, _i32, _i64, _vp, _i64, _vp]
_lib.dd_corner_turn.restype = _i32
DD_SURVEY_TIME_MAJOR = 1
_lib.dd_survey_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(Range), _i32, _i32, ctypes.POINTER(_vp)]
_lib.dd_survey_create.restype = _i32
_lib.dd_survey_plan.argtypes = [_vp, _i32, ctypes.POINTER(_vp)]
_lib.dd_survey_plan.restype = _i32
_lib.dd_survey_workspace_bytes.argtypes = [_vp, ctypes.POINTER(_sz)]
_lib.dd_survey_workspace_bytes.restype = _i32
_lib.dd_survey_bind.argtypes = [_vp, _vp, _sz, _vp]
_lib.dd_survey_bind.restype = _i32
_lib.dd_survey_autotune.argtypes = [_vp, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_i64), _vp]
_lib.dd_survey_autotune.restype = _i32
_lib.dd_survey_execute.argtypes = [_vp, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_i64), _vp]
_lib.dd_survey_execute.restype = _i32
_lib.dd_survey_destroy.argtypes = [_vp]
_lib.dd_survey_destroy.restype = None
_lib.dd_status_string.argtypes = [_i32]
_lib.dd_status_string.restype = ctypes.c_char_p
_lib.dd_last_error.argtypes = []
_lib.dd_last_error.restype = ctypes.c_char_p


class DDError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        detail = (_lib.dd_last_error() or b"").decode()
        super().__init__("%s: %s (%s)" % (where, self.name, detail))


def _check(rc: int, where: str) -> None:
    if rc != 0:
        raise DDError(rc, where)


def _stream_handle(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _round_up(v: int, a: int) -> int:
    return (v + a - 1) // a * a


def _desc(n_chan, n_samp, dtype, f_high, chan_bw, t_samp, dm_start, dm_step, n_dm, freqs, in_pitch_bytes):
    d = PlanDesc()
    d.n_chan, d.n_samp, d.dtype = int(n_chan), int(n_samp), _DTYPES[dtype]
    d.f_high_mhz, d.chan_bw_mhz, d.t_samp_s = float(f_high), float(chan_bw), float(t_samp)
    d.dm_start, d.dm_step, d.n_dm = float(dm_start), float(dm_step), int(n_dm)
    d.in_pitch_bytes = int(in_pitch_bytes)
    if freqs is not None:
        d.chan_freq_mhz = freqs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d


class Plan:
    """A dedispersion plan bound to the current device.

    Mirrors dd_plan_desc.  ``in_pitch_bytes`` of 0 means tightly packed rows.
    The FP64 shift table is built on the host by dd_plan_create; its device
    copy lives in a torch uint8 tensor owned by the plan.
    """

    def __init__(self, n_chan, n_samp, dtype, f_high, chan_bw, t_samp, dm_start, dm_step, n_dm,
                 chan_freq=None, in_pitch_bytes=0, device=None, bind=True):
        self.dtype = dtype
        self._freqs = None if chan_freq is None else np.ascontiguousarray(chan_freq, dtype=np.float64)
        d = _desc(n_chan, n_samp, dtype, f_high, chan_bw, t_samp, dm_start, dm_step, n_dm, self._freqs,
                  in_pitch_bytes)
        h = _vp()
        _check(_lib.dd_plan_create(ctypes.byref(d), ctypes.byref(h)), "dd_plan_create")
        self._h = h
        self._query()
        info = self.info
        self.n_chan, self.n_samp, self.n_dm = int(n_chan), int(n_samp), int(n_dm)
        self.n_out = int(info.n_out)
        self.max_shift = int(info.max_shift)
        self.in_pitch_bytes = int(info.in_pitch_bytes)
        self.out_pitch = _round_up(self.n_out, 4)
        self.workspace = None
        self.device = None
        if bind:
            self.bind(device)

    def _query(self):
        info = PlanInfo()
        _check(_lib.dd_plan_query(self._h, ctypes.byref(info)), "dd_plan_query")
        self.info = info

    @property
    def n_shapes(self) -> int:
        n = _i32()
        _check(_lib.dd_plan_shape_count(self._h, ctypes.byref(n)), "dd_plan_shape_count")
        return int(n.value)

    def tiles(self, direction=0) -> dict:
        """Current tile choice of the forward (0) or adjoint (1) kernel."""
        t = Tiles()
        _check(_lib.dd_plan_get_tiles(self._h, int(direction), ctypes.byref(t)), "dd_plan_get_tiles")
        return t.as_dict()

    def set_tiles(self, direction, shape, order=0, stream=None):
        """Switch to compiled shape `shape` with workgroup order `order` and re-bind."""
        _check(_lib.dd_plan_set_tiles(self._h, int(direction), int(shape), int(order)), "dd_plan_set_tiles")
        self._query()
        if self.device is not None:
            self.bind(self.device, stream)

    def autotune(self, src, dst, direction=0, stream=None) -> dict:
        """Time every feasible tile choice on (src, dst) and keep the fastest (dd_plan_autotune).

        Forward: src = input, dst = output [n_dm][>= n_out].  Adjoint: src = y
        [n_dm][>= n_out], dst = gradient [n_chan][in_row_elems].  dst is overwritten."""
        if direction == 0:
            self._check_input(src)
            self._check_output(dst)
            pitch = dst.stride(0)
        else:
            self._check_y(src)
            self._check_grad(dst)
            pitch = src.stride(0)
        with torch.cuda.device(self.device):
            ws = torch.empty(int(self.info.tune_ws_bytes), dtype=torch.uint8, device=self.device)
            rep = TuneReport()
            _check(_lib.dd_plan_autotune(self._h, int(direction), src.data_ptr(), dst.data_ptr(), pitch, ws.data_ptr(),
                                         ws.numel(), _stream_handle(stream), ctypes.byref(rep)), "dd_plan_autotune")
        self._query()
        self.bind(self.device, stream)  # a workspace of the winner's size
        return {"n_tried": int(rep.n_tried), "best": rep.best.as_dict(), "best_ms": rep.best_ms,
                "default_ms": rep.default_ms, "timed_out_samples": int(rep.timed_out_samples)}

    @property
    def shift(self) -> np.ndarray:
        """Copy of the host shift table, int32 [n_dm][n_chan]."""
        a = np.ctypeslib.as_array(self.info.host_shift, shape=(self.n_dm * self.n_chan,))
        return a.reshape(self.n_dm, self.n_chan).copy()

    def bind(self, device=None, stream=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(dev):
            ws = torch.empty(int(self.info.dev_table_bytes), dtype=torch.uint8, device=dev)
            _check(_lib.dd_plan_bind(self._h, ws.data_ptr(), ws.numel(), _stream_handle(stream)), "dd_plan_bind")
        self.workspace, self.device = ws, dev

    @property
    def in_row_elems(self) -> int:
        return self.in_pitch_bytes // _IN_TORCH[self.dtype][1]

    def empty_input(self):
        dt = _IN_TORCH[self.dtype][0]
        return torch.empty((self.n_chan, self.in_row_elems), dtype=dt, device=self.device)

    def _check_input(self, x):
        dt = _IN_TORCH[self.dtype][0]
        if x.dtype != dt or x.device != self.device or x.dim() != 2 or x.shape[0] != self.n_chan:
            raise ValueError("input must be %s [n_chan][...] on %s" % (dt, self.device))
        if x.stride(1) != 1 or x.stride(0) * x.element_size() != self.in_pitch_bytes:
            raise ValueError("input rows must be contiguous with pitch %d bytes" % self.in_pitch_bytes)
        need = self.n_samp // 2 if self.dtype == "u4" else self.n_samp
        if x.shape[1] < need:
            raise ValueError("input rows are shorter than n_samp")

    def _check_output(self, out):
        if (out.dtype != torch.float32 or out.device != self.device or out.dim() != 2 or out.shape[0] != self.n_dm
                or out.shape[1] < self.n_out or out.stride(1) != 1):
            raise ValueError("out must be float32 [n_dm][>= n_out] with contiguous rows on %s" % self.device)

    def _check_y(self, y):
        if (y.dtype != torch.float32 or y.device != self.device or y.dim() != 2 or y.shape[0] != self.n_dm
                or y.shape[1] < self.n_out or y.stride(1) != 1 or y.stride(0) < self.n_out):
            raise ValueError("y must be float32 [n_dm][>= n_out] with contiguous rows on %s" % self.device)

    def _check_grad(self, g):
        if (g.dtype != torch.float32 or g.device != self.device or g.dim() != 2 or g.shape[0] != self.n_chan
                or g.shape[1] < self.n_samp or g.stride(1) != 1 or g.stride(0) * 4 != self.in_pitch_bytes):
            raise ValueError("gradient buffer must be float32 [n_chan][in_row_elems] on %s" % self.device)

    def forward(self, x, out=None, stream=None):
        """S = dedisperse(x): float32 [n_dm][n_out] (a view of an [n_dm][out_pitch] buffer)."""
        self._check_input(x)
        if out is None:
            out = torch.empty((self.n_dm, self.out_pitch), dtype=torch.float32, device=self.device)
        self._check_output(out)
        _check(_lib.dd_execute(self._h, x.data_ptr(), out.data_ptr(), out.stride(0), _stream_handle(stream)),
               "dd_execute")
        return out[:, : self.n_out]

    def forward_noalloc(self, x, out, stream=None):
        """dd_execute_noalloc: the forward transform with the plan's tables in the library's
        static device area instead of a bound workspace; allocates nothing (`out` is required).
        Works on an unbound plan (bind=False), which then takes x's device for its checks."""
        if self.device is None:
            self.device = x.device
        self._check_input(x)
        self._check_output(out)
        _check(_lib.dd_execute_noalloc(self._h, x.data_ptr(), out.data_ptr(), out.stride(0), _stream_handle(stream)),
               "dd_execute_noalloc")
        return out[:, : self.n_out]

    def adjoint(self, y, out=None, stream=None):
        """g = A^T y for float32 plans: float32 [n_chan][n_samp] (view of a pitched buffer).

        y may have any row pitch >= n_out (a gradient tensor is passed as is)."""
        self._check_y(y)
        if out is None:
            out = torch.empty((self.n_chan, self.in_row_elems), dtype=torch.float32, device=self.device)
        self._check_grad(out)
        _check(_lib.dd_execute_adjoint(self._h, y.data_ptr(), y.stride(0), out.data_ptr(), _stream_handle(stream)),
               "dd_execute_adjoint")
        return out[:, : self.n_samp]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dd_plan_destroy(h)
            self._h = None


def dedisperse(x, plan: Plan, out=None):
    """Forward transform of ``x`` with ``plan`` on the current stream."""
    return plan.forward(x, out=out)


class DedisperseFn(torch.autograd.Function):
    """Differentiable forward transform for float32 plans; backward is dd_execute_adjoint.

    x is float32 [n_chan][m] with the plan's row pitch, m >= n_samp (the plan's
    whole pitched buffer or a view of its first columns).  The forward returns
    an [n_dm][n_out] view of a pitched output buffer.  The backward passes the
    incoming gradient to the adjoint as it is (any row pitch; only a gradient
    without contiguous rows, such as the expanded ones of a plain sum, is
    materialised first) and writes the input gradient straight into a buffer of
    the plan's pitch; columns n_samp..m-1, which no output reads, are zeroed only
    when x has them."""

    @staticmethod
    def forward(ctx, x, plan):
        if plan.dtype != "f32":
            raise TypeError("autograd needs a float32 plan")
        ctx.plan = plan
        ctx.x_cols = int(x.shape[1])
        return plan.forward(x)

    @staticmethod
    def backward(ctx, grad_out):
        plan = ctx.plan
        g = grad_out
        if g.stride(1) != 1 or g.stride(0) < plan.n_out or g.data_ptr() % 4:
            g = g.contiguous()
        gx = torch.empty((plan.n_chan, plan.in_row_elems), dtype=torch.float32, device=plan.device)
        plan.adjoint(g, out=gx)
        if ctx.x_cols > plan.n_samp:
            gx[:, plan.n_samp: ctx.x_cols].zero_()
        return gx[:, : ctx.x_cols], None


class Batch:
    """Many beams (one plan each) in persistent, graph-replayed launches (one per tile shape in use)."""

    def __init__(self, plans, inputs, outputs=None, stream=None):
        n = len(plans)
        self.plans = list(plans)
        arr = (_vp * n)(*[p._h for p in plans])
        h = _vp()
        _check(_lib.dd_batch_create(arr, n, ctypes.byref(h)), "dd_batch_create")
        self._h = h
        nbytes = _sz()
        _check(_lib.dd_batch_workspace_bytes(h, ctypes.byref(nbytes)), "dd_batch_workspace_bytes")
        dev = plans[0].device
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
        for p, x in zip(plans, inputs):
            p._check_input(x)
        self.inputs = list(inputs)
        if outputs is None:
            outputs = [torch.empty((p.n_dm, p.out_pitch), dtype=torch.float32, device=dev) for p in plans]
        self.outputs = list(outputs)
        self.bind(stream)

    def _bind_args(self):
        n = len(self.plans)
        return ((_vp * n)(*[x.data_ptr() for x in self.inputs]), (_vp * n)(*[o.data_ptr() for o in self.outputs]),
                (_i64 * n)(*[o.stride(0) for o in self.outputs]))

    def bind(self, stream=None):
        ins, outs, pitches = self._bind_args()
        _check(_lib.dd_batch_bind(self._h, ins, outs, pitches, self.workspace.data_ptr(), self.workspace.numel(),
                                  _stream_handle(stream)), "dd_batch_bind")

    def tiles(self) -> dict:
        """The shape every beam runs (shape -1 when the beams run different shapes)."""
        t = Tiles()
        _check(_lib.dd_batch_get_tiles(self._h, ctypes.byref(t)), "dd_batch_get_tiles")
        return t.as_dict()

    def beam_tiles(self, beam) -> dict:
        """The shape beam `beam` runs."""
        t = Tiles()
        _check(_lib.dd_batch_get_beam_tiles(self._h, int(beam), ctypes.byref(t)), "dd_batch_get_beam_tiles")
        return t.as_dict()

    def set_tiles(self, shape, stream=None):
        """Put every beam on compiled shape `shape` (staged or direct-read) and re-bind."""
        _check(_lib.dd_batch_set_tiles(self._h, int(shape)), "dd_batch_set_tiles")
        self.bind(stream)

    def autotune(self, stream=None) -> dict:
        """Time the per-beam default shapes and the shared staged and direct-read shapes on the whole
        batch and keep the fastest (dd_batch_autotune); outputs are overwritten."""
        ins, outs, pitches = self._bind_args()
        rep = TuneReport()
        _check(_lib.dd_batch_autotune(self._h, ins, outs, pitches, self.workspace.data_ptr(), self.workspace.numel(),
                                      _stream_handle(stream), ctypes.byref(rep)), "dd_batch_autotune")
        return {"n_tried": int(rep.n_tried), "best": rep.best.as_dict(), "best_ms": rep.best_ms,
                "default_ms": rep.default_ms}

    def run(self, stream=None):
        _check(_lib.dd_execute_batched(self._h, _stream_handle(stream)), "dd_execute_batched")
        return [o[:, : p.n_out] for o, p in zip(self.outputs, self.plans)]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dd_batch_destroy(h)
            self._h = None


#: Output encoding of time binning per input encoding (dd_bin_out_dtype).
BIN_OUT = {"u8": "u16", "u4": "u16", "u16": "f32", "f32": "f32"}
#: Encoding a survey's binned range is dedispersed in: binned 16-bit input is kept as two
#: exact uint16 planes (low and high halves of the sums) and runs the 16-bit kernel on each.
SURVEY_BIN_DTYPE = {"u8": "u16", "u4": "u16", "u16": "u16", "f32": "f32"}


def _row_bytes(dtype, n_samp):
    return {"u8": n_samp, "u4": (n_samp + 1) // 2, "u16": 2 * n_samp, "f32": 4 * n_samp}[dtype]


def _check_rows(x, dtype, n_rows, n_samp, what):
    tdt, eb = _IN_TORCH[dtype]
    if x.dtype != tdt or x.dim() != 2 or x.shape[0] != n_rows or x.stride(1) != 1 or x.device.type != "cuda":
        raise ValueError("%s must be a %s [%d][...] CUDA tensor with contiguous rows" % (what, tdt, n_rows))
    if x.shape[1] * eb < _row_bytes(dtype, n_samp):
        raise ValueError("%s rows are shorter than %d samples" % (what, n_samp))
    if (x.stride(0) * eb) % 16 or x.data_ptr() % 16:
        raise ValueError("%s must be 16-byte aligned with a row pitch that is a multiple of 16 bytes" % what)


def bin_time(x, dtype, n_samp, factor, out=None, stream=None):
    """Time binning (dd_bin_time): sums of ``factor`` consecutive samples of every row.

    x: [n_chan][>= row] tensor in encoding ``dtype``; returns the binned rows,
    encoding BIN_OUT[dtype], as a [n_chan][n_samp // factor] view of ``out``
    (allocated with 16-byte rows when not given)."""
    n_chan = x.shape[0]
    _check_rows(x, dtype, n_chan, n_samp, "input")
    n_bins = n_samp // factor
    odt = BIN_OUT[dtype]
    ot, ob = _IN_TORCH[odt]
    if out is None:
        out = torch.empty((n_chan, _round_up(max(n_bins, 1) * ob, 16) // ob), dtype=ot, device=x.device)
    _check_rows(out, odt, n_chan, n_bins, "out")
    with torch.cuda.device(x.device):
        _check(_lib.dd_bin_time(_DTYPES[dtype], x.data_ptr(), x.stride(0) * _IN_TORCH[dtype][1], n_chan, n_samp,
                                int(factor), out.data_ptr(), out.stride(0) * ob, _stream_handle(stream)),
               "dd_bin_time")
    return out[:, :n_bins]


def _spectrum_bytes(dtype, n_chan):
    return (n_chan + 1) // 2 if dtype == "u4" else n_chan * _IN_TORCH[dtype][1]


def _check_spectra(x, dtype, n_chan, n_samp, what="spectra"):
    tdt, eb = _IN_TORCH[dtype]
    if x.dtype != tdt or x.dim() != 2 or x.shape[0] < n_samp or x.stride(1) != 1 or x.device.type != "cuda":
        raise ValueError("%s must be a %s [n_samp][...] CUDA tensor with contiguous rows" % (what, tdt))
    if x.shape[1] * eb < _spectrum_bytes(dtype, n_chan):
        raise ValueError("%s hold fewer than %d channels" % (what, n_chan))
    if (x.stride(0) * eb) % 16 or x.data_ptr() % 16:
        raise ValueError("%s must be 16-byte aligned with a pitch that is a multiple of 16 bytes" % what)


def corner_turn(spectra, dtype, n_chan, n_samp, out=None, stream=None):
    """Time-major spectra [n_samp][...] to channel-major rows [n_chan][...] (dd_corner_turn).

    Returns ``out`` (allocated with 16-byte rows when not given); 4-bit rows
    hold n_samp // 2 bytes."""
    _check_spectra(spectra, dtype, n_chan, n_samp)
    tdt, eb = _IN_TORCH[dtype]
    row = _row_bytes(dtype, n_samp)
    if out is None:
        out = torch.empty((n_chan, _round_up(row, 16) // eb), dtype=tdt, device=spectra.device)
    _check_rows(out, dtype, n_chan, n_samp, "out")
    with torch.cuda.device(spectra.device):
        _check(_lib.dd_corner_turn(_DTYPES[dtype], spectra.data_ptr(), spectra.stride(0) * eb, n_chan, n_samp,
                                   out.data_ptr(), out.stride(0) * eb, _stream_handle(stream)), "dd_corner_turn")
    return out


class Survey:
    """Several DM ranges over one filterbank, each with its own step and time binning (dd_survey_*).

    ranges: sequence of (dm_start, dm_step, n_dm, bin).  Range r is dedispersed
    from the input binned by ``bin`` (n_samp // bin samples of t_samp * bin);
    ``run`` returns one float32 [n_dm_r][n_out_r] view per range.  With
    ``time_major`` the input is spectra [n_samp][...] (``in_pitch_bytes`` between
    spectra), corner-turned on the device first."""

    def __init__(self, n_chan, n_samp, dtype, f_high, chan_bw, t_samp, ranges, chan_freq=None,
                 in_pitch_bytes=0, device=None, stream=None, bind=True, time_major=False):
        self.dtype = dtype
        self.time_major = bool(time_major)
        self.n_chan, self.n_samp = int(n_chan), int(n_samp)
        self._freqs = None if chan_freq is None else np.ascontiguousarray(chan_freq, dtype=np.float64)
        d = _desc(n_chan, n_samp, dtype, f_high, chan_bw, t_samp, 0.0, 0.0, 1, self._freqs, in_pitch_bytes)
        rs = (Range * len(ranges))()
        for i, (start, step, n_dm, b) in enumerate(ranges):
            rs[i].dm_start, rs[i].dm_step, rs[i].n_dm, rs[i].bin = float(start), float(step), int(n_dm), int(b)
        h = _vp()
        _check(_lib.dd_survey_create(ctypes.byref(d), rs, len(ranges), DD_SURVEY_TIME_MAJOR if time_major else 0,
                                     ctypes.byref(h)), "dd_survey_create")
        self._h = h
        self.ranges = [tuple(r) for r in ranges]
        self.in_pitch_bytes = int(in_pitch_bytes) or (_spectrum_bytes(dtype, self.n_chan) if time_major
                                                       else _row_bytes(dtype, self.n_samp))
        self.range_info = []
        for r, (start, step, n_dm, b) in enumerate(self.ranges):
            ph = _vp()
            _check(_lib.dd_survey_plan(h, r, ctypes.byref(ph)), "dd_survey_plan")
            info = PlanInfo()
            _check(_lib.dd_plan_query(ph, ctypes.byref(info)), "dd_plan_query")
            n_out = int(info.n_out)
            self.range_info.append({"n_dm": int(n_dm), "bin": int(b), "n_out": n_out, "out_pitch": _round_up(n_out, 4),
                                    "n_samp": self.n_samp // int(b), "t_samp": float(t_samp) * int(b),
                                    "dtype": dtype if int(b) == 1 else SURVEY_BIN_DTYPE[dtype],
                                    "split_planes": dtype == "u16" and int(b) > 1,
                                    "max_shift": int(info.max_shift)})
        nbytes = _sz()
        _check(_lib.dd_survey_workspace_bytes(h, ctypes.byref(nbytes)), "dd_survey_workspace_bytes")
        self.workspace_bytes = int(nbytes.value)
        self.workspace = self.device = None
        if bind:
            self.bind(device, stream)

    def bind(self, device=None, stream=None):
        """Allocate the workspace on ``device`` and bind (dd_survey_bind)."""
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        nbytes = self.workspace_bytes
        h = self._h
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=self.device)
            _check(_lib.dd_survey_bind(h, self.workspace.data_ptr(), self.workspace.numel(), _stream_handle(stream)),
                   "dd_survey_bind")

    def tiles(self, r) -> dict:
        """Forward tile choice of range r's plan."""
        ph = _vp()
        _check(_lib.dd_survey_plan(self._h, r, ctypes.byref(ph)), "dd_survey_plan")
        t = Tiles()
        _check(_lib.dd_plan_get_tiles(ph, 0, ctypes.byref(t)), "dd_plan_get_tiles")
        return t.as_dict()

    def shift(self, r) -> np.ndarray:
        """Copy of range r's shift table (in binned samples), int32 [n_dm][n_chan]."""
        ph = _vp()
        _check(_lib.dd_survey_plan(self._h, r, ctypes.byref(ph)), "dd_survey_plan")
        info = PlanInfo()
        _check(_lib.dd_plan_query(ph, ctypes.byref(info)), "dd_plan_query")
        n_dm = self.range_info[r]["n_dm"]
        a = np.ctypeslib.as_array(info.host_shift, shape=(n_dm * self.n_chan,))
        return a.reshape(n_dm, self.n_chan).copy()

    def empty_outputs(self):
        return [torch.empty((ri["n_dm"], ri["out_pitch"]), dtype=torch.float32, device=self.device)
                for ri in self.range_info]

    def _args(self, x, outs):
        if self.time_major:
            _check_spectra(x, self.dtype, self.n_chan, self.n_samp, "input")
        else:
            _check_rows(x, self.dtype, self.n_chan, self.n_samp, "input")
        if x.device != self.device:
            raise ValueError("input must be on %s" % self.device)
        if x.stride(0) * x.element_size() != self.in_pitch_bytes:
            raise ValueError("input pitch must be the survey's %d bytes" % self.in_pitch_bytes)
        if outs is None:
            outs = self.empty_outputs()
        if len(outs) != len(self.range_info):
            raise ValueError("one output per range")
        for o, ri in zip(outs, self.range_info):
            if (o.dtype != torch.float32 or o.device != self.device or o.dim() != 2 or o.shape[0] != ri["n_dm"]
                    or o.shape[1] < ri["n_out"] or o.stride(1) != 1):
                raise ValueError("outputs must be float32 [n_dm][>= n_out] with contiguous rows on %s" % self.device)
        n = len(outs)
        return outs, (_vp * n)(*[o.data_ptr() for o in outs]), (_i64 * n)(*[o.stride(0) for o in outs])

    def run(self, x, outs=None, stream=None):
        outs, ptrs, pitches = self._args(x, outs)
        with torch.cuda.device(self.device):
            _check(_lib.dd_survey_execute(self._h, x.data_ptr(), ptrs, pitches, _stream_handle(stream)),
                   "dd_survey_execute")
        return [o[:, : ri["n_out"]] for o, ri in zip(outs, self.range_info)]

    def autotune(self, x, outs=None, stream=None):
        """Tune every range's forward tiles on its own (binned) input; outputs are overwritten."""
        outs, ptrs, pitches = self._args(x, outs)
        with torch.cuda.device(self.device):
            _check(_lib.dd_survey_autotune(self._h, x.data_ptr(), ptrs, pitches, _stream_handle(stream)),
                   "dd_survey_autotune")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dd_survey_destroy(h)
            self._h = None

