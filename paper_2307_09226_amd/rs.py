"""Python binding of librs (include/rs.h): argument marshalling only.

Every step of the synthesis runs in the library's gfx950 kernels.  PyTorch
supplies device memory (tensor data pointers) and HIP streams; nothing here
computes any part of the cube.  If librs.so is missing this module raises on
import: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# RS_LIBRARY selects another build of the library (e.g. an instrumented one)
LIB_PATH = os.environ.get("RS_LIBRARY") or os.path.join(_PKG, "librs.so")

RS_OK, RS_E_INVALID, RS_E_NOMEM, RS_E_DEVICE, RS_E_UNSUPPORTED, RS_E_BUSY, RS_E_NOT_FOUND = range(7)
RS_FORM_FP64_DIRECT, RS_FORM_MFMA_SPLIT16, RS_FORM_NUFFT = 0, 1, 2
RS_C64, RS_C128 = 0, 1
RS_STATIC_SCRATCH_BYTES = 64 << 20  # include/rs.h: workspace of rs_beat_synthesize_noalloc
RS_REQ_QUEUED, RS_REQ_RUNNING, RS_REQ_DONE, RS_REQ_FAILED, RS_REQ_CANCELLED = range(5)
RS_SCHED_SHORTEST, RS_SCHED_EQUAL = 0, 1
RS_MODEL_FAR_FIELD, RS_MODEL_TDM_SLOT, RS_MODEL_INTRA_CHIRP, RS_MODEL_RVP, RS_MODEL_BLOCK_STRENGTH = 1, 2, 4, 8, 16
STATUS_NAMES = {0: "RS_OK", 1: "RS_E_INVALID", 2: "RS_E_NOMEM", 3: "RS_E_DEVICE",
                4: "RS_E_UNSUPPORTED", 5: "RS_E_BUSY", 6: "RS_E_NOT_FOUND"}


class RSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class rs_radar(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("N", ctypes.c_int32), ("Ns", ctypes.c_int32),
                ("L", ctypes.c_int32), ("fc", ctypes.c_double), ("mu", ctypes.c_double),
                ("Fs", ctypes.c_double), ("Tb", ctypes.c_double), ("c0", ctypes.c_double),
                ("tx_xyz", ctypes.POINTER(ctypes.c_double)),
                ("rx_xyz", ctypes.POINTER(ctypes.c_double)),
                ("carrier_phase", ctypes.c_int32), ("model", ctypes.c_int32)]


class rs_pixels(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("amp", ctypes.c_void_p), ("vr", ctypes.c_void_p)]


class rs_session_opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("hbm_budget", ctypes.c_size_t),
                ("max_slots", ctypes.c_int32), ("queue_cap", ctypes.c_int32),
                ("slice_items", ctypes.c_int32), ("policy", ctypes.c_int32),
                ("strict_fifo", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("slice_terms", ctypes.c_double)]


class rs_timing(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class rs_session_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("done", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("queued_now", ctypes.c_int64), ("running_now", ctypes.c_int64),
                ("footprint_now", ctypes.c_size_t), ("footprint_peak", ctypes.c_size_t),
                ("terms_done", ctypes.c_double), ("request_bytes_now", ctypes.c_size_t),
                ("request_bytes_peak", ctypes.c_size_t), ("device_error", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class rs_scene(ctypes.Structure):
    _fields_ = [("room_w", ctypes.c_double), ("room_d", ctypes.c_double), ("room_h", ctypes.c_double),
                ("pedestrian", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("centre", ctypes.c_double * 3), ("velocity", ctypes.c_double * 3),
                ("semi_axes", ctypes.c_double * 3)]


class rs_rd_peak(ctypes.Structure):
    _fields_ = [("range_bin", ctypes.c_int32), ("doppler_bin", ctypes.c_int32),
                ("power", ctypes.c_float), ("range_m", ctypes.c_float),
                ("velocity_mps", ctypes.c_float), ("reserved", ctypes.c_float)]


# numpy view of an rs_rd_peak array (same layout)
RD_PEAK_DTYPE = np.dtype([("range_bin", np.int32), ("doppler_bin", np.int32), ("power", np.float32),
                          ("range_m", np.float32), ("velocity_mps", np.float32),
                          ("reserved", np.float32)])


# Every symbol declared in include/rs.h: name -> (restype, argtypes)
_VP = ctypes.c_void_p
SIGNATURES = {
    "rs_cube_plan": (ctypes.c_int, [ctypes.POINTER(rs_radar), ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int64, ctypes.POINTER(_VP)]),
    "rs_cube_plan_nufft": (ctypes.c_int, [ctypes.POINTER(rs_radar), ctypes.c_int, ctypes.c_int64,
                                          ctypes.c_double, ctypes.POINTER(_VP)]),
    "rs_plan_workspace_bytes": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "rs_plan_describe": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_char_p, ctypes.c_size_t]),
    "rs_plan_tune": (ctypes.c_int, [_VP, ctypes.POINTER(rs_pixels), _VP, ctypes.c_int32, _VP,
                                    ctypes.c_char_p, ctypes.c_size_t]),
    "rs_plan_tune_cached": (ctypes.c_int, [_VP, ctypes.POINTER(rs_pixels), _VP, ctypes.c_int32, _VP,
                                           ctypes.c_char_p, ctypes.c_char_p, ctypes.c_size_t]),
    "rs_plan_set_tile": (ctypes.c_int, [_VP, ctypes.c_char_p]),
    "rs_beat_synthesize": (ctypes.c_int, [_VP, ctypes.POINTER(rs_pixels), _VP, _VP]),
    "rs_beat_synthesize_ws": (ctypes.c_int, [_VP, ctypes.POINTER(rs_pixels), _VP, _VP,
                                             ctypes.c_size_t, _VP]),
    "rs_beat_synthesize_noalloc": (ctypes.c_int, [_VP, ctypes.POINTER(rs_pixels), _VP, _VP]),
    "rs_beat_synthesize_batch": (ctypes.c_int, [_VP, ctypes.POINTER(rs_pixels), ctypes.c_int32,
                                                _VP, _VP]),
    "rs_plan_destroy": (None, [_VP]),
    "rs_session_create": (ctypes.c_int, [ctypes.POINTER(rs_session_opts), ctypes.POINTER(_VP)]),
    "rs_session_submit": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(rs_pixels), _VP,
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "rs_session_poll": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(rs_timing)]),
    "rs_session_cancel": (ctypes.c_int, [_VP, ctypes.c_uint64]),
    "rs_session_drain": (ctypes.c_int, [_VP]),
    "rs_session_stats_get": (ctypes.c_int, [_VP, ctypes.POINTER(rs_session_stats)]),
    "rs_session_destroy": (None, [_VP]),
    "rs_session_inject_failure": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "rs_session_inject_device_error": (ctypes.c_int, [_VP]),
    "rs_range_doppler": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP, _VP]),
    "rs_range_doppler_ws": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP, _VP,
                                           ctypes.c_size_t, _VP]),
    "rs_range_doppler_workspace_bytes": (ctypes.c_size_t, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "rs_render_scenes": (ctypes.c_int, [ctypes.POINTER(rs_scene), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "rs_kernel_timer_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_VP)]),
    "rs_kernel_timer_attach": (ctypes.c_int, [_VP]),
    "rs_kernel_timer_read": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32)]),
    "rs_kernel_timer_destroy": (None, [_VP]),
    "rs_last_error": (ctypes.c_char_p, []),
    "rs_version": (ctypes.c_char_p, []),
}


def _load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"librs.so not found at {path}: build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    # PyTorch ships its own copy of the HIP runtime.  Loading it first makes
    # librs.so bind to that same copy (its soname matches); loaded the other
    # way round the process would hold two HIP runtimes, and whichever
    # initialises the GPU second finds no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status: int):
    if status != RS_OK:
        raise RSError(status, lib.rs_last_error().decode())


def rs_version() -> str:
    return lib.rs_version().decode()


def rs_last_error() -> str:
    return lib.rs_last_error().decode()


# ----------------------------------------------------------------------------
def _stream_handle(stream) -> int:
    """HIP stream handle of a torch stream (None = torch's current stream)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _ptr(t) -> int:
    return int(t.data_ptr())


class DevicePixels:
    """Float32 structure-of-arrays pixels resident in device memory."""

    def __init__(self, x, y, z, amp, vr):
        self.x, self.y, self.z, self.amp, self.vr = x, y, z, amp, vr
        self.P = int(x.numel())

    @classmethod
    def from_host(cls, px, device="cuda:0") -> "DevicePixels":
        """amp may be [P] or, for plans with RS_MODEL_BLOCK_STRENGTH, [L][P]."""
        import torch
        arrs = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
                for a in (px.x, px.y, px.z, px.amp, px.vr)]
        return cls(*arrs)

    def struct(self, plan: Optional["Plan"] = None) -> rs_pixels:
        """C view of the arrays.  With a plan, amp must hold L * P values when
        the plan's model has RS_MODEL_BLOCK_STRENGTH and P otherwise."""
        if self.P == 0:
            return rs_pixels(0, None, None, None, None, None)
        rows = 1
        if plan is not None and int(getattr(plan.radar, "model", 0)) & RS_MODEL_BLOCK_STRENGTH:
            rows = int(plan.radar.L)
        for i, a in enumerate((self.x, self.y, self.z, self.amp, self.vr)):
            want = self.P * (rows if i == 3 else 1)
            if i == 3 and plan is None and a.numel() % self.P == 0:
                want = a.numel()
            if a.numel() != want or not a.is_contiguous() or str(a.dtype) != "torch.float32":
                raise ValueError(f"pixel array {i}: {a.numel()} contiguous float32 values, expected {want}")
        return rs_pixels(self.P, _ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.amp),
                         _ptr(self.vr))


class Plan:
    """Owner of an rs_plan handle (rs_cube_plan / rs_plan_destroy)."""

    def __init__(self, handle: int, radar, form: int, dtype: int, max_pixels: int):
        self.handle = handle
        self.radar = radar
        self.form = form
        self.dtype = dtype
        self.max_pixels = max_pixels

    @property
    def cube_shape(self):
        return (self.radar.M * self.radar.N, self.radar.L, self.radar.Ns)

    @property
    def torch_dtype(self):
        import torch
        return torch.complex128 if self.dtype == RS_C128 else torch.complex64

    def describe(self, P: int) -> str:
        buf = ctypes.create_string_buffer(1024)
        _check(lib.rs_plan_describe(self.handle, P, buf, 1024))
        return buf.value.decode()

    def workspace_bytes(self, P: int) -> int:
        out = ctypes.c_size_t()
        _check(lib.rs_plan_workspace_bytes(self.handle, P, ctypes.byref(out)))
        return int(out.value)

    def close(self):
        if self.handle:
            lib.rs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _radar_struct(radar):
    tx = np.ascontiguousarray(radar.tx, dtype=np.float64).reshape(-1)
    rx = np.ascontiguousarray(radar.rx, dtype=np.float64).reshape(-1)
    if tx.size < 3 * max(radar.M, 0) or rx.size < 3 * max(radar.N, 0):
        raise ValueError("antenna arrays must hold M x 3 and N x 3 positions")
    st = rs_radar(int(radar.M), int(radar.N), int(radar.Ns), int(radar.L), float(radar.fc),
                  float(radar.mu), float(radar.Fs), float(radar.Tb), float(radar.c0),
                  tx.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                  rx.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                  int(radar.carrier_phase), int(getattr(radar, "model", 0)))
    return st, (tx, rx)


def rs_cube_plan(radar, form: int = RS_FORM_MFMA_SPLIT16, dtype: int = RS_C64,
                 max_pixels: int = 1 << 20) -> Plan:
    st, keep = _radar_struct(radar)
    h = ctypes.c_void_p()
    _check(lib.rs_cube_plan(ctypes.byref(st), form, dtype, max_pixels, ctypes.byref(h)))
    return Plan(h.value, radar, form, dtype, max_pixels)


def rs_cube_plan_nufft(radar, dtype: int = RS_C64, max_pixels: int = 1 << 20,
                       tolerance: float = 1e-6) -> Plan:
    st, keep = _radar_struct(radar)
    h = ctypes.c_void_p()
    _check(lib.rs_cube_plan_nufft(ctypes.byref(st), dtype, max_pixels, float(tolerance), ctypes.byref(h)))
    return Plan(h.value, radar, RS_FORM_NUFFT, dtype, max_pixels)


def new_cube(plan: Plan, device="cuda:0", count: Optional[int] = None):
    import torch
    shape = plan.cube_shape if count is None else (count,) + plan.cube_shape
    return torch.empty(shape, dtype=plan.torch_dtype, device=device)


def rs_plan_set_tile(plan: Plan, tile: str) -> None:
    """Sets the matrix-core tile configuration ("WNxTLxNW", optional 'i'
    suffix for the pipelined schedule of 8-wave shapes)."""
    _check(lib.rs_plan_set_tile(plan.handle, tile.encode()))


def rs_plan_tune(plan: Plan, pixels: DevicePixels, cube, reps: int = 3, stream=None) -> str:
    """Times every matrix-core tile shape on these pixels and keeps the
    fastest in the plan; returns it as "WNxTLxNW"."""
    ps = pixels.struct(plan)
    buf = ctypes.create_string_buffer(32)
    _check(lib.rs_plan_tune(plan.handle, ctypes.byref(ps), _ptr(cube), int(reps), _stream_handle(stream),
                            buf, 32))
    return buf.value.decode()


def rs_plan_tune_cached(plan: Plan, pixels: DevicePixels, cube, cache_path: str, reps: int = 3,
                        stream=None) -> str:
    """rs_plan_tune with the persistent tile cache at cache_path (a hit sets
    the stored shape and launches nothing); returns the shape."""
    ps = pixels.struct(plan)
    buf = ctypes.create_string_buffer(32)
    _check(lib.rs_plan_tune_cached(plan.handle, ctypes.byref(ps), _ptr(cube), int(reps), _stream_handle(stream),
                                   os.fsencode(cache_path), buf, 32))
    return buf.value.decode()


def rs_beat_synthesize(plan: Plan, pixels: DevicePixels, cube, stream=None):
    ps = pixels.struct(plan)
    _check(lib.rs_beat_synthesize(plan.handle, ctypes.byref(ps), _ptr(cube),
                                  _stream_handle(stream)))
    return cube


def rs_beat_synthesize_ws(plan: Plan, pixels: DevicePixels, cube, workspace, stream=None):
    ps = pixels.struct(plan)
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib.rs_beat_synthesize_ws(plan.handle, ctypes.byref(ps), _ptr(cube),
                                     _ptr(workspace) if nbytes else None, nbytes,
                                     _stream_handle(stream)))
    return cube


def rs_beat_synthesize_noalloc(plan: Plan, pixels: DevicePixels, cube, stream=None):
    """rs_beat_synthesize with the library's static device scratch as its
    workspace: nothing is allocated (see include/rs.h)."""
    ps = pixels.struct(plan)
    _check(lib.rs_beat_synthesize_noalloc(plan.handle, ctypes.byref(ps), _ptr(cube), _stream_handle(stream)))
    return cube


def rs_range_doppler(plan: Plan, cubes, skip_static: bool = True, power=None, doppler_time=None,
                     peaks=None, stream=None):
    """Range-Doppler processing of cubes [F][C][L][Ns] (a single cube [C][L][Ns]
    counts as F = 1).  power (float32 [F][Ns][L]), doppler_time (float32
    [F][L]) and peaks (uint8 [F * 24], rs_rd_peak records) are device tensors
    or None."""
    nframes = 1 if cubes.dim() == 3 else int(cubes.shape[0])
    _check(lib.rs_range_doppler(plan.handle, _ptr(cubes), nframes, 1 if skip_static else 0,
                                _ptr(power) if power is not None else None,
                                _ptr(doppler_time) if doppler_time is not None else None,
                                _ptr(peaks) if peaks is not None else None,
                                _stream_handle(stream)))


def rs_range_doppler_workspace_bytes(plan: Plan, nframes: int, power_given: bool = True) -> int:
    return int(lib.rs_range_doppler_workspace_bytes(plan.handle, int(nframes), 1 if power_given else 0))


def rs_range_doppler_ws(plan: Plan, cubes, skip_static: bool, power, doppler_time, peaks, workspace,
                        stream=None):
    """rs_range_doppler with a caller's device workspace (a uint8 tensor of
    at least rs_range_doppler_workspace_bytes): nothing is allocated."""
    nframes = 1 if cubes.dim() == 3 else int(cubes.shape[0])
    _check(lib.rs_range_doppler_ws(plan.handle, _ptr(cubes), nframes, 1 if skip_static else 0,
                                   _ptr(power) if power is not None else None,
                                   _ptr(doppler_time) if doppler_time is not None else None,
                                   _ptr(peaks) if peaks is not None else None,
                                   _ptr(workspace) if workspace is not None else None,
                                   int(workspace.numel() * workspace.element_size()) if workspace is not None else 0,
                                   _stream_handle(stream)))


def range_doppler(plan: Plan, cubes, skip_static: bool = True, stream=None):
    """rs_range_doppler into new device tensors; returns (power [F][Ns][L],
    doppler_time [F][L], peaks) with peaks a numpy record array (this
    synchronises the stream)."""
    import torch
    nframes = 1 if cubes.dim() == 3 else int(cubes.shape[0])
    r = plan.radar
    power = torch.empty((nframes, r.Ns, r.L), dtype=torch.float32, device=cubes.device)
    dtime = torch.empty((nframes, r.L), dtype=torch.float32, device=cubes.device)
    peaks = torch.empty(nframes * RD_PEAK_DTYPE.itemsize, dtype=torch.uint8, device=cubes.device)
    rs_range_doppler(plan, cubes, skip_static, power, dtime, peaks, stream)
    pk = np.frombuffer(peaks.cpu().numpy().tobytes(), dtype=RD_PEAK_DTYPE)
    return power, dtime, pk


def scene_struct(room, ped=None) -> rs_scene:
    """rs_scene of a room (W, D, H) and an optional pedestrian (centre,
    velocity, semi_axes), e.g. the seeded input generator's Room and
    Pedestrian."""
    s = rs_scene()
    s.room_w, s.room_d, s.room_h = float(room.W), float(room.D), float(room.H)
    s.pedestrian = 0 if ped is None else 1
    if ped is not None:
        for k in range(3):
            s.centre[k] = float(ped.centre[k])
            s.velocity[k] = float(ped.velocity[k])
            s.semi_axes[k] = float(ped.semi_axes[k])
    return s


def scene_array(scenes_: Sequence[rs_scene]):
    """ctypes array of rs_scene records (build once, render many times)."""
    return (rs_scene * max(1, len(scenes_)))(*scenes_)


def rs_render_scenes(scenes_, g_az: int, g_el: int, noise=None, device="cuda:0",
                     stream=None, out=None) -> List[DevicePixels]:
    """Ray-cast len(scenes_) frames on the device.  scenes_: rs_scene records
    or a scene_array(); noise: device float32 [F * P] strength factors or
    None; out: five float32 [F * P] device tensors to fill, or None for new
    ones.  Returns one DevicePixels per frame (views into the five tensors)."""
    import torch
    F = len(scenes_)
    P = int(g_az) * int(g_el)
    outs = out if out is not None else [torch.empty(F * P, dtype=torch.float32, device=device)
                                        for _ in range(5)]
    arr = scenes_ if isinstance(scenes_, ctypes.Array) else scene_array(scenes_)
    _check(lib.rs_render_scenes(arr, F, int(g_az), int(g_el),
                                _ptr(noise) if noise is not None else None,
                                *[_ptr(o) for o in outs], _stream_handle(stream)))
    return [DevicePixels(*(o[f * P:(f + 1) * P] for o in outs)) for f in range(F)]


def rs_beat_synthesize_batch(plan: Plan, frames: Sequence[DevicePixels], cubes, stream=None):
    arr = (rs_pixels * max(1, len(frames)))()
    for i, f in enumerate(frames):
        arr[i] = f.struct(plan)
    _check(lib.rs_beat_synthesize_batch(plan.handle, arr, len(frames), _ptr(cubes),
                                        _stream_handle(stream)))
    return cubes


# ----------------------------------------------------------------------------
class Session:
    """Owner of an rs_session handle (continuous-batching serving loop)."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_slots: int = 16,
                 queue_cap: int = 4096, slice_items: int = 0, policy: int = RS_SCHED_SHORTEST,
                 strict_fifo: bool = False, slice_terms: float = 0.0):
        opts = rs_session_opts(device, hbm_budget, max_slots, queue_cap, slice_items, policy,
                               1 if strict_fifo else 0, 0, float(slice_terms))
        h = ctypes.c_void_p()
        _check(lib.rs_session_create(ctypes.byref(opts), ctypes.byref(h)))
        self.handle = h.value
        self._keep = {}

    def submit(self, plan: Plan, pixels: DevicePixels, cube) -> int:
        ps = pixels.struct(plan)
        t = ctypes.c_uint64()
        _check(lib.rs_session_submit(self.handle, plan.handle, ctypes.byref(ps), _ptr(cube),
                                     ctypes.byref(t)))
        self._keep[t.value] = (plan, pixels, cube)
        return int(t.value)

    def try_submit(self, plan: Plan, pixels: DevicePixels, cube) -> Optional[int]:
        """submit, or None when the queue is full (RS_E_BUSY)."""
        try:
            return self.submit(plan, pixels, cube)
        except RSError as e:
            if e.status == RS_E_BUSY:
                return None
            raise

    def poll(self, ticket: int):
        state = ctypes.c_int32()
        tm = rs_timing()
        _check(lib.rs_session_poll(self.handle, ticket, ctypes.byref(state), ctypes.byref(tm)))
        if state.value in (RS_REQ_DONE, RS_REQ_FAILED, RS_REQ_CANCELLED):
            self._keep.pop(ticket, None)
        return state.value, (tm.t_submit_ns, tm.t_admit_ns, tm.t_done_ns)

    def cancel(self, ticket: int):
        _check(lib.rs_session_cancel(self.handle, ticket))

    def drain(self):
        _check(lib.rs_session_drain(self.handle))

    def stats(self) -> dict:
        st = rs_session_stats()
        _check(lib.rs_session_stats_get(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in rs_session_stats._fields_}

    def inject_failure(self, count: int = 1):
        _check(lib.rs_session_inject_failure(self.handle, count))

    def inject_device_error(self):
        _check(lib.rs_session_inject_device_error(self.handle))

    def close(self):
        if self.handle:
            lib.rs_session_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rs_session_create(**kw) -> Session:
    return Session(**kw)


class KernelTimer:
    """HIP-event durations of main-kernel launches made from this thread
    (rs_kernel_timer_*)."""

    def __init__(self, capacity: int = 4096):
        h = ctypes.c_void_p()
        _check(lib.rs_kernel_timer_create(capacity, ctypes.byref(h)))
        self.handle = h.value
        self.capacity = capacity

    def __enter__(self):
        _check(lib.rs_kernel_timer_attach(self.handle))
        return self

    def __exit__(self, *exc):
        lib.rs_kernel_timer_attach(None)

    def read(self) -> List[float]:
        buf = (ctypes.c_double * self.capacity)()
        n = ctypes.c_int32()
        _check(lib.rs_kernel_timer_read(self.handle, buf, self.capacity, ctypes.byref(n)))
        return [buf[i] for i in range(min(n.value, self.capacity))]

    def close(self):
        if self.handle:
            lib.rs_kernel_timer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
