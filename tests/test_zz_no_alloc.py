"""rs_beat_synthesize_noalloc: the synthesis call that allocates nothing (its
workspace is the library's static device scratch), called through the C ABI
and checked against rs_beat_synthesize on two calls in a row, the second with
a smaller input, plus the oracle on sampled entries or full cubes."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2307_09226_amd import scenes
from gpu_util import GATE_MFMA, GATE_PLAIN_C128, errors, sample_indices

pytestmark = pytest.mark.gpu


def _rs():
    from paper_2307_09226_amd import rs
    return rs


def _noalloc(rs, plan, dpx, cube):
    """One call of the entry point through the raw C ABI; returns its status."""
    ps = dpx.struct(plan)
    return rs.lib.rs_beat_synthesize_noalloc(plan.handle, ctypes.byref(ps), cube.data_ptr(),
                                             rs._stream_handle(None))


def _existing(rs, plan, dpx):
    import torch
    cube = rs.new_cube(plan)
    rs.rs_beat_synthesize(plan, dpx, cube)
    torch.cuda.synchronize()
    return cube.cpu().numpy()


def _run_pair(rs, plan, frames, check):
    """Two calls in a row on one plan (the second with fewer pixels), each
    compared bitwise with rs_beat_synthesize and then by `check`."""
    import torch
    for px in frames:
        print(f"noalloc form={plan.form} P={px.P} workspace={plan.workspace_bytes(px.P)}", flush=True)
        dpx = rs.DevicePixels.from_host(px)
        cube = rs.new_cube(plan)
        cube.fill_(complex(3.0, -5.0))
        assert _noalloc(rs, plan, dpx, cube) == rs.RS_OK, rs.rs_last_error()
        torch.cuda.synchronize()
        got = cube.cpu().numpy()
        want = _existing(rs, plan, dpx)
        assert np.array_equal(got, want), f"P={px.P}: differs from rs_beat_synthesize"
        check(px, got)


def test_matrix_core_frame_then_smaller():
    """The 65,536-pixel frame (3 x 4 array, Ns 256, L 128), then a ragged
    9,001-pixel scene on the same plan."""
    rs = _rs()
    radar, frame = scenes.workload_frame()
    small = scenes.tiny_scene(501, 9001, vmax=6.0)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=frame.P)
    assert plan.workspace_bytes(frame.P) <= rs.RS_STATIC_SCRATCH_BYTES

    def check(px, got):
        idx = sample_indices(got.shape, 96, seed=px.P)
        ref = oracle.entries(radar, px, *idx)
        rel, mx = errors(got[idx], ref)
        print(f"  vs oracle (sampled): relL2={rel:.3e} maxabs={mx:.3e}", flush=True)
        assert rel <= GATE_MFMA and mx <= GATE_MFMA

    _run_pair(rs, plan, [frame, small], check)
    plan.close()


def test_plain_complex128_small_workload_then_smaller():
    """The small workload (2 x 4, Ns 64, L 32, 4,096 pixels) in binary64,
    then 1,337 pixels: full cubes against the oracle at 1e-12."""
    rs = _rs()
    radar, px = scenes.workload_small()
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_FP64_DIRECT, rs.RS_C128, max_pixels=px.P)

    def check(p, got):
        rel, mx = errors(got, oracle.cube(radar, p))
        print(f"  vs oracle (full cube): relL2={rel:.3e} maxabs={mx:.3e}", flush=True)
        assert rel <= GATE_PLAIN_C128 and mx <= GATE_PLAIN_C128

    _run_pair(rs, plan, [px, px.take(np.arange(0, px.P, 3)[:1337])], check)
    plan.close()


def test_nufft_plan_then_smaller():
    """A NUFFT plan (tolerance 1e-6) on the frame and on its first 30,001
    pixels (grid order keeps each 256-pixel block's box inside its tile slot,
    so the cubes repeat bit for bit)."""
    rs = _rs()
    radar, frame = scenes.workload_frame()
    plan = rs.rs_cube_plan_nufft(radar, rs.RS_C64, max_pixels=frame.P, tolerance=1e-6)
    assert plan.workspace_bytes(frame.P) <= rs.RS_STATIC_SCRATCH_BYTES

    def check(px, got):
        idx = sample_indices(got.shape, 64, seed=7 + px.P)
        ref = oracle.entries(radar, px, *idx)
        rel, _ = errors(got[idx], ref)
        print(f"  vs oracle (sampled): relL2={rel:.3e}", flush=True)
        assert rel <= 1e-6 + 2e-6

    _run_pair(rs, plan, [frame, frame.take(np.arange(30001))], check)
    plan.close()


def test_too_large_is_refused_without_writing():
    """The binary64 plain form of the frame needs more than the static
    scratch: RS_E_INVALID, nothing launched, the cube untouched; an empty
    scene still gives the exact zero cube."""
    import torch
    rs = _rs()
    radar, frame = scenes.workload_frame()
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_FP64_DIRECT, rs.RS_C64, max_pixels=frame.P)
    assert plan.workspace_bytes(frame.P) > rs.RS_STATIC_SCRATCH_BYTES
    dpx = rs.DevicePixels.from_host(frame)
    cube = rs.new_cube(plan)
    cube.fill_(complex(1.0, 2.0))
    assert _noalloc(rs, plan, dpx, cube) == rs.RS_E_INVALID
    assert "static scratch" in rs.rs_last_error()
    empty = rs.DevicePixels(*(torch.zeros(0, dtype=torch.float32, device="cuda:0") for _ in range(5)))
    torch.cuda.synchronize()
    assert np.all(cube.cpu().numpy() == complex(1.0, 2.0))
    assert _noalloc(rs, plan, empty, cube) == rs.RS_OK
    torch.cuda.synchronize()
    assert np.all(cube.cpu().numpy() == 0)
    plan.close()
