"""Error handling and edge cases of the C ABI on the GPU."""
import ctypes

import numpy as np
import pytest

from paper_2307_09226_amd import scenes
from gpu_util import synth

pytestmark = pytest.mark.gpu


def _rs():
    from paper_2307_09226_amd import rs
    return rs


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("dtype", [0, 1])
def test_empty_scene_gives_exact_zero_cube(form, dtype):
    import torch
    rs = _rs()
    radar = scenes.radar_small()
    plan = rs.rs_cube_plan(radar, form, dtype, max_pixels=10)
    cube = rs.new_cube(plan)
    cube.fill_(complex(7.0, -3.0))
    empty = rs.DevicePixels(*(torch.zeros(0, dtype=torch.float32, device="cuda:0") for _ in range(5)))
    rs.rs_beat_synthesize(plan, empty, cube)
    torch.cuda.synchronize()
    out = cube.cpu().numpy()
    assert np.all(out == 0)
    assert plan.workspace_bytes(0) == 0


def test_invalid_calls_do_not_launch_or_write():
    import torch
    rs = _rs()
    radar = scenes.radar_small()
    px = scenes.tiny_scene(1, 100)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=50)
    dpx = rs.DevicePixels.from_host(px)
    cube = rs.new_cube(plan)
    cube.fill_(complex(1.0, 2.0))
    with pytest.raises(rs.RSError) as e:
        rs.rs_beat_synthesize(plan, dpx, cube)  # P = 100 > max_pixels = 50
    assert e.value.status == rs.RS_E_INVALID and "max_pixels" in str(e.value)
    # NULL pixel pointer with P > 0
    ps = rs.rs_pixels(10, None, dpx.y.data_ptr(), dpx.z.data_ptr(), dpx.amp.data_ptr(), dpx.vr.data_ptr())
    code = rs.lib.rs_beat_synthesize(plan.handle, ctypes.byref(ps), cube.data_ptr(), None)
    assert code == rs.RS_E_INVALID
    # NULL cube
    ps = dpx.struct()
    ps.P = 10
    assert rs.lib.rs_beat_synthesize(plan.handle, ctypes.byref(ps), None, None) == rs.RS_E_INVALID
    # workspace too small / misaligned
    buf = torch.empty(1024, dtype=torch.uint8, device="cuda:0")
    need = plan.workspace_bytes(10)
    assert need > 0
    code = rs.lib.rs_beat_synthesize_ws(plan.handle, ctypes.byref(ps), cube.data_ptr(),
                                        buf.data_ptr(), 16, None)
    assert code == rs.RS_E_INVALID
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda:0")
    code = rs.lib.rs_beat_synthesize_ws(plan.handle, ctypes.byref(ps), cube.data_ptr(),
                                        big.data_ptr() + 8, need, None)
    assert code == rs.RS_E_INVALID
    code = rs.lib.rs_beat_synthesize_batch(plan.handle, None, -1, cube.data_ptr(), None)
    assert code == rs.RS_E_INVALID
    torch.cuda.synchronize()
    assert np.all(cube.cpu().numpy() == complex(1.0, 2.0))


def test_stream_ordering_and_two_streams_share_a_plan():
    import torch
    rs = _rs()
    radar = scenes.radar_for(2, 2, 128, 64, Fs=10e6, Tb=80e-6)
    px = scenes.tiny_scene(5, 4000)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=px.P)
    dpx = rs.DevicePixels.from_host(px)
    ref = rs.new_cube(plan)
    rs.rs_beat_synthesize(plan, dpx, ref)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a, b = rs.new_cube(plan), rs.new_cube(plan)
    with torch.cuda.stream(s1):
        rs.rs_beat_synthesize(plan, dpx, a, stream=s1)
        a2 = a * 2  # ordered after the synthesis on s1
    with torch.cuda.stream(s2):
        rs.rs_beat_synthesize(plan, dpx, b, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(a, ref) and torch.equal(b, ref) and torch.equal(a2, ref * 2)


def test_plan_describe_and_workspace():
    rs = _rs()
    radar, px = scenes.workload_frame()
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=px.P)
    import json
    d = json.loads(plan.describe(px.P))
    assert d["form"] == "mfma_split16" and d["chunks"] >= 1
    # partial sums of every chunk (the kernel finds the chunk scales itself)
    assert plan.workspace_bytes(px.P) == d["chunks"] * 12 * 128 * 256 * 8
    # with strengths per block, plus one scale exponent per chunk (256-byte padded)
    import dataclasses
    bplan = rs.rs_cube_plan(dataclasses.replace(radar, model=16), rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64,
                            max_pixels=px.P)
    db = json.loads(bplan.describe(px.P))
    scale_bytes = (db["chunks"] * 4 + 255) // 256 * 256
    assert bplan.workspace_bytes(px.P) == db["chunks"] * 12 * 128 * 256 * 8 + scale_bytes
    bplan.close()
    # a pixel count whose chunks would exceed 2^30 pixels is refused, not wrapped
    big = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=1 << 40)
    with pytest.raises(rs.RSError) as e:
        big.workspace_bytes(1 << 40)
    assert e.value.status == rs.RS_E_INVALID
    big.close()
    plan.close()


def test_ws_variant_equals_allocating_variant():
    rs = _rs()
    radar = scenes.radar_for(3, 4, 256, 128, Fs=10e6, Tb=120e-6)
    px = scenes.scene_small(seed=1, grid=96, pedestrian=True)
    for form in (0, 1):
        a = synth(radar, px, form, 0)
        b = synth(radar, px, form, 0, ws=True)
        assert np.array_equal(a, b)


def test_library_first_then_torch_share_one_runtime():
    """A process that loads the binding and creates a plan before touching
    torch's GPU state must still see the device from torch (one HIP runtime
    in the process)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_2307_09226_amd import rs, scenes\n"
            "plan = rs.rs_cube_plan(scenes.radar_small(), rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=64)\n"
            "import torch\n"
            "assert torch.cuda.is_available()\n"
            "cube = rs.new_cube(plan)\n"
            "px = rs.DevicePixels.from_host(scenes.tiny_scene(1, 64))\n"
            "rs.rs_beat_synthesize(plan, px, cube)\n"
            "torch.cuda.synchronize()\n"
            "print('ok')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "ok" in r.stdout, r.stderr[-2000:]
