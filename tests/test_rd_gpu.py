"""Range-Doppler maps on the GPU (rs_range_doppler) against the CPU oracle
applied to the same input cubes, and the walking-circle Doppler-time series
against the pedestrian's ground truth."""
import ctypes

import numpy as np
import pytest

from oracle import rd
from paper_2307_09226_amd import scenes
from gpu_util import synth

pytestmark = pytest.mark.gpu

TOL_POWER = 1e-5   # float32 FFTs: relative L2 of the power map


def _rs():
    from paper_2307_09226_amd import rs
    return rs


def check_rd(radar, plan, cubes_dev, skip_static):
    """GPU maps, peaks and Doppler-time rows vs the oracle on the same cubes."""
    rs = _rs()
    power, dtime, pk = rs.range_doppler(plan, cubes_dev, skip_static=skip_static)
    host = cubes_dev.cpu().numpy()
    ref = rd.range_doppler_power(host)
    got = power.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"rd power relL2={rel:.3e}")
    assert rel <= TOL_POWER
    kr, dr = rd.peaks(ref, skip_static=skip_static)
    L = radar.L
    for f in range(ref.shape[0]):
        k, ds = int(pk["range_bin"][f]), int(pk["doppler_bin"][f])
        d = ds % L
        if (k, d) != (kr[f], dr[f]):
            # a near tie decided in float32: the GPU's cell must be as strong
            # as the oracle's maximum to within the map tolerance
            assert ref[f, k, d] >= ref[f, kr[f], dr[f]] * (1 - 10 * TOL_POWER), (f, k, d, kr[f], dr[f])
        if skip_static:
            assert d != 0
        assert pk["power"][f] == pytest.approx(got[f, k, d], rel=1e-6)
        assert pk["velocity_mps"][f] == pytest.approx(rd.bin_velocity(ds, radar), rel=1e-6, abs=1e-6)
        assert pk["range_m"][f] == pytest.approx(rd.bin_range(k, radar), rel=1e-6, abs=1e-6)
        assert np.array_equal(dtime.cpu().numpy()[f], power.cpu().numpy()[f, k, :])
    return pk


@pytest.mark.parametrize("form,dtype", [(0, 1), (1, 0)])
def test_small_workload(form, dtype):
    import torch
    rs = _rs()
    radar, px = scenes.workload_small()
    plan = rs.rs_cube_plan(radar, form, dtype, max_pixels=px.P)
    cube = torch.from_numpy(synth(radar, px, form, dtype)).to("cuda:0")
    for skip in (True, False):
        check_rd(radar, plan, cube, skip)


def test_walk_frames_batch_and_optional_outputs():
    import torch
    rs = _rs()
    radar = scenes.radar_frame()
    cw = scenes.circle_walk(frame_ids=[5, 30, 61], grid=128)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64,
                           max_pixels=max(f.P for f in cw.frames))
    cubes = rs.new_cube(plan, count=len(cw.frames))
    rs.rs_beat_synthesize_batch(plan, [rs.DevicePixels.from_host(f) for f in cw.frames], cubes)
    pk = check_rd(radar, plan, cubes, True)
    # peaks alone (no power or Doppler-time output) give the same records
    peaks = torch.zeros(len(cw.frames) * rs.RD_PEAK_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    rs.rs_range_doppler(plan, cubes, True, None, None, peaks)
    alone = np.frombuffer(peaks.cpu().numpy().tobytes(), dtype=rs.RD_PEAK_DTYPE)
    assert np.array_equal(alone, pk)


def _random_cubes(plan, F, seed):
    """Seeded complex Gaussian cubes [F][C][L][Ns] on the device."""
    import torch
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    cubes = _rs().new_cube(plan, count=F)
    real = torch.float64 if cubes.dtype == torch.complex128 else torch.float32
    cubes.copy_(torch.complex(torch.randn(cubes.shape, generator=g, device="cuda:0", dtype=real),
                              torch.randn(cubes.shape, generator=g, device="cuda:0", dtype=real)))
    return cubes


def check_rd_frames(radar, plan, cubes, frames, skip_static=True):
    """GPU maps and peaks of a batch against the oracle on a subset of its
    frames (each frame's map depends on that frame's cube alone)."""
    rs = _rs()
    power, dtime, pk = rs.range_doppler(plan, cubes, skip_static=skip_static)
    host = cubes[frames].cpu().numpy()
    ref = rd.range_doppler_power(host)
    got = power[frames].cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"rd power relL2={rel:.3e} over frames {frames}")
    assert rel <= TOL_POWER
    kr, dr = rd.peaks(ref, skip_static=skip_static)
    L = radar.L
    dt = dtime.cpu().numpy()
    for j, f in enumerate(frames):
        k, d = int(pk["range_bin"][f]), int(pk["doppler_bin"][f]) % L
        if (k, d) != (kr[j], dr[j]):
            assert ref[j, k, d] >= ref[j, kr[j], dr[j]] * (1 - 10 * TOL_POWER), (f, k, d, kr[j], dr[j])
        assert pk["power"][f] == pytest.approx(got[j, k, d], rel=1e-6)
        assert np.array_equal(dt[f], power[f, k, :].cpu().numpy())


@pytest.mark.parametrize("L,dtype", [(16, 0), (32, 1), (64, 0), (128, 1)])
def test_fused_shapes(L, dtype):
    """Every fast-time-256 shape of the fused path, both input precisions,
    on seeded random cubes (7 frames of 12 channels)."""
    rs = _rs()
    radar = scenes.radar_for(3, 4, 256, L, Fs=10e6, Tb=3 * 40e-6)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, dtype, max_pixels=16)
    cubes = _random_cubes(plan, 7, seed=L + dtype)
    check_rd_frames(radar, plan, cubes, list(range(7)))


def test_fused_runs_across_frames():
    """300 frames: the workgroups' runs of (frame, channel) items start and
    end inside frames and span up to three of them, so frames are merged
    from partial maps of up to four workgroups; frames at run boundaries,
    the first and the last are checked."""
    rs = _rs()
    radar = scenes.radar_frame()
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=16)
    cubes = _random_cubes(plan, 300, seed=11)
    check_rd_frames(radar, plan, cubes, [0, 1, 2, 13, 149, 150, 151, 298, 299], skip_static=False)


@pytest.mark.parametrize("L", [64, 128])
def test_workspace_variant_matches(L):
    """rs_range_doppler_ws with a caller's workspace gives the bits of
    rs_range_doppler, with and without a power map; short or misaligned
    workspaces are refused."""
    import torch
    rs = _rs()
    radar = scenes.radar_for(3, 4, 256, L, Fs=10e6, Tb=3 * 40e-6)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=16)
    F = 9
    cubes = _random_cubes(plan, F, seed=5)
    power, dtime, pk = rs.range_doppler(plan, cubes, skip_static=True)
    need = rs.rs_range_doppler_workspace_bytes(plan, F, True)
    need_np = rs.rs_range_doppler_workspace_bytes(plan, F, False)
    assert need_np == need + (F * radar.Ns * L * 4 + 255) // 256 * 256
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    p2 = torch.empty_like(power)
    d2 = torch.empty_like(dtime)
    k2 = torch.empty(F * rs.RD_PEAK_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    rs.rs_range_doppler_ws(plan, cubes, True, p2, d2, k2, ws)
    assert torch.equal(p2, power) and torch.equal(d2, dtime)
    assert np.array_equal(np.frombuffer(k2.cpu().numpy().tobytes(), dtype=rs.RD_PEAK_DTYPE), pk)
    # without a power map the workspace holds it
    ws2 = torch.empty(need_np, dtype=torch.uint8, device="cuda:0")
    k3 = torch.zeros_like(k2)
    rs.rs_range_doppler_ws(plan, cubes, True, None, None, k3, ws2)
    assert torch.equal(k3, k2)
    code = rs.lib.rs_range_doppler_ws(plan.handle, cubes.data_ptr(), F, 1, p2.data_ptr(), None, None,
                                      ws.data_ptr(), need - 1, None)
    assert code == rs.RS_E_INVALID and "needed" in rs.rs_last_error()
    code = rs.lib.rs_range_doppler_ws(plan.handle, cubes.data_ptr(), F, 1, p2.data_ptr(), None, None,
                                      ws.data_ptr() + 8, need, None)
    assert code == rs.RS_E_INVALID and "aligned" in rs.rs_last_error()
    torch.cuda.synchronize()


def test_unsupported_and_invalid():
    import torch
    rs = _rs()
    r = scenes.radar_for(1, 2, 50, 32, Fs=10e6, Tb=40e-6)
    plan = rs.rs_cube_plan(r, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=10)
    cube = rs.new_cube(plan)
    code = rs.lib.rs_range_doppler(plan.handle, cube.data_ptr(), 1, 1, None, None, None, None)
    assert code == rs.RS_E_UNSUPPORTED and "powers of two" in rs.rs_last_error()
    r2 = scenes.radar_small()
    plan2 = rs.rs_cube_plan(r2, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=10)
    assert rs.lib.rs_range_doppler(plan2.handle, None, 1, 1, None, None, None, None) == rs.RS_E_INVALID
    assert rs.lib.rs_range_doppler(plan2.handle, None, -1, 1, None, None, None, None) == rs.RS_E_INVALID
    assert rs.lib.rs_range_doppler(plan2.handle, None, 0, 1, None, None, None, None) == rs.RS_OK
    torch.cuda.synchronize()


def test_walking_circle_doppler_time():
    """The 100-frame walking circle (Sec. III scenario) through synthesis and
    range-Doppler maps on the GPU: the max-power velocity of every CPI follows
    the pedestrian centre's radial velocity."""
    import torch
    rs = _rs()
    radar = scenes.radar_frame()
    cw = scenes.circle_walk()
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64,
                           max_pixels=max(f.P for f in cw.frames))
    cubes = rs.new_cube(plan, count=len(cw.frames))
    rs.rs_beat_synthesize_batch(plan, [rs.DevicePixels.from_host(f) for f in cw.frames], cubes)
    _, _, pk = rs.range_doppler(plan, cubes, skip_static=True)
    v_est = pk["velocity_mps"].astype(np.float64)
    dv = rd.bin_velocity(1, radar)
    err = np.abs(v_est - cw.v_radial)
    ev = rd.e_velo(v_est, cw.v_radial)
    print(f"E_velo = {ev:.3f} m/s (bin {dv:.3f} m/s), max error {err.max():.3f} m/s")
    assert ev <= 2 * dv
    assert err.max() <= 6 * dv
    assert np.corrcoef(v_est, cw.v_radial)[0, 1] > 0.99
    rng_true = np.linalg.norm(cw.centres, axis=1)
    assert np.all(np.abs(pk["range_m"] - rng_true) <= 0.6)
