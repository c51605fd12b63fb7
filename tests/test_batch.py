"""Batched animation frames in one persistent launch."""
import numpy as np
import pytest

import oracle
from paper_2307_09226_amd import scenes
from gpu_util import GATE_MFMA, GATE_PLAIN_C128, errors, marginal_ratio, sample_indices

pytestmark = pytest.mark.gpu


def _rs():
    from paper_2307_09226_amd import rs
    return rs


def _frames(n, p_max=30000):
    return scenes.animation_frames(seed=3, nframes=n, p_min=2048, p_max=p_max)


@pytest.mark.parametrize("form,dtype", [(1, 0), (0, 1)])
def test_batch_equals_single_frames_bitwise(form, dtype):
    import torch
    rs = _rs()
    radar = scenes.radar_batch()
    frames = _frames(6)
    plan = rs.rs_cube_plan(radar, form, dtype, max_pixels=max(f.P for f in frames))
    dfr = [rs.DevicePixels.from_host(f) for f in frames]
    cubes = rs.new_cube(plan, count=len(frames))
    rs.rs_beat_synthesize_batch(plan, dfr, cubes)
    singles = []
    for d in dfr:
        c = rs.new_cube(plan)
        rs.rs_beat_synthesize(plan, d, c)
        singles.append(c)
    torch.cuda.synchronize()
    for i in range(len(frames)):
        assert torch.equal(cubes[i], singles[i]), i


def test_batch_parity_sampled_and_marginals():
    import torch
    rs = _rs()
    radar = scenes.radar_batch()
    frames = _frames(4, p_max=60000)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64,
                           max_pixels=max(f.P for f in frames))
    dfr = [rs.DevicePixels.from_host(f) for f in frames]
    cubes = rs.new_cube(plan, count=len(frames))
    rs.rs_beat_synthesize_batch(plan, dfr, cubes)
    torch.cuda.synchronize()
    out = cubes.cpu().numpy()
    for i, f in enumerate(frames):
        c, l, n = sample_indices(radar.cube_shape(), 300, seed=i)
        ref = oracle.entries(radar, f, c, l, n)
        rel, mx = errors(out[i][c, l, n], ref)
        assert rel <= GATE_MFMA and mx <= GATE_MFMA, (i, rel, mx)
        assert marginal_ratio(out[i], oracle.marginal_n(radar, f), 2) <= GATE_MFMA
        assert marginal_ratio(out[i], oracle.marginal_l(radar, f), 1) <= GATE_MFMA


def test_batch_with_empty_frames():
    import torch
    rs = _rs()
    radar = scenes.radar_batch()
    f = scenes.tiny_scene(3, 1000)
    empty = scenes.Pixels(*(np.zeros(0, np.float32) for _ in range(5)))
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=1000)
    dfr = [rs.DevicePixels.from_host(x) for x in (empty, f, empty)]
    cubes = rs.new_cube(plan, count=3)
    cubes.fill_(5)
    rs.rs_beat_synthesize_batch(plan, dfr, cubes)
    torch.cuda.synchronize()
    out = cubes.cpu().numpy()
    assert np.all(out[0] == 0) and np.all(out[2] == 0)
    ref = oracle.cube(radar, f)
    assert errors(out[1], ref)[0] <= GATE_MFMA


def test_full_animation_batch_one_launch():
    """The 64-frame animation (3 x 4 array, Ns 256, L 64; 2,304 .. 235,225
    pixels per frame, 3.0 M in all) in one persistent launch: a few frames,
    the smallest and the largest among them, bitwise equal to single-frame
    calls; every frame within the matrix-core gate on sampled entries; the
    largest frame summed over fast time and over slow time within the bound
    the gate implies for the closed-form marginals (gpu_util.marginal_ratio)."""
    import torch
    rs = _rs()
    radar = scenes.radar_batch()
    frames = scenes.animation_frames(seed=3, nframes=64)
    sizes = np.array([f.P for f in frames])
    big, small = int(np.argmax(sizes)), int(np.argmin(sizes))
    print(f"animation: {len(frames)} frames, P {sizes.min()} .. {sizes.max()}, total {sizes.sum()}", flush=True)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=int(sizes.max()))
    dfr = [rs.DevicePixels.from_host(f) for f in frames]
    cubes = rs.new_cube(plan, count=len(frames))
    rs.rs_beat_synthesize_batch(plan, dfr, cubes)
    torch.cuda.synchronize()
    for i in sorted({0, small, big, len(frames) - 1}):
        c = rs.new_cube(plan)
        rs.rs_beat_synthesize(plan, dfr[i], c)
        torch.cuda.synchronize()
        assert torch.equal(cubes[i], c), i
    out = cubes.cpu().numpy()
    worst = 0.0
    for i, f in enumerate(frames):
        idx = sample_indices(radar.cube_shape(), 32, seed=100 + i)
        rel, mx = errors(out[i][idx], oracle.entries(radar, f, *idx))
        worst = max(worst, rel, mx)
        assert rel <= GATE_MFMA and mx <= GATE_MFMA, (i, rel, mx)
    mn, ml = oracle.marginal_n(radar, frames[big]), oracle.marginal_l(radar, frames[big])
    rn, rl = marginal_ratio(out[big], mn, 2), marginal_ratio(out[big], ml, 1)
    g = out[big].astype(np.complex128)
    print(f"animation: worst sampled error {worst:.2e}; largest frame marginals (bound ratio) "
          f"{rn:.2e} / {rl:.2e} (relative L2 of the marginals {errors(g.sum(axis=2), mn)[0]:.2e} / "
          f"{errors(g.sum(axis=1), ml)[0]:.2e})", flush=True)
    assert rn <= GATE_MFMA and rl <= GATE_MFMA
