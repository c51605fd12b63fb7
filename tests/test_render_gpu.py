"""Scenes ray-cast on the device (rs_render_scenes) against the seeded
input generator's CPU renderer, and the whole path rendered on the device."""
import math

import numpy as np
import pytest

import oracle
from paper_2307_09226_amd import scenes
from gpu_util import GATE_MFMA, errors, sample_indices

pytestmark = pytest.mark.gpu


def _rs():
    from paper_2307_09226_amd import rs
    return rs


def _compare(dev, ref):
    """float32 outputs of binary64 geometry: equal to a few float32 ulp."""
    for f in ("x", "y", "z", "amp", "vr"):
        g = getattr(dev, f).cpu().numpy().astype(np.float64)
        r = getattr(ref, f).astype(np.float64)
        scale = np.maximum(np.abs(r), 1e-6 if f != "amp" else 0.0)
        tol = 4 * 2.0 ** -24 * np.maximum(np.abs(r), np.max(np.abs(r)) * 1e-6) + (1e-9 if f == "vr" else 0.0)
        bad = np.abs(g - r) > tol
        assert not np.any(bad), (f, int(bad.sum()), float(np.max(np.abs(g - r) / np.maximum(scale, 1e-30))))


@pytest.mark.parametrize("grid,ped", [((37, 23), False), ((64, 64), True), ((256, 256), True)])
def test_matches_cpu_renderer(grid, ped):
    import torch
    rs = _rs()
    g_az, g_el = grid
    rng = np.random.default_rng(11)
    room = scenes.draw_room(rng)
    pedestrian = scenes.draw_pedestrian(rng, room) if ped else None
    seed = 123
    noise = np.random.default_rng(seed).lognormal(0.0, 0.5, g_az * g_el).astype(np.float32)
    ref = scenes.render(np.random.default_rng(seed), room, pedestrian, g_az, g_el)
    dn = torch.from_numpy(noise).to("cuda:0")
    (dev,) = rs.rs_render_scenes([rs.scene_struct(room, pedestrian)], g_az, g_el, dn)
    torch.cuda.synchronize()
    _compare(dev, ref)
    if ped:
        assert np.count_nonzero(dev.vr.cpu().numpy()) == int(ref.is_ped.sum()) > 0


def test_batch_of_walk_frames_and_no_noise():
    import torch
    rs = _rs()
    # five frames: a thread casts its pixel into up to four frames, so the
    # fifth starts a second, ragged group
    ids = [0, 17, 50, 83, 99]
    cw = scenes.circle_walk(frame_ids=ids, grid=96)
    room = scenes.Room(W=12.0, D=10.0)
    structs = [rs.scene_struct(room, scenes.Pedestrian(centre=c, velocity=v))
               for c, v in zip(cw.centres, cw.velocities)]
    frames = rs.rs_render_scenes(structs, 96, 96)   # noise = 1
    torch.cuda.synchronize()
    for k, f in enumerate(ids):
        ref = scenes.render(_OnesRng(), room, scenes.Pedestrian(centre=cw.centres[k], velocity=cw.velocities[k]),
                            96, 96)
        _compare(frames[k], ref)
        single = rs.rs_render_scenes([structs[k]], 96, 96)[0]
        torch.cuda.synchronize()
        for a in ("x", "y", "z", "amp", "vr"):
            assert torch.equal(getattr(single, a), getattr(frames[k], a))


class _OnesRng:
    """Stands in for the generator where the CPU renderer draws its strength
    factors: all ones."""

    @staticmethod
    def lognormal(mean, sigma, size):
        return np.ones(size)


def test_rendered_on_device_through_synthesis():
    """Device-rendered frame -> split-fp16 synthesis, against the oracle on
    the CPU-rendered pixels of the same scene."""
    import torch
    rs = _rs()
    radar = scenes.radar_for(2, 4, 128, 64, Fs=10e6, Tb=80e-6)
    rng = np.random.default_rng(5)
    room = scenes.draw_room(rng)
    ped = scenes.draw_pedestrian(rng, room)
    noise = np.random.default_rng(6).lognormal(0.0, 0.5, 48 * 40).astype(np.float32)
    ref_px = scenes.render(np.random.default_rng(6), room, ped, 48, 40)
    (dev,) = rs.rs_render_scenes([rs.scene_struct(room, ped)], 48, 40,
                                 torch.from_numpy(noise).to("cuda:0"))
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=dev.P)
    cube = rs.new_cube(plan)
    rs.rs_beat_synthesize(plan, dev, cube)
    torch.cuda.synchronize()
    c, l, n = sample_indices(radar.cube_shape(), 300, seed=3)
    ref = oracle.entries(radar, ref_px, c, l, n)
    rel, mx = errors(cube.cpu().numpy()[c, l, n], ref)
    assert rel <= GATE_MFMA and mx <= GATE_MFMA


def test_invalid_arguments():
    import ctypes
    rs = _rs()
    bad = rs.scene_struct(scenes.Room(W=4.0, D=5.0), scenes.Pedestrian(centre=np.array([0, 2.0, 0]),
                                                                       velocity=np.zeros(3),
                                                                       semi_axes=np.array([0.2, 0.0, 0.8])))
    with pytest.raises(rs.RSError) as e:
        rs.rs_render_scenes([bad], 8, 8)
    assert e.value.status == rs.RS_E_INVALID
