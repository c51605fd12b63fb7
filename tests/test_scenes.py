"""The seeded input generator: reproducibility and geometric sanity."""
import math

import numpy as np

from paper_2307_09226_amd import scenes


def test_seed_reproducible():
    a = scenes.scene_small(seed=1, grid=32, pedestrian=True)
    b = scenes.scene_small(seed=1, grid=32, pedestrian=True)
    for f in ("x", "y", "z", "amp", "vr"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = scenes.scene_small(seed=2, grid=32, pedestrian=True)
    assert not np.array_equal(a.amp, c.amp)


def test_float32_soa():
    px = scenes.scene_small(seed=0, grid=16)
    for f in ("x", "y", "z", "amp", "vr"):
        a = getattr(px, f)
        assert a.dtype == np.float32 and a.flags.c_contiguous and a.shape == (256,)


def test_room_hits_inside_room():
    rng = np.random.default_rng(0)
    room = scenes.draw_room(rng)
    px = scenes.render(rng, room, None, 40, 30)
    eps = 1e-4
    assert np.all(np.abs(px.x) <= room.W / 2 + eps)
    assert np.all((px.y >= -eps) & (px.y <= room.D + eps))
    assert np.all(np.abs(px.z) <= room.H / 2 + eps)
    # every wall pixel lies on one of the five visible planes
    on = ((np.abs(np.abs(px.x) - room.W / 2) < 1e-4) | (np.abs(px.y - room.D) < 1e-4)
          | (np.abs(np.abs(px.z) - room.H / 2) < 1e-4))
    assert np.all(on)
    assert np.all(px.vr == 0) and np.all(px.amp > 0)


def test_pixel_grid_directions():
    px = scenes.scene_small(seed=0, grid=8)
    pos = np.stack([px.x, px.y, px.z], 1).astype(np.float64)
    u = pos / np.linalg.norm(pos, axis=1, keepdims=True)
    az = np.degrees(np.arctan2(u[:, 0], u[:, 1]))
    el = np.degrees(np.arcsin(u[:, 2]))
    want_az = -60 + 120 * (np.arange(8) + 0.5) / 8
    want_el = -30 + 60 * (np.arange(8) + 0.5) / 8
    assert np.allclose(az.reshape(8, 8), want_az[None, :], atol=1e-4)
    assert np.allclose(el.reshape(8, 8), want_el[:, None], atol=1e-4)


def test_pedestrian_occludes_and_moves():
    rng = np.random.default_rng(1)
    room = scenes.draw_room(rng)
    ped = scenes.draw_pedestrian(rng, room)
    px = scenes.render(rng, room, ped, 128, 128)
    assert px.is_ped.sum() > 0
    pos = np.stack([px.x, px.y, px.z], 1).astype(np.float64)
    # pedestrian pixels lie on the ellipsoid and in front of the wall behind
    q = (pos[px.is_ped] - ped.centre) / ped.semi_axes
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-5)
    # radial velocity is -(v . u), positive when approaching
    u = pos / np.linalg.norm(pos, axis=1, keepdims=True)
    want = -(u @ ped.velocity)
    assert np.allclose(px.vr[px.is_ped], want[px.is_ped], atol=1e-6)
    assert np.all(px.vr[~px.is_ped] == 0)
    assert 0.5 <= np.linalg.norm(ped.velocity) <= 1.5


def test_animation_counts_and_bounds():
    frames = scenes.animation_frames(seed=3, nframes=6)
    counts = [f.P for f in frames]
    assert all(2000 <= c <= 262144 for c in counts)
    again = scenes.animation_frames(seed=3, nframes=6)
    assert all(np.array_equal(a.amp, b.amp) for a, b in zip(frames, again))


def test_serving_mix():
    reqs = scenes.serving_requests(12)
    assert {(r.radar.M, r.radar.N) for r in reqs} <= {(1, 4), (3, 4), (12, 16)}
    for r in reqs:
        assert r.radar.Ns in (128, 256, 512) and r.radar.L in (64, 128, 256)
        assert math.isclose(r.radar.Fs, r.radar.Ns / 25.6e-6)
        assert 3000 <= r.pixels.P <= 262144
    t = scenes.poisson_arrivals(1000, 50.0)
    assert np.all(np.diff(t) > 0) and abs(1000 / t[-1] - 50) < 6


def test_ula_geometry():
    tx, rx = scenes.ula_geometry(2, 4, 0.004)
    assert np.allclose(rx[:, 0], [0, 0.002, 0.004, 0.006])
    assert np.allclose(tx[:, 0], [0, 0.008])  # Tx spacing 2 lambda for N = 4
    assert np.all(tx[:, 1:] == 0) and np.all(rx[:, 1:] == 0)
