"""NUFFT form on the GPU: against the NUFFT oracle (same kernel, grid and
modes; differences are float32 rounding) and against the exact direct sum
(differences are the tolerance plus that rounding).

Gates.  The float32 path rounds each strength and weight (2^-24 relative),
sums up to a few hundred weighted points per grid cell and runs two float32
FFTs of log2(n) <= 12 radix-2 stages; with errors adding in quadrature that
is a few 1e-7 relative L2, so 2e-6 against the NUFFT oracle leaves a
margin of several times.  Against the exact sum the gate is the tolerance
plus that float32 term."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import nufft as onufft
from paper_2307_09226_amd import scenes
from gpu_util import errors, sample_indices

pytestmark = pytest.mark.gpu

GATE_FP32 = 2e-6


def _rs():
    from paper_2307_09226_amd import rs
    return rs


def _synth(r, px, tol, dtype=0, ws=False):
    import torch
    rs = _rs()
    plan = rs.rs_cube_plan_nufft(r, dtype, max_pixels=max(px.P, 1), tolerance=tol)
    cube = rs.new_cube(plan)
    dpx = rs.DevicePixels.from_host(px)
    if ws:
        buf = torch.empty(max(plan.workspace_bytes(px.P), 1), dtype=torch.uint8, device="cuda:0")
        rs.rs_beat_synthesize_ws(plan, dpx, cube, buf)
    else:
        rs.rs_beat_synthesize(plan, dpx, cube)
    torch.cuda.synchronize()
    out = cube.cpu().numpy()
    plan.close()
    return out


RADARS = {
    "odd": lambda: scenes.radar_for(2, 3, 37, 11, Fs=10e6, Tb=120e-6),
    "ragged": lambda: scenes.radar_for(3, 2, 72, 40, Fs=10e6, Tb=120e-6),
    "frame_shape": lambda: scenes.radar_for(3, 4, 256, 128, Fs=10e6, Tb=120e-6),
}


@pytest.mark.parametrize("name", list(RADARS))
@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-6])
def test_against_nufft_oracle_and_exact(name, tol):
    r = RADARS[name]()
    px = scenes.tiny_scene(400 + len(name), 2500, vmax=6.0)
    got = _synth(r, px, tol)
    ref_nu = onufft.nufft_cube(r, px, tol)
    ref = oracle.cube(r, px)
    rel_nu, _ = errors(got, ref_nu)
    rel, mx = errors(got, ref)
    print(f"nufft {name} tol={tol:g}: vs NUFFT oracle {rel_nu:.2e}, vs exact {rel:.2e} (max {mx:.2e})",
          flush=True)
    assert rel_nu <= GATE_FP32
    assert rel <= tol + GATE_FP32


@pytest.mark.parametrize("model,carrier", [(15, 1), (1, 1), (1, 0), (2 | 4 | 8, 1)])
def test_variants_and_complex128(model, carrier):
    r = dataclasses.replace(RADARS["ragged"](), model=model, carrier_phase=carrier)
    px = scenes.tiny_scene(420 + model, 1500, vmax=6.0)
    got = _synth(r, px, 1e-5, dtype=1, ws=True)
    assert got.dtype == np.complex128
    rel, _ = errors(got, oracle.cube(r, px))
    rel_nu, _ = errors(got, onufft.nufft_cube(r, px, 1e-5))
    print(f"nufft model={model} carrier={carrier}: vs exact {rel:.2e}, vs NUFFT oracle {rel_nu:.2e}", flush=True)
    assert rel_nu <= GATE_FP32 and rel <= 1e-5 + GATE_FP32


def test_points_across_the_grid_and_its_edge():
    """Points spread over every frequency, several beyond Nyquist (wrapped):
    the blocks' bounding boxes are wider than the grid and the weights go
    straight to it; beat frequencies at +-1/2 cycle straddle its periodic
    edge."""
    rng = np.random.default_rng(430)
    r = RADARS["ragged"]()
    P = 5000
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    Kb = 2 * r.mu / (r.c0 * r.Fs)
    rr = rng.uniform(0.3, 1.2 / Kb, P)           # beat frequencies 0 .. 1.2 cycles
    az = rng.uniform(-1.0, 1.0, P)
    px = scenes.Pixels(f32(rr * np.sin(az)), f32(rr * np.cos(az)), f32(rng.uniform(-1, 1, P)),
                       f32(rng.lognormal(0, 0.5, P)), f32(rng.uniform(-9, 9, P)))
    got = _synth(r, px, 1e-6)
    rel_nu, _ = errors(got, onufft.nufft_cube(r, px, 1e-6))
    rel, _ = errors(got, oracle.cube(r, px))
    print(f"nufft spread-out points: vs NUFFT oracle {rel_nu:.2e}, vs exact {rel:.2e}", flush=True)
    assert rel_nu <= GATE_FP32 and rel <= 1e-6 + GATE_FP32


def test_frame_sampled():
    """The 65,536-pixel frame (3 x 4, Ns 256, L 128) at tolerance 1e-6:
    sampled entries against the exact sum."""
    radar, px = scenes.workload_frame()
    got = _synth(radar, px, 1e-6)
    c, l, n = sample_indices(radar.cube_shape(), 300, seed=12)
    rel, mx = errors(got[c, l, n], oracle.entries(radar, px, c, l, n))
    print(f"nufft frame: relL2 {rel:.2e} maxabs {mx:.2e}", flush=True)
    assert rel <= 1e-6 + GATE_FP32


def test_edge_sizes_and_refusals():
    """P = 0 gives an exact zero cube; one pixel and a pixel count that
    leaves a partial block match the oracle; sessions and strengths per
    block are refused."""
    import ctypes
    import torch
    rs = _rs()
    r = RADARS["odd"]()
    empty = scenes.Pixels(*(np.zeros(0, np.float32) for _ in range(5)))
    assert np.all(_synth(r, empty, 1e-6) == 0)
    for P in (1, 2049):
        px = scenes.tiny_scene(440 + P, P, vmax=5.0)
        rel, _ = errors(_synth(r, px, 1e-6), oracle.cube(r, px))
        assert rel <= 1e-6 + GATE_FP32, (P, rel)
    plan = rs.rs_cube_plan_nufft(r, 0, max_pixels=10, tolerance=1e-4)
    d = rs.DevicePixels.from_host(scenes.tiny_scene(450, 10))
    cubes = rs.new_cube(plan, count=2)
    sess = rs.Session(hbm_budget=1 << 28, max_slots=1)
    with pytest.raises(rs.RSError) as e:
        sess.submit(plan, d, cubes[0])
    assert e.value.status == rs.RS_E_UNSUPPORTED
    sess.close()
    torch.cuda.synchronize()
    st, keep = rs._radar_struct(dataclasses.replace(r, model=16))
    h = ctypes.c_void_p()
    assert rs.lib.rs_cube_plan_nufft(ctypes.byref(st), 0, 10, 1e-6, ctypes.byref(h)) == rs.RS_E_UNSUPPORTED
    assert "NUFFT" in plan.describe(10) or "nufft" in plan.describe(10)


def test_more_blocks_than_one_coverage_pass():
    """600,000 pixels (2,344 blocks of 256, more than the 1,024 blocks one
    coverage pass of the assembly lists) on a small radar: the cube still
    matches the NUFFT oracle and the exact sum."""
    rng = np.random.default_rng(460)
    z = np.zeros((1, 3))
    r = scenes.Radar(M=1, N=1, Ns=16, L=8, fc=77e9, mu=30e12, Fs=10e6, Tb=120e-6, tx=z, rx=z.copy())
    P = 600_000
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    rr = rng.uniform(1.0, 6.0, P)
    az = rng.uniform(-1.0, 1.0, P)
    px = scenes.Pixels(f32(rr * np.sin(az)), f32(rr * np.cos(az)), f32(rng.uniform(-1, 1, P)),
                       f32(rng.lognormal(0, 0.5, P)), f32(np.where(rng.random(P) < 0.9, 0.0, rng.uniform(-2, 2, P))))
    got = _synth(r, px, 1e-6)
    rel_nu, _ = errors(got, onufft.nufft_cube(r, px, 1e-6))
    rel, _ = errors(got, oracle.cube(r, px))
    print(f"nufft 600k pixels: vs NUFFT oracle {rel_nu:.2e}, vs exact {rel:.2e}", flush=True)
    assert rel_nu <= GATE_FP32 and rel <= 1e-6 + GATE_FP32


def _two_group_scene(r, P, seed):
    """Pixels whose blocks of 256 each hold static scatterers (v = 0) and
    moving ones in a narrow Doppler band a quarter cycle away, ranges rising
    slowly with the index (as along an image row): every block's box is
    tall, and its start rows fall into two groups a wide gap apart."""
    rng = np.random.default_rng(seed)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    Kd = 2 * r.fc * r.Tb / r.c0                       # cycles per block per (m/s)
    rr = 1.0 + 5.0 * np.arange(P) / P + rng.uniform(0, 0.02, P)
    az = rng.uniform(-0.5, 0.5, P)
    v = np.where(np.arange(P) % 2 == 0, 0.0, (0.25 + 30.0) / Kd + rng.uniform(-2e-4, 2e-4, P))
    return scenes.Pixels(f32(rr * np.sin(az)), f32(rr * np.cos(az)), f32(rng.uniform(-0.3, 0.3, P)),
                         f32(rng.lognormal(0, 0.5, P)), f32(v))


def _split_blocks(r, px, tol):
    """Blocks (of channel 0) whose box is taller than 16 rows and whose start
    rows split at the widest gap into two groups of at most 16 rows each."""
    w, _ = onufft.es_params(tol)
    n2 = onufft.fine_size(r.L, w)
    _, _, beta = oracle.default().chan_args(r, px, 0)
    v = -beta - np.rint(-beta)
    m2 = np.ceil(v * n2 - w / 2.0).astype(np.int64)
    count = 0
    for b0 in range(0, px.P, 256):
        rows = np.unique(m2[b0:b0 + 256])
        if rows[-1] - rows[0] + w <= 16:
            continue
        k = int(np.argmax(np.diff(rows)))
        if rows[k] - rows[0] + w <= 16 and rows[-1] - rows[k + 1] + w <= 16:
            count += 1
    return count, (px.P + 255) // 256


@pytest.mark.parametrize("name", ["ragged", "frame_shape"])
@pytest.mark.parametrize("tol", [1e-2, 1e-6])
def test_blocks_split_into_two_sub_boxes(name, tol):
    """Blocks mixing static and moving scatterers: their tall boxes are split
    into two sub-boxes; the cube still matches the NUFFT oracle and the exact
    sum, and a second run gives the same bits."""
    r = RADARS[name]()
    px = _two_group_scene(r, 2048 + 77, seed=470)
    split, nblk = _split_blocks(r, px, tol)
    assert split == nblk, (split, nblk)              # the scene exercises the split in every block
    got = _synth(r, px, tol)
    again = _synth(r, px, tol)
    rel_nu, _ = errors(got, onufft.nufft_cube(r, px, tol))
    rel, _ = errors(got, oracle.cube(r, px))
    print(f"nufft two groups {name} tol={tol:g}: vs NUFFT oracle {rel_nu:.2e}, vs exact {rel:.2e}", flush=True)
    assert np.array_equal(got, again)
    assert rel_nu <= GATE_FP32 and rel <= tol + GATE_FP32


def test_largest_serving_request_sampled():
    """The largest serving-size request (12 x 16 channels, N_s 512, 234,256
    pixels; a quarter of its blocks take the two-sub-box split) at tolerance
    1e-6: sampled entries against the exact sum."""
    big = max((q for q in scenes.serving_requests(48) if q.radar.C == 192),
              key=lambda q: q.pixels.P * q.radar.Ns * q.radar.L)
    got = _synth(big.radar, big.pixels, 1e-6)
    c, l, n = sample_indices(big.radar.cube_shape(), 128, seed=13)
    rel, mx = errors(got[c, l, n], oracle.entries(big.radar, big.pixels, c, l, n))
    print(f"nufft largest request: relL2 {rel:.2e} maxabs {mx:.2e}", flush=True)
    assert rel <= 1e-6 + GATE_FP32
    # every box fits a tile slot (after the splits): the sums have a fixed order
    assert np.array_equal(got, _synth(big.radar, big.pixels, 1e-6))


def test_boxes_wider_than_the_gathered_columns():
    """A radar with N_s 512 (grid 1024 columns) and blocks whose points span
    about 640 window columns: wider than the 512 columns a block gathers, not
    wider than the grid; their weights go to the grid with atomics."""
    rng = np.random.default_rng(480)
    z = np.zeros((1, 3))
    r = scenes.Radar(M=1, N=1, Ns=512, L=16, fc=77e9, mu=30e12, Fs=10e6, Tb=120e-6, tx=z, rx=z.copy())
    P = 1024
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    Kb = 2 * r.mu / (r.c0 * r.Fs)
    # beat frequencies 0.7 .. 1.3 cycles per sample (1.33 for odd pixels):
    # reduced to -0.3 .. 0.33 around 0: 637-641 columns per block
    span = np.where(np.arange(P) % 2 == 0, 0.6, 0.63)
    rr = (0.7 + rng.uniform(0.0, 1.0, P) * span) / Kb
    px = scenes.Pixels(f32(rr), f32(np.zeros(P)), f32(np.zeros(P)), f32(rng.lognormal(0, 0.5, P)),
                       f32(rng.uniform(-0.02, 0.02, P)))
    got = _synth(r, px, 1e-6)
    rel_nu, _ = errors(got, onufft.nufft_cube(r, px, 1e-6))
    rel, _ = errors(got, oracle.cube(r, px))
    print(f"nufft wide boxes: vs NUFFT oracle {rel_nu:.2e}, vs exact {rel:.2e}", flush=True)
    assert rel_nu <= GATE_FP32 and rel <= 1e-6 + GATE_FP32


def test_batch_equals_single_frames_bitwise():
    """Frames of different pixel counts (room+pedestrian renders: every box
    fits its tile slot, so the sums have a fixed order; one frame empty, one
    a partial block) through one batched call give each frame's single-call
    cube bit for bit, in complex64 and complex128."""
    import torch
    rs = _rs()
    r, full = scenes.workload_frame()
    frames = [full.take(np.arange(9000)), scenes.Pixels(*(np.zeros(0, np.float32) for _ in range(5))),
              full.take(np.arange(30000, 30077)), full]
    for dtype in (0, 1):
        plan = rs.rs_cube_plan_nufft(r, dtype, max_pixels=max(f.P for f in frames), tolerance=1e-5)
        dev = [rs.DevicePixels.from_host(f) for f in frames]
        cubes = rs.new_cube(plan, count=len(frames))
        cubes.fill_(complex(5.0, 5.0))
        rs.rs_beat_synthesize_batch(plan, dev, cubes)
        for i, d in enumerate(dev):
            one = rs.new_cube(plan)
            rs.rs_beat_synthesize(plan, d, one)
            torch.cuda.synchronize()
            assert torch.equal(cubes[i], one), (dtype, i)
        assert torch.all(cubes[1] == 0)
        rel, _ = errors(cubes[2].cpu().numpy(), oracle.cube(r, frames[2]))
        assert rel <= 1e-5 + GATE_FP32
        plan.close()
