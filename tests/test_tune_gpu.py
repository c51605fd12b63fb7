"""Tile tuning by measurement (rs_plan_tune): the chosen shape is one the
library builds, the plan describes it, and cubes computed with it still
match the oracle."""
import json

import numpy as np
import pytest

import oracle
from paper_2307_09226_amd import scenes
from gpu_util import GATE_MFMA, errors, sample_indices

pytestmark = pytest.mark.gpu

SHAPES = {"64x128x4", "32x128x4", "32x128x8", "32x64x4", "32x64x8", "64x64x4", "64x64x8", "128x64x4",
          # the 8-wave shapes with the software-pipelined schedule
          "32x128x8i", "32x64x8i", "64x64x8i"}


def _tile_of(desc):
    """Configuration string of a plan description."""
    pipe = desc["waves"] == 8 and desc["schedule"] == "pipelined"
    return f"{desc['wave_rows']}x{desc['tile_l']}x{desc['waves']}" + ("i" if pipe else "")


def test_tune_picks_a_built_shape_and_keeps_parity():
    import torch
    from paper_2307_09226_amd import rs
    radar = scenes.radar_for(3, 4, 256, 64, Fs=10e6, Tb=120e-6)
    px = scenes.tiny_scene(501, 9000, vmax=6.0)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=px.P)
    d = rs.DevicePixels.from_host(px)
    cube = rs.new_cube(plan)
    chosen = rs.rs_plan_tune(plan, d, cube, reps=2)
    print("tuned tile", chosen, flush=True)
    assert chosen in SHAPES
    desc = json.loads(plan.describe(px.P))
    assert _tile_of(desc) == chosen
    # the cube left by the tuning call and a fresh one both match the oracle
    c, l, n = sample_indices(radar.cube_shape(), 200, seed=5)
    ref = oracle.entries(radar, px, c, l, n)
    for got in (cube.cpu().numpy(), None):
        if got is None:
            out = rs.new_cube(plan)
            rs.rs_beat_synthesize(plan, d, out)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
        rel, mx = errors(got[c, l, n], ref)
        assert rel <= GATE_MFMA and mx <= GATE_MFMA


def test_tune_leaves_other_forms_alone():
    from paper_2307_09226_amd import rs
    radar = scenes.radar_small()
    px = scenes.tiny_scene(502, 100)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_FP64_DIRECT, rs.RS_C64, max_pixels=px.P)
    before = plan.describe(px.P)
    rs.rs_plan_tune(plan, rs.DevicePixels.from_host(px), rs.new_cube(plan), reps=1)
    assert plan.describe(px.P) == before


def test_tune_cache_miss_then_hit(tmp_path):
    """rs_plan_tune_cached: a miss tunes and appends one entry; a later plan
    with the same key takes the stored shape without launching anything and
    then computes the same bits; lines that do not parse or name a shape the
    library does not build are skipped; another pixel-count bucket misses."""
    import torch
    from paper_2307_09226_amd import rs
    radar = scenes.radar_for(3, 4, 256, 64, Fs=10e6, Tb=120e-6)
    px = scenes.tiny_scene(503, 9000, vmax=6.0)
    d = rs.DevicePixels.from_host(px)
    path = str(tmp_path / "tiles.txt")
    plan1 = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=px.P)
    cube1 = rs.new_cube(plan1)
    shape = rs.rs_plan_tune_cached(plan1, d, cube1, path, reps=2)
    assert shape in SHAPES
    lines = open(path).read().splitlines()
    assert lines == [f"12 256 64 16384 {shape}"]
    # noise after the entry: skipped
    with open(path, "a") as f:
        f.write("garbage line\n12 256 64 16384 48x128x8\n")
    plan2 = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=px.P)
    cube2 = rs.new_cube(plan2)
    cube2.fill_(complex(3.0, -1.0))
    assert rs.rs_plan_tune_cached(plan2, d, cube2, path, reps=2) == shape
    torch.cuda.synchronize()
    assert torch.all(cube2 == complex(3.0, -1.0))          # a hit launches nothing
    desc = json.loads(plan2.describe(px.P))
    assert _tile_of(desc) == shape
    rs.rs_beat_synthesize(plan2, d, cube2)
    torch.cuda.synchronize()
    assert torch.equal(cube1, cube2)
    assert len(open(path).read().splitlines()) == 3
    # 20,000 pixels fall in the next bucket: a miss, one more entry
    px3 = scenes.tiny_scene(504, 20000, vmax=6.0)
    plan3 = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=px3.P)
    s3 = rs.rs_plan_tune_cached(plan3, rs.DevicePixels.from_host(px3), rs.new_cube(plan3), path, reps=1)
    assert open(path).read().splitlines()[-1] == f"12 256 64 32768 {s3}"
    for p in (plan1, plan2, plan3):
        p.close()


@pytest.mark.parametrize("model", [0, 16])
def test_every_tile_shape_full_cube(tmp_path, model):
    """Each tile configuration the library builds (both schedules of the
    8-wave shapes), forced through the tile cache, on a radar whose n and l
    axes leave ragged tiles for every shape: the full cube matches the
    oracle, a second run gives the same bits, and the two schedules of an
    8-wave shape give the same bits (a missing barrier or a wrong tail guard
    in one shape shows up here)."""
    import dataclasses
    import torch
    from paper_2307_09226_amd import rs
    radar = dataclasses.replace(scenes.radar_for(2, 2, 130, 70, Fs=10e6, Tb=80e-6), model=model)
    px = scenes.tiny_scene(505, 2333, vmax=6.0)
    if model & 16:
        px = scenes.block_strengths(px, radar.L, seed=6)
    ref = oracle.cube(radar, px)
    d = rs.DevicePixels.from_host(px)
    first = {}
    for shape in sorted(SHAPES):
        path = str(tmp_path / f"tiles_{shape}.txt")
        with open(path, "w") as f:
            f.write(f"4 130 70 4096 {shape}\n")
        plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=px.P)
        cube = rs.new_cube(plan)
        assert rs.rs_plan_tune_cached(plan, d, cube, path, reps=1) == shape
        rs.rs_beat_synthesize(plan, d, cube)
        again = rs.new_cube(plan)
        rs.rs_beat_synthesize(plan, d, again)
        torch.cuda.synchronize()
        got = cube.cpu().numpy()
        rel, mx = errors(got, ref)
        print(f"tile {shape} model={model}: relL2 {rel:.2e} maxabs {mx:.2e}", flush=True)
        assert rel <= GATE_MFMA and mx <= GATE_MFMA, shape
        assert torch.equal(cube, again), shape
        # the two schedules of one shape chunk the pixels alike: same bits
        base = shape.rstrip("i")
        if base in first:
            assert torch.equal(cube, first[base]), shape
        first[base] = cube
        plan.close()


def test_set_tile_and_refusals():
    """rs_plan_set_tile takes every built configuration (the plan describes
    it) and refuses strings that are not one, leaving the plan unchanged;
    plans of the other forms refuse it."""
    import json
    from paper_2307_09226_amd import rs
    radar = scenes.radar_frame()
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=1000)
    assert json.loads(plan.describe(1000))["schedule"] == "phase_shifted"   # the rule's 32x128x8
    for t in sorted(SHAPES):
        rs.rs_plan_set_tile(plan, t)
        assert _tile_of(json.loads(plan.describe(1000))) == t
    rs.rs_plan_set_tile(plan, "64x64x4i")                                    # accepted, no effect
    assert _tile_of(json.loads(plan.describe(1000))) == "64x64x4"
    for bad in ("48x128x8", "32x128x8x", "32x128", "", "32x128x8j", "64x128x8"):
        with pytest.raises(rs.RSError) as e:
            rs.rs_plan_set_tile(plan, bad)
        assert e.value.status == rs.RS_E_INVALID
    assert _tile_of(json.loads(plan.describe(1000))) == "64x64x4"
    pplan = rs.rs_cube_plan(scenes.radar_small(), rs.RS_FORM_FP64_DIRECT, rs.RS_C64, max_pixels=10)
    with pytest.raises(rs.RSError) as e:
        rs.rs_plan_set_tile(pplan, "32x128x8")
    assert e.value.status == rs.RS_E_UNSUPPORTED
    plan.close()
    pplan.close()
