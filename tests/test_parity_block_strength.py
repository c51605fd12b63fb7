"""Strength per TDM block (eq. (1)'s sigma varying with the block l, flag 16)
on the GPU against the CPU oracle: both forms, ragged tiles, the frame
workload, batched frames and the serving loop."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2307_09226_amd import scenes
from gpu_util import (GATE_MFMA, GATE_PLAIN_C128, GATE_PLAIN_C64, GATE_PLAIN_C64_MAX, errors,
                      sample_indices, synth)

pytestmark = pytest.mark.gpu

BS = 16


def _rs():
    from paper_2307_09226_amd import rs
    return rs


def _radar(model=BS):
    # Ns = 72 and L = 40 leave ragged n and l tiles
    r = scenes.radar_for(3, 2, 72, 40, Fs=10e6, Tb=120e-6)
    return dataclasses.replace(r, model=model)


def _scene(seed, P, L):
    return scenes.block_strengths(scenes.tiny_scene(seed, P, vmax=6.0), L, seed=seed + 1000, depth=0.8)


@pytest.mark.parametrize("model", [BS, 31])
def test_plain_c128_full_cube(model):
    rs = _rs()
    r = _radar(model)
    px = _scene(160 + model, 517, r.L)
    ref = oracle.cube(r, px)
    got = synth(r, px, rs.RS_FORM_FP64_DIRECT, rs.RS_C128)
    rel, mx = errors(got, ref)
    print(f"plain block-strength model={model} relL2={rel:.3e} maxabs={mx:.3e}", flush=True)
    assert rel <= GATE_PLAIN_C128 and mx <= GATE_PLAIN_C128


def test_plain_c64_full_cube():
    rs = _rs()
    r = _radar()
    px = _scene(171, 333, r.L)
    ref = oracle.cube(r, px)
    got = synth(r, px, rs.RS_FORM_FP64_DIRECT, rs.RS_C64)
    rel, mx = errors(got, ref)
    print(f"plain c64 block-strength relL2={rel:.3e} maxabs={mx:.3e}", flush=True)
    assert rel <= GATE_PLAIN_C64 and mx <= GATE_PLAIN_C64_MAX


@pytest.mark.parametrize("model", [BS, 31])
def test_mfma_full_cube(model):
    rs = _rs()
    r = _radar(model)
    px = _scene(180 + model, 2111, r.L)
    ref = oracle.cube(r, px)
    got = synth(r, px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64)
    rel, mx = errors(got, ref)
    print(f"mfma block-strength model={model} relL2={rel:.3e} maxabs={mx:.3e}", flush=True)
    assert rel <= GATE_MFMA and mx <= GATE_MFMA


def test_mfma_frame_sampled():
    """The 65,536-pixel frame (3 x 4, Ns 256, L 128) with strengths per block,
    in the headline launch configuration: sampled entries against the
    oracle."""
    rs = _rs()
    radar, px0 = scenes.workload_frame()
    r = dataclasses.replace(radar, model=BS)
    px = scenes.block_strengths(px0, r.L, seed=7)
    got = synth(r, px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64)
    c, l, n = sample_indices(r.cube_shape(), 300, seed=11)
    ref = oracle.entries(r, px, c, l, n)
    rel, mx = errors(got[c, l, n], ref)
    print(f"mfma frame block-strength relL2={rel:.3e} maxabs={mx:.3e}", flush=True)
    assert rel <= GATE_MFMA and mx <= GATE_MFMA


def test_batch_and_session_bitwise():
    """Batched frames with strengths per block equal single calls bitwise;
    in the serving loop a request with strengths per block and one without
    share launches, and each cube equals its single call bitwise."""
    import time
    import torch
    rs = _rs()
    r = _radar()
    frames = [_scene(190 + i, 300 + 410 * i, r.L) for i in range(3)]
    plan = rs.rs_cube_plan(r, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=max(f.P for f in frames))
    cubes = rs.new_cube(plan, count=3)
    rs.rs_beat_synthesize_batch(plan, [rs.DevicePixels.from_host(f) for f in frames], cubes)
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        assert np.array_equal(cubes[i].cpu().numpy(), synth(r, f, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64)), i

    rf = scenes.radar_for(3, 4, 256, 128, Fs=10e6, Tb=120e-6)
    reqs = [(dataclasses.replace(rf, model=BS), scenes.block_strengths(scenes.tiny_scene(201, 9000), 128, seed=202)),
            (rf, scenes.tiny_scene(203, 7000))]
    plans = [rs.rs_cube_plan(q, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=p.P) for q, p in reqs]
    dpx = [rs.DevicePixels.from_host(p) for _, p in reqs]
    alone = []
    for p, d in zip(plans, dpx):
        c = rs.new_cube(p)
        rs.rs_beat_synthesize(p, d, c)
        alone.append(c)
    torch.cuda.synchronize()
    sess = rs.Session(hbm_budget=2 << 30, max_slots=4, slice_items=200)
    outs = [rs.new_cube(p) for p in plans]
    tickets = [sess.submit(p, d, c) for p, d, c in zip(plans, dpx, outs)]
    t0 = time.time()
    while time.time() - t0 < 60:
        states = [sess.poll(t)[0] for t in tickets]
        if all(s in (rs.RS_REQ_DONE, rs.RS_REQ_FAILED) for s in states):
            break
        time.sleep(0.002)
    assert all(s == rs.RS_REQ_DONE for s in states), states
    for i, (a, b) in enumerate(zip(alone, outs)):
        assert torch.equal(a, b), i
    q, p = reqs[0]
    c, l, n = sample_indices(q.cube_shape(), 100, seed=3)
    rel, mx = errors(outs[0].cpu().numpy()[c, l, n], oracle.entries(q, p, c, l, n))
    assert rel <= GATE_MFMA and mx <= GATE_MFMA
    sess.close()


def test_binding_checks_strength_rows():
    """The binding refuses strengths of the wrong length for the plan before
    anything reaches the library."""
    rs = _rs()
    r = _radar()
    px = scenes.tiny_scene(210, 64)
    plan = rs.rs_cube_plan(r, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=64)
    cube = rs.new_cube(plan)
    with pytest.raises(ValueError):
        rs.rs_beat_synthesize(plan, rs.DevicePixels.from_host(px), cube)
    plain = rs.rs_cube_plan(_radar(0), rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=64)
    with pytest.raises(ValueError):
        rs.rs_beat_synthesize(plain, rs.DevicePixels.from_host(scenes.block_strengths(px, r.L, 1)), cube)
