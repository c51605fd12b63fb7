"""Signal-model variants (far field as eq. (2), Tx slot timing, Doppler within
the chirp, residual video phase) on the GPU against the CPU oracle.  The far
field runs both with the carrier phase (its far-field-limit reading) and
without it (eq. (2) as printed)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2307_09226_amd import scenes
from gpu_util import GATE_MFMA, GATE_PLAIN_C128, errors, synth

pytestmark = pytest.mark.gpu

# (model flags, carrier phase)
MODELS = [(1, 1), (1, 0), (2, 1), (4, 1), (8, 1), (15, 1), (15, 0)]
IDS = [f"model{m}-carrier{c}" for m, c in MODELS]


def _rs():
    from paper_2307_09226_amd import rs
    return rs


def _radar(model, carrier=1):
    r = scenes.radar_for(3, 2, 72, 40, Fs=10e6, Tb=120e-6, carrier_phase=carrier)
    return dataclasses.replace(r, model=model)


@pytest.mark.parametrize("model,carrier", MODELS, ids=IDS)
def test_plain_c128_full_cube(model, carrier):
    rs = _rs()
    r = _radar(model, carrier)
    px = scenes.tiny_scene(60 + model, 517, vmax=6.0)
    ref = oracle.cube(r, px)
    got = synth(r, px, rs.RS_FORM_FP64_DIRECT, rs.RS_C128)
    rel, mx = errors(got, ref)
    print(f"plain model={model} carrier={carrier} relL2={rel:.3e} maxabs={mx:.3e}")
    assert rel <= GATE_PLAIN_C128 and mx <= GATE_PLAIN_C128


@pytest.mark.parametrize("model,carrier", MODELS, ids=IDS)
def test_mfma_full_cube(model, carrier):
    rs = _rs()
    r = _radar(model, carrier)
    px = scenes.tiny_scene(70 + model, 2111, vmax=6.0)
    ref = oracle.cube(r, px)
    got = synth(r, px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64)
    rel, mx = errors(got, ref)
    print(f"mfma model={model} carrier={carrier} relL2={rel:.3e} maxabs={mx:.3e}")
    assert rel <= GATE_MFMA and mx <= GATE_MFMA


def test_variants_change_the_cube_and_batch_is_bitwise():
    """Each variant changes a moving scene's cube (it is not silently
    ignored), and batched frames equal single calls bitwise."""
    import torch
    rs = _rs()
    px = scenes.tiny_scene(81, 700, vmax=6.0)
    base = synth(_radar(0), px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64)
    for m in (1, 2, 4, 8):
        got = synth(_radar(m), px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64)
        assert np.linalg.norm(got - base) > 1e-3 * np.linalg.norm(base), m
    r = _radar(15)
    frames = [scenes.tiny_scene(90 + i, 300 + 250 * i, vmax=6.0) for i in range(3)]
    plan = rs.rs_cube_plan(r, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=max(f.P for f in frames))
    cubes = rs.new_cube(plan, count=3)
    rs.rs_beat_synthesize_batch(plan, [rs.DevicePixels.from_host(f) for f in frames], cubes)
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        assert np.array_equal(cubes[i].cpu().numpy(), synth(r, f, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64))


def test_unknown_model_flags_rejected():
    import ctypes
    rs = _rs()
    r = dataclasses.replace(scenes.radar_small(), model=32)
    st, keep = rs._radar_struct(r)
    h = ctypes.c_void_p()
    assert rs.lib.rs_cube_plan(ctypes.byref(st), 1, 0, 10, ctypes.byref(h)) == rs.RS_E_INVALID
    assert "model" in rs.rs_last_error()
