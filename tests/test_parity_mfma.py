"""Split-FP16 matrix-core form against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2307_09226_amd import scenes
from gpu_util import GATE_MFMA, errors, sample_indices, synth

pytestmark = pytest.mark.gpu


def _rs():
    from paper_2307_09226_amd import rs
    return rs


@pytest.mark.parametrize("shape", [
    (2, 4, 64, 32),    # small workload shape
    (1, 3, 50, 7),     # ragged n and l
    (2, 2, 130, 70),   # several n tiles, l tile 128 with tail
    (3, 1, 17, 129),   # two l tiles
    (1, 2, 512, 64),   # tall n
])
def test_full_cube_ragged(shape):
    rs = _rs()
    M, N, Ns, L = shape
    radar = scenes.radar_for(M, N, Ns, L, Fs=10e6, Tb=M * 40e-6)
    px = scenes.tiny_scene(11 + Ns, 2333)
    ref = oracle.cube(radar, px)
    got = synth(radar, px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64)
    rel, mx = errors(got, ref)
    print(f"mfma {shape} relL2={rel:.3e} maxabs={mx:.3e}")
    assert rel <= GATE_MFMA and mx <= GATE_MFMA


def test_small_workload_full_cube():
    rs = _rs()
    radar, px = scenes.workload_small()
    ref = oracle.cube(radar, px)
    for dtype in (rs.RS_C64, rs.RS_C128):
        got = synth(radar, px, rs.RS_FORM_MFMA_SPLIT16, dtype)
        rel, mx = errors(got, ref)
        assert rel <= GATE_MFMA and mx <= GATE_MFMA, (dtype, rel, mx)


def test_frame_workload_sampled_and_marginals():
    """The headline frame: 65,536 room+pedestrian pixels, 3x4, Ns=256, L=128."""
    rs = _rs()
    radar, px = scenes.workload_frame()
    got = synth(radar, px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64)
    c, l, n = sample_indices(radar.cube_shape(), 1500, seed=5)
    ref = oracle.entries(radar, px, c, l, n)
    rel, mx = errors(got[c, l, n], ref)
    print(f"frame mfma sampled relL2={rel:.3e} maxabs={mx:.3e}")
    assert rel <= GATE_MFMA and mx <= GATE_MFMA
    g = got.astype(np.complex128)
    rn, _ = errors(g.sum(axis=2), oracle.marginal_n(radar, px))
    rl, _ = errors(g.sum(axis=1), oracle.marginal_l(radar, px))
    print(f"frame mfma marginals relL2 n={rn:.3e} l={rl:.3e}")
    assert rn <= GATE_MFMA and rl <= GATE_MFMA


def test_single_scatterer_rank_one():
    rs = _rs()
    radar = scenes.radar_for(3, 4, 256, 128, Fs=10e6, Tb=120e-6)
    px = scenes.tiny_scene(2, 1)
    ref = oracle.cube(radar, px)
    got = synth(radar, px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64)
    rel, mx = errors(got, ref)
    assert rel <= GATE_MFMA and mx <= GATE_MFMA


def test_extreme_strength_span():
    """Strengths over 12 decades and tiny absolute values: the per-chunk
    power-of-two scaling keeps fp16 in range."""
    rs = _rs()
    radar = scenes.radar_for(1, 4, 64, 32, Fs=5e6, Tb=40e-6)
    px = scenes.tiny_scene(3, 3000)
    rng = np.random.default_rng(0)
    amp = (10.0 ** rng.uniform(-30, -18, px.P)).astype(np.float32)
    px = scenes.Pixels(px.x, px.y, px.z, amp, px.vr)
    ref = oracle.cube(radar, px)
    got = synth(radar, px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C128)
    rel, mx = errors(got, ref)
    assert rel <= GATE_MFMA and mx <= GATE_MFMA, (rel, mx)


def test_repeatable_bitwise():
    rs = _rs()
    radar = scenes.radar_for(2, 2, 128, 64, Fs=10e6, Tb=80e-6)
    px = scenes.tiny_scene(4, 5000)
    a = synth(radar, px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64)
    b = synth(radar, px, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, ws=True)
    assert np.array_equal(a, b)


def test_largest_serving_request_sampled():
    """The largest request shape of the serving mix (12 x 16 array, Ns 512,
    L 256, a 512 x 512-pixel frame): 192 channels, 6.6e12 terms, a 201 MB
    cube, alone and through a session, on sampled entries."""
    import torch
    rs = _rs()
    radar = scenes.radar_for(12, 16, 512, 256, Fs=512 / 25.6e-6, Tb=12 * 40e-6)
    px = scenes.scene_small(seed=9, grid=512, pedestrian=True)
    assert px.P == 512 * 512
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=px.P)
    dpx = rs.DevicePixels.from_host(px)
    cube = rs.new_cube(plan)
    rs.rs_beat_synthesize(plan, dpx, cube)
    torch.cuda.synchronize()
    c, l, n = sample_indices(radar.cube_shape(), 160, seed=9)
    got = cube[torch.as_tensor(c, device="cuda:0").long(), torch.as_tensor(l, device="cuda:0").long(),
               torch.as_tensor(n, device="cuda:0").long()].cpu().numpy()
    ref = oracle.entries(radar, px, c, l, n)
    rel, mx = errors(got, ref)
    print(f"largest request relL2={rel:.3e} maxabs={mx:.3e}")
    assert rel <= GATE_MFMA and mx <= GATE_MFMA
    sess = rs.Session(hbm_budget=2 << 30, max_slots=2)
    cube2 = rs.new_cube(plan)
    t = sess.submit(plan, dpx, cube2)
    sess.drain()
    assert sess.poll(t)[0] == rs.RS_REQ_DONE
    assert torch.equal(cube, cube2)
    sess.close()
