"""Plain form (binary64 on the vector ALUs) against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2307_09226_amd import scenes
from gpu_util import (GATE_PLAIN_C128, GATE_PLAIN_C64, GATE_PLAIN_C64_MAX, errors,
                      sample_indices, synth)

pytestmark = pytest.mark.gpu


def _rs():
    from paper_2307_09226_amd import rs
    return rs


def test_small_workload_full_cube_c128():
    """64x64 room pixels, 2x4 array, Ns=64, L=32, v=0: the whole cube."""
    rs = _rs()
    radar, px = scenes.workload_small()
    ref = oracle.cube(radar, px)
    got = synth(radar, px, rs.RS_FORM_FP64_DIRECT, rs.RS_C128)
    rel, mx = errors(got, ref)
    print(f"small c128 relL2={rel:.3e} maxabs={mx:.3e}")
    assert rel <= GATE_PLAIN_C128 and mx <= GATE_PLAIN_C128
    # v = 0 everywhere: identical slow-time slices, as in the oracle
    assert np.all(got == got[:, :1, :])


@pytest.mark.parametrize("shape", [(1, 3, 50, 7), (2, 2, 130, 70), (3, 1, 17, 129)])
def test_ragged_tiles_full_cube(shape):
    """Sizes that leave ragged tails in every tile dimension and the pixel chunks."""
    rs = _rs()
    M, N, Ns, L = shape
    radar = scenes.radar_for(M, N, Ns, L, Fs=10e6, Tb=M * 40e-6)
    px = scenes.tiny_scene(7 + Ns, 1237)
    ref = oracle.cube(radar, px)
    got = synth(radar, px, rs.RS_FORM_FP64_DIRECT, rs.RS_C128)
    rel, mx = errors(got, ref)
    assert rel <= GATE_PLAIN_C128 and mx <= GATE_PLAIN_C128, (rel, mx)


def test_frame_workload_sampled_c128_and_c64():
    """256x256 room + pedestrian, 3x4 array, Ns=256, L=128: sampled entries
    (direct sums in the oracle) and both closed-form marginals over the
    whole cube."""
    rs = _rs()
    radar, px = scenes.workload_frame()
    c, l, n = sample_indices(radar.cube_shape(), 1500, seed=3)
    ref = oracle.entries(radar, px, c, l, n)
    got = synth(radar, px, rs.RS_FORM_FP64_DIRECT, rs.RS_C128)
    rel, mx = errors(got[c, l, n], ref)
    print(f"frame c128 sampled relL2={rel:.3e} maxabs={mx:.3e}")
    assert rel <= GATE_PLAIN_C128 and mx <= GATE_PLAIN_C128
    mn = oracle.marginal_n(radar, px)
    ml = oracle.marginal_l(radar, px)
    assert errors(got.sum(axis=2), mn)[0] <= GATE_PLAIN_C128
    assert errors(got.sum(axis=1), ml)[0] <= GATE_PLAIN_C128
    got64 = synth(radar, px, rs.RS_FORM_FP64_DIRECT, rs.RS_C64)
    rel, mx = errors(got64[c, l, n], ref)
    assert rel <= GATE_PLAIN_C64 and mx <= GATE_PLAIN_C64_MAX
    # complex64 output is the rounded complex128 output
    assert np.array_equal(got64, got.astype(np.complex64))


def test_single_scatterer_no_carrier():
    rs = _rs()
    radar = scenes.radar_for(1, 4, 64, 16, Fs=5e6, Tb=40e-6, carrier_phase=0)
    px = scenes.tiny_scene(1, 1)
    ref = oracle.cube(radar, px)
    got = synth(radar, px, rs.RS_FORM_FP64_DIRECT, rs.RS_C128)
    assert errors(got, ref)[0] <= GATE_PLAIN_C128
