"""Pins of the CPU range-Doppler oracle (Sec. III) against brute force,
closed forms and the physical ground truth of a moving scatterer."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import rd
from paper_2307_09226_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sec3_walking_scenario.json")


def brute_power(cube):
    """Double DFT written out term by term (tiny sizes only)."""
    C, L, Ns = cube.shape
    out = np.zeros((Ns, L))
    for k in range(Ns):
        for d in range(L):
            for c in range(C):
                s = 0j
                for l in range(L):
                    for n in range(Ns):
                        s += cube[c, l, n] * np.exp(-2j * np.pi * k * n / Ns) * np.exp(2j * np.pi * d * l / L)
                out[k, d] += abs(s) ** 2
    return out


def tone_cube(C, L, Ns, comps):
    """sum of a * exp(j2pi(psi + b n - beta l)) over comps = [(a, psi, b, beta)]."""
    n = np.arange(Ns)[None, None, :]
    l = np.arange(L)[None, :, None]
    y = np.zeros((C, L, Ns), dtype=np.complex128)
    for a, psi, b, beta in comps:
        y += a * np.exp(2j * np.pi * (psi + b * n - beta * l))
    return y


def check_brute_force(mod):
    rng = np.random.default_rng(0)
    cube = rng.normal(size=(2, 4, 8)) + 1j * rng.normal(size=(2, 4, 8))
    got = mod.range_doppler_power(cube)[0]
    want = brute_power(cube)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(want)


def check_single_tone(mod, k0, d0):
    """An on-bin tone lands in exactly one cell with power C a^2 (Ns L)^2; an
    approaching scatterer (beta > 0) has a positive Doppler bin."""
    C, L, Ns = 3, 16, 32
    a = 0.7
    cube = tone_cube(C, L, Ns, [(a, 0.3, k0 / Ns, d0 / L)])
    p = mod.range_doppler_power(cube)[0]
    k, d = mod.peaks(p[None], skip_static=False)
    assert k[0] == k0 % Ns and mod.signed_bin(d, L)[0] == d0
    assert p[k0 % Ns, d0 % L] == pytest.approx(C * a * a * (Ns * L) ** 2, rel=1e-12)
    rest = p.copy()
    rest[k0 % Ns, d0 % L] = 0
    assert rest.max() <= 1e-20 * p.max()


def check_parseval(mod):
    rng = np.random.default_rng(1)
    cube = rng.normal(size=(2, 3, 16, 8)) + 1j * rng.normal(size=(2, 3, 16, 8))
    p = mod.range_doppler_power(cube)
    for f in range(2):
        assert p[f].sum() == pytest.approx(16 * 8 * np.sum(np.abs(cube[f]) ** 2), rel=1e-12)


def check_skip_static_and_ties(mod):
    C, L, Ns = 2, 16, 16
    cube = tone_cube(C, L, Ns, [(1.0, 0.0, 4 / Ns, 3 / L), (10.0, 0.1, 9 / Ns, 0.0)])
    p = mod.range_doppler_power(cube)
    k, d = mod.peaks(p, skip_static=True)
    assert (k[0], d[0]) == (4, 3)
    k, d = mod.peaks(p, skip_static=False)
    assert (k[0], d[0]) == (9, 0)
    # equal maxima: the first in k L + d order wins
    tie = np.zeros((1, 4, 4))
    tie[0, 2, 1] = tie[0, 1, 3] = 5.0
    k, d = mod.peaks(tie, skip_static=True)
    assert (k[0], d[0]) == (1, 3)


def check_bin_conversions(mod):
    r = scenes.radar_for(1, 1, 64, 32, Fs=10e6, Tb=120e-6)
    # b = 2 mu R / (c0 Fs) = k / Ns  and  beta = 2 fc Tb v / c0 = d / L
    R = 7 * r.c0 * r.Fs / (2 * r.mu * r.Ns)
    v = -5 * r.c0 / (2 * r.fc * r.Tb * r.L)
    assert mod.bin_range(7, r) == pytest.approx(R, rel=1e-15)
    assert mod.bin_velocity(-5, r) == pytest.approx(v, rel=1e-15)
    assert 2 * r.mu * R / (r.c0 * r.Fs) * r.Ns == pytest.approx(7, rel=1e-12)
    assert 2 * r.fc * r.Tb * v / r.c0 * r.L == pytest.approx(-5, rel=1e-12)


def test_walking_speed_matches_the_paper():
    g = json.load(open(GOLDEN))
    cw = scenes.circle_walk(frame_ids=[0], grid=8)
    assert round(cw.speed, g["S_walk_decimals"]) == g["S_walk_mps"]
    assert cw.speed == pytest.approx(2 * np.pi * g["radius_m"] * g["fps"] / g["frames"], rel=1e-15)


def check_walk(mod, cubes, r, cw):
    p = mod.range_doppler_power(cubes)
    k, d = mod.peaks(p, skip_static=True)
    v_est = mod.bin_velocity(mod.signed_bin(d, r.L), r)
    dv = mod.bin_velocity(1, r)
    err = np.abs(v_est - cw.v_radial)
    assert np.all(err <= dv * (1 + 1e-9)), (v_est, cw.v_radial)  # bin 0 is skipped: v ~ 0 reads as +-1 bin
    assert mod.e_velo(v_est, cw.v_radial) <= 0.5 * dv
    # the peak's range bin holds the pedestrian
    rng_est = mod.bin_range(k, r)
    rng_true = np.linalg.norm(cw.centres, axis=1)
    assert np.all(np.abs(rng_est - rng_true) <= 2 * mod.bin_range(1, r))
    dt = mod.doppler_time(p, k)
    assert dt.shape == (len(cw.frames), r.L)
    assert np.all(dt[np.arange(len(k)), d] == p[np.arange(len(k)), k, d])


def check_e_velo(mod):
    """Sec. III: the mean over CPIs of |v_est - v_true| (errors of opposite
    sign do not cancel)."""
    assert mod.e_velo([1.0, -1.0, 0.5], [0.0, 0.0, 0.0]) == pytest.approx(2.5 / 3, rel=1e-15)
    assert mod.e_velo([3.0], [3.0]) == 0.0


_WALK = {}


def walk_inputs():
    """Every 11th frame of the 100-frame walk, small grid and array, and
    their oracle cubes (computed once)."""
    if not _WALK:
        r = scenes.radar_for(1, 4, 64, 32, Fs=10e6, Tb=120e-6)
        cw = scenes.circle_walk(frame_ids=range(3, 100, 11), grid=48)
        o = oracle.default()
        _WALK["v"] = (np.stack([o.cube(r, f) for f in cw.frames]), r, cw)
    return _WALK["v"]


CHECKS = [check_brute_force, lambda m: check_single_tone(m, 5, 3), lambda m: check_single_tone(m, 13, -6),
          check_parseval, check_skip_static_and_ties, check_bin_conversions, check_e_velo,
          lambda m: check_walk(m, *walk_inputs())]


def test_matches_brute_force_dft():
    check_brute_force(rd)


@pytest.mark.parametrize("k0,d0", [(5, 3), (0, 7), (13, -6), (31, -8)])
def test_single_tone_on_bin(k0, d0):
    check_single_tone(rd, k0, d0)


def test_parseval():
    check_parseval(rd)


def test_skip_static_and_ties():
    check_skip_static_and_ties(rd)


def test_bin_conversions_invert_the_signal_model():
    check_bin_conversions(rd)


def test_e_velo_definition():
    check_e_velo(rd)


def test_doppler_time_tracks_ground_truth():
    """Oracle synthesis of the walking scenario (every 11th frame of the
    100-frame walk, small grid and array), then range-Doppler maps: the
    max-power velocity of each CPI follows the pedestrian's radial velocity
    to within one Doppler bin, with the right sign."""
    check_walk(rd, *walk_inputs())
