"""The NUFFT oracle against the exact direct sum and the kernel's own
mathematics; planted mistakes in a copy of its source must be caught.

The direct-sum oracle (pinned in test_oracle_pins.py) is the reference: a
type-1 NUFFT with an exponential-of-semicircle kernel of width w on a grid
oversampled at least twofold reaches a relative L2 error below the
tolerance it was sized for."""
import dataclasses
import importlib.util
import os

import numpy as np
import pytest

import oracle
from oracle import nufft
from paper_2307_09226_amd import scenes


def _relerr(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _odd_radar(model=0):
    # odd Ns and L: the centred modes floor(N/2) are exercised
    r = scenes.radar_for(2, 3, 37, 11, Fs=10e6, Tb=120e-6)
    return dataclasses.replace(r, model=model)


def pin_matches_exact_sum(nu):
    """Relative L2 error against the exact sum below the tolerance, for
    tolerances 1e-2 .. 1e-12, with and without the phase variants."""
    for model in (0, 15):
        r = _odd_radar(model)
        px = scenes.tiny_scene(301 + model, 400, vmax=6.0)
        ref = oracle.cube(r, px)
        for tol in (1e-2, 1e-4, 1e-6, 1e-9, 1e-12):
            err = _relerr(nu.nufft_cube(r, px, tol), ref)
            assert err < tol, (model, tol, err)


def pin_converges(nu):
    """Each extra digit of tolerance (one more kernel cell) cuts the error by
    at least 4x, down to 1e-13."""
    r = scenes.radar_for(3, 2, 64, 32, Fs=10e6, Tb=120e-6)
    px = scenes.tiny_scene(311, 300, vmax=6.0)
    ref = oracle.cube(r, px)
    errs = [_relerr(nu.nufft_cube(r, px, 10.0 ** -d), ref) for d in range(2, 13)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 4, errs


def pin_kernel_transform(nu):
    """phi_hat by quadrature equals a fine Riemann sum of phi(x) cos(k x) over
    its support (another route to the same integral), for several w, k."""
    for tol in (1e-3, 1e-6, 1e-10):
        w, beta = nu.es_params(tol)
        n = 128
        h = 2 * np.pi / n
        x = np.linspace(-w * h / 2, w * h / 2, 400001)
        dx = x[1] - x[0]
        phi = nu.es(x / h, w, beta)
        for k in (0, 1, 17, 40):
            want = float(np.sum(phi * np.cos(k * x)) * dx)
            got = float(nu.es_hat(np.array([k]), w, beta, n)[0])
            assert abs(got - want) < 1e-6 * abs(want), (tol, k, got, want)


def pin_wraps_at_nyquist(nu):
    """Beat frequencies and Doppler phases next to +-1/2 cycle (the grid's
    periodic edge) are spread across the wrap correctly: the error stays at
    the tolerance's scale (3 tol: three points do not average the error as a
    scene does); a wrap handled wrongly gives errors of order 1."""
    z = np.zeros((1, 3))
    r = scenes.Radar(M=1, N=1, Ns=32, L=16, fc=77e9, mu=30e12, Fs=10e6, Tb=120e-6, tx=z, rx=z.copy())
    Kb = 2 * r.mu / (r.c0 * r.Fs)              # cycles per sample per metre
    Kd = 2 * r.fc * r.Tb / r.c0                # cycles per block per (m/s)
    dists = [0.4995 / Kb, 0.5005 / Kb, 0.25 / Kb]
    vels = [0.4997 / Kd, -0.4997 / Kd, 0.5003 / Kd]
    f = lambda a: np.array(a, dtype=np.float32)
    px = scenes.Pixels(f([0.0, 0.0, 0.0]), f(dists), f([0.0, 0.0, 0.0]), f([1.0, 0.7, 1.3]), f(vels))
    ref = oracle.cube(r, px)
    for tol in (1e-4, 1e-9):
        assert _relerr(nu.nufft_cube(r, px, tol), ref) < 3 * tol


def pin_empty_and_unsupported(nu):
    """No pixels give an exact zero cube; strengths per block are refused."""
    r = _odd_radar()
    px = scenes.Pixels(*(np.zeros(0, np.float32) for _ in range(5)))
    assert np.all(nu.nufft_cube(r, px, 1e-6) == 0)
    rb = _odd_radar(16)
    with pytest.raises(ValueError):
        nu.nufft_cube(rb, scenes.block_strengths(scenes.tiny_scene(1, 5), rb.L, 2), 1e-6)


PINS = [pin_matches_exact_sum, pin_converges, pin_kernel_transform, pin_wraps_at_nyquist,
        pin_empty_and_unsupported]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(nufft)


# (name, original text, replacement): a wrong sign, a dropped wrap, a wrong
# axis or scale, a mis-indexed mode, a shifted window
MUTANTS = [
    ("shift_sign", "theta = (psi - np.floor(psi)) + u * (Ns // 2) + v * (L // 2)",
     "theta = (psi - np.floor(psi)) - u * (Ns // 2) + v * (L // 2)"),
    ("no_wrap", "i1 = m1.astype(np.int64) % n1", "i1 = np.clip(m1.astype(np.int64), 0, n1 - 1)"),
    ("fft_sign", "G = np.fft.ifft2(grid) * (n1 * n2)", "G = np.fft.fft2(grid)"),
    ("mode_mirrored", "G[np.ix_(k2 % n2, k1 % n1)]", "G[np.ix_(k2 % n2, (-k1) % n1)]"),
    ("transform_half_width", "half = 0.5 * w * h", "half = w * h"),
    ("grid_axis_swapped", "t1, t2 = u * n1, v * n2", "t1, t2 = u * n1, v * n1"),
    ("window_floor", "m1 = np.ceil(t1 - w / 2.0)[:, None]", "m1 = np.floor(t1 - w / 2.0)[:, None]"),
    ("doppler_sign", "v = -bet - np.round(-bet)", "v = bet - np.round(bet)"),
    ("deconv_axes_swapped", "* d2[:, None] * d1[None, :]",
     "* deconv(L, n1, w, beta)[:, None] * deconv(Ns, n2, w, beta)[None, :]"),
]


def _load_mutant(tmp_path, old, new):
    src = open(nufft.__file__).read()
    assert src.count(old) == 1, old
    path = os.path.join(tmp_path, "nufft_mutant.py")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("nufft_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    mod = _load_mutant(tmp_path, old, new)
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError, IndexError):
            caught.append(pin.__name__)
    assert caught, f"mutant {name} survived every pin"
