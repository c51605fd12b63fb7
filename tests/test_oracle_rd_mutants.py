"""Plausible mistakes planted in a copy of the range-Doppler oracle must each
fail at least one of its pins (the pins are not blind to them)."""
import importlib.util
import os
import sys

import pytest

from test_oracle_rd_pins import CHECKS

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "rd.py")

MUTANTS = [
    ("doppler_forward_dft", "x = np.fft.ifft(x, axis=2) * L", "x = np.fft.fft(x, axis=2)"),
    ("doppler_normalised", "x = np.fft.ifft(x, axis=2) * L", "x = np.fft.ifft(x, axis=2)"),
    ("range_inverse_dft", "x = np.fft.fft(y, axis=3)", "x = np.fft.ifft(y, axis=3) * y.shape[3]"),
    ("axes_swapped", "x = np.fft.fft(y, axis=3)", "x = np.fft.fft(y, axis=2)"),
    ("one_channel_only", "p = np.sum(x.real ** 2 + x.imag ** 2, axis=1)", "p = x[:, 0].real ** 2 + x[:, 0].imag ** 2"),
    ("magnitude_not_power", "p = np.sum(x.real ** 2 + x.imag ** 2, axis=1)", "p = np.sum(np.abs(x), axis=1)"),
    ("no_transpose", "np.transpose(p, (0, 2, 1))", "p"),
    ("static_not_skipped", "p[:, :, 0] = -np.inf", "pass"),
    ("static_row_skipped", "p[:, :, 0] = -np.inf", "p[:, 0, :] = -np.inf"),
    ("last_on_ties", "flat = np.argmax(p.reshape(F, -1), axis=1)",
     "flat = p.reshape(F, -1).shape[1] - 1 - np.argmax(p.reshape(F, -1)[:, ::-1], axis=1)"),
    ("unsigned_bins", "return np.where(d >= L // 2, d - L, d)", "return d"),
    ("velocity_no_Tb", "radar.c0 / (2.0 * radar.fc * radar.Tb * radar.L)", "radar.c0 / (2.0 * radar.fc * radar.L)"),
    ("velocity_sign", "return np.asarray(d_signed, dtype=np.float64) * radar.c0",
     "return -np.asarray(d_signed, dtype=np.float64) * radar.c0"),
    ("range_full_path", "radar.c0 * radar.Fs / (2.0 * radar.mu * radar.Ns)", "radar.c0 * radar.Fs / (radar.mu * radar.Ns)"),
    ("e_velo_signed", "np.mean(np.abs(v_est - v_true))", "abs(np.mean(v_est - v_true))"),
]


def load_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = tmp_path / f"rd_{name}.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"rd_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_rd_mutant_is_caught(tmp_path, name, old, new):
    mod = load_mutant(tmp_path, name, old, new)
    caught = 0
    for check in CHECKS:
        try:
            check(mod)
        except Exception:
            caught += 1
    assert caught, f"mutant {name} passed every pin"
