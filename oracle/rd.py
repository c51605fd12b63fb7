"""CPU oracle of the range-Doppler step (Sec. III), numpy in float64.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this
module: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the GPU library.

Sec. III applies an FFT to the cube of each coherent processing interval to
get its range-Doppler map, takes the velocity of the map's strongest cell per
CPI (the Doppler-time series) and compares it with the ground truth by the
mean absolute error E_velo.  Written out, per frame:

  X_c[k][d] = sum_l sum_n Y[c][l][n] exp(-j2pi k n / Ns) exp(+j2pi d l / L)
  power[k][d] = sum_c |X_c[k][d]|^2

The sign over l makes an approaching scatterer (Y ~ exp(-j2pi beta l),
beta > 0) peak at d = beta L.  Bins are in natural order (d >= L/2 stands for
d - L).  The peak is argmax power over (k, d), over d != 0 when static
returns are skipped, first index k L + d on ties.
"""
from __future__ import annotations

import numpy as np


def range_doppler_power(cubes: np.ndarray) -> np.ndarray:
    """cubes [F][C][L][Ns] (or [C][L][Ns]) complex -> power [F][Ns][L] float64."""
    y = np.asarray(cubes, dtype=np.complex128)
    if y.ndim == 3:
        y = y[None]
    L = y.shape[2]
    x = np.fft.fft(y, axis=3)            # forward over fast time n
    x = np.fft.ifft(x, axis=2) * L       # exp(+j2pi d l / L), unnormalised
    p = np.sum(x.real ** 2 + x.imag ** 2, axis=1)   # [F][L][Ns], over channels
    return np.ascontiguousarray(np.transpose(p, (0, 2, 1)))


def peaks(power: np.ndarray, skip_static: bool = True):
    """(k, d) of the strongest cell of each frame, d in natural order."""
    p = np.array(power, dtype=np.float64, copy=True)
    if skip_static:
        p[:, :, 0] = -np.inf
    F, Ns, L = p.shape
    flat = np.argmax(p.reshape(F, -1), axis=1)      # first occurrence on ties
    return flat // L, flat % L


def signed_bin(d: np.ndarray, L: int) -> np.ndarray:
    d = np.asarray(d)
    return np.where(d >= L // 2, d - L, d)


def bin_velocity(d_signed, radar) -> np.ndarray:
    """Radial velocity of Doppler bin d: beta = d / L cycles per block and
    beta = 2 fc Tb v / c0 (eq. (1)'s f_D T_b)."""
    return np.asarray(d_signed, dtype=np.float64) * radar.c0 / (2.0 * radar.fc * radar.Tb * radar.L)


def bin_range(k, radar) -> np.ndarray:
    """Range of fast-time bin k: b = k / Ns cycles per sample and
    b = 2 mu R / (c0 Fs) (eq. (1)'s beat frequency)."""
    return np.asarray(k, dtype=np.float64) * radar.c0 * radar.Fs / (2.0 * radar.mu * radar.Ns)


def doppler_time(power: np.ndarray, k_peak: np.ndarray) -> np.ndarray:
    """Velocity spectrum at the peak's range bin, one row per frame [F][L]."""
    return np.stack([power[f, k_peak[f], :] for f in range(power.shape[0])])


def e_velo(v_est, v_true) -> float:
    """Mean absolute velocity error over the CPIs (Sec. III)."""
    v_est = np.asarray(v_est, dtype=np.float64)
    v_true = np.asarray(v_true, dtype=np.float64)
    return float(np.mean(np.abs(v_est - v_true)))
