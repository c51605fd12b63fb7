"""50-digit brute-force sums for tiny inputs (TEST INFRASTRUCTURE ONLY).

Two references pin the C oracle where exhaustive high-precision evaluation is
affordable (a few pixels, channels, samples and blocks):

* `cube_recipe`: the binary64 phase-argument recipe (ranges, carrier phase,
  beat and Doppler arguments, each reduced mod 1) evaluated step by step in
  NumPy float64, then everything after it -- the combined phase, the complex
  exponential and the sum over pixels -- carried out in 50-digit arithmetic.
  The C oracle must agree to a few ulp of the result.

* `cube_exact`: the signal model evaluated exactly from the float32 inputs
  (Sec. II, eq. (1) per virtual channel with the pixel sum of eq. (2)), with
  no binary64 rounding anywhere.  The C oracle must agree within the error
  bound of its binary64 phase arithmetic (`phase_error_bound`).
"""
from __future__ import annotations

import numpy as np
import mpmath as mp

DPS = 50


def _amp(px, p, l):
    """Strength of pixel p in block l: amp is [P], or [L][P] when the
    strength varies over the TDM blocks."""
    a = px.amp
    return float(a[l, p]) if a.ndim == 2 else float(a[p])


def _recipe_args(radar, px):
    f64 = np.float64
    Kc = (f64(2.0) * f64(radar.fc)) / f64(radar.c0) if radar.carrier_phase else f64(0.0)
    Kb = (f64(2.0) * f64(radar.mu)) / (f64(radar.c0) * f64(radar.Fs))
    Kd = ((f64(2.0) * f64(radar.fc)) * f64(radar.Tb)) / f64(radar.c0)
    x = px.x.astype(f64)
    y = px.y.astype(f64)
    z = px.z.astype(f64)

    def dist(ant):
        dx = x - f64(ant[0])
        dy = y - f64(ant[1])
        dz = z - f64(ant[2])
        return np.sqrt((dx * dx + dy * dy) + dz * dz)

    C = radar.M * radar.N
    R = np.empty((C, px.P), dtype=f64)
    for c in range(C):
        m, r = divmod(c, radar.N)
        R[c] = f64(0.5) * (dist(radar.tx[m]) + dist(radar.rx[r]))
    return Kc, Kb, Kd, R


def cube_recipe(radar, px, dps: int = DPS) -> np.ndarray:
    """Cube with binary64 phase arguments and an exact remainder."""
    Kc, Kb, Kd, R = _recipe_args(radar, px)
    C, L, Ns = radar.M * radar.N, radar.L, radar.Ns
    out = np.zeros((C, L, Ns), dtype=np.complex128)
    with mp.workdps(dps):
        for c in range(C):
            for l in range(L):
                for n in range(Ns):
                    s = mp.mpc(0)
                    for p in range(px.P):
                        psi = R[c, p] * Kc
                        psi_f = psi - np.floor(psi)
                        th = (R[c, p] * Kb) * np.float64(n)
                        th_f = th - np.floor(th)
                        ph = (np.float64(px.vr[p]) * Kd) * np.float64(l)
                        ph_f = ph - np.floor(ph)
                        phi = mp.mpf(float(psi_f)) + mp.mpf(float(th_f)) - mp.mpf(float(ph_f))
                        s += mp.mpf(_amp(px, p, l)) * mp.expj(2 * mp.pi * phi)
                    out[c, l, n] = complex(s)
    return out


def _exact_geometry(radar, px):
    C = radar.M * radar.N
    R = [[None] * px.P for _ in range(C)]
    for c in range(C):
        m, r = divmod(c, radar.N)
        for p in range(px.P):
            pos = [mp.mpf(float(px.x[p])), mp.mpf(float(px.y[p])), mp.mpf(float(px.z[p]))]
            t = [mp.mpf(float(v)) for v in radar.tx[m]]
            q = [mp.mpf(float(v)) for v in radar.rx[r]]
            rt = mp.sqrt(sum((pos[k] - t[k]) ** 2 for k in range(3)))
            rr = mp.sqrt(sum((pos[k] - q[k]) ** 2 for k in range(3)))
            R[c][p] = (rt + rr) / 2
    return R


def cube_exact(radar, px, dps: int = DPS) -> np.ndarray:
    """Cube evaluated exactly (to dps digits) from the float32 inputs."""
    C, L, Ns = radar.M * radar.N, radar.L, radar.Ns
    out = np.zeros((C, L, Ns), dtype=np.complex128)
    with mp.workdps(dps):
        fc, mu, Fs, Tb, c0 = (mp.mpf(float(v)) for v in
                               (radar.fc, radar.mu, radar.Fs, radar.Tb, radar.c0))
        R = _exact_geometry(radar, px)
        for c in range(C):
            for l in range(L):
                for n in range(Ns):
                    s = mp.mpc(0)
                    for p in range(px.P):
                        Rp = R[c][p]
                        sigma_phase = 2 * fc * Rp / c0 if radar.carrier_phase else mp.mpf(0)
                        beat = 2 * mu * Rp / c0 * n / Fs
                        fD = 2 * mp.mpf(float(px.vr[p])) * fc / c0
                        phi = sigma_phase + beat - fD * l * Tb
                        s += mp.mpf(_amp(px, p, l)) * mp.expj(2 * mp.pi * phi)
                    out[c, l, n] = complex(s)
    return out


def phase_error_bound(radar, px) -> np.ndarray:
    """Per-entry bound on |Y_binary64 - Y_exact| for the fixed recipe.

    Each rounded operation adds at most one unit roundoff u = 2^-53 of its
    result.  The range R carries a relative error of at most ~8u (three
    products and two sums per distance, a correctly rounded sqrt, the half
    sum); the argument psi = R*Kc inherits it on a magnitude |psi|, likewise
    b*n and beta*l, each plus a few rounding of the products and mod-1
    reductions.  With a 4x margin the per-term phase error (cycles) is taken
    as 32u(|psi| + |b n| + |beta l| + 4) and the cos/sin evaluation adds 4u.
    The entry bound is sum_p a_p (2 pi dphi_p + 4u).
    """
    u = 2.0 ** -53
    Kc, Kb, Kd, R = _recipe_args(radar, px)
    n = np.arange(radar.Ns, dtype=np.float64)
    l = np.arange(radar.L, dtype=np.float64)
    beta = np.abs(px.vr.astype(np.float64) * Kd)
    a = np.abs(px.amp.astype(np.float64))
    if a.ndim == 2:  # strengths per block: bound with the largest
        a = a.max(axis=0)
    C = radar.M * radar.N
    out = np.zeros((C, radar.L, radar.Ns))
    for c in range(C):
        psi = np.abs(R[c] * Kc)[:, None, None]
        bn = np.abs(R[c] * Kb)[:, None, None] * n[None, None, :]
        bl = beta[:, None, None] * l[None, :, None]
        dphi = 32 * u * (psi + bn + bl + 4.0)
        out[c] = np.sum(a[:, None, None] * (2 * np.pi * dphi + 4 * u), axis=0)
    return out
