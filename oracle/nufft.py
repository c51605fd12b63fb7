"""CPU oracle of the NUFFT form of the cube (numpy, float64).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this
module: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the GPU library.

The cube of Sec. II (eq. (1) per virtual channel, pixel sum of eq. (2)) is,
channel by channel, a two-dimensional type-1 non-uniform discrete Fourier
transform:

  Y[c][l][n] = sum_p s_p exp(j2pi (u_p n + v_p l))
  s_p = a_p exp(j2pi psi_p),  u_p = b_p (cycles per sample),  v_p = -beta_p

(phase arguments by the oracle's binary64 recipe).  This module evaluates it
the way a type-1 NUFFT does (spread, FFT, deconvolve; Barnett, Magland and
af Klinteberg, SIAM J. Sci. Comput. 41 (2019), the "exponential of
semicircle" kernel on a grid oversampled at least twofold), written out step
by step so that each can be checked against the exact sum:

  1. u' = u - round(u), v' = v - round(v) in [-1/2, 1/2] (the sum only sees
     u, v modulo 1); with n = k1 + floor(Ns/2), l = k2 + floor(L/2) the
     modes k are centred and the strengths pick up
     c_p = s_p exp(j2pi (u' floor(Ns/2) + v' floor(L/2))).
  2. Spread onto an n1 x n2 periodic grid (n1 >= 2 Ns, n2 >= 2 L, powers of
     two): grid cell (m1, m2) gets c_p phi(m1 - u' n1) phi(m2 - v' n2) for the
     w cells m = ceil(t - w/2) .. ceil(t - w/2) + w - 1 around each point t,
     phi(t) = exp(beta (sqrt(1 - (2t/w)^2) - 1)).
  3. FFT with the + sign: G[k] = sum_m grid[m] exp(+j2pi k m / n).
  4. Deconvolve: F[k] = G[k] h / phi_hat(k) per axis, h = 2pi / n,
     phi_hat(k) = integral of phi (in radians, support w h / 2 each side)
     times cos(k x), by Gauss-Legendre quadrature.
Kernel width and shape for a tolerance eps (twofold oversampling):
w = ceil(log10(1/eps)) + 1, beta = 2.30 w (2.20 w, 2.26 w, 2.38 w for
w = 2, 3, 4), as that paper chooses them.
"""
from __future__ import annotations

import math

import numpy as np

_BETA_PER_W = {2: 2.20, 3: 2.26, 4: 2.38}


def es_params(tol: float):
    """Kernel width w (grid cells) and shape beta for tolerance tol."""
    if not (1e-15 < tol < 1):
        raise ValueError("tolerance must lie in (1e-15, 1)")
    w = int(math.ceil(math.log10(1.0 / tol))) + 1
    w = min(max(w, 2), 16)
    return w, _BETA_PER_W.get(w, 2.30) * w


def fine_size(N: int, w: int) -> int:
    """Smallest power of two >= max(2 N, 2 w)."""
    n = 1
    while n < max(2 * N, 2 * w):
        n *= 2
    return n


def es(t, w, beta):
    """phi(t) on grid offsets t (cells), zero outside |t| <= w/2."""
    z = 2.0 * np.asarray(t, dtype=np.float64) / w
    inside = np.abs(z) <= 1.0
    out = np.zeros_like(z)
    out[inside] = np.exp(beta * (np.sqrt(1.0 - z[inside] ** 2) - 1.0))
    return out


def es_hat(k, w, beta, n, nodes: int = 200):
    """phi_hat(k) = int phi(x) exp(-j k x) dx over radians x, phi even,
    for integer modes k on an n-point grid (cell width h = 2pi / n)."""
    h = 2.0 * np.pi / n
    z, q = np.polynomial.legendre.leggauss(nodes)   # nodes on [-1, 1]
    half = 0.5 * w * h                               # support half-width (radians)
    phi = np.exp(beta * (np.sqrt(1.0 - z * z) - 1.0))
    k = np.asarray(k, dtype=np.float64)
    return half * np.cos(np.outer(k, z * half)) @ (q * phi)


def deconv(N: int, n: int, w: int, beta: float) -> np.ndarray:
    """h / phi_hat(k) for the centred modes k = i - floor(N/2), i < N."""
    k = np.arange(N) - N // 2
    return (2.0 * np.pi / n) / es_hat(k, w, beta, n)


def nufft_cube(radar, px, tol: float, orc=None) -> np.ndarray:
    """Cube Y[C][L][Ns] (complex128) by spreading, FFT and deconvolution."""
    import oracle
    if int(getattr(radar, "model", 0)) & 16:
        raise ValueError("strengths per block do not factor into one NUFFT per channel")
    o = orc or oracle.default()
    w, beta = es_params(tol)
    C, L, Ns = radar.M * radar.N, radar.L, radar.Ns
    n1, n2 = fine_size(Ns, w), fine_size(L, w)
    d1, d2 = deconv(Ns, n1, w, beta), deconv(L, n2, w, beta)
    k1 = np.arange(Ns) - Ns // 2
    k2 = np.arange(L) - L // 2
    amp = np.asarray(px.amp, dtype=np.float64)
    out = np.zeros((C, L, Ns), dtype=np.complex128)
    off = np.arange(w)
    for c in range(C):
        psi, b, bet = o.chan_args(radar, px, c)
        u = b - np.round(b)
        v = -bet - np.round(-bet)
        theta = (psi - np.floor(psi)) + u * (Ns // 2) + v * (L // 2)
        cp = amp * np.exp(2j * np.pi * theta)
        t1, t2 = u * n1, v * n2
        m1 = np.ceil(t1 - w / 2.0)[:, None] + off[None, :]      # [P][w]
        m2 = np.ceil(t2 - w / 2.0)[:, None] + off[None, :]
        f1 = es(m1 - t1[:, None], w, beta)
        f2 = es(m2 - t2[:, None], w, beta)
        i1 = m1.astype(np.int64) % n1
        i2 = m2.astype(np.int64) % n2
        grid = np.zeros((n2, n1), dtype=np.complex128)
        for j in range(w):
            for i in range(w):
                np.add.at(grid, (i2[:, j], i1[:, i]), cp * f2[:, j] * f1[:, i])
        G = np.fft.ifft2(grid) * (n1 * n2)          # + sign, unnormalised
        out[c] = G[np.ix_(k2 % n2, k1 % n1)] * d2[:, None] * d1[None, :]
    return out
