"""Pins of the CPU oracle: checks that come from the mathematics of the
signal model (Sec. II, eq. (1) per virtual channel, pixel sum of eq. (2)),
not from the oracle's own code.

Each pin takes an `oracle.Oracle` and raises AssertionError when the oracle
disagrees.  `test_oracle_pins.py` runs them on the real oracle and
`test_oracle_mutants.py` runs them on deliberately broken copies of the
oracle's C source to show that each plausible mistake is caught.
"""
from __future__ import annotations

import math

import numpy as np
import mpmath as mp

from paper_2307_09226_amd import scenes
from oracle import brute

C0 = scenes.C0


def relerr(a, b):
    d = np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
    n = np.linalg.norm(np.asarray(b).ravel())
    return d / n if n > 0 else d


def _one_pixel(x, y, z, amp, vr):
    f = lambda v: np.array([v], dtype=np.float32)
    return scenes.Pixels(f(x), f(y), f(z), f(amp), f(vr))


def _colocated_radar(Ns=64, L=32, Fs=5e6, Tb=80e-6, fc=77e9, mu=30e12):
    z = np.zeros((1, 3))
    return scenes.Radar(M=1, N=1, Ns=Ns, L=L, fc=fc, mu=mu, Fs=Fs, Tb=Tb, tx=z, rx=z.copy())


def _random_antennas(rng, M, N, lam):
    """Non-collinear antenna positions (all three coordinates non-zero)."""
    tx = rng.uniform(-4 * lam, 4 * lam, (M, 3))
    rx = rng.uniform(-4 * lam, 4 * lam, (N, 3))
    return tx, rx


# ----------------------------------------------------------------------------
def pin_empty_scene(o):
    """No pixels: the sum is empty, every entry is exactly zero."""
    r = scenes.radar_small()
    px = scenes.Pixels(*(np.zeros(0, np.float32) for _ in range(5)))
    Y = o.cube(r, px)
    assert Y.shape == (8, 32, 64)
    assert np.all(Y == 0) and not np.any(np.signbit(Y.real) & (Y.real != 0))


def pin_single_scatterer_closed_form(o):
    """One scatterer gives the rank-1 cube a exp(j2pi(psi_c + b_c n - beta l))
    with psi, b, beta evaluated exactly (mpmath) from the float32 inputs."""
    r = scenes.radar_small()
    px = _one_pixel(0.7, 3.3, -0.4, 0.8, 1.7)
    Y = o.cube(r, px)
    mp.mp.dps = 40
    pos = [mp.mpf(float(v)) for v in (px.x[0], px.y[0], px.z[0])]
    fc, mu, Fs, Tb, c0 = (mp.mpf(float(v)) for v in (r.fc, r.mu, r.Fs, r.Tb, r.c0))
    v = mp.mpf(float(px.vr[0]))
    beta = float(2 * v * fc * Tb / c0)
    n = np.arange(r.Ns)
    l = np.arange(r.L)
    for c in range(r.C):
        m, q = divmod(c, r.N)
        dt = mp.sqrt(sum((pos[k] - mp.mpf(float(r.tx[m][k]))) ** 2 for k in range(3)))
        dr = mp.sqrt(sum((pos[k] - mp.mpf(float(r.rx[q][k]))) ** 2 for k in range(3)))
        R = (dt + dr) / 2
        psi = 2 * fc * R / c0
        psi_f = float(psi - mp.floor(psi))
        b = float(2 * mu * R / (c0 * Fs))
        phase = psi_f + b * n[None, :] - beta * l[:, None]
        ref = float(px.amp[0]) * np.exp(2j * np.pi * phase)
        assert relerr(Y[c], ref) < 1e-10, (c, relerr(Y[c], ref))


def pin_range_and_doppler_peaks(o):
    """Co-located Tx/Rx, one scatterer at range R = k0 c0 Fs / (2 mu Ns) and
    radial velocity v with f_D Tb L = j0: the forward DFT over fast time
    peaks at bin k0 = 2 mu R Ns / (c0 Fs), every bin has the Dirichlet
    magnitude a |G_Ns(b - k/Ns)|, and the inverse DFT over slow time peaks
    at bin j0 = f_D Tb L (exp(-j2pi beta l) puts the forward-DFT peak at
    -j0 mod L)."""
    r = _colocated_radar()
    k0, j0 = 10, 5
    R = k0 * r.c0 * r.Fs / (2 * r.mu * r.Ns)
    v = j0 * r.c0 / (2 * r.fc * r.Tb * r.L)
    a = 0.5
    px = _one_pixel(0.0, R, 0.0, a, v)
    Y = o.cube(r, px)[0]  # [L][Ns]
    Rf = float(np.float32(R))
    b = 2 * r.mu * Rf / (r.c0 * r.Fs)
    spec = np.fft.fft(Y, axis=1)  # over n
    k = np.arange(r.Ns)
    x = b - k / r.Ns
    with np.errstate(invalid="ignore", divide="ignore"):
        G = np.where(np.abs(np.sin(np.pi * x)) < 1e-15, r.Ns,
                     np.abs(np.sin(np.pi * r.Ns * x) / np.sin(np.pi * x)))
    for l in range(r.L):
        assert int(np.argmax(np.abs(spec[l]))) == k0
        assert np.max(np.abs(np.abs(spec[l]) - a * G)) < 1e-9 * a * r.Ns
    dop = np.fft.ifft(Y, axis=0)  # over l
    for n in range(r.Ns):
        assert int(np.argmax(np.abs(dop[:, n]))) == j0
    fwd = np.fft.fft(Y[:, 0])
    assert int(np.argmax(np.abs(fwd))) == (-j0) % r.L


def pin_marginals(o):
    """Fast- and slow-time sums of the direct cube equal the geometric-series
    closed forms sum_p a e^{j2pi(psi - beta l)} G_Ns(b) and
    sum_p a e^{j2pi(psi + b n)} G_L(-beta)."""
    rng = np.random.default_rng(5)
    r = scenes.radar_for(2, 3, 16, 8, Fs=5e6, Tb=80e-6)
    r.tx, r.rx = _random_antennas(rng, 2, 3, r.wavelength)
    px = scenes.tiny_scene(11, 37)
    Y = o.cube(r, px)
    assert relerr(Y.sum(axis=2), o.marginal_n(r, px)) < 1e-11
    assert relerr(Y.sum(axis=1), o.marginal_l(r, px)) < 1e-11


def pin_linearity(o):
    """Superposition over disjoint pixel sets, exact power-of-two scaling of
    the strengths, and invariance under pixel permutation."""
    r = scenes.radar_for(2, 2, 16, 8, Fs=5e6, Tb=80e-6)
    px = scenes.tiny_scene(3, 40)
    A, B = px.take(np.arange(0, 17)), px.take(np.arange(17, 40))
    Y = o.cube(r, px)
    assert relerr(Y, o.cube(r, A) + o.cube(r, B)) < 1e-13
    twice = scenes.Pixels(px.x, px.y, px.z, (px.amp * np.float32(2)).astype(np.float32), px.vr)
    assert np.array_equal(o.cube(r, twice), 2 * Y)
    perm = np.random.default_rng(1).permutation(px.P)
    assert relerr(o.cube(r, px.take(perm)), Y) < 1e-13


def pin_static_scene_slices(o):
    """v = 0 for every pixel: all slow-time slices are identical."""
    r = scenes.radar_for(2, 2, 16, 6, Fs=5e6, Tb=80e-6)
    px = scenes.tiny_scene(4, 25)
    px = scenes.Pixels(px.x, px.y, px.z, px.amp, np.zeros_like(px.vr))
    Y = o.cube(r, px)
    for l in range(1, r.L):
        assert np.array_equal(Y[:, l], Y[:, 0])


def pin_doppler_alias(o):
    """Adding the blind speed c0/(2 fc Tb) to every velocity moves each
    Doppler phase by a whole cycle per block: the cube is unchanged.  The
    block period is chosen so the blind speed is 16 m/s and both velocity
    sets are exact in float32."""
    fc = 77e9
    Tb = C0 / (2 * fc * 16.0)
    r = scenes.radar_for(1, 2, 8, 16, Fs=5e6, Tb=Tb, fc=fc)
    px = scenes.tiny_scene(6, 20)
    v = np.round(px.vr * 64) / 64
    p1 = scenes.Pixels(px.x, px.y, px.z, px.amp, v.astype(np.float32))
    p2 = scenes.Pixels(px.x, px.y, px.z, px.amp, (v + 16.0).astype(np.float32))
    assert relerr(o.cube(r, p2), o.cube(r, p1)) < 1e-11
    # a non-alias shift does change it
    p3 = scenes.Pixels(px.x, px.y, px.z, px.amp, (v + 8.0).astype(np.float32))
    assert relerr(o.cube(r, p3), o.cube(r, p1)) > 0.1


def _eq2_as_printed(r, px, q):
    """Eq. (2) for Rx n = q + 1 written out with its own 1-based indices and
    evaluated in 40-digit arithmetic from the float32 pixels:
      H[l][n_s] = sum_p sum_{m=1..M} P_r exp(j2pi(2 mu R/c (n_s-1)/F_s
                  - 2 f V/c (l-1) T_b + ((m-1)N + n - 1) dd sin(theta)/lambda))
    with R = |x| the pixel's range, dd = lambda/2, the Doppler of eq. (1)
    (f = f_c, no 1/L: the garbles read as such) and sin(theta) = -x/R, the
    direction cosine along the array axis with theta measured toward -x
    (the sign that makes eq. (2)'s '+' agree with a phase that grows with
    the path length)."""
    out = np.zeros((r.L, r.Ns), dtype=np.complex128)
    with mp.workdps(40):
        c0, fc, mu, Fs, Tb = (mp.mpf(float(v)) for v in (r.c0, r.fc, r.mu, r.Fs, r.Tb))
        lam = c0 / fc
        dd = lam / 2
        n = q + 1
        for p in range(px.P):
            pos = [mp.mpf(float(v)) for v in (px.x[p], px.y[p], px.z[p])]
            R = mp.sqrt(sum(t * t for t in pos))
            sin_t = -pos[0] / R
            V = mp.mpf(float(px.vr[p]))
            Pr = mp.mpf(float(px.amp[p]))
            for l in range(1, r.L + 1):
                for ns in range(1, r.Ns + 1):
                    acc = mp.mpc(0)
                    for m in range(1, r.M + 1):
                        ph = (2 * mu * R / c0 * (ns - 1) / Fs - 2 * fc * V / c0 * (l - 1) * Tb
                              + ((m - 1) * r.N + n - 1) * dd / lam * sin_t)
                        acc += Pr * mp.expj(2 * mp.pi * ph)
                    out[l - 1, ns - 1] += complex(acc)
    return out


def pin_eq2_literal(o):
    """The far-field variant without the carrier phase is eq. (2) as printed:
    for each Rx, the sum of its virtual channels over the Tx equals eq. (2)'s
    H_{T_n} (written out above, independently of the oracle) within the
    binary64 rounding of the phase arguments, on a small moving scene and
    the A11 virtual ULA."""
    r = _with_model(scenes.radar_for(2, 3, 6, 4, Fs=10e6, Tb=120e-6, carrier_phase=0), 1)
    px = scenes.tiny_scene(91, 4, vmax=4.0)
    Y = o.cube(r, px)
    scale = r.M * float(np.sum(px.amp))
    for q in range(r.N):
        got = sum(Y[m * r.N + q] for m in range(r.M))
        want = _eq2_as_printed(r, px, q)
        assert np.max(np.abs(got - want)) < 1e-12 * scale, (q, float(np.max(np.abs(got - want))))


def pin_eq1_per_rx(o):
    """Summing the virtual channels of one Rx over the Tx gives eq. (1) for
    that Rx, written out with its own 1-based indices and evaluated in
    40-digit arithmetic: h_{T,n}(n_s; l) = sum_m sigma_{m,n}
    exp(j2pi(2 mu R_{m,n}/c (n_s-1)/F_s - f_D (l-1) T_b)), summed over the
    pixels, with sigma = a exp(j2pi 2 f_c R_{m,n}/c) (the carrier phase) and
    f_D = 2 v f_c / c.  Random non-collinear antennas, so a transposed
    channel index or a Tx/Rx mix-up shows."""
    rng = np.random.default_rng(8)
    r = scenes.radar_for(2, 3, 4, 3, Fs=10e6, Tb=120e-6)
    r.tx, r.rx = _random_antennas(rng, 2, 3, r.wavelength)
    px = scenes.tiny_scene(9, 3)
    Y = o.cube(r, px)
    with mp.workdps(40):
        c0, fc, mu, Fs, Tb = (mp.mpf(float(v)) for v in (r.c0, r.fc, r.mu, r.Fs, r.Tb))
        for n in range(1, r.N + 1):
            want = np.zeros((r.L, r.Ns), dtype=np.complex128)
            for p in range(px.P):
                pos = [mp.mpf(float(v)) for v in (px.x[p], px.y[p], px.z[p])]
                fD = 2 * mp.mpf(float(px.vr[p])) * fc / c0
                for m in range(1, r.M + 1):
                    tx = [mp.mpf(float(v)) for v in r.tx[m - 1]]
                    rx = [mp.mpf(float(v)) for v in r.rx[n - 1]]
                    R = (mp.sqrt(sum((pos[k] - tx[k]) ** 2 for k in range(3)))
                         + mp.sqrt(sum((pos[k] - rx[k]) ** 2 for k in range(3)))) / 2
                    sigma = mp.mpf(float(px.amp[p])) * mp.expj(2 * mp.pi * 2 * fc * R / c0)
                    for l in range(1, r.L + 1):
                        for ns in range(1, r.Ns + 1):
                            want[l - 1, ns - 1] += complex(sigma * mp.expj(
                                2 * mp.pi * (2 * mu * R / c0 * (ns - 1) / Fs - fD * (l - 1) * Tb)))
            got = sum(Y[(m - 1) * r.N + (n - 1)] for m in range(1, r.M + 1))
            scale = r.M * float(np.sum(px.amp))
            assert np.max(np.abs(got - want)) < 1e-10 * scale, (n, float(np.max(np.abs(got - want))))


def pin_far_field_literal_one_pixel(o):
    """One pixel, far-field variant, no carrier phase: channel 0 (Tx 0 and
    Rx 0 at the origin) at n = l = 0 is exactly the real strength (eq. (2)
    has no common phase), and channel c is a exp(j2pi c sin(theta) / 2)
    (eq. (2)'s angle term with dd = lambda/2) at any distance, near or far;
    along fast time the phase advances by 2 mu R / (c0 Fs) per sample."""
    r = _with_model(scenes.radar_for(3, 4, 8, 4, Fs=10e6, Tb=120e-6, carrier_phase=0), 1)
    for dist in (1.5, 300.0):
        az, el = math.radians(-25.0), math.radians(8.0)
        u = np.array([math.cos(el) * math.sin(az), math.cos(el) * math.cos(az), math.sin(el)])
        px = _one_pixel(*(dist * u), 0.75, 0.0)
        Y = o.cube(r, px)
        assert Y[0, 0, 0] == complex(0.75, 0.0), Y[0, 0, 0]
        x = np.array([float(px.x[0]), float(px.y[0]), float(px.z[0])])
        R = np.linalg.norm(x)
        sin_t = -x[0] / R
        for c in range(r.C):
            want = 0.75 * np.exp(2j * np.pi * c * sin_t / 2)
            assert abs(Y[c, 0, 0] - want) < 1e-13, (dist, c, Y[c, 0, 0], want)
        b = 2 * r.mu * R / (r.c0 * r.Fs)
        step = Y[7, 0, 1:] / Y[7, 0, :-1]
        assert np.max(np.abs(np.angle(step / np.exp(2j * np.pi * b)))) < 1e-12


def pin_far_field(o):
    """A distant scatterer at azimuth az, elevation el: across the virtual
    ULA (element c at c lambda/2 on +x) the channel ratio at n = l = 0 tends
    to exp(-j2pi c (lambda/2) cos(el) sin(az) / lambda), eq. (2)'s array
    term, with the sign that follows from a carrier phase of +2R/lambda."""
    r = scenes.radar_for(3, 4, 4, 2, Fs=10e6, Tb=120e-6)
    az, el, dist = math.radians(20.0), math.radians(10.0), 5000.0
    u = np.array([math.cos(el) * math.sin(az), math.cos(el) * math.cos(az), math.sin(el)])
    px = _one_pixel(*(dist * u), 1.0, 0.0)
    Y = o.cube(r, px)
    lam = r.wavelength
    for c in range(r.C):
        want = np.exp(-2j * np.pi * c * (lam / 2) * u[0] / lam)
        got = Y[c, 0, 0] / Y[0, 0, 0]
        assert abs(abs(got) - 1) < 1e-12
        assert abs(np.angle(got / want)) < 1e-3, (c, np.angle(got / want))


def pin_entries_match_cube(o):
    """Selected entries equal the same entries of the full cube."""
    r = scenes.radar_for(2, 3, 16, 8, Fs=5e6, Tb=80e-6)
    px = scenes.tiny_scene(12, 30)
    Y = o.cube(r, px)
    rng = np.random.default_rng(2)
    c = rng.integers(0, r.C, 50)
    l = rng.integers(0, r.L, 50)
    n = rng.integers(0, r.Ns, 50)
    assert np.array_equal(o.entries(r, px, c, l, n), Y[c, l, n])


def pin_brute_recipe(o):
    """Tiny scene: binary64 phase arguments with an exact remainder agree
    with the oracle to a few ulp of the entries' scale."""
    rng = np.random.default_rng(21)
    r = scenes.radar_for(1, 2, 4, 3, Fs=5e6, Tb=80e-6)
    r.tx, r.rx = _random_antennas(rng, 1, 2, r.wavelength)
    px = scenes.tiny_scene(22, 3)
    ref = brute.cube_recipe(r, px)
    Y = o.cube(r, px)
    scale = float(np.sum(px.amp))
    assert np.max(np.abs(Y - ref)) < 16 * 2.0 ** -52 * scale


def pin_brute_exact(o):
    """Tiny scene against the exact (50-digit) sum from the float32 inputs:
    every entry within the binary64 phase-error bound."""
    rng = np.random.default_rng(31)
    r = scenes.radar_for(2, 2, 4, 3, Fs=5e6, Tb=80e-6)
    r.tx, r.rx = _random_antennas(rng, 2, 2, r.wavelength)
    px = scenes.tiny_scene(32, 4)
    ref = brute.cube_exact(r, px)
    bound = brute.phase_error_bound(r, px)
    Y = o.cube(r, px)
    assert np.all(np.abs(Y - ref) <= bound), float(np.max(np.abs(Y - ref) / bound))


def pin_brute_exact_no_carrier(o):
    """As above with the carrier phase switched off (sigma = a)."""
    rng = np.random.default_rng(41)
    r = scenes.radar_for(1, 3, 4, 3, Fs=5e6, Tb=80e-6, carrier_phase=0)
    r.tx, r.rx = _random_antennas(rng, 1, 3, r.wavelength)
    px = scenes.tiny_scene(42, 3)
    ref = brute.cube_exact(r, px)
    bound = brute.phase_error_bound(r, px)
    assert np.all(np.abs(o.cube(r, px) - ref) <= bound)


# ----------------------------------------------------------------------------
# Signal-model variants (flags: 1 far field, 2 Tx slot timing, 4 Doppler
# within the chirp, 8 residual video phase)
def _with_model(r, model):
    import dataclasses
    return dataclasses.replace(r, model=model)


def pin_model_zero_is_default(o):
    """Variants that vanish for a static scene or a single Tx leave the cube
    bitwise unchanged: slot timing with M = 1 or v = 0, intra-chirp Doppler
    with v = 0."""
    r = scenes.radar_for(1, 3, 8, 4, Fs=5e6, Tb=80e-6)
    px = scenes.tiny_scene(51, 5)
    base = o.cube(r, px)
    assert np.array_equal(o.cube(_with_model(r, 2), px), base)
    r2 = scenes.radar_for(2, 2, 8, 4, Fs=5e6, Tb=80e-6)
    px0 = scenes.tiny_scene(52, 5, vmax=0.0)
    base2 = o.cube(r2, px0)
    assert np.array_equal(o.cube(_with_model(r2, 2 | 4), px0), base2)


def pin_slot_timing_alias(o):
    """Tx m fires at l Tb + m Tb / M.  One extra Doppler cycle per block
    (v + c0 / (2 fc Tb)) then turns channel m by exactly exp(-j2pi m / M),
    and M extra cycles per block leave every channel unchanged."""
    r = _with_model(scenes.radar_for(3, 2, 8, 4, Fs=5e6, Tb=120e-6), 2)
    v0 = 1.3
    dv = r.c0 / (2 * r.fc * r.Tb)
    Ya = o.cube(r, _one_pixel(0.4, 3.1, 0.2, 1.0, v0))
    Yb = o.cube(r, _one_pixel(0.4, 3.1, 0.2, 1.0, np.float32(v0 + dv)))
    Yc = o.cube(r, _one_pixel(0.4, 3.1, 0.2, 1.0, np.float32(v0 + r.M * dv)))
    vb = float(np.float32(v0 + dv)) - float(np.float32(v0))
    vc = float(np.float32(v0 + r.M * dv)) - float(np.float32(v0))
    for c in range(r.C):
        m = c // r.N
        for l in range(r.L):
            # the float32 velocities are off the exact alias by a few ulp:
            # remove that residual Doppler before comparing
            res_b = np.exp(-2j * np.pi * ((vb - dv) * 2 * r.fc * r.Tb / r.c0) * (l + m / r.M))
            res_c = np.exp(-2j * np.pi * ((vc - r.M * dv) * 2 * r.fc * r.Tb / r.c0) * (l + m / r.M))
            want_b = Ya[c, l] * np.exp(-2j * np.pi * m / r.M) * res_b
            assert np.max(np.abs(Yb[c, l] - want_b)) < 1e-6, (c, l)
            assert np.max(np.abs(Yc[c, l] - Ya[c, l] * res_c)) < 1e-6, (c, l)


def pin_dechirp_physics(o):
    """The dechirped echo of one moving scatterer written from the FMCW
    chirp itself: s(t) = exp(j2pi(fc t + mu t^2 / 2)), echo delay
    tau(t) = 2 (R0 - v t) / c0, y = s(t) conj(s(t - tau)) over the first
    chirp.  With the residual-video-phase and intra-chirp-Doppler variants
    the cube's l = 0 row follows y to within the second-order terms the
    model leaves out (-2 mu v t^2 / c0, a few thousandths of a cycle here);
    without them it does not."""
    z = np.zeros((1, 3))
    r = scenes.Radar(M=1, N=1, Ns=64, L=2, fc=77e9, mu=30e12, Fs=5e6, Tb=80e-6, tx=z, rx=z.copy())
    px = _one_pixel(1.2, 6.5, 0.3, 1.0, 100.0)
    with mp.workdps(40):
        pos = [mp.mpf(float(v)) for v in (px.x[0], px.y[0], px.z[0])]
        R0 = mp.sqrt(sum(q * q for q in pos))
        v = mp.mpf(float(px.vr[0]))
        want = []
        for n in range(r.Ns):
            t = mp.mpf(n) / r.Fs
            tau = 2 * (R0 - v * t) / r.c0
            ph = (r.fc * t + r.mu * t * t / 2) - (r.fc * (t - tau) + r.mu * (t - tau) ** 2 / 2)
            want.append(complex(mp.expj(2 * mp.pi * ph)))
    want = np.array(want)
    full = o.cube(_with_model(r, 4 | 8), px)[0, 0]
    cyc = np.abs(np.angle(full / want)) / (2 * np.pi)
    assert cyc.max() < 0.01, cyc.max()
    plain = o.cube(r, px)[0, 0]
    assert (np.abs(np.angle(plain / want)) / (2 * np.pi)).max() > 0.02


def pin_far_field_model(o):
    """Far-field variant with the carrier phase (the far-field limit of the
    exact model): across the virtual ULA the channels differ at n = l = 0 by
    exactly eq. (2)'s angle term exp(-j2pi c (lambda/2) u_x / lambda) at any
    distance (the common phase 2 |x| / lambda cancels in the ratio); along
    fast time the phase advances by 2 mu |x| / (c0 Fs) per sample, the range
    from the array origin; and the variant approaches the exact model as
    1/distance."""
    r = _with_model(scenes.radar_for(3, 4, 16, 2, Fs=10e6, Tb=120e-6), 1)
    lam = r.wavelength
    for dist in (2.0, 40.0):
        az, el = math.radians(-25.0), math.radians(8.0)
        u = np.array([math.cos(el) * math.sin(az), math.cos(el) * math.cos(az), math.sin(el)])
        px = _one_pixel(*(dist * u), 1.0, 0.0)
        Y = o.cube(r, px)
        x = np.array([float(px.x[0]), float(px.y[0]), float(px.z[0])])
        Rp = np.linalg.norm(x)
        ux = x[0] / Rp
        for c in range(r.C):
            got = Y[c, 0, 0] / Y[0, 0, 0]
            want = np.exp(-2j * np.pi * c * (lam / 2) * ux / lam)
            assert abs(np.angle(got / want)) < 1e-8, (dist, c)
        b = 2 * r.mu * Rp / (r.c0 * r.Fs)
        got = Y[5, 0, 1:] / Y[5, 0, :-1]
        assert np.max(np.abs(np.angle(got / np.exp(2j * np.pi * b)))) < 1e-8
    # convergence to the exact model
    errs = []
    rr = scenes.radar_for(3, 4, 16, 2, Fs=10e6, Tb=120e-6, carrier_phase=1)
    for dist in (20.0, 2000.0):
        u = np.array([0.3, 0.9, 0.1]) / np.linalg.norm([0.3, 0.9, 0.1])
        px = _one_pixel(*(dist * u), 1.0, 0.0)
        d = o.cube(_with_model(rr, 1), px)[:, 0, 0] / o.cube(rr, px)[:, 0, 0]
        errs.append(np.max(np.abs(np.angle(d))))
    assert errs[1] < errs[0] / 30, errs


# ----------------------------------------------------------------------------
# Strength per TDM block (flag 16): eq. (1)'s sigma_{m,n,l} varying with l
def _block_amp(px, rows):
    """Pixels whose [L][P] strengths are `rows` (float32)."""
    return scenes.Pixels(px.x, px.y, px.z, np.ascontiguousarray(rows, dtype=np.float32), px.vr)


def pin_block_strength_reductions(o):
    """Equal rows reproduce the constant-strength cube bitwise; power-of-two
    row factors g_l scale block l of the cube by exactly g_l (every term of
    block l is scaled by g_l, a power of two)."""
    rng = np.random.default_rng(61)
    r = scenes.radar_for(2, 3, 8, 6, Fs=5e6, Tb=80e-6)
    r.tx, r.rx = _random_antennas(rng, 2, 3, r.wavelength)
    px = scenes.tiny_scene(62, 13)
    base = o.cube(r, px)
    rb = _with_model(r, 16)
    same = _block_amp(px, np.tile(px.amp, (r.L, 1)))
    assert np.array_equal(o.cube(rb, same), base)
    g = 2.0 ** rng.integers(-3, 4, r.L)
    scaled = _block_amp(px, g[:, None] * px.amp[None, :])
    assert np.array_equal(o.cube(rb, scaled), g[None, :, None] * base)


def pin_block_strength_sidebands(o):
    """One scatterer whose strength follows 1 + cos(2pi k0 l / L) over the
    blocks: its slow-time spectrum is the carrier line G_L(d/L - beta) plus
    two half-height sidebands G_L((d -+ k0)/L - beta) / 2, where
    G_L(x) = sum_l exp(j2pi x l), here evaluated in 40-digit arithmetic with
    beta from the float32 velocity."""
    r = _with_model(_colocated_radar(Ns=16, L=32), 16)
    px = _one_pixel(0.3, 4.1, -0.2, 1.0, 2.3)
    k0 = 5
    l = np.arange(r.L)
    px = _block_amp(px, (1.0 + np.cos(2 * np.pi * k0 * l / r.L))[:, None])
    Y = o.cube(r, px)
    spec = np.fft.ifft(Y[0, :, 0]) * r.L   # sum_l Y[l] exp(+j2pi d l / L)
    with mp.workdps(40):
        beta = 2 * mp.mpf(r.fc) * mp.mpf(r.Tb) * mp.mpf(float(px.vr[0])) / mp.mpf(r.c0)
        G = lambda x: mp.fsum(mp.expj(2 * mp.pi * x * j) for j in range(r.L))
        want = [G(mp.mpf(d) / r.L - beta) + (G(mp.mpf(d - k0) / r.L - beta) + G(mp.mpf(d + k0) / r.L - beta)) / 2
                for d in range(r.L)]
    want = np.array([complex(w) for w in want])
    # the float32 row values (1 + cos) carry ~6e-8 relative rounding
    assert np.max(np.abs(np.abs(spec) - np.abs(want))) < 1e-6 * r.L
    top = sorted(np.argsort(np.abs(spec))[-3:])
    j0 = int(round(float(beta) * r.L)) % r.L
    assert top == sorted({j0, (j0 + k0) % r.L, (j0 - k0) % r.L}), (top, j0)


def pin_block_strength_brute(o):
    """Tiny scene with random strengths per block against the exact (50-digit)
    sum: every entry within the binary64 phase-error bound; the entries and
    both marginals (the slow-time one summed per pixel over l) agree with
    the cube."""
    rng = np.random.default_rng(71)
    r = _with_model(scenes.radar_for(2, 2, 4, 3, Fs=5e6, Tb=80e-6), 16)
    r.tx, r.rx = _random_antennas(rng, 2, 2, r.wavelength)
    base = scenes.tiny_scene(72, 4)
    px = _block_amp(base, rng.lognormal(0.0, 0.7, (r.L, base.P)))
    ref = brute.cube_exact(r, px)
    bound = brute.phase_error_bound(r, px)
    Y = o.cube(r, px)
    assert np.all(np.abs(Y - ref) <= bound), float(np.max(np.abs(Y - ref) / bound))
    c = rng.integers(0, r.C, 20)
    ll = rng.integers(0, r.L, 20)
    n = rng.integers(0, r.Ns, 20)
    assert np.array_equal(o.entries(r, px, c, ll, n), Y[c, ll, n])
    r2 = _with_model(scenes.radar_for(2, 3, 16, 8, Fs=5e6, Tb=80e-6), 16)
    px2 = scenes.block_strengths(scenes.tiny_scene(73, 29), r2.L, seed=74)
    Y2 = o.cube(r2, px2)
    assert relerr(Y2.sum(axis=2), o.marginal_n(r2, px2)) < 1e-11
    assert relerr(Y2.sum(axis=1), o.marginal_l(r2, px2)) < 1e-11


ALL_PINS = [pin_block_strength_reductions, pin_block_strength_sidebands, pin_block_strength_brute,
            pin_model_zero_is_default, pin_slot_timing_alias, pin_dechirp_physics,
            pin_far_field_model, pin_empty_scene, pin_single_scatterer_closed_form, pin_range_and_doppler_peaks,
            pin_marginals, pin_linearity, pin_static_scene_slices, pin_doppler_alias,
            pin_eq1_per_rx, pin_eq2_literal, pin_far_field_literal_one_pixel, pin_far_field, pin_entries_match_cube, pin_brute_recipe,
            pin_brute_exact, pin_brute_exact_no_carrier]
