"""Seeded synthetic inputs: radar parameter sets and rendered-pixel scatterers.

The paper renders each animation frame of a Blender scene into an
N_az x N_el image whose pixels carry range, strength, angle of arrival and
velocity (Sec. II, the paragraph after eq. (1) and the symbol list of
eq. (2)); every pixel is then one point target.  Blender is not available
here, so this module stands in for the rendering stage with a seeded ray
caster over an axis-aligned room and an ellipsoid pedestrian.

This module holds only input generation.  It evaluates no part of the beat
signal model: no range to an antenna, no phase and no phasor.  Both the CPU
oracle and the GPU library consume its output, and neither imports the
other.

Conventions
-----------
* Radar frame: the array sits on the back wall (y = 0) at the origin, the
  array axis is +x, boresight is +y, +z is up.
* Pixel p = n_el * G_az + n_az; azimuth spans +-60 deg, elevation +-30 deg,
  pixel centres at half-pixel offsets.
* A pixel position is x_p = t * u(az, el) with t the first hit along the ray.
* Strength a_p = |cos(incidence)| / t^2 * lognormal(0, 0.5).
* Radial velocity v_p = -(v . u) (positive when approaching).
* Everything is computed in float64 and stored as float32 (structure of
  arrays x, y, z, amp, vr).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

C0 = 299_792_458.0  # m/s

__all__ = [
    "C0", "Radar", "Pixels", "Room", "Pedestrian", "ula_geometry", "radar_for",
    "draw_room", "draw_pedestrian", "render", "cull", "concat", "scene_small",
    "scene_frame", "animation_frames", "serving_requests", "poisson_arrivals",
    "ServingRequest", "tiny_scene", "CircleWalk", "circle_walk",
]


# ----------------------------------------------------------------------------
# Radar parameter sets (eq. (1) symbols), virtual ULA geometry
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Radar:
    """Parameters of the eq. (1) signal model, SI units.

    M, N: Tx and Rx counts; Ns fast-time samples per chirp; L TDM blocks per
    CPI.  fc carrier [Hz], mu chirp slope [Hz/s], Fs sampling rate [Hz],
    Tb block period [s] (one block holds M chirps), c0 [m/s].
    tx, rx: antenna positions [M][3], [N][3] in metres (float64).
    carrier_phase: 1 puts the exact carrier phase 2 fc R / c0 into sigma.
    model: signal-model variant flags (1 far field as eq. (2), 2 Tx slot
    timing, 4 Doppler within the chirp, 8 residual video phase).
    """

    M: int
    N: int
    Ns: int
    L: int
    fc: float
    mu: float
    Fs: float
    Tb: float
    tx: np.ndarray
    rx: np.ndarray
    c0: float = C0
    carrier_phase: int = 1
    model: int = 0

    @property
    def C(self) -> int:
        return self.M * self.N

    @property
    def wavelength(self) -> float:
        return self.c0 / self.fc

    def cube_shape(self) -> Tuple[int, int, int]:
        return (self.C, self.L, self.Ns)


def ula_geometry(M: int, N: int, wavelength: float) -> Tuple[np.ndarray, np.ndarray]:
    """Virtual uniform linear array on +x.

    Rx r at x = r * lambda/2 and Tx m at x = m * N * lambda/2, so that virtual
    element (m, r) sits at (m*N + r) * lambda/2 (the index of eq. (2)'s
    far-field term with spacing lambda/2).  For N = 4 the Tx spacing is
    2 lambda.
    """
    d = wavelength / 2.0
    tx = np.zeros((M, 3), dtype=np.float64)
    rx = np.zeros((N, 3), dtype=np.float64)
    tx[:, 0] = np.arange(M, dtype=np.float64) * N * d
    rx[:, 0] = np.arange(N, dtype=np.float64) * d
    return tx, rx


def radar_for(M: int, N: int, Ns: int, L: int, Fs: float, Tb: float,
              fc: float = 77e9, mu: float = 30e6 / 1e-6,
              carrier_phase: int = 1) -> Radar:
    tx, rx = ula_geometry(M, N, C0 / fc)
    return Radar(M=M, N=N, Ns=Ns, L=L, fc=fc, mu=mu, Fs=Fs, Tb=Tb, tx=tx, rx=rx,
                 carrier_phase=carrier_phase)


# ----------------------------------------------------------------------------
# Pixels
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Pixels:
    """Structure of arrays of float32 scatterers (one per rendered pixel)."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    amp: np.ndarray
    vr: np.ndarray
    # float64 incidence cosine, kept for culling and tests only
    cos_inc: Optional[np.ndarray] = None
    is_ped: Optional[np.ndarray] = None

    @property
    def P(self) -> int:
        return int(self.x.shape[0])

    def take(self, idx) -> "Pixels":
        amp = self.amp[:, idx] if self.amp.ndim == 2 else self.amp[idx]
        return Pixels(self.x[idx], self.y[idx], self.z[idx], amp, self.vr[idx],
                      None if self.cos_inc is None else self.cos_inc[idx],
                      None if self.is_ped is None else self.is_ped[idx])

    def arrays(self) -> Tuple[np.ndarray, ...]:
        return (self.x, self.y, self.z, self.amp, self.vr)


def concat(parts: Sequence[Pixels]) -> Pixels:
    return Pixels(*(np.ascontiguousarray(np.concatenate([getattr(p, f) for p in parts]))
                    for f in ("x", "y", "z", "amp", "vr")))


# ----------------------------------------------------------------------------
# Room and pedestrian
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Room:
    W: float  # x extent, room spans [-W/2, W/2]
    D: float  # y depth, room spans [0, D]
    H: float = 3.0  # height, room spans [-H/2, H/2]


@dataclasses.dataclass
class Pedestrian:
    centre: np.ndarray  # (3,) float64, metres
    velocity: np.ndarray  # (3,) float64, m/s (horizontal)
    semi_axes: np.ndarray = dataclasses.field(
        default_factory=lambda: np.array([0.20, 0.15, 0.85]))


def draw_room(rng: np.random.Generator) -> Room:
    W = rng.uniform(3.0, 8.0)
    D = rng.uniform(3.0, 8.0)
    return Room(W=float(W), D=float(D))


def draw_pedestrian(rng: np.random.Generator, room: Room) -> Pedestrian:
    """Ellipsoid 0.4 x 0.3 x 1.7 m standing on the floor, at ground range
    U[1,6] m (clipped to D - 0.3) and azimuth U[-40, 40] deg (clipped so the
    centre stays 0.3 m from the side walls), speed U[0.5,1.5] m/s with a
    uniform heading in the x-y plane."""
    semi = np.array([0.20, 0.15, 0.85])
    rho = rng.uniform(1.0, 6.0)
    az = math.radians(rng.uniform(-40.0, 40.0))
    speed = rng.uniform(0.5, 1.5)
    heading = rng.uniform(0.0, 2.0 * math.pi)
    rho = min(rho, room.D - 0.3)
    xc = rho * math.sin(az)
    lim = room.W / 2.0 - 0.3
    xc = max(-lim, min(lim, xc))
    yc = math.sqrt(max(rho * rho - xc * xc, 0.09))
    yc = max(0.3, min(room.D - 0.3, yc))
    zc = -room.H / 2.0 + semi[2]
    centre = np.array([xc, yc, zc], dtype=np.float64)
    vel = np.array([speed * math.cos(heading), speed * math.sin(heading), 0.0])
    return Pedestrian(centre=centre, velocity=vel, semi_axes=semi)


def _pixel_directions(g_az: int, g_el: int) -> np.ndarray:
    """Unit ray per pixel, p = j * g_az + i, shape [P, 3] float64."""
    i = np.arange(g_az, dtype=np.float64)
    j = np.arange(g_el, dtype=np.float64)
    az = np.deg2rad(-60.0 + 120.0 * (i + 0.5) / g_az)
    el = np.deg2rad(-30.0 + 60.0 * (j + 0.5) / g_el)
    AZ, EL = np.meshgrid(az, el)  # [g_el, g_az]
    u = np.stack([np.cos(EL) * np.sin(AZ), np.cos(EL) * np.cos(AZ), np.sin(EL)], axis=-1)
    return u.reshape(-1, 3)


def _wall_hits(u: np.ndarray, room: Room) -> Tuple[np.ndarray, np.ndarray]:
    """Nearest positive hit on the room's walls for rays from the origin."""
    big = np.inf
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = np.where(u[:, 0] > 0, (room.W / 2) / u[:, 0],
                      np.where(u[:, 0] < 0, (-room.W / 2) / u[:, 0], big))
        ty = np.where(u[:, 1] > 0, room.D / u[:, 1], big)
        tz = np.where(u[:, 2] > 0, (room.H / 2) / u[:, 2],
                      np.where(u[:, 2] < 0, (-room.H / 2) / u[:, 2], big))
    T = np.stack([tx, ty, tz], axis=1)
    k = np.argmin(T, axis=1)
    t = T[np.arange(T.shape[0]), k]
    cos_inc = np.abs(u[np.arange(u.shape[0]), k])
    return t, cos_inc


def _ellipsoid_hits(u: np.ndarray, ped: Pedestrian) -> Tuple[np.ndarray, np.ndarray]:
    """First positive hit of rays from the origin on the ellipsoid
    |(x - c)/s| = 1; inf where missed.  Returns (t, |cos incidence|)."""
    s = ped.semi_axes
    o = -ped.centre / s
    d = u / s
    a = np.einsum("ij,ij->i", d, d)
    b = 2.0 * (d @ o)
    cc = float(o @ o) - 1.0
    disc = b * b - 4.0 * a * cc
    t = np.full(u.shape[0], np.inf)
    hit = disc > 0
    sq = np.sqrt(np.where(hit, disc, 0.0))
    t1 = (-b - sq) / (2.0 * a)
    t2 = (-b + sq) / (2.0 * a)
    tt = np.where(t1 > 0, t1, t2)
    ok = hit & (tt > 0)
    t[ok] = tt[ok]
    xs = u * np.where(ok, t, 0.0)[:, None]
    nrm = (xs - ped.centre) / (s * s)
    nrm /= np.maximum(np.linalg.norm(nrm, axis=1, keepdims=True), 1e-300)
    cos_inc = np.abs(np.einsum("ij,ij->i", u, nrm))
    return t, cos_inc


def render(rng: np.random.Generator, room: Room, ped: Optional[Pedestrian],
           g_az: int, g_el: int) -> Pixels:
    """Ray-cast the pixel grid into the room (and pedestrian), then draw the
    per-pixel lognormal(0, 0.5) strength factor in pixel order."""
    u = _pixel_directions(g_az, g_el)
    t, cos_inc = _wall_hits(u, room)
    vr = np.zeros(u.shape[0])
    is_ped = np.zeros(u.shape[0], dtype=bool)
    if ped is not None:
        te, ce = _ellipsoid_hits(u, ped)
        is_ped = te < t
        t = np.where(is_ped, te, t)
        cos_inc = np.where(is_ped, ce, cos_inc)
        vr = np.where(is_ped, -(u @ ped.velocity), 0.0)
    pos = u * t[:, None]
    amp = cos_inc / (t * t) * rng.lognormal(0.0, 0.5, size=u.shape[0])
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Pixels(f32(pos[:, 0]), f32(pos[:, 1]), f32(pos[:, 2]), f32(amp), f32(vr),
                  cos_inc=cos_inc, is_ped=is_ped)


def cull(px: Pixels, rel_floor: float = 1e-6, cos_floor: float = 1e-3) -> Pixels:
    """Drop zero-return pixels: strength below rel_floor * max strength or a
    grazing incidence cosine below cos_floor.  Occluded wall points are never
    emitted by `render` in the first place."""
    a = px.amp.astype(np.float64)
    keep = a >= rel_floor * (a.max() if a.size else 0.0)
    if px.cos_inc is not None:
        keep &= px.cos_inc >= cos_floor
    return px.take(np.nonzero(keep)[0])


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------
def scene_small(seed: int = 0, grid: int = 64, pedestrian: bool = False) -> Pixels:
    """Single frame: seeded room, grid x grid pixels, optional pedestrian."""
    rng = np.random.default_rng(seed)
    room = draw_room(rng)
    ped = draw_pedestrian(rng, room) if pedestrian else None
    return render(rng, room, ped, grid, grid)


def scene_frame(seed: int, grid: int, pedestrian: bool = True) -> Pixels:
    return scene_small(seed, grid, pedestrian)


def _advance(ped: Pedestrian, room: Room, dt: float) -> Pedestrian:
    """Move the pedestrian by v*dt; the heading reflects 0.3 m from a wall."""
    c = ped.centre + ped.velocity * dt
    v = ped.velocity.copy()
    lo = np.array([-room.W / 2 + 0.3, 0.3])
    hi = np.array([room.W / 2 - 0.3, room.D - 0.3])
    for k in range(2):
        if c[k] > hi[k]:
            c[k] = 2 * hi[k] - c[k]
            v[k] = -v[k]
        elif c[k] < lo[k]:
            c[k] = 2 * lo[k] - c[k]
            v[k] = -v[k]
    return Pedestrian(centre=c, velocity=v, semi_axes=ped.semi_axes)


def animation_frames(seed: int = 3, nframes: int = 64, dt: float = 1.0 / 30.0,
                     p_min: int = 2048, p_max: int = 262144,
                     max_grid: int = 512) -> List[Pixels]:
    """Animated room-plus-pedestrian frames.  The room and the pedestrian's
    start come from `seed`; frame f draws its grid side (log-uniform pixel
    target in [p_min, p_max]) and its strengths from the generator seeded by
    (seed, f).  Each frame is culled."""
    rng = np.random.default_rng(seed)
    room = draw_room(rng)
    ped = draw_pedestrian(rng, room)
    frames = []
    for f in range(nframes):
        if f:
            ped = _advance(ped, room, dt)
        frng = np.random.default_rng([seed, f])
        target = math.exp(frng.uniform(math.log(p_min), math.log(p_max)))
        side = int(min(max_grid, max(1, round(math.sqrt(target)))))
        frames.append(cull(render(frng, room, ped, side, side)))
    return frames


@dataclasses.dataclass
class CircleWalk:
    """Frames of the walking-circle scenario and the pedestrian's ground
    truth per frame: centre [F][3], velocity [F][3] and the radial velocity of
    the centre seen from the radar (positive when approaching)."""
    frames: List[Pixels]
    centres: np.ndarray
    velocities: np.ndarray
    v_radial: np.ndarray
    speed: float
    fps: float


def circle_walk(seed: int = 5, nframes: int = 100, fps: float = 24.0, radius: float = 3.0,
                centre_xy: Tuple[float, float] = (0.0, 5.5), grid: int = 256,
                room_wd: Tuple[float, float] = (12.0, 10.0), theta0: float = 0.0,
                frame_ids: Optional[Sequence[int]] = None) -> CircleWalk:
    """Stand-in for the walking scenario of Sec. III: the ellipsoid pedestrian
    walks counter-clockwise at constant speed around a circle of `radius`
    metres centred at `centre_xy`, one full turn over `nframes` frames at
    `fps` (2 pi 3 m / (100 / 24 s) = 4.52 m/s for the paper's numbers), in a
    fixed room of width x depth `room_wd`.  Frame f renders the pedestrian at
    angle theta0 + 2 pi f / nframes with strengths drawn from the generator
    seeded by (seed, f).  frame_ids renders only those frames of the walk."""
    room = Room(W=float(room_wd[0]), D=float(room_wd[1]))
    semi = np.array([0.20, 0.15, 0.85])
    zc = -room.H / 2.0 + semi[2]
    speed = 2.0 * math.pi * radius * fps / nframes
    frames, centres, vels, vrad = [], [], [], []
    for f in (range(nframes) if frame_ids is None else frame_ids):
        th = theta0 + 2.0 * math.pi * f / nframes
        c = np.array([centre_xy[0] + radius * math.cos(th), centre_xy[1] + radius * math.sin(th), zc])
        v = np.array([-speed * math.sin(th), speed * math.cos(th), 0.0])
        ped = Pedestrian(centre=c, velocity=v, semi_axes=semi)
        frng = np.random.default_rng([seed, f])
        frames.append(cull(render(frng, room, ped, grid, grid)))
        centres.append(c)
        vels.append(v)
        vrad.append(-float(v @ (c / np.linalg.norm(c))))
    return CircleWalk(frames=frames, centres=np.array(centres), velocities=np.array(vels),
                      v_radial=np.array(vrad), speed=speed, fps=fps)


@dataclasses.dataclass
class ServingRequest:
    index: int
    radar: Radar
    pixels: Pixels

    @property
    def terms(self) -> int:
        return self.pixels.P * self.radar.C * self.radar.Ns * self.radar.L


SERVING_ARRAYS = ((1, 4), (3, 4), (12, 16))
SERVING_NS = (128, 256, 512)
SERVING_L = (64, 128, 256)


def serving_requests(count: int, base_seed: int = 1000, p_min: int = 4096,
                     p_max: int = 262144, start: int = 0) -> List[ServingRequest]:
    """Mixed cube requests.  Request i uses seed base_seed + i and draws its
    array (1x4, 3x4 or 12x16), Ns, L and a log-uniform pixel target; the
    sampling rate is Ns / 25.6 us, the block period M x 40 us, the chirp slope
    30 MHz/us and the carrier 77 GHz."""
    out = []
    for i in range(start, start + count):
        rng = np.random.default_rng(base_seed + i)
        M, N = SERVING_ARRAYS[int(rng.integers(0, 3))]
        Ns = SERVING_NS[int(rng.integers(0, 3))]
        L = SERVING_L[int(rng.integers(0, 3))]
        target = math.exp(rng.uniform(math.log(p_min), math.log(p_max)))
        side = int(min(512, max(1, round(math.sqrt(target)))))
        room = draw_room(rng)
        ped = draw_pedestrian(rng, room)
        px = cull(render(rng, room, ped, side, side))
        radar = radar_for(M, N, Ns, L, Fs=Ns / 25.6e-6, Tb=M * 40e-6)
        out.append(ServingRequest(index=i, radar=radar, pixels=px))
    return out


def poisson_arrivals(count: int, rate_hz: float, seed: int = 7) -> np.ndarray:
    """Arrival times [s] of a Poisson process (exponential gaps), seeded."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=count))


def tiny_scene(seed: int, P: int, span: float = 6.0, vmax: float = 3.0) -> Pixels:
    """Free-floating scatterers for small brute-force and property tests."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-span / 2, span / 2, P)
    y = rng.uniform(0.5, span, P)
    z = rng.uniform(-1.0, 1.0, P)
    amp = rng.lognormal(0.0, 0.5, P)
    vr = rng.uniform(-vmax, vmax, P)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Pixels(f32(x), f32(y), f32(z), f32(amp), f32(vr))


def block_strengths(px: Pixels, L: int, seed: int, depth: float = 0.5) -> Pixels:
    """The same scatterers with a strength per TDM block (float32 [L][P],
    row l = block l): each pixel's strength swings slowly over the CPI,
    a_p (1 + depth sin(2pi (f_p l / L) + phase_p)) with f_p ~ U[0, 3) cycles
    per CPI and phase_p ~ U[0, 2pi), as an aspect-dependent return would."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.0, 3.0, px.P)
    ph = rng.uniform(0.0, 2 * np.pi, px.P)
    l = np.arange(L, dtype=np.float64)[:, None]
    a = px.amp.astype(np.float64)[None, :] * (1.0 + depth * np.sin(2 * np.pi * f[None, :] * l / L + ph[None, :]))
    return Pixels(px.x, px.y, px.z, np.ascontiguousarray(a, dtype=np.float32), px.vr,
                  px.cos_inc, px.is_ped)


# ----------------------------------------------------------------------------
# The five workload recipes (small plain case, headline single frame, the
# animation batch and the serving mix share these radars)
# ----------------------------------------------------------------------------
def radar_small() -> Radar:
    """2 Tx x 4 Rx, Ns=64, L=32, Fs=5 MHz, Tb=2x40 us."""
    return radar_for(2, 4, 64, 32, Fs=5e6, Tb=2 * 40e-6)


def radar_frame() -> Radar:
    """3 Tx x 4 Rx, Ns=256, L=128, Fs=10 MHz, Tb=3x40 us."""
    return radar_for(3, 4, 256, 128, Fs=10e6, Tb=3 * 40e-6)


def radar_batch() -> Radar:
    """3 Tx x 4 Rx, Ns=256, L=64, Fs=10 MHz, Tb=3x40 us."""
    return radar_for(3, 4, 256, 64, Fs=10e6, Tb=3 * 40e-6)


def workload_small() -> Tuple[Radar, Pixels]:
    """64x64 room pixels, no pedestrian (v = 0), seed 0."""
    return radar_small(), scene_small(seed=0, grid=64, pedestrian=False)


def workload_frame() -> Tuple[Radar, Pixels]:
    """256x256 room-plus-pedestrian pixels, seed 1."""
    return radar_frame(), scene_small(seed=1, grid=256, pedestrian=True)
