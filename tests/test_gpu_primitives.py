"""Device primitives the synthesis kernels rest on, checked element by element
against the host through a test-only library (tests/csrc/rs_prims.hip, built
with the library's flags by build.py; librs.so is not involved):

* binary64 sqrt and the per-antenna distance of the phase-argument recipe are
  bitwise those of the host (IEEE correctly rounded sqrt, no contraction), so
  the GPU's ranges are bitwise the oracle's;
* v_fract_f64 is v - floor(v) held below 1, and the recipe's rs_frac is
  v - floor(v) exactly (1.0 for tiny negative v);
* the hardware binary32 sin / cos, input in revolutions, over [0, 1): its
  largest error against the binary64 sin / cos of 2 pi x is bounded by
  SINCOS_MAX_ABS (the bound the matrix-core form's error budget uses);
* the fp16 split of a binary32 pair is hi = rne16(x), lo = rne16(x - hi),
  bitwise equal to NumPy's round-to-nearest-even conversions, and that
  split times j is the split of (-y, x) (the imaginary D column).
"""
import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "csrc", "librs_prims.so")

# Largest error of the hardware sin / cos on revolution inputs in [0, 1),
# absolute, against sin / cos of 2 pi x in binary64: 2^-22 (measured on
# MI355X: 1.24e-7, about 2^-23, with an RMS of 3.5e-8).
SINCOS_MAX_ABS = 2.0 ** -22


@pytest.fixture(scope="module")
def prims():
    import torch  # one HIP runtime in the process: torch's, loaded first
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} missing: build it first (__graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    lib.prim_distance.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, vp]
    lib.prim_sqrt.argtypes = [vp, vp, ctypes.c_int, vp]
    lib.prim_fract.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp]
    lib.prim_sincos.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.prim_split16.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.prim_split16j.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    for f in (lib.prim_distance, lib.prim_sqrt, lib.prim_fract, lib.prim_sincos, lib.prim_split16,
              lib.prim_split16j):
        f.restype = ctypes.c_int
    return lib


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _empty(n, dtype):
    import torch
    return torch.empty(n, dtype=dtype, device="cuda:0")


def _run(fn, *args):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    assert fn(*[a.data_ptr() if hasattr(a, "data_ptr") else a for a in args], stream) == 0
    torch.cuda.synchronize()


def test_sqrt_bitwise(prims):
    """2^20 seeded doubles: squared ranges of the workloads (1e-4 .. 1e4 m^2,
    log-uniform), exact squares, and positive doubles of every exponent
    (subnormals included)."""
    import torch
    rng = np.random.default_rng(11)
    n = 1 << 20
    r2 = np.exp(rng.uniform(np.log(1e-4), np.log(1e4), n // 2))
    sq = np.square(rng.uniform(0.0, 100.0, n // 8))
    bits = rng.integers(1, 0x7FEFFFFFFFFFFFFF, n - n // 2 - n // 8, dtype=np.int64)
    v = np.concatenate([r2, sq, bits.view(np.float64)])
    out = _empty(n, torch.float64)
    _run(prims.prim_sqrt, _dev(v), out, n)
    got = out.cpu().numpy()
    want = np.sqrt(v)
    bad = np.flatnonzero(got.view(np.int64) != want.view(np.int64))
    assert bad.size == 0, (bad.size, v[bad[:4]], got[bad[:4]], want[bad[:4]])


def test_distance_recipe_bitwise(prims):
    """rs_distance of float32 positions to binary64 antennas equals the
    recipe sqrt((dx*dx + dy*dy) + dz*dz), dx = (double)x - a.x, evaluated by
    NumPy in binary64 (no contraction) bit for bit."""
    import torch
    rng = np.random.default_rng(12)
    n = 1 << 18
    pos = [rng.uniform(-20.0, 20.0, n).astype(np.float32) for _ in range(3)]
    lam = 299792458.0 / 77e9
    for ant in (np.zeros(3), np.array([11 * lam / 2, 0.0, 0.0]), rng.uniform(-0.05, 0.05, 3)):
        out = _empty(n, torch.float64)
        _run(prims.prim_distance, _dev(pos[0]), _dev(pos[1]), _dev(pos[2]), _dev(ant.astype(np.float64)),
             out, n)
        d = [p.astype(np.float64) - a for p, a in zip(pos, ant)]
        want = np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
        assert np.array_equal(out.cpu().numpy().view(np.int64), want.view(np.int64)), ant


def test_fract_semantics(prims):
    """v_fract_f64 returns v - floor(v) held below 1 (the largest double
    below 1 where v - floor(v) rounds to 1); rs_frac returns v - floor(v)
    exactly; their binary32 rounding is what the phasors use."""
    import torch
    rng = np.random.default_rng(13)
    below1 = np.nextafter(1.0, 0.0)
    edges = np.array([0.0, 1.0, -1.0, 0.5, -0.5, 0.25, -1e-17, -1e-300, -5e-324, 5e-324, below1, -below1,
                      1.0 + 2.0 ** -52, 6000.123456789, -6000.123456789, 2.0 ** 52 + 0.5, 2.0 ** 53,
                      1e20, -1e20, 3.0, -3.0, -2.5, 1e-310])
    v = np.concatenate([edges, rng.uniform(-1e4, 1e4, 1 << 16), rng.uniform(-1.0, 1.0, 1 << 16),
                        -np.exp(rng.uniform(-700, -1, 1 << 12))])
    n = v.size
    hw, sub, f32 = _empty(n, torch.float64), _empty(n, torch.float64), _empty(n, torch.float32)
    _run(prims.prim_fract, _dev(v), hw, sub, f32, n)
    exact = v - np.floor(v)
    hw, sub, f32 = hw.cpu().numpy(), sub.cpu().numpy(), f32.cpu().numpy()
    assert np.array_equal(sub, exact)
    assert np.array_equal(hw, np.minimum(exact, below1))
    assert np.all((hw >= 0.0) & (hw < 1.0))
    assert np.array_equal(f32, hw.astype(np.float32))
    # tiny negative values: exact difference rounds to 1, the hardware keeps it below
    k = list(edges).index(-1e-17)
    assert sub[k] == 1.0 and hw[k] == below1


def test_hardware_sincos_on_revolutions(prims):
    """Largest absolute error of the binary32 hardware sin / cos (input in
    revolutions) over [0, 1), against binary64 sin / cos of 2 pi x."""
    import torch
    rng = np.random.default_rng(14)
    n = 1 << 20
    x = np.concatenate([rng.uniform(0.0, 1.0, n - 8).astype(np.float32),
                        np.array([0.0, 0.125, 0.25, 0.5, 0.75, np.nextafter(np.float32(1), np.float32(0)),
                                  2.0 ** -24, 0.999], dtype=np.float32)])
    s, c = _empty(n, torch.float32), _empty(n, torch.float32)
    _run(prims.prim_sincos, _dev(x), s, c, n)
    xd = x.astype(np.float64)
    es = np.abs(s.cpu().numpy().astype(np.float64) - np.sin(2 * np.pi * xd))
    ec = np.abs(c.cpu().numpy().astype(np.float64) - np.cos(2 * np.pi * xd))
    print(f"hardware sin/cos on [0,1) revolutions: max abs error sin {es.max():.3e} cos {ec.max():.3e}, "
          f"rms {np.sqrt(np.mean(es ** 2)):.3e} / {np.sqrt(np.mean(ec ** 2)):.3e}", flush=True)
    assert es.max() <= SINCOS_MAX_ABS and ec.max() <= SINCOS_MAX_ABS


def test_split16_round_to_nearest_even(prims):
    """hi = rne16(x) and lo = rne16(x - hi) of binary32 pairs, bitwise equal
    to NumPy's conversions, over phasor components in [-1, 1], the
    chunk-scaled strengths up to 2^15 and small values; x - hi is exact in
    binary32 and hi + lo recovers x to 2^-22 of |x| where x - hi stays a
    normal fp16 number."""
    import torch
    rng = np.random.default_rng(15)
    n = 1 << 19
    unit = rng.uniform(-1.0, 1.0, n)
    scaled = rng.uniform(-1.0, 1.0, n) * 2.0 ** rng.integers(-14, 15, n)
    tiny = rng.uniform(-1.0, 1.0, n // 4) * 2.0 ** rng.integers(-30, -14, n // 4)
    x = np.concatenate([unit, scaled, tiny, [0.0, -0.0, 1.0, -1.0, 65504.0, 2.0 ** -24]]).astype(np.float32)
    if x.size % 2:
        x = np.append(x, np.float32(0.5))
    pairs = x.size // 2
    hi, lo = _empty(pairs, torch.int32), _empty(pairs, torch.int32)
    _run(prims.prim_split16, _dev(x), hi, lo, pairs)
    got_hi = hi.cpu().numpy().view(np.uint16)  # (x, y) per pair, x first
    got_lo = lo.cpu().numpy().view(np.uint16)
    want_hi = x.astype(np.float16)
    resid = x - want_hi.astype(np.float32)
    assert np.array_equal(resid.astype(np.float64), x.astype(np.float64) - want_hi.astype(np.float64))
    want_lo = resid.astype(np.float16)
    assert np.array_equal(got_hi, want_hi.view(np.uint16))
    assert np.array_equal(got_lo, want_lo.view(np.uint16))
    # where x - hi stays a normal fp16 number, hi + lo carries 22 bits
    big = np.abs(x) >= 2.0 ** -2
    rec = want_hi.astype(np.float64) + want_lo.astype(np.float64)
    assert np.all(np.abs(rec - x)[big] <= 2.0 ** -22 * np.abs(x.astype(np.float64))[big])


def test_split16_times_j(prims):
    """The imaginary D column (-w, u) is the split of (u, w) times j: hi
    halves bitwise rne16(-w), rne16(u); lo halves rne16(-w - rne16(-w)),
    rne16(u - rne16(u)) equal in value, bitwise wherever nonzero (a zero lo
    half may carry either sign).  Pairs include exact fp16 values, whose lo
    halves are zero, and fp16 subnormal residuals."""
    import torch
    rng = np.random.default_rng(16)
    n = 1 << 18
    unit = rng.uniform(-1.0, 1.0, n)
    scaled = rng.uniform(-1.0, 1.0, n) * 2.0 ** rng.integers(-14, 15, n)
    tiny = rng.uniform(-1.0, 1.0, n // 4) * 2.0 ** rng.integers(-30, -14, n // 4)
    exact = rng.uniform(-1.0, 1.0, n // 4).astype(np.float16).astype(np.float64)
    x = np.concatenate([unit, scaled, tiny, exact, [0.0, -0.0, 1.0, -1.0, 65504.0, 2.0 ** -24]])
    x = rng.permutation(x).astype(np.float32)
    if x.size % 2:
        x = np.append(x, np.float32(0.5))
    pairs = x.size // 2
    hi, lo = _empty(pairs, torch.int32), _empty(pairs, torch.int32)
    _run(prims.prim_split16j, _dev(x), hi, lo, pairs)
    got_hi = hi.cpu().numpy().view(np.float16)  # (-y, x) per pair
    got_lo = lo.cpu().numpy().view(np.float16)
    xy = x.reshape(-1, 2)
    xj = np.stack([-xy[:, 1], xy[:, 0]], axis=1).reshape(-1)  # (-y, x), binary32
    want_hi = xj.astype(np.float16)
    want_lo = (xj - want_hi.astype(np.float32)).astype(np.float16)
    assert np.array_equal(got_hi.view(np.uint16), want_hi.view(np.uint16))
    assert np.array_equal(got_lo, want_lo)  # by value: +0 == -0
    nz = want_lo != 0
    assert np.array_equal(got_lo.view(np.uint16)[nz], want_lo.view(np.uint16)[nz])
    assert np.count_nonzero(~nz) > n // 8  # the zero-lo case is exercised
