"""Helpers of the GPU parity tests (GPU path through the C ABI, CPU oracle)."""
from __future__ import annotations

import numpy as np

# Parity gates (relative L2 norm and max-abs relative to the largest entry of
# the reference), per form and output type.
GATE_PLAIN_C128 = 1e-12
GATE_PLAIN_C64 = 1e-7
GATE_PLAIN_C64_MAX = 2.0 ** -23
GATE_MFMA = 1e-4


def errors(got, ref):
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    d = got - ref
    rel = float(np.linalg.norm(d.ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))
    mx = float(np.max(np.abs(d)) / max(np.max(np.abs(ref)), 1e-300)) if d.size else 0.0
    return rel, mx


def marginal_ratio(cube, ref_marginal, axis):
    """The cube's error seen through a closed-form marginal.  Summing the
    cube over `axis` (2: fast time, 1: slow time, n entries per row) turns an
    error dY into dM with ||dM||_2 <= sqrt(n) ||dY||_2 and
    max |dM| <= n max |dY| (Cauchy-Schwarz), so a cube within relative L2
    error g and max-abs error g (relative to its largest entry) gives
    max(||dM||_2 / (sqrt(n) ||Y||_2), max |dM| / (n max |Y|)) <= g; this
    returns that maximum, to be held to the cube's gate.  (A plain relative
    error of the marginal is not implied by the gates: where the pixels'
    phases cancel over a row the marginal is far smaller than the row, and
    the entries' rounding, which does not cancel, dominates it.)"""
    cube = np.asarray(cube, dtype=np.complex128)
    d = cube.sum(axis=axis) - np.asarray(ref_marginal)
    n = cube.shape[axis]
    l2 = np.linalg.norm(d.ravel()) / max(np.sqrt(n) * np.linalg.norm(cube.ravel()), 1e-300)
    mx = np.max(np.abs(d)) / max(n * np.max(np.abs(cube)), 1e-300)
    return float(max(l2, mx))


def synth(radar, px, form, dtype, device="cuda:0", max_pixels=None, ws=False):
    import torch
    from paper_2307_09226_amd import rs
    plan = rs.rs_cube_plan(radar, form, dtype, max_pixels=max(px.P, 1) if max_pixels is None else max_pixels)
    dpx = rs.DevicePixels.from_host(px, device)
    cube = rs.new_cube(plan, device)
    if ws:
        nb = plan.workspace_bytes(px.P)
        buf = torch.empty(max(nb, 1), dtype=torch.uint8, device=device)
        rs.rs_beat_synthesize_ws(plan, dpx, cube, buf)
    else:
        rs.rs_beat_synthesize(plan, dpx, cube)
    torch.cuda.synchronize()
    out = cube.cpu().numpy()
    plan.close()
    return out


def sample_indices(shape, k, seed=0, include_corners=True):
    """k seeded (c, l, n) indices, plus the first and last entries."""
    rng = np.random.default_rng(seed)
    C, L, Ns = shape
    c = rng.integers(0, C, k)
    l = rng.integers(0, L, k)
    n = rng.integers(0, Ns, k)
    if include_corners:
        c = np.concatenate([c, [0, C - 1, C - 1, 0]])
        l = np.concatenate([l, [0, L - 1, 0, L - 1]])
        n = np.concatenate([n, [0, Ns - 1, Ns - 1, 0]])
    return c.astype(np.int32), l.astype(np.int32), n.astype(np.int32)
