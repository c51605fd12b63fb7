"""Serving loop: continuous batching, admission, back-pressure, failures."""
import time

import numpy as np
import pytest

import oracle
from paper_2307_09226_amd import scenes
from gpu_util import GATE_MFMA, errors, sample_indices

pytestmark = pytest.mark.gpu


def _rs():
    from paper_2307_09226_amd import rs
    return rs


def _wait(sess, tickets, timeout=60.0):
    rs = _rs()
    t0 = time.time()
    states = {}
    while time.time() - t0 < timeout:
        states = {t: sess.poll(t)[0] for t in tickets}
        if all(s in (rs.RS_REQ_DONE, rs.RS_REQ_FAILED, rs.RS_REQ_CANCELLED) for s in states.values()):
            return states
        time.sleep(0.002)
    raise TimeoutError(states)


def _requests(n, start=0, p_max=40000):
    return scenes.serving_requests(n, start=start, p_max=p_max)


def test_alone_vs_mix_bitwise_and_parity():
    """Each request's cube is the same alone (rs_beat_synthesize) and when
    served in a mix of concurrently admitted requests; sampled entries match
    the oracle."""
    import torch
    rs = _rs()
    reqs = _requests(8)
    plans = [rs.rs_cube_plan(q.radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=q.pixels.P)
             for q in reqs]
    dpx = [rs.DevicePixels.from_host(q.pixels) for q in reqs]
    alone = []
    for p, d in zip(plans, dpx):
        c = rs.new_cube(p)
        rs.rs_beat_synthesize(p, d, c)
        alone.append(c)
    torch.cuda.synchronize()
    sess = rs.Session(hbm_budget=2 << 30, max_slots=8, slice_items=300)
    cubes = [rs.new_cube(p) for p in plans]
    tickets = [sess.submit(p, d, c) for p, d, c in zip(plans, dpx, cubes)]
    states = _wait(sess, tickets)
    assert all(s == rs.RS_REQ_DONE for s in states.values())
    st = sess.stats()
    assert st["done"] == len(reqs) and st["launches"] >= 2
    for i, (a, b) in enumerate(zip(alone, cubes)):
        assert torch.equal(a, b), i
    for i in (0, 3, 7):
        q = reqs[i]
        c, l, n = sample_indices(q.radar.cube_shape(), 200, seed=i)
        ref = oracle.entries(q.radar, q.pixels, c, l, n)
        rel, mx = errors(cubes[i].cpu().numpy()[c, l, n], ref)
        assert rel <= GATE_MFMA and mx <= GATE_MFMA
    sess.close()


# Full-size requests of the serving pool (base seed 1000): the four largest
# (2.95e12, 1.62e12, 1.17e12 and 1.02e12 terms, 192 channels each) and four
# smaller ones, 3x4 and 1x4 arrays among them.
FULL_MIX = (17, 31, 10, 41, 32, 3, 5, 8)


def test_full_size_mix_bitwise_and_parity():
    """A mix of full-size pool requests served together (slices of the
    default size, shortest-remaining shares) gives each request the cube it
    gets alone, bit for bit, and sampled entries of every request match the
    oracle."""
    import torch
    rs = _rs()
    reqs = [scenes.serving_requests(1, start=i)[0] for i in FULL_MIX]
    assert max(q.radar.C * q.radar.Ns * q.radar.L * q.pixels.P for q in reqs) > 2.9e12
    plans = [rs.rs_cube_plan(q.radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=q.pixels.P)
             for q in reqs]
    dpx = [rs.DevicePixels.from_host(q.pixels) for q in reqs]
    alone = []
    for p, d in zip(plans, dpx):
        c = rs.new_cube(p)
        rs.rs_beat_synthesize(p, d, c)
        alone.append(c)
    torch.cuda.synchronize()
    sess = rs.Session(hbm_budget=12 << 30, max_slots=8)
    cubes = [rs.new_cube(p) for p in plans]
    tickets = [sess.submit(p, d, c) for p, d, c in zip(plans, dpx, cubes)]
    states = _wait(sess, tickets, timeout=120.0)
    assert all(s == rs.RS_REQ_DONE for s in states.values())
    st = sess.stats()
    assert st["done"] == len(reqs) and st["launches"] >= len(reqs)
    for i, (a, b) in enumerate(zip(alone, cubes)):
        assert torch.equal(a, b), FULL_MIX[i]
    for i, q in enumerate(reqs):
        c, l, n = sample_indices(q.radar.cube_shape(), 128, seed=100 + i)
        ref = oracle.entries(q.radar, q.pixels, c, l, n)
        rel, mx = errors(cubes[i].cpu().numpy()[c, l, n], ref)
        print(f"request {FULL_MIX[i]}: C={q.radar.C} Ns={q.radar.Ns} L={q.radar.L} P={q.pixels.P} "
              f"relL2={rel:.3e} maxabs={mx:.3e}", flush=True)
        assert rel <= GATE_MFMA and mx <= GATE_MFMA, FULL_MIX[i]
    sess.close()


def test_admission_respects_budget_and_backpressure():
    import torch
    rs = _rs()
    reqs = _requests(6)
    plans = [rs.rs_cube_plan(q.radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=q.pixels.P)
             for q in reqs]
    dpx = [rs.DevicePixels.from_host(q.pixels) for q in reqs]
    need = max(p.workspace_bytes(q.pixels.P) for p, q in zip(plans, reqs))
    # room for exactly one request's partial sums at a time
    sess = rs.Session(hbm_budget=need, max_slots=4, queue_cap=3)
    cubes = [rs.new_cube(p) for p in plans]
    tickets = []
    busy = 0
    for p, d, c in zip(plans, dpx, cubes):
        t = sess.try_submit(p, d, c)
        if t is None:
            busy += 1
            _wait(sess, tickets)
            t = sess.submit(p, d, c)
        tickets.append(t)
    _wait(sess, tickets)
    st = sess.stats()
    assert st["footprint_peak"] <= need
    assert st["done"] == len(reqs)
    # a request that can never fit is rejected at submit
    small = rs.Session(hbm_budget=1024, max_slots=2)
    with pytest.raises(rs.RSError) as e:
        small.submit(plans[0], dpx[0], cubes[0])
    assert e.value.status == rs.RS_E_INVALID
    small.close()
    sess.close()


def test_injected_failure_only_marks_affected_requests():
    import torch
    rs = _rs()
    reqs = _requests(4)
    plans = [rs.rs_cube_plan(q.radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=q.pixels.P)
             for q in reqs]
    dpx = [rs.DevicePixels.from_host(q.pixels) for q in reqs]
    sess = rs.Session(hbm_budget=4 << 30, max_slots=1)
    sess.inject_failure(1)
    cubes = [rs.new_cube(p) for p in plans]
    tickets = [sess.submit(p, d, c) for p, d, c in zip(plans, dpx, cubes)]
    states = _wait(sess, tickets)
    assert states[tickets[0]] == rs.RS_REQ_FAILED
    assert all(states[t] == rs.RS_REQ_DONE for t in tickets[1:])
    ref = rs.new_cube(plans[2])
    rs.rs_beat_synthesize(plans[2], dpx[2], ref)
    torch.cuda.synchronize()
    assert torch.equal(ref, cubes[2])
    assert sess.stats()["failed"] == 1
    sess.close()


def test_cancel_queued_and_not_found():
    rs = _rs()
    reqs = _requests(3)
    plans = [rs.rs_cube_plan(q.radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=q.pixels.P)
             for q in reqs]
    dpx = [rs.DevicePixels.from_host(q.pixels) for q in reqs]
    sess = rs.Session(hbm_budget=4 << 30, max_slots=1)
    cubes = [rs.new_cube(p) for p in plans]
    tickets = [sess.submit(p, d, c) for p, d, c in zip(plans, dpx, cubes)]
    try:
        sess.cancel(tickets[2])
        cancelled = True
    except rs.RSError as e:  # already admitted
        assert e.status == rs.RS_E_BUSY
        cancelled = False
    states = _wait(sess, tickets)
    if cancelled:
        assert states[tickets[2]] == rs.RS_REQ_CANCELLED
    with pytest.raises(rs.RSError) as e:
        sess.poll(123456789)
    assert e.value.status == rs.RS_E_NOT_FOUND
    sess.close()


def test_plain_plan_rejected_and_zero_pixel_request():
    import torch
    rs = _rs()
    q = _requests(1)[0]
    plain = rs.rs_cube_plan(q.radar, rs.RS_FORM_FP64_DIRECT, rs.RS_C64, max_pixels=q.pixels.P)
    mf = rs.rs_cube_plan(q.radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=q.pixels.P)
    d = rs.DevicePixels.from_host(q.pixels)
    sess = rs.Session(hbm_budget=1 << 30, max_slots=2)
    with pytest.raises(rs.RSError) as e:
        sess.submit(plain, d, rs.new_cube(plain))
    assert e.value.status == rs.RS_E_UNSUPPORTED
    empty = rs.DevicePixels(*(torch.zeros(0, dtype=torch.float32, device="cuda:0") for _ in range(5)))
    cube = rs.new_cube(mf)
    cube.fill_(3)
    t = sess.submit(mf, empty, cube)
    assert _wait(sess, [t])[t] == rs.RS_REQ_DONE
    assert torch.count_nonzero(cube).item() == 0
    sess.close()


def test_both_policies_give_the_alone_cubes():
    """Shortest-remaining-first and equal shares, in arrival order or with
    overtaking, give every request the cube it has alone, bit for bit; the
    stats count the requests' whole HBM (pixels, cubes, partial sums)."""
    import torch
    rs = _rs()
    reqs = _requests(6)
    plans = [rs.rs_cube_plan(q.radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=q.pixels.P)
             for q in reqs]
    dpx = [rs.DevicePixels.from_host(q.pixels) for q in reqs]
    alone = []
    for p, d in zip(plans, dpx):
        c = rs.new_cube(p)
        rs.rs_beat_synthesize(p, d, c)
        alone.append(c)
    torch.cuda.synchronize()
    for policy, strict in ((rs.RS_SCHED_SHORTEST, False), (rs.RS_SCHED_EQUAL, True)):
        sess = rs.Session(hbm_budget=2 << 30, max_slots=4, policy=policy, strict_fifo=strict,
                          slice_terms=2e10)
        cubes = [rs.new_cube(p) for p in plans]
        tickets = [sess.submit(p, d, c) for p, d, c in zip(plans, dpx, cubes)]
        states = _wait(sess, tickets)
        assert all(s == rs.RS_REQ_DONE for s in states.values()), (policy, states)
        for i, (a, b) in enumerate(zip(alone, cubes)):
            assert torch.equal(a, b), (policy, i)
        st = sess.stats()
        assert st["request_bytes_peak"] > st["footprint_peak"] > 0
        assert st["request_bytes_now"] == 0 and st["footprint_now"] == 0 and st["device_error"] == 0
        sess.close()
    with pytest.raises(rs.RSError) as e:
        rs.Session(policy=7)
    assert e.value.status == rs.RS_E_INVALID


def test_device_error_stops_the_session():
    """A device error seen at a completion check (injected from the host;
    the device is untouched): every admitted and queued request ends FAILED,
    later submits are refused with RS_E_DEVICE, and drain and close return."""
    rs = _rs()
    reqs = _requests(5, p_max=60000)
    plans = [rs.rs_cube_plan(q.radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=q.pixels.P)
             for q in reqs]
    dpx = [rs.DevicePixels.from_host(q.pixels) for q in reqs]
    sess = rs.Session(hbm_budget=4 << 30, max_slots=1, slice_terms=2e9)
    cubes = [rs.new_cube(p) for p in plans]
    tickets = [sess.submit(p, d, c) for p, d, c in zip(plans, dpx, cubes)]
    sess.inject_device_error()
    states = _wait(sess, tickets)
    sess.drain()
    st = sess.stats()
    print("states after the device error:", states, st, flush=True)
    assert st["device_error"] == 1
    assert any(s == rs.RS_REQ_FAILED for s in states.values())
    assert all(s in (rs.RS_REQ_DONE, rs.RS_REQ_FAILED) for s in states.values())
    assert st["done"] + st["failed"] == len(reqs)
    assert st["running_now"] == 0 and st["queued_now"] == 0 and st["footprint_now"] == 0
    with pytest.raises(rs.RSError) as e:
        sess.submit(plans[0], dpx[0], cubes[0])
    assert e.value.status == rs.RS_E_DEVICE and "device error" in str(e.value)
    sess.close()
