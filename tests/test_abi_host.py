"""The C ABI library on the host: it loads and exports every function that
include/rs.h declares (no compute call is made; no GPU is needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rs_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rs_cube_plan", "rs_beat_synthesize", "rs_beat_synthesize_batch",
                 "rs_session_create", "rs_session_submit", "rs_session_poll", "rs_range_doppler",
                 "rs_render_scenes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2307_09226_amd import rs
    lib = ctypes.CDLL(rs.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every declared function with the same name
    assert set(declared_functions()) <= set(rs.SIGNATURES)


def test_version_and_error_text():
    from paper_2307_09226_amd import rs
    assert "gfx950" in rs.rs_version()
    assert isinstance(rs.rs_last_error(), str)


def test_invalid_plan_arguments_rejected_on_host():
    """Argument validation happens before any device call."""
    import numpy as np
    from paper_2307_09226_amd import rs, scenes
    r = scenes.radar_small()
    bad = [
        dict(M=0), dict(N=0), dict(Ns=0), dict(L=0), dict(Fs=0.0), dict(Tb=-1.0),
        dict(c0=0.0), dict(fc=float("nan")), dict(mu=float("inf")), dict(model=32), dict(model=-1),
    ]
    for kw in bad:
        rr = scenes.Radar(**{**r.__dict__, **kw})
        st, keep = rs._radar_struct(rr)
        h = ctypes.c_void_p()
        code = rs.lib.rs_cube_plan(ctypes.byref(st), rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, 100,
                                   ctypes.byref(h))
        assert code == rs.RS_E_INVALID, kw
        assert h.value is None
    st, keep = rs._radar_struct(r)
    h = ctypes.c_void_p()
    assert rs.lib.rs_cube_plan(ctypes.byref(st), 7, rs.RS_C64, 100, ctypes.byref(h)) == rs.RS_E_INVALID
    assert rs.lib.rs_cube_plan(ctypes.byref(st), 0, 5, 100, ctypes.byref(h)) == rs.RS_E_INVALID
    assert rs.lib.rs_cube_plan(ctypes.byref(st), 0, 0, -1, ctypes.byref(h)) == rs.RS_E_INVALID
    assert rs.lib.rs_cube_plan(None, 0, 0, 1, ctypes.byref(h)) == rs.RS_E_INVALID
    assert "NULL" in rs.rs_last_error()
    st.tx_xyz = ctypes.POINTER(ctypes.c_double)()
    assert rs.lib.rs_cube_plan(ctypes.byref(st), 0, 0, 1, ctypes.byref(h)) == rs.RS_E_INVALID
    # NULL handles
    assert rs.lib.rs_beat_synthesize(None, None, None, None) == rs.RS_E_INVALID
    assert rs.lib.rs_session_submit(None, None, None, None, None) == rs.RS_E_INVALID
    assert rs.lib.rs_range_doppler(None, None, 1, 1, None, None, None, None) == rs.RS_E_INVALID
    assert rs.lib.rs_render_scenes(None, 1, 8, 8, None, None, None, None, None, None, None) == rs.RS_E_INVALID
    sc = (rs.rs_scene * 1)()
    sc[0].room_w, sc[0].room_d, sc[0].room_h = 4.0, -1.0, 3.0
    fake = ctypes.c_void_p(256)   # never dereferenced: validation fails first
    assert rs.lib.rs_render_scenes(sc, 1, 8, 8, None, fake, fake, fake, fake, fake, None) == rs.RS_E_INVALID
    assert rs.lib.rs_render_scenes(sc, -1, 8, 8, None, fake, fake, fake, fake, fake, None) == rs.RS_E_INVALID
    sc[0].room_d = 5.0
    assert rs.lib.rs_render_scenes(sc, 1, 0, 8, None, fake, fake, fake, fake, fake, None) == rs.RS_E_INVALID
    out = ctypes.c_size_t()
    assert rs.lib.rs_plan_workspace_bytes(None, 0, ctypes.byref(out)) == rs.RS_E_INVALID
    rs.lib.rs_plan_destroy(None)
    rs.lib.rs_session_destroy(None)


def test_nufft_plan_arguments_rejected_on_host():
    """The NUFFT form's tolerance range and limits are checked before any
    device call."""
    import dataclasses
    from paper_2307_09226_amd import rs, scenes
    r = scenes.radar_small()
    st, keep = rs._radar_struct(r)
    h = ctypes.c_void_p()
    for tol in (0.0, 1e-8, 0.5, 2.0, float("nan"), -1e-3):
        assert rs.lib.rs_cube_plan_nufft(ctypes.byref(st), 0, 10, tol, ctypes.byref(h)) == rs.RS_E_INVALID, tol
        assert h.value is None
    for kw, code in ((dict(model=16), rs.RS_E_UNSUPPORTED), (dict(Ns=4096), rs.RS_E_UNSUPPORTED),
                     (dict(L=4096), rs.RS_E_UNSUPPORTED), (dict(model=64), rs.RS_E_INVALID)):
        st2, keep2 = rs._radar_struct(dataclasses.replace(r, **kw))
        assert rs.lib.rs_cube_plan_nufft(ctypes.byref(st2), 0, 10, 1e-6, ctypes.byref(h)) == code, kw
        assert rs.lib.rs_cube_plan(ctypes.byref(st2), rs.RS_FORM_NUFFT, 0, 10, ctypes.byref(h)) == code, kw
    assert rs.lib.rs_cube_plan_nufft(ctypes.byref(st), 0, 1 << 31, 1e-6, ctypes.byref(h)) == rs.RS_E_UNSUPPORTED
    # 16,384 channels: 2^25 grid rows (L 1024, grid 2048) or 2^24 fast-time
    # samples (Ns 1024) over all channels are refused before any device call
    for Ns, L, code in ((64, 1024, rs.RS_E_UNSUPPORTED), (1024, 64, rs.RS_E_UNSUPPORTED)):
        st3, keep3 = rs._radar_struct(scenes.radar_for(128, 128, Ns, L, Fs=10e6, Tb=120e-6))
        assert rs.lib.rs_cube_plan_nufft(ctypes.byref(st3), 0, 10, 1e-6, ctypes.byref(h)) == code, (Ns, L)
        assert "2^24" in rs.rs_last_error()


def test_tune_arguments_rejected_on_host():
    from paper_2307_09226_amd import rs
    assert rs.lib.rs_plan_tune(None, None, None, 3, None, None, 0) == rs.RS_E_INVALID
    assert rs.lib.rs_plan_tune_cached(None, None, None, 3, None, b"/tmp/x", None, 0) == rs.RS_E_INVALID
