"""The C ABI: the library loads, exports every entry point the header declares, and rejects
invalid arguments on the host before launching anything (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1803_10045_amd import inputs
from paper_1803_10045_amd import kcs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "kcs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kcs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_entry_point():
    L = kcs.lib()
    names = header_functions()
    assert set(names) == set(kcs.ENTRY_POINTS)
    for n in names:
        assert hasattr(L, n), n


def geometry():
    return kcs.Geometry.from_config(inputs.disk64())


def frames(M=24):
    t0, t1 = inputs.frame_times()
    return kcs.Frames(t0[:M], t1[:M], np.ones(M), np.zeros(M))


def call_project(g, f, q=0, Q=4, x=1, y=1):
    gc, fc = g.c(), f.c()
    return kcs.lib().kcs_project(ctypes.byref(gc), ctypes.byref(fc), ctypes.c_void_p(x), q, Q, ctypes.c_void_p(y),
                                 None)


def test_workspace_sizes():
    g = geometry()
    w4 = kcs.kcs_workspace_bytes(g, 24, 4)
    w1 = kcs.kcs_workspace_bytes(g, 24, 1)
    w0 = kcs.kcs_workspace_bytes(g, 24, 0)
    assert w0 < w4 < w1
    # the ratio buffer holds the largest subset's sinogram
    assert w1 - w0 >= g.nz * g.n_ang * g.n_bin * 24 * 4
    assert kcs.kcs_study_footprint_bytes(g, 24, 4) > w4
    assert kcs.kcs_workspace_bytes(None, 24, 0) > 0


@pytest.mark.parametrize("bad,code", [
    (dict(q=4, Q=4), kcs.KCS_EINVAL), (dict(q=0, Q=0), kcs.KCS_EINVAL), (dict(q=0, Q=61), kcs.KCS_EINVAL),
    (dict(x=0), kcs.KCS_EINVAL), (dict(y=0), kcs.KCS_EINVAL)])
def test_project_rejects_bad_arguments(bad, code):
    assert call_project(geometry(), frames(), **bad) == code
    assert kcs.kcs_last_error() != ""


def test_bad_geometry_and_frames():
    g = geometry()
    bad = kcs.Geometry(0, 64, 1, 4.0, 60, 64, 4.0)
    assert call_project(bad, frames()) == kcs.KCS_EINVAL
    neg = kcs.Geometry(64, 64, 1, -1.0, 60, 64, 4.0)
    assert call_project(neg, frames()) == kcs.KCS_EINVAL
    assert call_project(g, frames(M=12)) == kcs.KCS_ESHAPE
    t0, t1 = inputs.frame_times()
    unsorted = kcs.Frames(t0[::-1].copy(), t1[::-1].copy(), np.ones(24), np.zeros(24))
    assert call_project(g, unsorted) == kcs.KCS_EINVAL
    negscale = kcs.Frames(t0, t1, -np.ones(24), np.zeros(24))
    assert call_project(g, negscale) == kcs.KCS_EINVAL


def test_priors_and_lm_options_validated():
    g = geometry()
    f = frames()
    k = kcs.Kinetics(**inputs.FENG, vb=inputs.VB).c()
    gc, fc = g.c(), f.c()
    good_p = kcs.Prior(0.1, 0.01, 0.1, (1e-3,) * 3).c()
    good_l = kcs.LMOptions(5, 1e-3, 1e-8, 1e8, inputs.LM_LO, inputs.LM_HI).c()
    vp = ctypes.c_void_p
    work = ctypes.c_size_t(1 << 30)

    def lm(p, l):
        return kcs.lib().kcs_lm_fit(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(k), ctypes.byref(p),
                                    ctypes.byref(l), vp(256), vp(256), vp(256), vp(256), work, None)

    assert lm(kcs.Prior(1.0, 0.01, 0.1, (1e-3,) * 3).c(), good_l) == kcs.KCS_EINVAL  # beta_kp >= 1
    assert lm(kcs.Prior(0.1, 0.0, 0.1, (1e-3,) * 3).c(), good_l) == kcs.KCS_EINVAL  # eps_F = 0
    assert lm(kcs.Prior(0.1, 0.01, 0.1, (0.0, 1e-3, 1e-3)).c(), good_l) == kcs.KCS_EINVAL  # delta = 0
    assert lm(kcs.Prior(0.1, 0.01, 0.1, (1e-3,) * 3, True, -1.0).c(), good_l) == kcs.KCS_EINVAL  # plane_ratio < 0
    assert lm(kcs.Prior(0.1, 0.01, 0.1, (1e-3,) * 3, True, float('nan')).c(), good_l) == kcs.KCS_EINVAL
    assert lm(good_p, kcs.LMOptions(5, 1e-3, 1e-8, 1e8, (0, 0, 0), inputs.LM_HI).c()) == kcs.KCS_EINVAL
    assert lm(good_p, kcs.LMOptions(5, 1e-3, 1.0, 0.1, inputs.LM_LO, inputs.LM_HI).c()) == kcs.KCS_EINVAL
    small = ctypes.c_size_t(1024)
    rc = kcs.lib().kcs_lm_fit(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(k), ctypes.byref(good_p),
                              ctypes.byref(good_l), vp(256), vp(256), vp(256), vp(256), small, None)
    assert rc == kcs.KCS_EWORKSPACE
    misaligned = kcs.lib().kcs_lm_fit(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(k), ctypes.byref(good_p),
                                      ctypes.byref(good_l), vp(256), vp(256), vp(256), vp(260), work, None)
    assert misaligned == kcs.KCS_EINVAL


def c_study(g, f, Q=4, s0=0, s1=1, ptr=256, work_bytes=1 << 32):
    k = kcs.Kinetics(**inputs.FENG, vb=inputs.VB)
    p = kcs.Prior(0.1, 0.01, 0.1, (1e-3,) * 3)
    lm = kcs.LMOptions(5, 1e-3, 1e-8, 1e8, inputs.LM_LO, inputs.LM_HI, 1e-3)
    vp = ctypes.c_void_p
    return kcs.c_study(g.c(), f.c(), k.c(), p.c(), lm.c(), Q, s0, s1, vp(ptr), vp(ptr), vp(ptr), vp(ptr), vp(ptr),
                       work_bytes)


@pytest.mark.parametrize("bad", ["none", "sweeps", "subsets", "null", "workspace", "second"])
def test_plan_create_rejects_bad_studies(bad):
    """Plans validate every study on the host and name the one at fault; nothing is launched."""
    g, f = geometry(), frames()
    good = c_study(g, f)
    studies = {"none": [], "sweeps": [c_study(g, f, s0=3, s1=2)], "subsets": [c_study(g, f, Q=0)],
               "null": [c_study(g, f, ptr=0)], "workspace": [c_study(g, f, work_bytes=16)],
               "second": [good, c_study(g, f, Q=61)]}[bad]
    arr = (kcs.c_study * max(len(studies), 1))(*studies)
    out = ctypes.c_void_p()
    rc = kcs.lib().kcs_plan_create(arr, len(studies), 0, None, ctypes.byref(out))
    assert rc in (kcs.KCS_EINVAL, kcs.KCS_EWORKSPACE)
    assert out.value is None
    msg = kcs.kcs_last_error()
    if bad != "none":
        assert ("study 1" if bad == "second" else "study 0") in msg
    kcs.lib().kcs_plan_destroy(None)  # NULL is ignored


def test_ki_map_validates_before_launching():
    L = kcs.lib()
    assert L.kcs_ki_map(None, -1, None, None) == kcs.KCS_EINVAL
    assert L.kcs_ki_map(None, 10, None, None) == kcs.KCS_EINVAL
    assert L.kcs_ki_map(ctypes.c_void_p(256), 1 << 40, ctypes.c_void_p(256), None) == kcs.KCS_EINVAL
    assert L.kcs_ki_map(None, 0, None, None) == kcs.KCS_OK  # empty: nothing to do


def test_frame_starts_within_rounding_of_the_previous_end_are_accepted():
    """A schedule built as end - duration may start a frame an ulp before the previous end: it
    counts as starting there.  A real overlap is still rejected (validation runs before the
    pointer checks, so the messages tell the two apart)."""
    t0, t1 = inputs.frame_times()
    t0u = t0.copy()
    t0u[1:] = np.nextafter(t1[:-1], -np.inf)  # an ulp before the previous end
    g = geometry()
    assert call_project(g, kcs.Frames(t0u, t1, np.ones(24), np.zeros(24)), x=0, y=0) == kcs.KCS_EINVAL
    assert "frames" not in kcs.lib().kcs_last_error().decode()
    t0o = t0.copy()
    t0o[5] = t1[4] - 1e-6
    assert call_project(g, kcs.Frames(t0o, t1, np.ones(24), np.zeros(24)), x=0, y=0) == kcs.KCS_EINVAL
    assert "sorted and disjoint" in kcs.lib().kcs_last_error().decode()


def test_limits_rejected_before_launching():
    """Beyond the supported shapes: more than 1024 angles in a subset, bins more than 6 times
    narrower than pixels."""
    g = kcs.Geometry(16, 16, 1, 3.0, 2050, 32, 3.0)
    assert call_project(g, frames(), q=0, Q=2, x=0, y=0) == kcs.KCS_ESHAPE  # 1025 angles in subset 0
    g = kcs.Geometry(12, 12, 1, 3.0, 30, 120, 0.45)
    assert call_project(g, frames(), q=0, Q=3, x=0, y=0) == kcs.KCS_ESHAPE  # 6.7 times narrower


def test_plane_of_more_than_2_31_values_rejected():
    """Offsets within one plane's image are 32-bit in the kernels: a plane of nx * ny * M >= 2^31
    values is refused on the host (16384 x 16384 pixels with 8 frames) while one below passes the
    shape checks (it fails later, on the NULL pointers)."""
    big = kcs.Geometry(16384, 16384, 1, 1.0, 60, 64, 1.0)
    assert call_project(big, frames(M=8), x=0, y=0) == kcs.KCS_ESHAPE
    assert "2^31" in kcs.kcs_last_error()
    ok = kcs.Geometry(16384, 8192, 1, 1.0, 60, 64, 1.0)
    assert call_project(ok, frames(M=8), x=0, y=0) == kcs.KCS_EINVAL


def test_footprint_counts_the_correction_sinogram():
    g = geometry()
    gc = g.c()
    plain = kcs.lib().kcs_study_footprint_bytes(ctypes.byref(gc), 24, 4)
    gc.d_mult = ctypes.c_void_p(256)
    with_mult = kcs.lib().kcs_study_footprint_bytes(ctypes.byref(gc), 24, 4)
    assert with_mult - plain == g.nz * g.n_ang * g.n_bin * 4


def test_lm_options_carry_the_restart_flag():
    assert kcs.LMOptions(5, 1e-3, 1e-8, 1e8, inputs.LM_LO, inputs.LM_HI).c().restart == 1
    assert kcs.LMOptions(5, 1e-3, 1e-8, 1e8, inputs.LM_LO, inputs.LM_HI, 1e-3, False).c().restart == 0


def test_noalloc_sweep_rejects_studies_beyond_its_static_scratch():
    """kcs_icm_sweep_noalloc refuses, on the host and before touching the device, a study whose
    workspace exceeds the library's 256 MiB static scratch (128 x 128 x 60, 6 subsets)."""
    cfg = inputs.scaled(inputs.brain128(), nz=60)
    g = kcs.Geometry.from_config(cfg)
    assert kcs.kcs_workspace_bytes(g, 24, cfg.Q) > 256 << 20
    f = frames()
    k = kcs.Kinetics(**inputs.FENG, vb=inputs.VB).c()
    p = kcs.Prior(0.1, 0.01, 0.1, (1e-3,) * 3).c()
    lm = kcs.LMOptions(5, 1e-3, 1e-8, 1e8, inputs.LM_LO, inputs.LM_HI).c()
    gc, fc = g.c(), f.c()
    vp = ctypes.c_void_p
    rc = kcs.lib().kcs_icm_sweep_noalloc(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(k), ctypes.byref(p),
                                         ctypes.byref(lm), vp(256), cfg.Q, 0, vp(256), vp(256), vp(256), None)
    assert rc == kcs.KCS_EWORKSPACE
    assert "static scratch" in kcs.kcs_last_error()
    rc = kcs.lib().kcs_icm_sweep_noalloc(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(k), ctypes.byref(p),
                                         ctypes.byref(lm), vp(0), cfg.Q, 0, vp(256), vp(256), vp(256), None)
    assert rc == kcs.KCS_EINVAL  # argument checks come first


def test_blood_fraction_options_validated():
    """With fit_vb the fourth Huber threshold and the blood-fraction box are checked (the box must
    lie in [0, 1]); fit_vb takes 0 or 1; kcs_init_state takes 3 or 4 initial maps; plans do not
    fit the blood fraction.  All refused on the host."""
    g, f = geometry(), frames()
    gc, fc = g.c(), f.c()
    vp = ctypes.c_void_p
    work = ctypes.c_size_t(1 << 30)
    kv = kcs.Kinetics(**inputs.FENG, vb=inputs.VB, fit_vb=True)
    p4 = kcs.Prior(0.1, 0.01, 0.1, (1e-3,) * 4)
    lo4, hi4 = inputs.LM_LO + (0.0,), inputs.LM_HI + (1.0,)

    def lm(k, p, l):
        kc, pc, lc = k.c(), p.c(), l.c()
        return kcs.lib().kcs_lm_fit(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(kc), ctypes.byref(pc),
                                    ctypes.byref(lc), vp(256), vp(256), vp(256), vp(256), work, None)

    good = kcs.LMOptions(5, 1e-3, 1e-8, 1e8, lo4, hi4)
    assert lm(kv, kcs.Prior(0.1, 0.01, 0.1, (1e-3, 1e-3, 1e-3, 0.0)), good) == kcs.KCS_EINVAL
    assert "delta" in kcs.kcs_last_error()
    assert lm(kv, p4, kcs.LMOptions(5, 1e-3, 1e-8, 1e8, inputs.LM_LO + (-0.1,), hi4)) == kcs.KCS_EINVAL
    assert "blood fraction" in kcs.kcs_last_error()
    assert lm(kv, p4, kcs.LMOptions(5, 1e-3, 1e-8, 1e8, lo4, inputs.LM_HI + (1.5,))) == kcs.KCS_EINVAL
    # three maps: the fourth entries are not read
    k3 = kcs.Kinetics(**inputs.FENG, vb=inputs.VB)
    kc = k3.c()
    kc.fit_vb = 2
    pc, lc = p4.c(), good.c()
    assert kcs.lib().kcs_lm_fit(ctypes.byref(gc), ctypes.byref(fc), ctypes.byref(kc), ctypes.byref(pc),
                                ctypes.byref(lc), vp(256), vp(256), vp(256), vp(256), work, None) == kcs.KCS_EINVAL
    assert "fit_vb" in kcs.kcs_last_error()
    xi = (ctypes.c_double * 5)(0.08, 0.12, 0.05, 0.05, 0.05)
    rc = kcs.lib().kcs_init_state(ctypes.byref(gc), ctypes.byref(fc), vp(256), xi, 5, vp(256), vp(256), vp(256),
                                  vp(256), work, None)
    assert rc == kcs.KCS_EINVAL and "n_maps" in kcs.kcs_last_error()
    st = c_study(g, f)
    st.k = kv.c()
    arr = (kcs.c_study * 1)(st)
    out = ctypes.c_void_p()
    assert kcs.lib().kcs_plan_create(arr, 1, 0, None, ctypes.byref(out)) == kcs.KCS_EINVAL
    assert "fit_vb" in kcs.kcs_last_error() and out.value is None


def test_rebin_arguments_validated():
    """Single-slice rebinning refuses bad ring counts, ring differences, sizes and NULL pointers on
    the host."""
    L = kcs.lib()
    vp = ctypes.c_void_p
    assert L.kcs_rebin_ssrb(0, 0, 4, 4, 1, vp(256), vp(256), None, None) == kcs.KCS_EINVAL
    assert L.kcs_rebin_ssrb(8, 8, 4, 4, 1, vp(256), vp(256), None, None) == kcs.KCS_EINVAL  # D > R - 1
    assert L.kcs_rebin_ssrb(8, -1, 4, 4, 1, vp(256), vp(256), None, None) == kcs.KCS_EINVAL
    assert L.kcs_rebin_ssrb(8, 2, 0, 4, 1, vp(256), vp(256), None, None) == kcs.KCS_EINVAL
    assert L.kcs_rebin_ssrb(8, 2, 4, 4, 1, None, vp(256), None, None) == kcs.KCS_EINVAL
    assert "NULL" in kcs.kcs_last_error()
    assert L.kcs_rebin_ssrb(4096, 10, 4096, 4096, 32, vp(256), vp(256), None, None) == kcs.KCS_ESHAPE
