"""Host-side checks of libhog355 that need no GPU: every declared symbol is
exported, the host tables match the oracle, and argument errors are
reported before any work is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import hog as oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libhog355.h")


@pytest.fixture(scope="module")
def L():
    from paper_2006_00816_amd import build, hog355
    if not os.path.exists(hog355.LIB_PATH):
        build.build()
    return hog355.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hog_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_function(L):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_version_and_strerror(L):
    assert L.hog_version() >= 100
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert L.hog_strerror(code)
    assert L.hog_strerror(-99) == b"unknown status"


def test_orientation_table_matches_oracle_bitwise(L):
    from paper_2006_00816_amd import hog355
    c, s = hog355.orientation_table()
    oc, os_ = oracle.orientation_table()
    assert np.array_equal(c.view(np.uint64), oc.view(np.uint64))
    assert np.array_equal(s.view(np.uint64), os_.view(np.uint64))


@pytest.mark.parametrize("h,w,u", [(240, 320, 1), (480, 640, 1), (80, 80, 1), (1080, 1920, 2),
                                   (97, 331, 1), (4096, 4096, 2), (4096, 81, 1), (100, 120, 2), (79, 500, 1)])
def test_pyramid_matches_oracle(L, h, w, u):
    from paper_2006_00816_amd import hog355
    got = hog355.pyramid(h, w, u, 5)
    want = oracle.pyramid(h, w, u)
    assert [(g["h"], g["w"]) for g in got] == [(l.h, l.w) for l in want]
    assert [g["sig"] for g in got] == [oracle.inverse_scale_fixed(l) for l in want]
    off = 0
    for g in got:
        assert g["feat_offset"] == off
        off += g["cy"] * g["cx"] * 31
        assert g["rows"] == g["cy"] - 9 and g["cols"] == g["cx"] - 9


@pytest.mark.parametrize("h,w,u", [(480, 640, 1), (240, 320, 2), (97, 331, 1), (1080, 1920, 2), (80, 80, 1)])
def test_cascade_pyramid_matches_oracle(L, h, w, u):
    """Recursive pyramid sizes (floor(5x/6) of the previous level) and the
    same nominal inverse scales as the direct pyramid."""
    from paper_2006_00816_amd import hog355
    got = hog355.pyramid(h, w, u | hog355.CASCADE, 5)
    want = oracle.pyramid_cascade(h, w, u)
    assert [(g["h"], g["w"]) for g in got] == [(l.h, l.w) for l in want]
    assert [g["sig"] for g in got] == [oracle.inverse_scale_fixed(l) for l in want]
    # level images of every level but a level 0 that is the frame itself
    # (the other regions shrink a little with the smaller recursive sizes)
    if len(want) > 1 or u == 2:
        assert hog355.workspace_bytes(h, w, u | hog355.CASCADE, 2, 5) > hog355.workspace_bytes(h, w, u, 2, 5)
    assert L.hog_workspace_bytes(h, w, u | 0x200, 1, 5) == 0
    assert L.hog_workspace_bytes(h, w, 3 | hog355.CASCADE, 1, 5) == 0


def test_workspace_bytes(L):
    from paper_2006_00816_amd import hog355
    a = hog355.workspace_bytes(480, 640, 1, 1, 5)
    b = hog355.workspace_bytes(480, 640, 1, 64, 5)
    assert 0 < a < b
    assert L.hog_workspace_bytes(480, 640, 3, 1, 5) == 0       # bad upsample
    assert L.hog_workspace_bytes(5000, 640, 1, 1, 5) == 0      # too large
    assert L.hog_workspace_bytes(480, 640, 1, 0, 5) == 0       # no frames


def _detect(L, prm=True, frame=1, h=240, w=320, pitch=320, filt=1, bias=1, nf=1, dets=1, cap=16, nd=1,
            ws=1, ws_bytes=1 << 40, iou=0.5, up=1):
    from paper_2006_00816_amd import hog355
    p = hog355.hog_params(up, 0.0, iou)
    v = lambda x: ctypes.c_void_p(x) if x else None
    return L.hog_detect(ctypes.byref(p) if prm else None, v(frame), h, w, pitch, v(filt), v(bias), nf, v(dets),
                        cap, v(nd), v(ws), ws_bytes, None)


def test_argument_errors_reported_before_launch(L):
    # Every call below fails a host-side check; the dummy pointers are
    # never dereferenced and no GPU is touched.
    assert _detect(L, prm=False) == -1
    assert _detect(L, frame=0) == -1
    assert _detect(L, pitch=100) == -1
    assert _detect(L, nf=0) == -1
    assert _detect(L, nf=33) == -2
    assert _detect(L, cap=0) == -4
    assert _detect(L, cap=5000) == -4
    assert _detect(L, iou=1.0) == -1
    assert _detect(L, iou=0.3) == -1
    assert _detect(L, h=5000, w=5000, pitch=5000) == -2
    assert _detect(L, up=3) == -1
    assert _detect(L, ws_bytes=16) == -3
    assert _detect(L, ws=0) == -1


def test_static_entry_point_checks_before_launch(L):
    """hog_detect_batch_static: argument errors and shapes beyond the fixed
    scratch array are rejected on the host (dummy pointers, no GPU)."""
    from paper_2006_00816_amd import hog355
    v = ctypes.c_void_p

    def call(n, h, w, nf=5, frame=1):
        p = hog355.hog_params(1, 0.0, 0.5)
        return L.hog_detect_batch_static(ctypes.byref(p), v(frame) if frame else None, n, h, w, w, h * w, v(1),
                                         v(1), nf, v(1), 16, v(1), None)
    assert call(64, 480, 640) == hog355.HOG_E_SCRATCH == -8
    assert call(1, 1080, 1920) == -8
    assert hog355.workspace_bytes(480, 640, 1, 64, 5) > hog355.STATIC_SCRATCH_BYTES
    assert call(1, 480, 640, frame=0) == -1
    assert call(1, 480, 640, nf=0) == -1
    assert call(0, 480, 640) == -1
    assert L.hog_strerror(-8) == b"the call needs more workspace than the library's fixed scratch array"


def test_region_and_level_arguments_checked_before_launch(L):
    """min_face out of range and bad hog_track_regions arguments are
    rejected on the host (dummy pointers, no GPU); hog_params has the
    header's layout."""
    from paper_2006_00816_amd import hog355
    assert ctypes.sizeof(hog355.hog_params) == 32 and hog355.hog_params.regions.offset == 16
    assert hog355.hog_params.score_arith.offset == 24
    v = ctypes.c_void_p
    for mf, want in ((-1, -1), (65537, -1)):
        p = hog355.hog_params(1, 0.0, 0.5, mf, None)
        assert L.hog_detect(ctypes.byref(p), v(1), 240, 320, 320, v(1), v(1), 1, v(1), 16, v(1), v(1), 1 << 40,
                            None) == want
    # the scoring arithmetic: HOG_ARITH_F32 (0) or HOG_ARITH_F16X3 (1)
    for ar in (-1, 2, 7):
        p = hog355.hog_params(1, 0.0, 0.5, 0, None, ar)
        assert L.hog_detect(ctypes.byref(p), v(1), 240, 320, 320, v(1), v(1), 1, v(1), 16, v(1), v(1), 1 << 40,
                            None) == -1, ar
        assert L.hog_scores_arith(v(1), 240, 320, 320, 1, v(1), v(1), 1, ar, v(1), 1 << 30, v(1), 1 << 40,
                                  None) == -1, ar
    p = hog355.hog_params(1, 0.0, 0.5, 0, None, hog355.ARITH_F16X3)
    assert L.hog_detect_topk(ctypes.byref(p), v(1), 1, 240, 320, 320, 0, v(1), v(1), 1, v(1), 16, v(1), 1, v(1),
                             v(1), v(1), 1 << 40, None) == -1
    d = hog355.hog_params(7, 1.0, 0.9, 5, 3, 9)
    assert L.hog_params_default(ctypes.byref(d)) == 0
    assert (d.upsample, d.thresh, d.iou, d.min_face, d.regions, d.score_arith) == (1, 0.0, 0.5, 0, None, 0)
    ok = dict(dets=v(1), nd=v(1), n=2, cap=16, h=480, w=640, margin=8, span=1, regs=v(1))

    def track(**kw):
        a = {**ok, **kw}
        return L.hog_track_regions(a["dets"], a["nd"], a["n"], a["cap"], a["h"], a["w"], a["margin"], a["span"],
                                   a["regs"], None)
    for bad in (dict(dets=None), dict(nd=None), dict(regs=None), dict(n=0), dict(cap=0), dict(cap=5000),
                dict(h=0), dict(w=5000), dict(margin=-1), dict(span=-1), dict(span=29)):
        assert track(**bad) == -1, bad


def test_pipeline_config_checked_before_any_allocation(L):
    """Invalid pipeline configurations are rejected before the library
    touches the GPU or allocates (dummy pointers)."""
    from paper_2006_00816_amd import hog355
    v = ctypes.c_void_p
    prm = hog355.hog_params(1, 0.0, 0.5, 0, None)
    good = dict(h=480, w=640, batch=4, depth=2, cap=16, consumer_threads=1, staging=1)
    for bad in (dict(batch=0), dict(batch=2000), dict(depth=0), dict(depth=17), dict(cap=0), dict(cap=5000),
                dict(consumer_threads=0), dict(staging=2), dict(h=5000), dict(w=0)):
        c = {**good, **bad}
        cfg = hog355.hog_pipeline_config(c["h"], c["w"], c["batch"], c["depth"], c["cap"], c["consumer_threads"],
                                         c["staging"], 0, hog355.CONSUMER_FN(), None)
        out = v()
        assert L.hog_pipeline_create(ctypes.byref(out), ctypes.byref(prm), ctypes.byref(cfg), v(1), v(1), 5) == -1, bad
        assert not out.value
    cfg = hog355.hog_pipeline_config(480, 640, 4, 2, 16, 1, 1, 0, hog355.CONSUMER_FN(), None)
    prm_r = hog355.hog_params(1, 0.0, 0.5, 0, 1)   # regions are not supported by the pipeline
    assert L.hog_pipeline_create(ctypes.byref(v()), ctypes.byref(prm_r), ctypes.byref(cfg), v(1), v(1), 5) == -1
    prm_a = hog355.hog_params(1, 0.0, 0.5, 0, None, 5)   # no such scoring arithmetic
    assert L.hog_pipeline_create(ctypes.byref(v()), ctypes.byref(prm_a), ctypes.byref(cfg), v(1), v(1), 5) == -1
    assert L.hog_pipeline_submit(None, v(1), 1, 0) == -1 and L.hog_pipeline_drain(None) == -1


@pytest.mark.parametrize("h,w,u", [(480, 640, 1), (97, 331, 1), (240, 320, 2), (1080, 1920, 2)])
def test_region_windows_match_oracle(L, h, w, u):
    """The anchor ranges the kernels derive from a search region select
    exactly the windows whose boxes the oracle finds inside it (random
    regions, also partly or wholly outside the frame and empty ones)."""
    from paper_2006_00816_amd import hog355
    rng = np.random.default_rng(h + w + u)
    levels = oracle.pyramid(h, w, u)
    for _ in range(60):
        x0, x1 = sorted(rng.integers(-60, w + 60, 2))
        y0, y1 = sorted(rng.integers(-60, h + 60, 2))
        if rng.random() < 0.2:
            x0, x1 = x1, x0
        reg = (int(x0), int(y0), int(x1), int(y1), int(rng.integers(0, 3)), int(rng.integers(1, 30)))
        for lv in levels[:: max(1, len(levels) // 4)]:
            r_lo, r_hi, c_lo, c_hi = hog355.region_windows(h, w, u, lv.k, reg)
            rr, cc = np.meshgrid(np.arange(lv.rows), np.arange(lv.cols), indexing="ij")
            want = oracle.window_in_region(lv, rr, cc, reg)
            got = (rr >= r_lo) & (rr <= r_hi) & (cc >= c_lo) & (cc <= c_hi)
            assert np.array_equal(got, want), (reg, lv.k, (r_lo, r_hi, c_lo, c_hi))


def test_level_table_limits(L):
    from paper_2006_00816_amd import hog355
    lv = hog355.pyramid(4096, 4096, 2, 32)
    assert len(lv) <= 28
    assert lv[0]["cx"] <= 1024


def test_tuning_table_roundtrip_and_validation(L):
    from paper_2006_00816_amd import hog355
    shape = (123, 321, 1, 5, 3)
    t, found = hog355.tuning_get(*shape)
    assert not found and t["fused"] == 0
    want = {"fused": 1, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 3, "split": 1, "nms_rounds": 3,
            "score_rows": 0, "stagger": 0}
    hog355.tuning_set(*shape, want)
    got, found = hog355.tuning_get(*shape)
    assert found and got == want
    # a scoring lag that does not follow the feature lag could wait on a
    # later ticket: rejected, as are queue counts outside 1..8
    for bad in ({**want, "lag_s": 1}, {**want, "lag_f": 0}, {**want, "queues": 9}, {**want, "queues": 0},
                {**want, "wg_per_queue": 0}, {**want, "fused": 2}, {**want, "split": 2},
                {**want, "fused": 0, "split": 0}, {**want, "fused": 0, "split": 5},
                {**want, "fused": 0, "nms_rounds": -1}, {**want, "fused": 0, "nms_rounds": 17},
                {**want, "fused": 0, "score_rows": 8}, {**want, "stagger": 1}, {**want, "fused": 0, "stagger": 3},
                {**want, "fused": 0, "stagger": -1}):
        with pytest.raises(hog355.HogError):
            hog355.tuning_set(*shape, bad)
    assert hog355.tuning_get(*shape)[0] == want
    hog355.tuning_set(*shape, None)
    assert not hog355.tuning_get(*shape)[1]


def test_params_default_and_constants(L):
    from paper_2006_00816_amd import hog355
    assert hog355.params_default() == {"upsample": 1, "thresh": 0.0, "iou": 0.5}
    c = hog355.constants()
    assert (c["cell_px"], c["bins"], c["features"], c["window_cells"], c["min_side"]) == (
        oracle.CELL, oracle.NBINS, oracle.NFEAT, oracle.WIN, oracle.MIN_SIDE)
    assert (c["scale_num"], c["scale_den"]) == (oracle.SCALE_NUM, oracle.SCALE_DEN)
    assert c["clip"] == np.float32(oracle.CLIP) and c["eps"] == np.float32(oracle.EPS)
    assert L.hog_params_default(None) == -1 and L.hog_constants_get(None) == -1


def test_windows_check_range(L):
    """The window range test the kernels apply, run on host records: every
    field at its first invalid value on either side is rejected, and the
    index of the first bad record is reported."""
    import torch
    from paper_2006_00816_amd import hog355
    h, w, u, n, nf = 240, 320, 1, 3, 2
    lv = oracle.pyramid(h, w, u)
    ok = [[0, 0, 0, 0, 0], [n - 1, nf - 1, len(lv) - 1, lv[-1].rows - 1, lv[-1].cols - 1],
          [1, 1, 0, lv[0].rows - 1, lv[0].cols - 1]]
    hog355.windows_check(torch.tensor(ok, dtype=torch.int32), n, h, w, nf, u)
    bad = [[-1, 0, 0, 0, 0], [n, 0, 0, 0, 0], [0, -1, 0, 0, 0], [0, nf, 0, 0, 0], [0, 0, -1, 0, 0],
           [0, 0, len(lv), 0, 0], [0, 0, 0, -1, 0], [0, 0, 0, lv[0].rows, 0], [0, 0, 0, 0, -1],
           [0, 0, 0, 0, lv[0].cols], [0, 0, len(lv) - 1, lv[-1].rows, 0], [0, 0, len(lv) - 1, 0, lv[-1].cols]]
    for rec in bad:
        arr = torch.tensor(ok + [rec] + ok, dtype=torch.int32)
        first = ctypes.c_int(-7)
        host = arr.contiguous()
        st = L.hog_windows_check(h, w, u, n, nf, ctypes.c_void_p(host.data_ptr()), int(host.shape[0]),
                                 ctypes.byref(first))
        assert st == -1 and first.value == len(ok), (rec, st, first.value)
        with pytest.raises(hog355.HogError):
            hog355.windows_check(arr, n, h, w, nf, u)
    assert L.hog_windows_check(h, w, u, n, nf, None, 0, None) == 0
    assert L.hog_windows_check(h, w, u, n, nf, None, 1, None) == -1
