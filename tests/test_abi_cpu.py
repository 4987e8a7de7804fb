"""C-ABI checks that need no GPU: the library loads, exports every function
include/famsa_lcs.h declares, and rejects invalid input with EINVAL before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1603_06958_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "famsa_lcs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(famsa_\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if not n.endswith("_fn")))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 19, names
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def plan_rc(codes, off, fam=None, nfam=0, **opt):
    L = B.lib()
    o = B.make_options(**opt)
    h = ctypes.c_void_p(123)
    codes = np.ascontiguousarray(codes, np.uint8)
    off = np.ascontiguousarray(off, np.uint64)
    cp = codes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if codes.size else None
    fp = None
    if fam is not None:
        fam = np.ascontiguousarray(fam, np.uint32)
        fp = fam.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    rc = L.famsa_lcs_plan(cp, off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), off.size - 1, fp, nfam,
                          ctypes.byref(o), ctypes.byref(h))
    if rc == 0:
        L.famsa_lcs_release(h)
    else:
        assert not h.value  # out is cleared on failure
    return rc, B.last_error()


def test_einval_code_out_of_alphabet():
    rc, msg = plan_rc([1, 2, 20], [0, 3])
    assert rc == B.EINVAL and "alphabet" in msg


def test_einval_alphabet_size():
    assert plan_rc([0], [0, 1], alphabet_size=0)[0] == B.EINVAL
    assert plan_rc([0], [0, 1], alphabet_size=33)[0] == B.EINVAL
    # codes up to 31 are fine with alphabet 32 (fails later only for lack of a GPU)
    assert plan_rc([31, 0], [0, 2], alphabet_size=32)[0] != B.EINVAL


def test_einval_offsets():
    assert plan_rc([0, 1, 2], [0, 2, 1])[0] == B.EINVAL
    long = np.zeros(B.MAX_LEN + 1, np.uint8)
    rc, msg = plan_rc(long, [0, long.size])
    assert rc == B.EINVAL and "length" in msg


def test_einval_families():
    c = np.zeros(4, np.uint8)
    off = [0, 1, 2, 3, 4]
    assert plan_rc(c, off, fam=[1, 4], nfam=1)[0] == B.EINVAL      # fam_off[0] != 0
    assert plan_rc(c, off, fam=[0, 3], nfam=1)[0] == B.EINVAL      # does not end at nseq
    assert plan_rc(c, off, fam=[0, 3, 2, 4], nfam=3)[0] == B.EINVAL  # decreasing


def test_options_layout_and_older_callers():
    # the Python mirror has the C layout, and a caller built before the last
    # field (step_cells) was added still gets a plan-time answer, not EINVAL
    o = B.make_options()
    assert o.struct_size == ctypes.sizeof(B.Options)
    o.struct_size = B.Options.step_cells.offset
    h = ctypes.c_void_p()
    off = np.array([0, 1], np.uint64)
    c = np.zeros(1, np.uint8)
    info = B.PlanInfo()
    rc = B.lib().famsa_lcs_plan_dry_run(c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                       off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), 1, None, 0,
                                       ctypes.byref(o), None, ctypes.byref(info))
    assert rc == 0, B.last_error()


def test_einval_options():
    assert plan_rc([0], [0, 1], tile_rows=0)[0] == B.EINVAL
    assert plan_rc([0], [0, 1], flags=0x800)[0] == B.EINVAL
    rc, msg = plan_rc([0], [0, 1], flags=B.ONE_STREAM | B.TWO_STREAMS)
    assert rc == B.EINVAL and "exclude" in msg
    rc, msg = plan_rc([0], [0, 1], flags=B.OUT_INDEL | B.OUT_SIM)
    assert rc == B.EINVAL and "exclude" in msg
    rc, msg = plan_rc([0], [0, 1], flags=B.PLAIN_ASYNC)
    assert rc == B.EINVAL and "needs FAMSA_LCS_PLAIN" in msg
    L = B.lib()
    o = B.make_options()
    o.struct_size = 4
    h = ctypes.c_void_p()
    off = np.array([0, 1], np.uint64)
    c = np.zeros(1, np.uint8)
    rc = L.famsa_lcs_plan(c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                          off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), 1, None, 0, ctypes.byref(o),
                          ctypes.byref(h))
    assert rc == B.EINVAL and "struct_size" in B.last_error()


def test_null_arguments():
    L = B.lib()
    off = np.array([0, 1], np.uint64)
    assert L.famsa_lcs_plan(None, off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), 1, None, 0, None,
                            None) == B.EINVAL
    h = ctypes.c_void_p()
    # residues present but codes NULL
    assert L.famsa_lcs_plan(None, off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), 1, None, 0, None,
                            ctypes.byref(h)) == B.EINVAL
    L.famsa_lcs_release(None)  # no-op
    assert L.famsa_lcs_tiles(None, 0, B.TILE_FN(lambda u, t: 0), None) == B.EINVAL
    assert L.famsa_lcs_plan_get_info(None, None) == B.EINVAL
    L.famsa_slink_destroy(None)
    L.famsa_lcs_server_destroy(None)


def test_no_gpu_is_edevice():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    rc, msg = plan_rc([0, 1, 2], [0, 3])
    assert rc == B.EDEVICE, msg


def test_valu_peak_rejects_bad_arguments():
    L = B.lib()
    r = B.PeakResult()
    assert L.famsa_valu_peak(0, 4, 8, 100, ctypes.byref(r)) == B.EINVAL
    assert L.famsa_valu_peak(0, 0, 0, 100, ctypes.byref(r)) == B.EINVAL
    assert L.famsa_valu_peak(0, 0, 8, 0, ctypes.byref(r)) == B.EINVAL
    assert L.famsa_valu_peak(0, 0, 8, 100, None) == B.EINVAL


def test_noalloc_rejects_on_the_host():
    # the allocation-free entry point checks its sizes before any HIP call
    L = B.lib()
    assert L.famsa_lcs_family_noalloc(1, 1, B.NOALLOC_MAX_SEQ + 1, 20, 1, None, 0, None) == B.EINVAL
    assert "scratch" in B.last_error()
    assert L.famsa_lcs_family_noalloc(1, 1, 10, 0, 1, None, 0, None) == B.EINVAL
    assert L.famsa_lcs_family_noalloc(1, None, 10, 20, 1, None, 0, None) == B.EINVAL
    assert L.famsa_lcs_family_noalloc(1, 1, 10, 20, None, None, 0, None) == B.EINVAL
    assert L.famsa_lcs_family_noalloc(1, 1, 10, 20, 1, None, -1, None) == B.EINVAL


def test_gap_costs_scaled_matches_the_oracle():
    # the library's host helper against the oracle's reading of g_scale
    from oracle import profile as OP
    for k in (1, 2, 44, 45, 46, 300, 100_000, 415_519):
        for base in ((10, 2, 14, 3), (7.5, 0.5, -3.5, 2.25), (0, 0, 0, 0)):
            assert B.gap_costs_scaled(k, base) == OP.scaled_gap_costs(k, base)
    with pytest.raises(B.FamsaError):
        B.gap_costs_scaled(0, (1, 1, 1, 1))


def test_profile_align_rejects_on_the_host():
    from paper_1603_06958_amd import inputs
    S = inputs.synthetic_subst(20, 1)
    p = inputs.profile_problem(10, 12, 2, np.random.default_rng(0))
    bad = p.rows.copy()
    bad[1, 3] = 21  # neither a gap nor a code below the alphabet size
    for probs, kw in [([(p.seq, bad)], {}), ([(p.seq, np.zeros((0, 12), np.uint8))], {}),
                      ([(np.array([20], np.uint8), p.rows)], {}), ([(p.seq, p.rows)], {"alphabet_size": 33})]:
        with pytest.raises(B.FamsaError) as e:
            B.profile_align(probs, S, (1, 1, 1, 1), **kw)
        assert e.value.code == B.EINVAL
    with pytest.raises(B.FamsaError) as e:
        B.profile_align([(p.seq, p.rows)], S, (1, 1, 1, 2 ** 21))
    assert e.value.code == B.EINVAL


def test_profile_align_accepts_valid_input_up_to_the_device():
    # negative scores and costs are valid; without a GPU the call fails only
    # at the device (EDEVICE), never in validation
    from paper_1603_06958_amd import inputs
    S = inputs.synthetic_subst(20, 1)
    p = inputs.profile_problem(10, 12, 2, np.random.default_rng(0))
    try:
        B.profile_align([(p.seq, p.rows)], S, (-3, 0, 2, -1))
    except B.FamsaError as e:
        assert e.code == B.EDEVICE, e
