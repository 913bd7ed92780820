"""The C ABI library loads, exports every symbol include/sfft.h declares, and
its host-only logic (unknown count, validation) is right. No compute calls."""
import ctypes
import os
import re

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfft.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sfft_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_three_calls():
    names = _declared()
    for n in ("sfft_build_system", "sfft_solve", "sfft_subtract"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2603_08593_amd as sf
    lib = sf.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_struct_sizes_match_header():
    import paper_2603_08593_amd as sf
    assert ctypes.sizeof(sf.Desc) == 56
    assert ctypes.sizeof(sf.SolveInfo) == 40


@pytest.mark.parametrize("L,DK,DB", [(1, 0, 0), (7, 0, 1), (11, 2, 2), (15, 2, 2), (3, 4, 4)])
def test_num_unknowns_matches_oracle(L, DK, DB):
    import paper_2603_08593_amd as sf
    d = sf.make_desc(64, 64, L, DK, DB)
    assert sf.sfft_num_unknowns(d) == O.n_unknowns(L, DK, DB)


def test_validation_codes():
    import paper_2603_08593_amd as sf
    ok = sf.make_desc(2048, 4096, 11, 2, 2)
    assert sf.sfft_validate(ok) == sf.SFFT_OK
    assert sf.sfft_validate(sf.make_desc(64, 64, 4, 0, 0)) == sf.SFFT_ERR_INVALID_ARG    # even L
    assert sf.sfft_validate(sf.make_desc(64, 64, 0, 0, 0)) == sf.SFFT_ERR_INVALID_ARG    # L = 0
    assert sf.sfft_validate(sf.make_desc(64, 64, 5, 5, 0)) == sf.SFFT_ERR_INVALID_ARG    # DK > 4
    assert sf.sfft_validate(sf.make_desc(16, 8, 9, 0, 0)) == sf.SFFT_ERR_INVALID_ARG     # L > min(W,H)
    assert sf.sfft_validate(sf.make_desc(64, 64, 5, 0, 0, ld=32)) == sf.SFFT_ERR_INVALID_ARG  # ld < W
    assert sf.sfft_validate(sf.make_desc(112, 64, 5, 0, 0)) == sf.SFFT_ERR_UNSUPPORTED   # 7 | W
    assert sf.sfft_validate(sf.make_desc(22, 64, 5, 0, 0)) == sf.SFFT_ERR_UNSUPPORTED    # 11 | W
    assert sf.sfft_validate(sf.make_desc(95, 64, 5, 0, 0)) == sf.SFFT_ERR_UNSUPPORTED    # W odd
    assert sf.sfft_validate(sf.make_desc(96, 64, 5, 0, 0)) == sf.SFFT_OK                 # 2^5 3
    assert sf.sfft_validate(sf.make_desc(1500, 64, 5, 0, 0)) == sf.SFFT_OK               # 2^2 3 5^3
    out = sf.make_desc(2048, 4096, 11, 2, 2, convention=sf.SFFT_CONV_OUTPUT_PIXEL)
    assert sf.sfft_validate(out) == sf.SFFT_OK                                          # output-pixel convention
    assert sf.sfft_validate(sf.make_desc(64, 64, 5, 0, 0, convention=2)) == sf.SFFT_ERR_INVALID_ARG
    assert sf.sfft_validate(sf.make_desc(64, 64, 5, 3, 0)) == sf.SFFT_ERR_UNSUPPORTED    # DK = 3
    assert sf.sfft_validate(sf.make_desc(64, 64, 17, 0, 0)) == sf.SFFT_ERR_UNSUPPORTED   # L > 15
    assert sf.sfft_validate(sf.make_desc(16, 64, 11, 0, 0)) == sf.SFFT_ERR_UNSUPPORTED   # W < 2L
    bad = sf.make_desc(64, 64, 5, 0, 0, ref_pedestal=float("nan"))
    assert sf.sfft_validate(bad) == sf.SFFT_ERR_INVALID_ARG


def test_status_strings():
    import paper_2603_08593_amd as sf
    assert sf.status_string(sf.SFFT_ERR_NOT_SPD) == "SFFT_ERR_NOT_SPD"
    assert sf.status_string(0) == "SFFT_OK"


def test_null_arguments_rejected_before_any_device_work():
    import paper_2603_08593_amd as sf
    lib = sf.lib()
    d = sf.make_desc(64, 64, 5, 0, 0)
    assert lib.sfft_create(None) == sf.SFFT_ERR_INVALID_ARG
    assert lib.sfft_build_system(None, ctypes.byref(d), None, None, None, None, None, 0, None) \
        == sf.SFFT_ERR_INVALID_ARG
    n = ctypes.c_size_t()
    assert lib.sfft_workspace_size(None, ctypes.byref(d), ctypes.byref(n)) == sf.SFFT_ERR_INVALID_ARG
    # the solve-team setting needs a handle
    assert lib.sfft_set_solve_team(None, 32) == sf.SFFT_ERR_INVALID_ARG
    t = ctypes.c_int32(-1)
    assert lib.sfft_get_solve_team(None, ctypes.byref(t)) == sf.SFFT_ERR_INVALID_ARG
    # so do the radix-order setting and the batch configuration
    assert lib.sfft_set_radix_order(None, 1) == sf.SFFT_ERR_INVALID_ARG
    assert lib.sfft_get_radix_order(None, ctypes.byref(t)) == sf.SFFT_ERR_INVALID_ARG
    k = sf.BatchKnobs(4, 0, 32, 0)
    assert lib.sfft_batch_set_knobs(None, ctypes.byref(k)) == sf.SFFT_ERR_INVALID_ARG
    assert lib.sfft_batch_get_knobs(None, ctypes.byref(k)) == sf.SFFT_ERR_INVALID_ARG
