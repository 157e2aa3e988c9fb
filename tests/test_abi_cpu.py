"""The C-ABI library builds, loads and exports every entry point that include/qed.h
declares; host-side argument checks work without a GPU; the Python binding refuses to run
without the library (no CPU fallback)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2306_11288_amd as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "qed.h")).read()
    return sorted(set(re.findall(r"^\s*(?:qed_status|int64_t|const char\s*\*)\s*(qed_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_exported_api():
    assert _declared() == sorted(Q.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = Q.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_table_sizes_match_the_oracle_specification():
    lib = Q.lib()
    for which in range(6):
        assert lib.qed_table_size(which) == oracle.lib().orc_tables_size(which)
    assert lib.qed_table_size(99) == -1


def test_null_arguments_are_rejected_without_touching_the_device():
    lib = Q.lib()
    assert lib.qed_destroy(None) == Q.QED_EARG
    assert lib.qed_read_status(None, None, None) == Q.QED_EARG
    assert lib.qed_gather(None, None, 0, None, None, 0, None) == Q.QED_EARG
    assert lib.qed_step_leptons(None, None, 0, None, None, 0, None) == Q.QED_EARG
    assert lib.qed_step_photons(None, None, 0, None, None, None, 0, None) == Q.QED_EARG
    assert lib.qed_compact_photons(None, None, None, None) == Q.QED_EARG
    assert lib.qed_last_error(None) == b"null context"
    # invalid configuration is rejected before any HIP call
    h = C.c_void_p()
    bad = Q.Config(Q.XI_L, Q.ALPHA, Q.A_E, -1.0, 0.1, 1, 0, Q.QED_FP64, 1)
    assert lib.qed_init_tables(C.byref(h), C.byref(bad), None) == Q.QED_EARG
    bad2 = Q.Config(Q.XI_L, Q.ALPHA, Q.A_E, 0.1, 0.1, 1, 0, 7, 1)
    assert lib.qed_init_tables(C.byref(h), C.byref(bad2), None) == Q.QED_EARG


def test_struct_layouts_match_the_header():
    # sizes of the ctypes mirrors follow the C structs' natural alignment
    assert C.sizeof(Q.Config) == 5 * 8 + 2 * 8 + 4 + 4
    assert C.sizeof(Q.CLeptons) == 12 * 8 + 8 + 8
    assert C.sizeof(Q.CPhotons) == 16 * 8 + 8
    assert C.sizeof(Q.Field) == 8 + 7 * 8 + 6 * 8 + 6 * 8 + 8 + 4 * 8
    assert C.sizeof(Q.Segment) == 16 + C.sizeof(Q.Field)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(Q, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(Q, "_lib", None)
    with pytest.raises(Q.QedError):
        Q.lib()
