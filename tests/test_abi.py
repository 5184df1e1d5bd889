"""The C-ABI library loads and exports every symbol include/gpa.h declares
(no device work: these run without a GPU)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "gpa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gpa_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("gpa_load_program", "gpa_attribute", "gpa_advise", "gpa_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2009_04061_amd import gpa
    L = gpa.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(gpa.EXPORTS) == _declared()


def test_null_arguments_are_rejected_without_device_work():
    from paper_2009_04061_amd import gpa
    L = gpa.lib()
    out = ct.c_void_p()
    assert L.gpa_load_program(None, None, ct.byref(out)) == -1
    assert b"NULL" in L.gpa_last_error()
    assert L.gpa_attribute(None, None, 0, 0, None, ct.byref(out)) == -1
    assert L.gpa_advise(None, None, ct.byref(out)) == -1
    assert L.gpa_blame_counts(None, None, None) == -1
    assert L.gpa_advice_topk(None, 5, None, None, None) == -1


def test_descriptor_scalars_checked_on_host():
    from paper_2009_04061_amd import gpa
    L = gpa.lib()
    d = gpa.ProgramDesc()
    out = ct.c_void_p()
    assert L.gpa_load_program(ct.byref(d), None, ct.byref(out)) == -1     # empty program
    d.n_instr, d.n_blocks, d.n_funcs, d.n_scopes = 10, 2, 1, 3
    d.n_regs, d.n_preds = 4, 17
    assert L.gpa_load_program(ct.byref(d), None, ct.byref(out)) == -6     # too many predicates
    d.n_preds, d.n_bars, d.n_regs = 2, 0, 2000
    assert L.gpa_load_program(ct.byref(d), None, ct.byref(out)) == -6     # too many locations
