"""The C-ABI library builds for gfx950, loads, and exports every function that
include/handrt.h declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

from paper_2107_05509_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "handrt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hr_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_calls():
    names = _declared()
    for n in ("hr_scene_create", "hr_skin", "hr_render", "hr_loss", "hr_backward", "hr_step"):
        assert n in names
    assert set(names) == set(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    assert os.path.exists(binding.LIB_PATH), "libhandrt.so not built"
    lib = ctypes.CDLL(binding.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    lib.hr_last_error.restype = ctypes.c_char_p
    assert lib.hr_last_error() == b""


def test_library_is_built_for_gfx950():
    data = open(binding.LIB_PATH, "rb").read()
    assert b"gfx950" in data
