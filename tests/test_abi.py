"""The C-ABI library loads and exports every function include/pasur.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pasur.h")
LIB = os.path.join(ROOT, "paper_2508_06559_amd", "libpasur.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pasur_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pasur_build_round_tree", "pasur_unfold_scores", "pasur_cfr_iterate",
                     "pasur_average_strategy", "pasur_round_values", "pasur_leaf_utilities",
                     "pasur_tree_values"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libpasur.so is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_library_has_gfx950_code_objects_only():
    data = open(LIB, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa-[-a-z0-9:+]*?(gfx[0-9a-z]+)", data))
    assert targets == {b"gfx950"}
