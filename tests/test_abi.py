"""CPU-side checks of the C-ABI library: it loads and exports every symbol
that include/pfsp.h declares.  No compute call is made here."""
import ctypes
import os
import re

import pytest

from paper_2012_09511_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(pfsp_[a-z0-9_]+)\s*\(", src))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("pfsp_load_instance", "pfsp_bound_children", "pfsp_search"):
        assert required in names
    assert names == set(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    for name in _declared():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_null_context_is_rejected():
    L = binding.lib()
    assert L.pfsp_pair_count(None) == binding.PFSP_EINVAL
    assert L.pfsp_set_option(None, b"pool_batch", 1) == binding.PFSP_EINVAL
    assert L.pfsp_last_error(None) == b"null context"
