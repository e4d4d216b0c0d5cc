"""The C-ABI library loads and exports every entry point declared in include/pdg.h
(no device calls)."""
import os
import re

from paper_2511_08020_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pdg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdg_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert set(_declared()) == set(binding.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_last_error_is_empty_string_initially():
    lib = binding.load_library()
    assert isinstance(lib.pdg_last_error(), bytes)
