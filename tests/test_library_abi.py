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


def test_error_codes_agree():
    text = open(os.path.join(ROOT, "include", "pdg.h")).read()
    block = re.search(r"enum \{ PDG_OK.*?\};", text, flags=re.S).group(0)
    codes = dict((k, int(v)) for k, v in re.findall(r"\b(PDG_[A-Z]+)\s*=\s*(-?\d+)", block))
    assert "PDG_ENONFINITE" in codes
    for name, value in codes.items():
        assert getattr(binding, name) == value, name
