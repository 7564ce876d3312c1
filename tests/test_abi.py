"""The C-ABI library loads and exports every symbol include/ch.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ch.h")
LIB = os.path.join(ROOT, "paper_2105_01865_amd", "libch.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ch_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("ch_create", "ch_step", "ch_mass", "ch_destroy", "ch_set_field", "ch_get_field",
                 "ch_set_stream", "ch_last_error", "ch_batch_create", "ch_batch_step",
                 "ch_batch_mass", "ch_batch_destroy", "ch_interp_create", "ch_step_multires"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libch.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (ch_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    L = ctypes.CDLL(LIB)          # loads without a GPU; nothing is called
    for n in declared():
        assert hasattr(L, n)


def test_binding_covers_every_declared_symbol():
    from paper_2105_01865_amd import ch
    assert sorted(ch.SIGNATURES) == declared()
    # the ctypes structures match the C layout
    assert ctypes.sizeof(ch.Grid) == 32 and ctypes.sizeof(ch.BC) == 12
    assert ch.Opts.kappa.offset == 8 and ch.Opts.x_general.offset == 48
    assert ch.Opts.dt_hint.offset == 56 and ctypes.sizeof(ch.Opts) == 64


def test_binding_fails_loudly_without_the_library(monkeypatch):
    from paper_2105_01865_amd import ch
    monkeypatch.setattr(ch, "_lib", None)
    monkeypatch.setattr(ch, "LIB_PATH", "/nonexistent/libch.so")
    with pytest.raises(RuntimeError, match="not built"):
        ch.lib()
