"""The C ABI: every function declared in include/isweno.h is exported by the
built library, the binding covers exactly those, and the struct layouts of
the binding match the header (checked on the CPU; no GPU call is made)."""
import ctypes as C
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "isweno.h"


def _declared():
    text = HEADER.read_text()
    return sorted(set(re.findall(r"ISWENO_API\s+[\w\s\*]*?\b(isweno_\w+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("isweno_rhs", "isweno_rk3_step", "isweno_batch_step", "isweno_create",
                 "isweno_destroy", "isweno_cfl_dt", "isweno_mlp_forward",
                 "isweno_mlp_loss_grad"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1707_00592_amd import isweno
    lib = C.CDLL(str(isweno.LIB_PATH))
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(isweno.EXPORTED) == _declared()


def test_binding_struct_layouts():
    from paper_1707_00592_amd import isweno
    # offsets follow the natural alignment of the header's structs
    assert C.sizeof(isweno.Grid) == 4 + 4 + 24 + 24 + 12 + 12
    assert isweno.Grid.n.offset == 8 and isweno.Grid.dx.offset == 32
    assert isweno.Grid.bc_lo.offset == 56 and isweno.Grid.bc_hi.offset == 68
    assert isweno.Opts.eps.offset == 16 and isweno.Opts.mlp_params.offset == 40
    assert C.sizeof(isweno.Opts) == 56
    assert C.sizeof(isweno.Stats) == 9 * 8 + 8


def test_version_string():
    from paper_1707_00592_amd import isweno
    lib = C.CDLL(str(isweno.LIB_PATH))
    lib.isweno_version.restype = C.c_char_p
    assert b"gfx950" in lib.isweno_version()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1707_00592_amd import isweno
    monkeypatch.setattr(isweno, "_lib", None)
    monkeypatch.setattr(isweno, "LIB_PATH", tmp_path / "nope.so")
    with pytest.raises(RuntimeError, match="missing"):
        isweno.load()
