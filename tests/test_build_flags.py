"""Which translation units may contract multiplies and adds.

The FP64 path equals the oracle bit for bit only if every FP64 expression
is evaluated as written (no fused multiply-add contraction); the float form
is held to an error bound and is built with contraction.  The build keeps
the two apart by translation unit: only the float-form units (*_f32.hip,
each instantiating float kernels only) are compiled with contraction.
"""
import re
from pathlib import Path

from paper_1707_00592_amd import build

CSRC = Path(build.__file__).resolve().parent / "csrc"


def test_default_flags_keep_every_operation_as_written():
    assert "-ffp-contract=off" in build.CFLAGS
    assert not any(f.startswith("-ffp-contract=") and f != "-ffp-contract=off"
                   for f in build.CFLAGS)
    assert "-packed-fp32-ops" in build.CFLAGS


def test_only_float_units_are_contracted():
    assert build.CONTRACTED <= set(build.SOURCES)
    for src in build.CONTRACTED:
        assert src.endswith("_f32.hip"), src
        text = (CSRC / src).read_text()
        # float instantiations only: no double-typed launch in these units
        assert "<double" not in text, src
        assert re.search(r"<float\b", text), src
    for src in build.SOURCES:
        if src not in build.CONTRACTED:
            assert not src.endswith("_f32.hip"), src


def test_every_source_is_built():
    on_disk = {p.name for p in CSRC.glob("*.hip")}
    assert on_disk == set(build.SOURCES)
