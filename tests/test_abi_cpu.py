"""Host-side checks that need no GPU: the library loads and exports every
function the public header declares, and the binding refuses to run
without it."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:sc_status|uint32_t|const char\*)\s+(sc_[a-z_0-9]+)\s*\(", src, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("sc_build_bvh", "sc_render", "sc_trace_photons", "sc_trace_rays", "sc_occluded"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2107_11008_amd as sc
    lib = sc.load()
    out = subprocess.run(["nm", "-D", "--defined-only", sc._sc.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (sc_[a-z_0-9]+)$", out, re.M))
    for n in _declared():
        assert n in exported, n
        assert hasattr(lib, n)
    assert lib.sc_abi_version() == sc._sc.ABI_VERSION == 6


def test_material_record_layout():
    """The 48-byte material record: header, binding and scene arrays agree."""
    import ctypes
    import paper_2107_11008_amd as sc
    import scenegen as sg
    hdr = open(os.path.join(ROOT, "include", "sc.h")).read()
    assert "} sc_material; /* 48 bytes */" in hdr
    assert ctypes.sizeof(sc._sc.Material) == 48 == sg.MATERIAL_DTYPE.itemsize
    for name, _ in sc._sc.Material._fields_:
        assert getattr(sc._sc.Material, name).offset == sg.MATERIAL_DTYPE.fields[name][1], name


def test_binding_lists_all_exports():
    import paper_2107_11008_amd as sc
    assert sorted(sc._sc.EXPORTS) == _declared()


def test_missing_library_raises(tmp_path):
    import paper_2107_11008_amd._sc as b
    saved = b._lib
    try:
        b._lib = None
        with pytest.raises(b.ScError):
            b.load(str(tmp_path / "nope.so"))
    finally:
        b._lib = saved
