"""The C-ABI library loads and exports every entry point the header declares
(CPU only: no compute call is made)."""
import os
import re

from paper_2311_17089_amd import msgs as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "msgs.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(msgs_[a-z_0-9]+)\s*\(", hdr)))


def test_header_declares_entry_points():
    names = _declared()
    assert "msgs_render" in names and "msgs_render_backward" in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    L = M.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_default_options():
    L = M.lib()
    assert L.msgs_version() == 1
    o = M.RenderOpts()
    L.msgs_default_opts(M.C.byref(o))
    assert (o.downscale, o.selective, o.update_range) == (1, 1, 0)
    assert abs(o.lowpass - 0.3) < 1e-7 and abs(o.near_z - 0.2) < 1e-7


def test_binding_declares_every_symbol():
    assert set(_declared()) <= set(M.EXPORTS)
