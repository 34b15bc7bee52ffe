"""The C-ABI library loads and exports every entry point that include/vp.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2204_10822_amd", "libvp.so")
HDRS = [os.path.join(ROOT, "include", h) for h in ("vp.h", "vpnet.h")]


def declared():
    names = set()
    for h in HDRS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(vp(?:net)?_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared()
    for n in ["vp_residual", "vp_newton_assemble", "vp_amg_setup", "vp_krylov_solve",
              "vp_newton_step", "vp_create", "vp_destroy", "vp_set_state"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvp.so not built")
def test_binding_signatures_cover_the_header():
    from paper_2204_10822_amd import vp
    assert set(declared()) <= set(vp.EXPORTED) | set(vp.EXPORTED_NET)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvp.so not built")
def test_create_rejects_bad_descriptions_without_touching_the_device():
    from paper_2204_10822_amd import vp
    d = vp.vp_problem_desc(1, 5, 512e3, 512e3, 900, 1.3, 1026, 1.2e-3, 5.5e-3, 27500, 20, 2, 0, 1800, 2e-9)
    h = ctypes.c_void_p()
    assert vp.LIB.vp_create(ctypes.byref(d), None, ctypes.byref(h)) == vp.VP_EINVAL
    assert b"nx" in vp.LIB.vp_last_error(None)
    d.nx, d.dt = 8, -1.0
    assert vp.LIB.vp_create(ctypes.byref(d), None, ctypes.byref(h)) == vp.VP_EINVAL


def header_constants():
    """NAME = value pairs of the enums in include/vp.h."""
    text = re.sub(r"/\*.*?\*/", "", open(HDRS[0]).read(), flags=re.S)
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(VP_[A-Z0-9_]+)\s*=\s*(-?\d+)", text)}


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvp.so not built")
def test_binding_constants_match_the_header():
    """Every enum value the binding defines equals the header's, and the profiling
    kernel ids cover the header's list (VP_KID_COUNT entries)."""
    from paper_2204_10822_amd import vp
    consts = header_constants()
    checked = 0
    for name, value in consts.items():
        if name.startswith("VP_KID_") or not hasattr(vp, name):
            continue
        assert getattr(vp, name) == value, name
        checked += 1
    assert checked >= 20
    kids = {k: v for k, v in consts.items() if k.startswith("VP_KID_") and k != "VP_KID_COUNT"}
    assert sorted(vp.VP_KID.values()) == sorted(kids.values()) == list(range(consts["VP_KID_COUNT"]))
    for name, value in vp.VP_KID.items():
        assert kids["VP_KID_" + name.upper()] == value, name
