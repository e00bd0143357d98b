"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/pfsm.h declares, and rejects invalid descriptors
before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pfsm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pfsm_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_1502_07806_amd as pf
    if not os.path.exists(pf.LIB_PATH):
        from paper_1502_07806_amd import build_lib
        build_lib.build(verbose=False)
    return pf.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "pfsm_solve" in names and "pfsm_backward" in names and "pfsm_plan_create" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in range(6):
        assert lib.pfsm_status_string(code).startswith(b"PFSM")
    assert b"unknown" in lib.pfsm_status_string(99)


def _desc(n=64, offs=(0, 32, 64), **kw):
    from paper_1502_07806_amd.binding import PfsmDesc
    arr = (ctypes.c_int64 * len(offs))(*offs)
    d = PfsmDesc(n, len(offs) - 1, arr, kw.get("halo", -1), kw.get("iterations", 3), kw.get("fs_power", 2),
                 kw.get("alpha", 0.0), kw.get("shift_mode", 0), kw.get("precision", 0), 0, kw.get("flags", 0),
                 kw.get("resid_tol", 0.0))
    return d, arr


@pytest.mark.parametrize("kw", [dict(n=0), dict(offs=(0, 40, 32, 64)), dict(offs=(0, 32, 60)), dict(offs=(1, 32, 64)),
                                dict(offs=(0, 32, 32, 64)), dict(fs_power=3), dict(iterations=-1),
                                dict(shift_mode=7), dict(precision=9), dict(flags=64), dict(alpha=float("nan")),
                                dict(resid_tol=-1.0), dict(resid_tol=float("nan"))])
def test_plan_rejects_invalid_descriptors(lib, kw):
    n = kw.pop("n", 64)
    offs = kw.pop("offs", (0, 32, 64))
    d, keep = _desc(n, offs, **kw)
    h = ctypes.c_void_p()
    assert lib.pfsm_plan_create(ctypes.byref(h), ctypes.byref(d)) == 1  # PFSM_INVALID_ARG
    assert not h.value


def test_mixed_with_rayleigh_shift_not_supported(lib):
    d, keep = _desc(64, (0, 32, 64), precision=1, shift_mode=1)
    h = ctypes.c_void_p()
    assert lib.pfsm_plan_create(ctypes.byref(h), ctypes.byref(d)) == 2  # PFSM_NOT_SUPPORTED


def test_mixed_residuals_need_the_refinement(lib):
    """The mixed path's residuals come from its refinement product: asking for
    them without the refinement is refused before touching a device."""
    for kw in (dict(flags=1 | 4), dict(flags=1, resid_tol=1e-3)):
        d, keep = _desc(64, (0, 32, 64), precision=1, **kw)
        h = ctypes.c_void_p()
        assert lib.pfsm_plan_create(ctypes.byref(h), ctypes.byref(d)) == 2  # PFSM_NOT_SUPPORTED


def test_null_arguments(lib):
    assert lib.pfsm_plan_create(None, None) == 1
    assert lib.pfsm_workspace_size(None, None) == 1
    assert lib.pfsm_solve(None, None, 0, None, 0, None, None, 0, None, 0, None, None) == 1
    assert lib.pfsm_backward(None, None, None, 0, None, None, 0, 0.0, None, 0, None, 0, None, None) == 1
    lib.pfsm_plan_destroy(None)


def test_g2s_argument_validation(lib):
    """Generalized -> standard conversion: workspace size and argument checks
    (all rejected on the host, before any device work)."""
    sz = ctypes.c_size_t(0)
    assert lib.pfsm_g2s_workspace_size(0, ctypes.byref(sz)) == 1
    assert lib.pfsm_g2s_workspace_size(1000, None) == 1
    assert lib.pfsm_g2s_workspace_size(1000, ctypes.byref(sz)) == 0
    assert sz.value >= 1000 * 1000 * 8 + 2 * 1000 * 8
    f = lib.pfsm_generalized_to_standard
    fake = 1 << 40  # never dereferenced: every call below fails validation first
    assert f(0, fake, 1, fake, 1, 3, fake + (1 << 32), 1, fake + (1 << 33), sz.value, None, fake, None) == 1
    assert f(1000, None, 1000, fake, 1000, 3, fake + (1 << 32), 1000, fake + (1 << 33), sz.value, None, fake, None) == 1
    assert f(1000, fake, 999, fake, 1000, 3, fake + (1 << 32), 1000, fake + (1 << 33), sz.value, None, fake, None) == 1
    assert f(1000, fake, 1000, fake, 1000, -1, fake + (1 << 32), 1000, fake + (1 << 33), sz.value, None, fake,
             None) == 1
    # Z overlapping A
    assert f(1000, fake, 1000, fake + (1 << 34), 1000, 3, fake + 8, 1000, fake + (1 << 33), sz.value, None, fake,
             None) == 1
    # workspace too small, misaligned workspace
    assert f(1000, fake, 1000, fake + (1 << 34), 1000, 3, fake + (1 << 32), 1000, fake + (1 << 33), sz.value - 1,
             None, fake, None) == 5
    assert f(1000, fake, 1000, fake + (1 << 34), 1000, 3, fake + (1 << 32), 1000, fake + (1 << 33) + 8, sz.value,
             None, fake, None) == 1
