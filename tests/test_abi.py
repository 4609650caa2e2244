"""The C-ABI library: it builds, loads, exports every entry point the
header declares, and rejects invalid arguments before any device work (no
compute call needs a GPU here)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmrcm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rmrcm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("rmrcm_setup", "rmrcm_solve", "rmrcm_destroy", "rmrcm_strerror",
              "rmrcm_set_stream", "rmrcm_get_stats", "rmrcm_get_interface"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2009_07965_amd import load_library, EXPORTS
    lib = load_library()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(EXPORTS) == set(declared_functions())


def test_params_layout_and_defaults():
    from paper_2009_07965_amd import rmrcm_default_params
    p = rmrcm_default_params()
    assert p.alpha == 1.0 and p.lx == 1.0 and p.precision == 0 and p.device == 0


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(sub_nx=5), dict(seg=3), dict(nx=96), dict(alpha=0.0),
    dict(alpha=float("nan")), dict(lx=-1.0),
])
def test_setup_rejects_invalid_geometry(bad):
    """EINVAL / ENOTSUP come from host validation before any HIP call."""
    from paper_2009_07965_amd import rmrcm_default_params, rmrcm_setup, RMRCMError
    p = rmrcm_default_params()
    p.nx = p.ny = 64
    p.sub_nx = p.sub_ny = 16
    p.seg = 4
    for k, v in bad.items():
        setattr(p, k, v)
    n = max(p.nx, 1) * p.ny
    with pytest.raises(RMRCMError) as ei:
        rmrcm_setup(p, np.ones(n), np.zeros(2 * max(p.nx, 1) + 2 * p.ny, np.int8))
    assert ei.value.status in (-1, -7)


def test_strerror_table():
    from paper_2009_07965_amd import rmrcm_strerror
    assert rmrcm_strerror(0) == "ok"
    assert "singular" in rmrcm_strerror(-4)
    assert rmrcm_strerror(12345) == "unknown status"
