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


def params(nx=64, b=16, seg=4, precision=0, **kw):
    from paper_2009_07965_amd import rmrcm_default_params
    p = rmrcm_default_params()
    p.nx = p.ny = nx
    p.sub_nx = p.sub_ny = b
    p.seg = seg
    p.precision = precision
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_memory_plan_counts_the_large_arrays():
    """The plan holds at least the basis (nslot columns of b^2 cells per
    subdomain), the factor store (b inverted b x b blocks per subdomain) and
    eight cell arrays (permeability, source, pressure, four fluxes, the
    particular solution), FP64; the traces and merge blocks of every level
    add less than as much again.  The mixed mode adds exactly its FP32
    factor store and sweep scratch and its per-subdomain residual, fallback
    (setup and solve) and refinement-history arrays."""
    from paper_2009_07965_amd import rmrcm_plan_bytes
    for nx, b, seg in [(64, 16, 4), (1024, 32, 8), (8192, 32, 8), (2048, 16, 4)]:
        nsub = (nx // b) ** 2
        R = 4 * b // seg
        fp64 = rmrcm_plan_bytes(params(nx, b, seg))
        low = 8 * nsub * (R * b * b + b * b * b) + 8 * 8 * nx * nx
        assert low < fp64 < 2 * low, (nx, fp64, low)
        mixed = rmrcm_plan_bytes(params(nx, b, seg, precision=1))
        extra = 4 * nsub * b * b * b + 4 * nsub * R * b * b + 8 * nsub + 2 * 4 * nsub + 4 * 4 + 8 * 2 * 16
        assert mixed - fp64 == extra


def test_memory_plan_rejects_what_setup_rejects():
    from paper_2009_07965_amd import rmrcm_plan_bytes, RMRCMError
    with pytest.raises(RMRCMError) as ei:
        rmrcm_plan_bytes(params(nx=96))
    assert ei.value.status == -1
    with pytest.raises(RMRCMError) as ei:
        rmrcm_plan_bytes(params(nx=96, b=12, seg=4))
    assert ei.value.status == -7


def test_memory_cap_gives_enomem_before_device_work():
    """A cap one byte below the plan: RMRCM_ENOMEM from the host, with no
    device (here there is none).  A cap at the plan passes that check, and
    the setup goes on to the device query (RMRCM_EDEVICE without a GPU)."""
    import torch
    from paper_2009_07965_amd import rmrcm_plan_bytes, rmrcm_setup, RMRCMError
    p = params()
    need = rmrcm_plan_bytes(p)
    K, t = np.ones(64 * 64), np.zeros(4 * 64, np.int8)
    t[:64] = 1
    p.mem_cap = need - 1
    with pytest.raises(RMRCMError) as ei:
        rmrcm_setup(p, K, t)
    assert ei.value.status == -2
    if not torch.cuda.is_available():
        p.mem_cap = need
        with pytest.raises(RMRCMError) as ei:
            rmrcm_setup(p, K, t)
        assert ei.value.status == -3


@pytest.mark.parametrize("bad", [
    dict(seg_u=3), dict(seg_p=32), dict(seg_u=8, seg_p=12, sub_nx=24, sub_ny=24, nx=96, ny=96),
    dict(seg_u=-4),
])
def test_general_spaces_rejected_by_validation(bad):
    """General interface spaces: U- and P-segment lengths that do not
    divide the subdomain, or that are not nested, are EINVAL (host
    validation, through the memory plan, before any device work)."""
    from paper_2009_07965_amd import rmrcm_plan_bytes, RMRCMError
    with pytest.raises(RMRCMError) as ei:
        rmrcm_plan_bytes(params(**bad))
    assert ei.value.status in (-1, -7)


def test_general_spaces_plan_and_noalloc():
    """The plan of general spaces holds the merge scratch of every level
    (more than the MuMM plan on the same pieces); the allocation-free step
    rejects them with ENOTSUP before looking at its arrays."""
    import ctypes
    from paper_2009_07965_amd import rmrcm_plan_bytes, load_library
    mumm = rmrcm_plan_bytes(params(256, 16, 4))
    gen = rmrcm_plan_bytes(params(256, 16, 4, seg_u=8))
    assert gen > mumm
    lib = load_library()
    p = params(256, 16, 4, seg_u=8)
    assert lib.rmrcm_step_noalloc(ctypes.byref(p), None, None, None, None, None, None, None) == -7


@pytest.mark.parametrize("bad,status", [
    (dict(nz=-1), -1), (dict(nz=4, lz=0.0), -1), (dict(nz=4, precision=1), -7),
    (dict(nz=8, sub_nx=16), -7), (dict(nz=4, seg_u=8), -7),
])
def test_3d_validation(bad, status):
    """3D problems (nz >= 1): FP64, MuMM spaces, sub_nx * nz <= 64."""
    from paper_2009_07965_amd import rmrcm_plan_bytes, RMRCMError
    p = params(64, 8, 4)
    p.lz = 1.0
    for k, v in bad.items():
        setattr(p, k, v)
    with pytest.raises(RMRCMError) as ei:
        rmrcm_plan_bytes(p)
    assert ei.value.status == status


def test_3d_plan_counts_the_columns():
    """The plan of a 3D problem holds its basis (R columns of the column's
    cells), factor store (by inverted blocks of (sub_nx nz)^2) and the six
    flux blocks."""
    from paper_2009_07965_amd import rmrcm_plan_bytes
    nx, b, seg, nz = 256, 8, 4, 8
    p = params(nx, b, seg)
    p.nz, p.lz = nz, 1.0
    nsub = (nx // b) ** 2
    R = 4 * b // seg
    n = b * b * nz
    low = 8 * nsub * (R * n + b * (b * nz) ** 2) + 8 * 10 * nx * nx * nz
    plan = rmrcm_plan_bytes(p)
    assert low < plan < 2 * low, (plan, low)
