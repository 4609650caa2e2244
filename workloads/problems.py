"""Problem records and the concrete synthetic workloads.

A :class:`Problem` is the 2D Darcy problem in mixed form (Section 2, the
model equations) on ``[0, lx] x [0, ly]`` discretised on a uniform
``nx x ny`` grid, together with the domain-decomposition parameters of the
method (subdomain size ``H`` in cells, interface segment ``Hbar`` in cells
and the Robin parameter ``alpha``).

Boundary data layout (shared by every consumer): one entry per boundary
face, ordered ``W (ny faces, bottom to top), E (ny), S (nx faces, left to
right), N (nx)``.  ``bc_type`` is 1 for Dirichlet (``bc_value`` is the
pressure) and 0 for Neumann (``bc_value`` is the outward *integrated* flux
through that face).  ``q`` is the cell-integrated source.
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

from .fields import lognormal_grf, channelized

BC_NEUMANN = 0
BC_DIRICHLET = 1


@dataclass
class Problem:
    nx: int
    ny: int
    K: np.ndarray                 # (ny, nx) permeability, > 0
    q: np.ndarray                 # (ny, nx) cell-integrated source
    bc_type: np.ndarray           # (2ny + 2nx,) int8
    bc_value: np.ndarray          # (2ny + 2nx,) float64
    sub_nx: int
    sub_ny: int
    seg: int
    alpha: float = 1.0
    lx: float = 1.0
    ly: float = 1.0
    name: str = ""
    meta: dict = field(default_factory=dict)
    # general MRCM interface spaces (Section 2, with the U and P spaces
    # chosen apart): piecewise constant U_H on segments of seg_u cells and
    # P_H on segments of seg_p cells; 0 = seg (the MuMM choice of Section 4,
    # both spaces on the same segments)
    seg_u: int = 0
    seg_p: int = 0

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny


def dirichlet_we(nx: int, ny: int, p_west: float = 1.0, p_east: float = 0.0):
    """p = p_west on x = 0, p = p_east on x = lx, no flow on y = 0 and y = ly
    (the boundary conditions of the paper's experiments, Section 5.1)."""
    t = np.zeros(2 * ny + 2 * nx, dtype=np.int8)
    v = np.zeros(2 * ny + 2 * nx, dtype=np.float64)
    t[:ny] = BC_DIRICHLET
    v[:ny] = p_west
    t[ny:2 * ny] = BC_DIRICHLET
    v[ny:2 * ny] = p_east
    return t, v


def five_spot(nx: int, ny: int):
    """No flow on the whole boundary, q = +1 in cell (0, 0) and -1 in cell
    (nx-1, ny-1): a quarter five-spot pair of wells."""
    t = np.zeros(2 * ny + 2 * nx, dtype=np.int8)
    v = np.zeros(2 * ny + 2 * nx, dtype=np.float64)
    q = np.zeros((ny, nx))
    q[0, 0] = 1.0
    q[ny - 1, nx - 1] = -1.0
    return q, t, v


def _grf_problem(n, lam, log_var, seed, sub, seg, alpha=1.0, name=""):
    K = lognormal_grf(n, n, lam, log_var, seed)
    t, v = dirichlet_we(n, n)
    return Problem(nx=n, ny=n, K=K, q=np.zeros((n, n)), bc_type=t, bc_value=v,
                   sub_nx=sub, sub_ny=sub, seg=seg, alpha=alpha, name=name,
                   meta=dict(lam=lam, log_var=log_var, seed=seed))


# The five synthetic workloads.  Each entry builds the Problem on demand.
CONFIGS = {
    1: dict(desc="64x64 GRF (corr 0.1, log-var 1), 4x4 subdomains of 16x16, "
                 "4-cell segments, alpha 1, p=1 W / p=0 E",
            build=lambda: _grf_problem(64, 0.1, 1.0, 1, 16, 4, name="grf64")),
    2: dict(desc="1024x1024 GRF (corr 0.05, log-var 4), 32x32 subdomains of "
                 "32x32, 8-cell segments, alpha 1, p=1 W / p=0 E",
            build=lambda: _grf_problem(1024, 0.05, 4.0, 2, 32, 8, name="grf1024")),
    4: dict(desc="2048x2048 GRF (corr 0.05, log-var 4), 128x128 subdomains "
                 "of 16x16, 4-cell segments, alpha 1",
            build=lambda: _grf_problem(2048, 0.05, 4.0, 4, 16, 4, name="grf2048")),
    5: dict(desc="8192x8192 channelized bimodal field, 256x256 subdomains of "
                 "32x32, 8-cell segments, alpha 1",
            build=lambda: _channel_problem(8192, 5, 32, 8)),
}


def _channel_problem(n, seed, sub, seg):
    K = channelized(n, seed)
    t, v = dirichlet_we(n, n)
    return Problem(nx=n, ny=n, K=K, q=np.zeros((n, n)), bc_type=t, bc_value=v,
                   sub_nx=sub, sub_ny=sub, seg=seg, alpha=1.0,
                   name="channel%d" % n, meta=dict(seed=seed))


def config_problem(k: int) -> Problem:
    return CONFIGS[k]["build"]()


def ensemble_member(m: int, n_override: Optional[int] = None) -> Problem:
    """Member ``m`` of the 256-realisation ensemble: grid n in {128,256,512},
    subdomain b in {8,16,32}, log-variance U[1,5], correlation U[0.02,0.2],
    segment b/4, alpha 1, quarter five-spot wells, no flow on the boundary."""
    rng = np.random.default_rng(3000 + m)
    n = int(rng.choice([128, 256, 512]))
    b = int(rng.choice([8, 16, 32]))
    log_var = float(rng.uniform(1.0, 5.0))
    lam = float(rng.uniform(0.02, 0.2))
    if n_override is not None:
        n = n_override
    K = lognormal_grf(n, n, lam, log_var, seed=100000 + m)
    q, t, v = five_spot(n, n)
    return Problem(nx=n, ny=n, K=K, q=q, bc_type=t, bc_value=v,
                   sub_nx=b, sub_ny=b, seg=max(b // 4, 1), alpha=1.0,
                   name="ens%d" % m, meta=dict(lam=lam, log_var=log_var, member=m))


@dataclass
class Problem3D:
    """The 3D Darcy problem of the paper's experiments (Section 5) on
    ``[0, lx] x [0, ly] x [0, lz]`` with an ``nx x ny x nz`` grid, split
    into ``sub_nx x sub_ny`` columns of cells with no division in z
    (Section 5.1: the finest decomposition has no z-division and
    Hbar_z = H_z, so a skeleton segment is ``seg`` faces along the interface
    by the full height).

    Arrays are ``(nz, ny, nx)``.  Boundary data, one entry per boundary
    face in the order W (ny*nz faces, index k*ny + j), E (same), S (nx*nz,
    index k*nx + i), N (same), B (z = 0, nx*ny, index j*nx + i), T (z = lz,
    same).  Types and values as in the 2D problem."""
    nx: int
    ny: int
    nz: int
    K: np.ndarray
    q: np.ndarray
    bc_type: np.ndarray
    bc_value: np.ndarray
    sub_nx: int
    sub_ny: int
    seg: int
    alpha: float = 1.0
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0
    name: str = ""

    def with_(self, **kw) -> "Problem3D":
        return replace(self, **kw)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz


def bc_faces3d(nx: int, ny: int, nz: int) -> int:
    return 2 * ny * nz + 2 * nx * nz + 2 * nx * ny


def dirichlet_we3d(nx: int, ny: int, nz: int, p_west: float = 1.0, p_east: float = 0.0):
    """p = p_west on x = 0, p = p_east on x = lx, no flow elsewhere (the
    boundary conditions of the paper's runs, Section 5.1)."""
    n = bc_faces3d(nx, ny, nz)
    t = np.zeros(n, dtype=np.int8)
    v = np.zeros(n, dtype=np.float64)
    t[:2 * ny * nz] = BC_DIRICHLET
    v[:ny * nz] = p_west
    v[ny * nz:2 * ny * nz] = p_east
    return t, v


def grf3d_problem(n: int = 512, nz: int = 8, b: int = 8, seg: int = 2, alpha: float = 1e3,
                  log_var: float = 4.0, lam: float = 0.05, seed: int = 11) -> "Problem3D":
    """The 3D benchmark workload: an n x n x nz log-normal field (the paper's
    field type) on [0,1] x [0,1] x [0, nz/n] (cubic cells), columns of
    b x b x nz cells (no z-division), segments of seg faces (Hbar = H/4 for
    seg = b/4, one of the paper's two choices), alpha 1e3 (the paper's
    scaling runs), p = 1 at x = 0 and 0 at x = 1, no flow elsewhere, no
    source."""
    from .fields import lognormal_grf3d
    lz = nz / n
    K = lognormal_grf3d(n, n, nz, lam, log_var, seed, lz=lz)
    t, v = dirichlet_we3d(n, n, nz)
    return Problem3D(nx=n, ny=n, nz=nz, K=K, q=np.zeros((nz, n, n)), bc_type=t, bc_value=v, sub_nx=b,
                     sub_ny=b, seg=seg, alpha=alpha, lz=lz,
                     name="grf3d_%dx%dx%d" % (n, n, nz))
