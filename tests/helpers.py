"""Small problem builders shared by the tests (inputs only, no arithmetic of
the method)."""

import numpy as np

from workloads import Problem, dirichlet_we, five_spot, lognormal_grf


def make_problem(nx, ny=None, b=4, by=None, seg=2, alpha=1.0, log_var=1.0,
                 lam=0.2, seed=7, bc="we", source=False, K=None):
    ny = ny or nx
    by = by or b
    if K is None:
        K = lognormal_grf(nx, ny, lam, log_var, seed) if log_var > 0 else np.ones((ny, nx))
    if bc == "we":
        t, v = dirichlet_we(nx, ny)
        q = np.zeros((ny, nx))
    elif bc == "fivespot":
        q, t, v = five_spot(nx, ny)
    elif bc == "mixed":
        # Dirichlet on W, a prescribed outflow on E, no flow on S/N
        rng = np.random.default_rng(seed + 11)
        t, v = dirichlet_we(nx, ny)
        t[ny:2 * ny] = 0
        v[ny:2 * ny] = rng.uniform(0.0, 2.0 / ny, ny)
        v[2 * ny:2 * ny + nx] = rng.uniform(-0.5 / nx, 0.5 / nx, nx)
        t[2 * ny + nx:] = 1
        v[2 * ny + nx:] = rng.uniform(0.0, 1.0, nx)
        q = np.zeros((ny, nx))
    else:
        raise ValueError(bc)
    if source:
        rng = np.random.default_rng(seed + 3)
        q = q + rng.standard_normal((ny, nx)) / (nx * ny)
    return Problem(nx=nx, ny=ny, K=K, q=q, bc_type=t, bc_value=v,
                   sub_nx=b, sub_ny=by, seg=seg, alpha=alpha)


def make_problem3d(nx, ny, nz, b=8, seg=2, alpha=1.0, log_var=2.0, lam=0.2, seed=3, bc="we",
                   source=True, lz=0.5):
    """A 3D problem (workloads.Problem3D): log-normal field, W/E Dirichlet
    data (bc="we"), a mixed set (Dirichlet W and T, prescribed fluxes E and
    S) or all-Neumann five-spot wells (bc="neumann")."""
    from workloads import Problem3D, dirichlet_we3d, lognormal_grf3d
    K = lognormal_grf3d(nx, ny, nz, lam, log_var, seed) if log_var > 0 else np.ones((nz, ny, nx))
    rng = np.random.default_rng(seed + 1)
    q = rng.standard_normal((nz, ny, nx)) / (nx * ny * nz) if source else np.zeros((nz, ny, nx))
    t, v = dirichlet_we3d(nx, ny, nz)
    if bc == "mixed":
        t[ny * nz:2 * ny * nz] = 0
        v[ny * nz:2 * ny * nz] = rng.uniform(0.0, 2.0 / (ny * nz), ny * nz)
        v[2 * ny * nz:2 * ny * nz + nx * nz] = rng.uniform(-0.5, 0.5, nx * nz) / (nx * nz)
        o = 2 * ny * nz + 2 * nx * nz + nx * ny
        t[o:] = 1
        v[o:] = rng.uniform(0.0, 1.0, nx * ny)
    elif bc == "neumann":
        t[:] = 0
        v[:] = 0.0
        q = np.zeros((nz, ny, nx))
        q[0, 0, 0], q[-1, -1, -1] = 1.0, -1.0
    return Problem3D(nx=nx, ny=ny, nz=nz, K=K, q=q, bc_type=t, bc_value=v, sub_nx=b, sub_ny=b, seg=seg,
                     alpha=alpha, lz=lz)
