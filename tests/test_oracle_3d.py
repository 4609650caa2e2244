"""Pins of the 3D oracle (oracle/three_d.py): the paper's experiments are
three-dimensional with no z-division of the finest decomposition and
Hbar_z = H_z (Section 5.1).

* closed forms: the fine seven-point solve gives the exactly linear
  pressure for homogeneous and z-layered permeability with W/E Dirichlet
  data; the MRCM gives it on vertical strips with K constant on every
  segment (the linear pressure then lies in the discrete spaces);
* extrusion: with K, sources and boundary data independent of z, every
  layer carries the solution of the 2D method on the same columns (the
  already pinned 2D oracle, with per-face fluxes scaled by the layer
  height), for the fine solve and for the MRCM;
* brute force: the non-recursive MRCM equals the face-by-face monolithic
  system (Dirichlet, mixed and all-Neumann data, alpha 1e-3 .. 1e3);
* per-cell conservation and eq. 13.2 / eq. 14.2 on every segment.
"""

import numpy as np
import pytest

from helpers import make_problem
from oracle.fine import fine_solve
from oracle.metrics import rel_l2
from oracle.mrcm import mrcm_solve
from oracle.three_d import fine_solve3d, mrcm_solve3d, monolithic_solve3d, Decomposition3D
from workloads import Problem3D, dirichlet_we3d, lognormal_grf3d, bc_faces3d


def problem3d(nx=16, ny=16, nz=3, b=8, seg=2, alpha=1.0, bc="we", seed=3, lz=0.5):
    K = lognormal_grf3d(nx, ny, nz, 0.2, 2.0, seed)
    rng = np.random.default_rng(seed + 1)
    q = rng.standard_normal((nz, ny, nx)) / (nx * ny * nz)
    t, v = dirichlet_we3d(nx, ny, nz)
    if bc == "mixed":
        # Dirichlet W, prescribed outflow E, a prescribed flux through S,
        # Dirichlet T
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
    return Problem3D(nx=nx, ny=ny, nz=nz, K=K, q=q, bc_type=t, bc_value=v, sub_nx=b, sub_ny=b,
                     seg=seg, alpha=alpha, lz=lz)


@pytest.mark.parametrize("layered", [False, True])
def test_fine3d_linear_pressure(layered):
    nx, ny, nz = 12, 6, 4
    t, v = dirichlet_we3d(nx, ny, nz)
    K = np.full((nz, ny, nx), 2.5)
    if layered:
        K = K * np.exp(np.arange(nz))[:, None, None]
    pr = Problem3D(nx=nx, ny=ny, nz=nz, K=K, q=np.zeros((nz, ny, nx)), bc_type=t, bc_value=v,
                   sub_nx=6, sub_ny=6, seg=2, lz=0.7)
    p, F = fine_solve3d(pr)
    xc = (np.arange(nx) + 0.5) / nx
    assert np.abs(p - (1 - xc)[None, None, :]).max() < 1e-13
    # the flux through every x-face of layer k is K_k * area * 1
    hy, hz = 1.0 / ny, 0.7 / nz
    assert np.allclose(F[1][:, :, :-1], (K[:, :, :-1] * hy * hz), rtol=1e-12)


@pytest.mark.parametrize("alpha", [0.1, 1.0, 100.0])
def test_mrcm3d_vertical_strips_exactly_linear(alpha):
    nx, ny, nz = 32, 8, 3
    t, v = dirichlet_we3d(nx, ny, nz)
    rng = np.random.default_rng(4)
    kseg = np.exp(rng.standard_normal(ny // 4))
    K = np.broadcast_to(np.repeat(kseg, 4)[None, :, None], (nz, ny, nx)).copy()
    pr = Problem3D(nx=nx, ny=ny, nz=nz, K=K, q=np.zeros((nz, ny, nx)), bc_type=t, bc_value=v,
                   sub_nx=8, sub_ny=8, seg=4, alpha=alpha)
    p, F, U, P, dec = mrcm_solve3d(pr)
    xc = (np.arange(nx) + 0.5) / nx
    assert np.abs(p - (1 - xc)[None, None, :]).max() < 1e-12


@pytest.mark.parametrize("bc", ["we", "mixed", "fivespot"])
def test_extruded_3d_equals_2d(bc):
    """Every layer of a z-independent 3D problem (lz = 1, nz layers) is the
    2D problem: pressures equal, lateral per-face fluxes and sources divided
    by nz, U and P equal."""
    nz = 3
    p2 = make_problem(16, b=8, seg=2, log_var=2.0, bc=bc, source=(bc != "fivespot"), seed=6)
    nx, ny = p2.nx, p2.ny
    K = np.broadcast_to(p2.K, (nz, ny, nx)).copy()
    q = np.broadcast_to(p2.q / nz, (nz, ny, nx)).copy()
    t = np.zeros(bc_faces3d(nx, ny, nz), dtype=np.int8)
    v = np.zeros(bc_faces3d(nx, ny, nz))
    for k in range(nz):
        for (o3, o2, n) in ((0, 0, ny), (ny * nz, ny, ny), (2 * ny * nz, 2 * ny, nx),
                            (2 * ny * nz + nx * nz, 2 * ny + nx, nx)):
            t[o3 + k * n:o3 + (k + 1) * n] = p2.bc_type[o2:o2 + n]
            vals = p2.bc_value[o2:o2 + n]
            v[o3 + k * n:o3 + (k + 1) * n] = np.where(p2.bc_type[o2:o2 + n] == 1, vals, vals / nz)
    pr = Problem3D(nx=nx, ny=ny, nz=nz, K=K, q=q, bc_type=t, bc_value=v, sub_nx=8, sub_ny=8, seg=2,
                   alpha=p2.alpha, lz=1.0)
    pf, Ff = fine_solve3d(pr)
    pf2, Ff2 = fine_solve(p2)
    r2 = mrcm_solve(p2)
    p, F, U, P, dec = mrcm_solve3d(pr)
    for k in range(nz):
        assert rel_l2(pf[k], pf2) < 1e-12 and rel_l2(nz * Ff[:4, k], Ff2) < 1e-12
        assert rel_l2(p[k], r2.p) < 1e-11 and rel_l2(nz * F[:4, k], r2.F) < 1e-11
    assert np.abs(F[4:]).max() < 1e-13 * np.abs(F).max()
    assert rel_l2(U, r2.U) < 1e-10 and rel_l2(P, r2.P) < 1e-10


@pytest.mark.parametrize("bc", ["we", "mixed", "neumann"])
@pytest.mark.parametrize("alpha", [1e-3, 1.0, 1e3])
def test_mrcm3d_matches_brute_force(bc, alpha):
    pr = problem3d(alpha=alpha, bc=bc)
    p, F, U, P, dec = mrcm_solve3d(pr)
    pm, Fm, Um, Pm = monolithic_solve3d(pr)
    assert rel_l2(p, pm) < 1e-11 and rel_l2(F, Fm) < 1e-11
    assert rel_l2(U, Um) < 1e-9 and rel_l2(P, Pm) < (1e-8 if alpha > 1 else 1e-10)


def test_mrcm3d_conservation_and_interface_equations():
    pr = problem3d(nx=32, ny=32, nz=4, b=16, seg=4, bc="mixed")
    p, F, U, P, dec = mrcm_solve3d(pr)
    bal = F.sum(axis=0) - pr.q
    assert np.abs(bal).max() < 1e-12 * np.abs(F).max()
    scale = np.abs(F).max()
    for e in range(dec.nseg):
        if e < dec.nv:
            I, s = e // dec.lines_v + 1, e % dec.lines_v
            js = slice(s * dec.sg, (s + 1) * dec.sg)
            flo, fhi = F[1][:, js, I * dec.bx - 1].sum(), F[0][:, js, I * dec.bx].sum()
        else:
            r = e - dec.nv
            J, s = r // dec.lines_h + 1, r % dec.lines_h
            is_ = slice(s * dec.sg, (s + 1) * dec.sg)
            flo, fhi = F[3][:, J * dec.by - 1, is_].sum(), F[2][:, J * dec.by, is_].sum()
        assert abs(flo + fhi) < 1e-12 * scale
        assert abs(flo - fhi - 2 * dec.seg_length[e] * U[e]) < 1e-12 * scale


def test_decomposition3d_segments():
    pr = problem3d(nx=32, ny=16, nz=2, b=8, seg=4)
    dec = Decomposition3D(pr)
    assert dec.nseg == 3 * (16 // 4) + 1 * (32 // 4)
    # area of a vertical segment: seg faces of hy x hz
    assert abs(dec.seg_length[0] - 4 * (1 / 16) * 2 * (0.5 / 2)) < 1e-15
