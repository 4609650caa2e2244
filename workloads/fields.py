"""Synthetic permeability fields.

* ``gaussian_field_exp`` — a stationary, zero-mean, unit-variance Gaussian
  random field with exponential covariance ``C(r) = exp(-|r| / lam)``
  sampled at cell centres by circulant embedding on a doubled torus
  (Dietrich & Newsam 1997).  Negative embedding eigenvalues are clipped to
  zero; the clipped fraction is returned for logging.
* ``lognormal_grf`` — ``K = exp(sigma * xi)`` with ``sigma**2`` the
  log-variance: the log-normal family the paper uses for its heterogeneous
  runs (Section 5, the log-normal permeability equation), here in 2D.
* ``channelized`` — a bimodal field of sinusoidal high-permeability channels
  on a low-permeability background with a small log-normal noise.

Arrays are ``float64`` of shape ``(ny, nx)``, row ``j`` is the ``j``-th
cell row in ``y`` and column ``i`` the ``i``-th cell in ``x``.
"""

from __future__ import annotations

import numpy as np


def gaussian_field_exp(nx: int, ny: int, lam: float, seed: int,
                       lx: float = 1.0, ly: float = 1.0,
                       return_clipped: bool = False):
    """Zero-mean unit-variance GRF with covariance exp(-|r|/lam)."""
    if nx <= 0 or ny <= 0:
        raise ValueError("grid must be non-empty")
    hx, hy = lx / nx, ly / ny
    mx, my = 2 * nx, 2 * ny
    ax = np.arange(mx)
    ay = np.arange(my)
    dx = np.minimum(ax, mx - ax) * hx
    dy = np.minimum(ay, my - ay) * hy
    r = np.sqrt(dy[:, None] ** 2 + dx[None, :] ** 2)
    c = np.exp(-r / lam)
    lam_eig = np.fft.fft2(c).real
    neg = lam_eig < 0
    clipped = float(-lam_eig[neg].sum() / np.abs(lam_eig).sum()) if neg.any() else 0.0
    lam_eig = np.where(neg, 0.0, lam_eig)
    rng = np.random.default_rng(seed)
    eps = rng.standard_normal((my, mx)) + 1j * rng.standard_normal((my, mx))
    w = np.fft.fft2(np.sqrt(lam_eig / (mx * my)) * eps)
    xi = np.ascontiguousarray(w.real[:ny, :nx])
    if return_clipped:
        return xi, clipped
    return xi


def lognormal_grf(nx: int, ny: int, lam: float, log_var: float, seed: int,
                  lx: float = 1.0, ly: float = 1.0) -> np.ndarray:
    """K = exp(sqrt(log_var) * xi), xi the exponential-covariance GRF."""
    xi = gaussian_field_exp(nx, ny, lam, seed, lx, ly)
    return np.exp(np.sqrt(log_var) * xi)


def channelized(n: int, seed: int, n_channels: int = 24,
                k_channel: float = 1000.0, k_background: float = 1.0,
                noise_frac: float = 0.05,
                width_cells=(8, 32)) -> np.ndarray:
    """Bimodal field of sinusoidal channels (square n x n grid, unit square).

    Channel ``c`` has centre line ``y_c(x) = c0 + A sin(2 pi x / wl + phi)``
    with ``A ~ U[0.02, 0.1]``, ``wl ~ U[0.25, 1]``, ``phi ~ U[0, 2 pi)``,
    ``c0 ~ U[0, 1]`` and a width drawn uniformly from ``width_cells`` (in
    cells).  ``log K = log k_channel`` inside a channel and
    ``log k_background`` outside, plus i.i.d. normal noise of standard
    deviation ``noise_frac * log(k_channel / k_background)``.
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    xc = (np.arange(n) + 0.5) * h
    yc = (np.arange(n) + 0.5) * h
    inside = np.zeros((n, n), dtype=bool)
    for _ in range(n_channels):
        c0 = rng.uniform(0.0, 1.0)
        amp = rng.uniform(0.02, 0.1)
        wl = rng.uniform(0.25, 1.0)
        phi = rng.uniform(0.0, 2 * np.pi)
        width = rng.integers(width_cells[0], width_cells[1] + 1) * h
        centre = c0 + amp * np.sin(2 * np.pi * xc / wl + phi)      # (nx,)
        inside |= np.abs(yc[:, None] - centre[None, :]) < 0.5 * width
    lk = np.where(inside, np.log(k_channel), np.log(k_background))
    span = np.log(k_channel / k_background)
    lk = lk + rng.standard_normal((n, n)) * (noise_frac * span)
    return np.exp(lk)


def lognormal_grf3d(nx: int, ny: int, nz: int, lam: float, log_var: float, seed: int,
                    lx: float = 1.0, ly: float = 1.0, lz: float = 1.0) -> np.ndarray:
    """3D log-normal field (the paper's field type, Section 5): K =
    exp(sqrt(log_var) xi) with xi the exponential-covariance GRF sampled by
    circulant embedding on the doubled 3D torus (negative eigenvalues
    clipped).  Shape (nz, ny, nx)."""
    hx, hy, hz = lx / nx, ly / ny, lz / nz
    m = (2 * nz, 2 * ny, 2 * nx)
    d = [np.minimum(np.arange(k), k - np.arange(k)) * h for k, h in zip(m, (hz, hy, hx))]
    r = np.sqrt(d[0][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[2][None, None, :] ** 2)
    lam_eig = np.fft.fftn(np.exp(-r / lam)).real
    lam_eig = np.where(lam_eig < 0, 0.0, lam_eig)
    rng = np.random.default_rng(seed)
    eps = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    w = np.fft.fftn(np.sqrt(lam_eig / lam_eig.size) * eps)
    xi = np.ascontiguousarray(w.real[:nz, :ny, :nx])
    return np.exp(np.sqrt(log_var) * xi)
