"""Seeded synthetic inputs: wave-speed models and right-hand sides.

This module only draws random media and sources.  It contains none of the
solver's arithmetic, so both the CPU reference implementation (``oracle/``)
and the GPU library's tests and benchmark may take their inputs from here.

Units are km and km/s.  Arrays use the solver's node ordering: axis 0 is the
sweep axis x (slowest), the last axis is the depth axis (fastest).  All
generators take an explicit integer seed and use ``numpy.random.default_rng``.

The paper's own media (Marmousi, SEG/EAGE salt) are not available; the
layered and smooth random models below stand in for them with the sizes,
speed range and correlation lengths of the paper's workloads.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter1d

C_MIN = 1.5
C_MAX = 4.5


def gaussian_random_field(shape, corr_len, seed):
    """Zero-mean, unit-std Gaussian random field with covariance exp(-r^2/l^2).

    White noise is filtered in Fourier space by the square root of the
    spectral density exp(-|k|^2 l^2 / 4) on a grid padded by 3 correlation
    lengths per axis (to suppress periodic wrap-around), then cropped and
    normalised to unit sample standard deviation.
    """
    rng = np.random.default_rng(seed)
    pad = int(np.ceil(3 * corr_len))
    big = tuple(s + 2 * pad for s in shape)
    noise = rng.standard_normal(big)
    spec = np.fft.fftn(noise)
    k2 = np.zeros(big)
    for ax, n in enumerate(big):
        kk = 2 * np.pi * np.fft.fftfreq(n)
        sh = [1] * len(big)
        sh[ax] = n
        k2 = k2 + kk.reshape(sh) ** 2
    filt = np.exp(-k2 * corr_len ** 2 / 8.0)
    field = np.real(np.fft.ifftn(spec * filt))
    sl = tuple(slice(pad, pad + s) for s in shape)
    field = field[sl]
    field = field - field.mean()
    std = field.std()
    return field / std if std > 0 else field


def layered_medium_2d(n_x, n_z, seed, n_layers=20, smooth_cells=2.0,
                      pert_amp=0.05, corr_len=20.0):
    """2-D smooth random layered model on an n_x x n_z node grid.

    ``n_layers`` equal-thickness horizontal layers (constant in x) with speeds
    drawn uniformly from [1.5, 4.5] km/s; interfaces smoothed along depth by a
    Gaussian of ``smooth_cells`` standard deviation; multiplied by
    (1 + pert_amp * g) with g a unit-std Gaussian random field of correlation
    length ``corr_len`` cells; clipped to [1.5, 4.5].
    """
    rng = np.random.default_rng(seed)
    speeds = rng.uniform(C_MIN, C_MAX, size=n_layers)
    idx = np.minimum((np.arange(n_z) * n_layers) // n_z, n_layers - 1)
    prof = speeds[idx]
    prof = gaussian_filter1d(prof, smooth_cells, mode="nearest")
    g = gaussian_random_field((n_x, n_z), corr_len, seed + 7919)
    c = prof[None, :] * (1.0 + pert_amp * g)
    return np.clip(c, C_MIN, C_MAX)


def smooth_medium_3d(n_x, n_y, n_z, seed, pert_amp=0.05, corr_len=10.0):
    """3-D smooth random model: linear depth trend 1.5 -> 4.5 km/s times
    (1 + pert_amp * g), g a unit-std 3-D Gaussian random field, clipped."""
    z = np.linspace(0.0, 1.0, n_z)
    bg = C_MIN + (C_MAX - C_MIN) * z
    g = gaussian_random_field((n_x, n_y, n_z), corr_len, seed)
    c = bg[None, None, :] * (1.0 + pert_amp * g)
    return np.clip(c, C_MIN, C_MAX)


def gaussian_anomaly(shape, centre, sigma_cells, amp):
    """Multiplicative Gaussian bump 1 + amp * exp(-|x - centre|^2 / (2 sigma^2))."""
    grids = np.meshgrid(*[np.arange(s, dtype=float) for s in shape], indexing="ij")
    r2 = sum((g - c) ** 2 for g, c in zip(grids, centre))
    return 1.0 + amp * np.exp(-r2 / (2.0 * sigma_cells ** 2))


def resample_nodes(c, n_new):
    """Bilinear resampling of a model given at the interior nodes of a unit
    square (n nodes per axis, spacing 1/(n+1)) onto n_new nodes per axis, so
    that grids of several resolutions carry the same medium."""
    c = np.asarray(c, dtype=float)
    out = c
    for ax in range(c.ndim):
        n = out.shape[ax]
        x_old = np.arange(1, n + 1) / (n + 1.0)
        x_new = np.arange(1, n_new + 1) / (n_new + 1.0)
        out = np.apply_along_axis(lambda v: np.interp(x_new, x_old, v), ax, out)
    return out


def extend_into_pml(c_interior, w):
    """Constant (edge-value) extension of an interior model by w nodes per side."""
    return np.pad(c_interior, w, mode="edge")


def point_source(shape, node, h, dim=None):
    """Discrete unit point source: 1/h^dim at one node (0-based node tuple)."""
    dim = len(shape) if dim is None else dim
    f = np.zeros(shape, dtype=np.complex128)
    f[tuple(node)] = 1.0 / h ** dim
    return f


def random_rhs(shape, seed, support=None):
    """Complex Gaussian right-hand side, optionally zero outside a boolean mask."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    if support is not None:
        f = np.where(support, f, 0.0)
    return f
