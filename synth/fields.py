"""Seeded random coefficient fields (log-permeability, Young's modulus)."""
import numpy as np


def lognormal_iid(dims, sigma, rng):
    """log k = sigma * xi with xi ~ N(0,1) independent per cell; x fastest."""
    n = int(np.prod(dims))
    return sigma * rng.standard_normal(n)


def channelised_logk(dims, sigma, n_channels, contrast, rng, slab=4, half_width=3.0):
    """Layered, channelised log-permeability on a 3D grid of `dims` cells.

    Each z-layer gets sigma * xi_z with xi_z ~ N(0,1).  Each channel occupies
    a z-slab of `slab` layers starting at a uniform layer, and in the x-y
    plane the cells within `half_width` (cell units) of the centreline
    y = y0 + A sin(2 pi x / lam + phi); y0 ~ U(0, ny), A ~ U(8, 24),
    lam ~ U(32, 128), phi ~ U(0, 2 pi).  Channel cells add ln(contrast).
    """
    nx, ny, nz = dims
    xi = rng.standard_normal(nz)
    logk = np.broadcast_to(sigma * xi[:, None, None], (nz, ny, nx)).copy()
    chan = np.zeros((nz, ny, nx), dtype=bool)
    xc = np.arange(nx) + 0.5
    yc = np.arange(ny) + 0.5
    for _ in range(n_channels):
        z0 = int(rng.integers(0, max(nz - slab, 0) + 1))
        y0 = rng.uniform(0, ny)
        amp = rng.uniform(8, 24)
        lam = rng.uniform(32, 128)
        phi = rng.uniform(0, 2 * np.pi)
        centre = y0 + amp * np.sin(2 * np.pi * xc / lam + phi)  # per x
        inside = np.abs(yc[:, None] - centre[None, :]) <= half_width  # (ny, nx)
        chan[z0:z0 + slab] |= inside[None]
    logk = logk + np.log(contrast) * chan
    return logk.ravel(), chan.ravel()


def gaussian_smoothed(dims, std_cells, rng, truncate=3.0):
    """White noise on `dims` cells convolved with a separable Gaussian of
    standard deviation `std_cells` (non-periodic, truncated at `truncate`
    sigma), then standardised to mean 0 and standard deviation 1."""
    g = rng.standard_normal(tuple(reversed(dims)))
    r = int(np.ceil(truncate * std_cells))
    t = np.arange(-r, r + 1)
    ker = np.exp(-0.5 * (t / std_cells) ** 2)
    ker /= ker.sum()
    for ax in range(g.ndim):
        # centred part of the full convolution (also for axes shorter than
        # the kernel)
        g = np.apply_along_axis(lambda v: np.convolve(v, ker, mode="full")[r:r + v.size], ax, g)
    g = (g - g.mean()) / g.std()
    return g.ravel()


def observation_cells(n, count, rng):
    """`count` distinct observation cells drawn uniformly."""
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)
