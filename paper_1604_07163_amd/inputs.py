"""Seeded synthetic inputs shaped like the structured-grid diffusion workloads.

This module holds input generators only: coefficient fields on grid links,
right-hand sides and sample draws.  It contains none of the solver's
arithmetic, so both the GPU path and the CPU oracle can be fed from it.

Conventions: N vertices per side on the unit cube, h = 1/(N-1), arrays in C
order (z, y, x) with x fastest.  Face (link) arrays:
  kx (N, N, N-1)  link (i,j,k)-(i+1,j,k)
  ky (N, N-1, N)  link (i,j,k)-(i,j+1,k)
  kz (N-1, N, N)  link (i,j,k)-(i,j,k+1)
All random draws use numpy.random.Generator(PCG64(seed)) in C order.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def face_shapes(n: int):
    return (n, n, n - 1), (n, n - 1, n), (n - 1, n, n)


def const_k(n: int, c: float = 1.0):
    sx, sy, sz = face_shapes(n)
    return np.full(sx, c), np.full(sy, c), np.full(sz, c)


def zero_boundary(v: np.ndarray) -> np.ndarray:
    v[0, :, :] = 0
    v[-1, :, :] = 0
    v[:, 0, :] = 0
    v[:, -1, :] = 0
    v[:, :, 0] = 0
    v[:, :, -1] = 0
    return v


def sine_rhs(n: int) -> np.ndarray:
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) at the vertices (boundary 0).

    The continuous solution of -lap(phi) = f with zero Dirichlet data is
    phi = sin(pi x) sin(pi y) sin(pi z)."""
    x = np.linspace(0.0, 1.0, n)
    s = np.sin(np.pi * x)
    f = 3.0 * np.pi ** 2 * s[:, None, None] * s[None, :, None] * s[None, None, :]
    return zero_boundary(f)


def sine_solution(n: int) -> np.ndarray:
    x = np.linspace(0.0, 1.0, n)
    s = np.sin(np.pi * x)
    return zero_boundary(s[:, None, None] * s[None, :, None] * s[None, None, :])


def uniform_rhs(n: int, seed: int) -> np.ndarray:
    """f ~ U(-1, 1) at interior vertices, 0 on the boundary."""
    f = rng(seed).uniform(-1.0, 1.0, size=(n, n, n))
    return zero_boundary(f)


def vertex_to_faces_log10(ell: np.ndarray):
    """Faces take the mean of the log10 values at their two end points
    (geometric mean of the vertex conductivities); returns k on the faces."""
    lx = 0.5 * (ell[:, :, :-1] + ell[:, :, 1:])
    ly = 0.5 * (ell[:, :-1, :] + ell[:, 1:, :])
    lz = 0.5 * (ell[:-1, :, :] + ell[1:, :, :])
    return 10.0 ** lx, 10.0 ** ly, 10.0 ** lz


def lognormal_log10_field(n: int, seed: int, width: float = 8.0, clip: float = 2.0) -> np.ndarray:
    """log10 k at the vertices: white N(0,1) noise smoothed by a Gaussian of
    standard deviation `width` cells (reflecting edges, truncated at 4 sigma),
    standardised to mean 0 / std 1, clipped to +-clip (contrast 10^(2 clip))."""
    from scipy.ndimage import gaussian_filter

    w = rng(seed).standard_normal(size=(n, n, n))
    g = gaussian_filter(w, sigma=width, mode="reflect", truncate=4.0)
    del w
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    np.clip(g, -clip, clip, out=g)
    return g


def gaussian_taps(width: float, truncate: float = 4.0) -> np.ndarray:
    """Normalised Gaussian taps exp(-x^2 / 2 width^2), |x| <= int(truncate*width + 0.5)."""
    r = int(truncate * float(width) + 0.5)
    x = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / width) ** 2)
    return w / w.sum()


def lognormal_log10_field_gpu(n: int, seed: int, width: float = 8.0, clip: float = 2.0, device="cuda"):
    """The same recipe as lognormal_log10_field, computed with torch on the GPU
    for large grids: identical white noise (the PCG64 stream drawn plane by
    plane in C order), separable Gaussian filtering with half-sample symmetric
    edges (scipy's 'reflect'), standardisation and clipping, in FP64."""
    import torch

    g = rng(seed)
    w = torch.empty((n, n, n), dtype=torch.float64, device=device)
    chunk = max(1, (1 << 27) // (n * n))
    for k0 in range(0, n, chunk):
        k1 = min(n, k0 + chunk)
        w[k0:k1] = torch.from_numpy(g.standard_normal(size=(k1 - k0, n, n))).to(device)
    taps = torch.from_numpy(gaussian_taps(width)).to(device)
    r = (taps.numel() - 1) // 2
    for axis in range(3):
        v = w.movedim(axis, -1)
        if r > n:
            raise ValueError("filter radius exceeds the grid")
        lo = v[..., :r].flip(-1)
        hi = v[..., -r:].flip(-1)
        padded = torch.cat([lo, v, hi], dim=-1)
        out = torch.zeros_like(v)
        for t in range(taps.numel()):
            out.add_(padded[..., t:t + n], alpha=float(taps[t]))
        w = out.movedim(-1, axis).contiguous()
        del padded, out, v, lo, hi
    w -= w.mean()
    sd = w.std(unbiased=False)
    if float(sd) > 0:
        w /= sd
    w.clamp_(-clip, clip)
    return w


def lognormal_k_gpu(n: int, seed: int, width: float = 8.0, clip: float = 2.0, device="cuda"):
    """Log-normal link conductivities on the GPU (torch float64 tensors)."""
    ell = lognormal_log10_field_gpu(n, seed, width, clip, device)
    kx = (10.0 ** (0.5 * (ell[:, :, :-1] + ell[:, :, 1:]))).contiguous()
    ky = (10.0 ** (0.5 * (ell[:, :-1, :] + ell[:, 1:, :]))).contiguous()
    kz = (10.0 ** (0.5 * (ell[:-1, :, :] + ell[1:, :, :]))).contiguous()
    del ell
    return kx, ky, kz


def uniform_rhs_gpu(n: int, seed: int, device="cuda"):
    """uniform_rhs drawn plane by plane (same stream) straight into GPU memory."""
    import torch

    g = rng(seed)
    f = torch.empty((n, n, n), dtype=torch.float64, device=device)
    chunk = max(1, (1 << 27) // (n * n))
    for k0 in range(0, n, chunk):
        k1 = min(n, k0 + chunk)
        f[k0:k1] = torch.from_numpy(g.uniform(-1.0, 1.0, size=(k1 - k0, n, n))).to(device)
    f[0] = f[-1] = 0
    f[:, 0] = f[:, -1] = 0
    f[:, :, 0] = f[:, :, -1] = 0
    return f


def lognormal_k(n: int, seed: int, width: float = 8.0, clip: float = 2.0):
    """Log-normal face conductivities (log10 k ~ N(0,1) smoothed, clipped)."""
    return vertex_to_faces_log10(lognormal_log10_field(n, seed, width, clip))


def inclusion_k(n: int, seed: int, rmin_cells: float = 4.0, rmax_cells: float = 16.0,
                frac: float = 0.20, k_in: float = 1e3, k_out: float = 1.0):
    """Two-phase conductivity: random spheres (centres U([0,1]^3), radii
    U(rmin, rmax) cells, overlaps allowed) are added until at least `frac` of
    the vertices lie inside one.  A face takes k_in when its midpoint lies
    inside any sphere, else k_out.  Returns (kx, ky, kz, n_spheres)."""
    g = rng(seed)
    h = 1.0 / (n - 1)
    sx, sy, sz = face_shapes(n)
    vin = np.zeros((n, n, n), dtype=bool)
    fx = np.zeros(sx, dtype=bool)
    fy = np.zeros(sy, dtype=bool)
    fz = np.zeros(sz, dtype=bool)
    target = frac * n ** 3
    count = 0
    nsph = 0
    while count < target:
        c = g.uniform(0.0, 1.0, size=3)  # (x, y, z)
        rad = g.uniform(rmin_cells, rmax_cells) * h
        nsph += 1
        lo = np.maximum(np.floor((c - rad) / h).astype(int) - 1, 0)
        hi = np.minimum(np.ceil((c + rad) / h).astype(int) + 1, n - 1)
        xs = np.arange(lo[0], hi[0] + 1) * h
        ys = np.arange(lo[1], hi[1] + 1) * h
        zs = np.arange(lo[2], hi[2] + 1) * h
        dx2 = (xs - c[0]) ** 2
        dy2 = (ys - c[1]) ** 2
        dz2 = (zs - c[2]) ** 2
        r2 = rad * rad
        inside = (dz2[:, None, None] + dy2[None, :, None] + dx2[None, None, :]) <= r2
        sub = vin[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        count += int(np.count_nonzero(inside & ~sub))
        sub |= inside
        # face midpoints: x-faces at (i+1/2) h for i in lo..min(hi, n-2)
        xm = (np.arange(lo[0], min(hi[0], n - 2) + 1) + 0.5) * h
        ym = (np.arange(lo[1], min(hi[1], n - 2) + 1) + 0.5) * h
        zm = (np.arange(lo[2], min(hi[2], n - 2) + 1) + 0.5) * h
        dxm2 = (xm - c[0]) ** 2
        dym2 = (ym - c[1]) ** 2
        dzm2 = (zm - c[2]) ** 2
        fx[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:lo[0] + len(xm)] |= (
            dz2[:, None, None] + dy2[None, :, None] + dxm2[None, None, :]) <= r2
        fy[lo[2]:hi[2] + 1, lo[1]:lo[1] + len(ym), lo[0]:hi[0] + 1] |= (
            dz2[:, None, None] + dym2[None, :, None] + dx2[None, None, :]) <= r2
        fz[lo[2]:lo[2] + len(zm), lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] |= (
            dzm2[:, None, None] + dy2[None, :, None] + dx2[None, None, :]) <= r2
    kx = np.where(fx, k_in, k_out)
    ky = np.where(fy, k_in, k_out)
    kz = np.where(fz, k_in, k_out)
    return kx, ky, kz, nsph


def sample_faces(n: int, count: int, seed: int):
    """`count` distinct active faces drawn uniformly without replacement.
    Returns a list of (axis, k, j, i) with axis 0=x, 1=y, 2=z (array index order)."""
    sizes = []
    for ax in range(3):
        # active links: both transverse indices interior, any index along the link
        sizes.append((n - 1) * (n - 2) * (n - 2))
    total = sum(sizes)
    picks = rng(seed).choice(total, size=count, replace=False)
    out = []
    for p in picks:
        ax = int(p // sizes[0])
        r = int(p % sizes[0])
        along = r % (n - 1)
        r //= (n - 1)
        t1 = r % (n - 2) + 1
        t2 = r // (n - 2) + 1
        if ax == 0:   # kx[k][j][i]: i along, j=t1, k=t2
            out.append((0, t2, t1, along))
        elif ax == 1:  # ky[k][j][i]: j along, i=t1, k=t2
            out.append((1, t2, along, t1))
        else:          # kz[k][j][i]: k along, i=t1, j=t2
            out.append((2, along, t2, t1))
    return out


# --------------------------------------------------------------------------
# the five synthetic workloads
# --------------------------------------------------------------------------
WORKLOADS = {
    "poisson33": dict(n=33, levels=4),
    "lognormal257": dict(n=257, levels=8, k_seed=2, f_seed=3),
    "inclusions513": dict(n=513, levels=9, k_seed=4, f_seed=5),
    "adjoint129": dict(n=129, levels=7, k_seed=6, kobs_seed=7, f_seed=8, face_seed=9),
    "lognormal1025": dict(n=1025, levels=10, k_seed=10, kobs_seed=11, f_seed=12, clip=3.0),
}
