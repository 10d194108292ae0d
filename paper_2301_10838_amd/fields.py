"""Seeded synthetic scalar fields for tests and benchmarks.

This module only draws inputs: it holds none of the merge-tree arithmetic and
is shared, as the one common piece, by the GPU path's tests and by the oracle
side.  Every generator is deterministic in its seed (numpy PCG64).

The paper evaluates on real simulation and CT volumes downsampled to 128^3,
256^3 and 512^3 (Sec. 4, Datasets); those are not available here, so these
fields stand in for them at the same sizes:

- ``uniform``: i.i.d. uniform [0, 1) float32 noise (maximal topological
  complexity: about one vertex in seven is a minimum in 3-D).
- ``bumps``: a sum of isotropic Gaussian bumps with signed amplitudes plus 1 %
  uniform noise (smooth simulation/CT-like fields with sparse large-scale
  topology and grid-scale noise).
- ``lognormal_grf``: a Gaussian random field with power spectrum k^-3 built
  by FFT, standardised and exponentiated (cosmology-density-like, standing in
  for the paper's Nyx dark-matter density).

Shapes follow the C order [nz][ny][nx] used throughout (a 2-D field is
[ny][nx]).
"""
from __future__ import annotations

import hashlib
import math
import os

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def uniform(shape, seed: int) -> np.ndarray:
    """i.i.d. uniform [0, 1) float32 (values on a 2^-24 grid, so ties occur)."""
    n = int(np.prod(shape))
    return _rng(seed).random(n, dtype=np.float32).reshape(shape)


def bumps(shape, seed: int, n_bumps: int = 64, sigma=(4.0, 16.0), noise: float = 0.01) -> np.ndarray:
    """Sum of Gaussian bumps + uniform noise, accumulated in float64, cast to float32.

    Centres are uniform over the grid box, widths sigma ~ U[sigma], amplitudes
    ~ U[-1, 1]; f = sum_i a_i exp(-|x - c_i|^2 / (2 sigma_i^2)) + noise * U[0, 1)
    at integer coordinates, non-periodic.  The Gaussian is separable, so the
    sum is formed as a product of per-axis factors.
    """
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    rng = _rng(seed)
    # per-bump centre in (x, y, z) order, then width, then amplitude
    cen = rng.random((n_bumps, dim)) * np.array(shape[::-1], dtype=np.float64)
    sig = rng.uniform(sigma[0], sigma[1], n_bumps)
    amp = rng.uniform(-1.0, 1.0, n_bumps)
    axes = []  # axes[d] : (n_bumps, shape_along_axis) for axis d in (x, y, z) order
    for d in range(dim):
        n = shape[dim - 1 - d]
        x = np.arange(n, dtype=np.float64)
        axes.append(np.exp(-((x[None, :] - cen[:, d:d + 1]) ** 2) / (2.0 * sig[:, None] ** 2)))
    if dim == 1:
        f = amp @ axes[0]
    elif dim == 2:
        f = (axes[1].T * amp[None, :]) @ axes[0]  # [ny, nb] @ [nb, nx]
    else:
        zy = (axes[2].T[:, None, :] * axes[1].T[None, :, :]) * amp[None, None, :]  # [nz, ny, nb]
        f = (zy.reshape(-1, n_bumps) @ axes[0]).reshape(shape)
    f = f.reshape(shape)
    f = f + noise * rng.random(shape)
    return f.astype(np.float32)


def lognormal_grf(shape, seed: int, slope: float = -3.0) -> np.ndarray:
    """exp of a standardised Gaussian random field with power spectrum |k|^slope.

    White noise N(0, 1) -> real FFT -> amplitude |k|^(slope/2) on integer
    wavenumbers (k = 0 removed) -> inverse FFT (periodic) -> mean 0, std 1 ->
    exp -> float32.
    """
    import scipy.fft as sfft

    shape = tuple(int(s) for s in shape)
    rng = _rng(seed)
    g = rng.standard_normal(shape)
    workers = max(1, min(16, os.cpu_count() or 1))
    G = sfft.rfftn(g, workers=workers)
    del g
    k2 = np.zeros(G.shape, dtype=np.float64)
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            k = np.fft.rfftfreq(n) * n
        else:
            k = np.fft.fftfreq(n) * n
        sh = [1] * len(shape)
        sh[ax] = k.size
        k2 = k2 + (k.reshape(sh) ** 2)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)  # |k|^(slope/2)
    del k2
    G *= amp
    del amp
    g = sfft.irfftn(G, s=shape, workers=workers)
    del G
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return np.exp(g).astype(np.float32)


def lognormal_grf_device(shape, seed: int, device, slope: float = -3.0):
    """The lognormal_grf recipe computed on a device with torch (float32 FFTs),
    for fields too large for a host FFT (e.g. 1300^3, 2.2 G vertices).

    Seeded with torch's generator on that device, so its values differ from
    lognormal_grf's for the same seed; returns a float32 torch tensor."""
    import torch

    shape = tuple(int(s) for s in shape)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    x = torch.randn(shape, generator=g, device=device, dtype=torch.float32)
    X = torch.fft.rfftn(x)
    del x
    k2 = None
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            k = torch.fft.rfftfreq(n, device=device) * n
        else:
            k = torch.fft.fftfreq(n, device=device) * n
        sh = [1] * len(shape)
        sh[ax] = k.numel()
        t = (k * k).reshape(sh)
        k2 = t if k2 is None else k2 + t
    amp = torch.where(k2 > 0, k2.clamp_min(1e-30) ** (slope / 4.0), torch.zeros_like(k2))
    del k2
    X *= amp
    del amp
    y = torch.fft.irfftn(X, s=shape)
    del X
    y -= y.mean(dtype=torch.float64).float()
    sd = y.std().float()
    if float(sd) > 0:
        y /= sd
    return torch.exp_(y)


# Adversarial structure ------------------------------------------------------
#
# Fields built to stress the parts of the build that the smooth workloads
# barely touch: deep chains across many tiles, the largest possible number of
# minima, large exact-tie plateaus next to noise (the sudden jump in sublevel
# volume and the suspected quadratic worst case the paper discusses for the
# Richtmyer-Meshkov data, Sec. 4), and nested plateaus.

def serpentine(shape, seed: int, descending: bool = False) -> np.ndarray:
    """One monotone path that snakes through the whole grid; every other
    vertex is higher than the whole path.

    3-D: the path runs along x in every row (y, z) with y and z even,
    alternating direction, steps to the next row through the vertex between
    them at the row's end, and to the next even z layer through the vertex
    above the layer's last row end.  Path vertex k (k-th along the path) gets
    value k (or its reverse with ``descending``); the rest get N + U[0, N),
    rounded to float32.  2-D uses the rows y even; 1-D is the whole line.
    """
    shape = tuple(int(s) for s in shape)
    rng = _rng(seed)
    n = int(np.prod(shape))
    f = (n + rng.random(n) * n).reshape(shape)
    if len(shape) == 1:
        order = np.arange(shape[0])
        coords = [order]
    else:
        nz = shape[0] if len(shape) == 3 else 1
        ny, nx = shape[-2], shape[-1]
        pts = []  # (z, y, x) along the path
        flip = False
        yrows = list(range(0, ny, 2))
        for zi, z in enumerate(range(0, nz, 2)):
            rows = yrows if zi % 2 == 0 else yrows[::-1]
            for ri, y in enumerate(rows):
                xs = range(nx - 1, -1, -1) if flip else range(nx)
                pts.extend((z, y, x) for x in xs)
                x_end = 0 if flip else nx - 1
                flip = not flip
                if ri + 1 < len(rows):  # through the vertex between this row and the next
                    ym = (y + rows[ri + 1]) // 2
                    pts.append((z, ym, x_end))
            if z + 2 < nz:  # up through the vertex above the layer's last point
                zl, yl, xl = pts[-1]
                pts.append((z + 1, yl, xl))
        p = np.array(pts)
        coords = [p[:, 0], p[:, 1], p[:, 2]] if len(shape) == 3 else [p[:, 1], p[:, 2]]
    k = np.arange(len(coords[0]), dtype=np.float64)
    if descending:
        k = k[::-1].copy()
    f[tuple(coords)] = k
    return f.astype(np.float32)


def tilted_checkerboard(shape, seed: int, tilt: float = 1e-3) -> np.ndarray:
    """Parity checkerboard (every even vertex a minimum: the most minima a grid
    graph can have) on a linear ramp along the linear id, plus a little noise,
    so that minima are ordered and elder-rule chains are long."""
    shape = tuple(int(s) for s in shape)
    idx = np.indices(shape)
    par = (idx.sum(axis=0) % 2).astype(np.float64)
    n = int(np.prod(shape))
    ramp = np.arange(n, dtype=np.float64).reshape(shape) / n
    noise = _rng(seed).random(shape) * tilt * 0.01
    return (par + tilt * ramp + noise).astype(np.float32)


def plateau_jump(shape, seed: int, noise: float = 0.0) -> np.ndarray:
    """Half of the domain (z below the middle) on one exact plateau at 0.5, the
    other half i.i.d. uniform [0, 1) on a coarse grid of 2^-12 steps (many
    ties), so that at level 0.5 the sublevel set jumps by half the volume.
    ``noise`` > 0 adds that much uniform noise to the plateau (values then
    almost, but not exactly, equal)."""
    shape = tuple(int(s) for s in shape)
    rng = _rng(seed)
    f = np.floor(rng.random(shape) * 4096.0) / 4096.0
    half = shape[0] // 2
    pl = np.full((half,) + shape[1:], 0.5)
    if noise > 0:
        pl = pl + noise * rng.random(pl.shape)
    f[:half] = pl
    return f.astype(np.float32)


def nested_plateaus(shape, seed: int, width: int = 6) -> np.ndarray:
    """Concentric shells of exact ties: floor(r / width) with r the distance
    to an off-centre point, with every other shell negated, plus blocks of
    random small integers in one octant (plateaus of several levels side by
    side)."""
    shape = tuple(int(s) for s in shape)
    rng = _rng(seed)
    idx = np.indices(shape).astype(np.float64)
    c = [s * 0.37 for s in shape]
    r = np.sqrt(sum((idx[i] - c[i]) ** 2 for i in range(len(shape))))
    shell = np.floor(r / width)
    f = np.where(shell % 2 == 0, shell, -shell)
    blk = max(2, width)
    coarse = rng.integers(0, 4, tuple((s + blk - 1) // blk for s in shape)).astype(np.float64)
    for ax in range(len(shape)):
        coarse = np.repeat(coarse, blk, axis=ax)
    coarse = coarse[tuple(slice(0, s) for s in shape)]
    octant = tuple(slice(0, s // 2) for s in shape)
    f[octant] = coarse[octant]
    return f.astype(np.float32)


def parity_lattice(shape) -> np.ndarray:
    """(x mod 2) + (y mod 2) + (z mod 2): the all-even vertices are the minima
    (one vertex in eight), every value is one of four, and each minimum's basin
    touches many others, so the in-tile table of basin pairs fills up."""
    shape = tuple(int(s) for s in shape)
    idx = np.indices(shape)
    return sum(i % 2 for i in idx).astype(np.float32)


def batch_shapes(seed: int = 4, n3: int = 32, n2: int = 16, r3=(32, 192), r2=(256, 2048)):
    """Uneven batch: n3 cubes with side log-uniform in r3, n2 squares log-uniform in r2."""
    rng = _rng(seed)
    s3 = np.rint(np.exp(rng.uniform(math.log(r3[0]), math.log(r3[1]), n3))).astype(int)
    s2 = np.rint(np.exp(rng.uniform(math.log(r2[0]), math.log(r2[1]), n2))).astype(int)
    return [(int(L), int(L), int(L)) for L in s3] + [(int(L), int(L)) for L in s2]


# Named workloads -------------------------------------------------------------

def workload(name: str, scale: float = 1.0):
    """Fields of a named workload; ``scale`` shrinks sides for quick tests.

    - ``uniform64``: 64^3 i.i.d. uniform, seed 1
    - ``bumps256``: 256^3 64 bumps sigma in [4, 16] + 1 % noise, seed 2
    - ``grf512``: 512^3 log-normal k^-3 field, seed 3
    - ``batch48``: 32 cubes (side 32..192) + 16 squares (side 256..2048) of
      log-normal fields, field i seeded 4000 + i
    - ``diff16x128``: 16 bump fields at 128^3, field i seeded 5000 + i
    """
    def sc(n):
        return max(2, int(round(n * scale)))

    if name == "uniform64":
        return [uniform((sc(64),) * 3, 1)]
    if name == "bumps256":
        return [bumps((sc(256),) * 3, 2)]
    if name == "grf512":
        return [lognormal_grf((sc(512),) * 3, 3)]
    if name == "batch48":
        out = []
        for i, shp in enumerate(batch_shapes(4)):
            out.append(lognormal_grf(tuple(sc(s) for s in shp), 4000 + i))
        return out
    if name == "diff16x128":
        return [bumps((sc(128),) * 3, 5000 + i) for i in range(16)]
    raise KeyError(name)


def generic_fd_field(shape, seed: int) -> np.ndarray:
    """Small bump field for finite-difference checks: 8 bumps, sigma in [1, 4], 1 % noise.

    Returned as float32; callers widen it to float64 for the FD base point.
    """
    return bumps(shape, seed, n_bumps=8, sigma=(1.0, 4.0), noise=0.01)
