"""Seeded synthetic grey-scale images in [0, 255].

The paper measures on 8-bit images from a public collection ("Checker",
"Testpat") and on a natural image, none of which are available here. These
generators stand in for their shape and structure: sharp binary edges,
piecewise-constant regions, smooth ramps and additive noise, clipped to the
8-bit range [L, U] = [0, 255] the paper uses (Section II, centring in
Section III-B).

All generators use numpy's PCG64 bit generator and return float64 arrays; the
caller casts. Nothing here knows about the filter.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "ramp_rectangles",
    "edge_rich",
    "checkerboard",
    "batch_specs",
    "diff_batch",
    "ImageSpec",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def ramp_rectangles(height: int = 256, width: int = 256, seed: int = 1,
                    n_rect: int = 12, noise_sigma: float = 10.0) -> np.ndarray:
    """Linear ramp 32..224 along a random direction, `n_rect` axis-aligned
    constant rectangles (sides U{16..96}, intensity U[0,255], painted in
    order), i.i.d. N(0, noise_sigma^2) noise, clipped to [0, 255]."""
    rng = _rng(seed)
    theta = rng.uniform(0.0, 2.0 * np.pi)
    rr, cc = np.meshgrid(np.arange(height, dtype=np.float64),
                         np.arange(width, dtype=np.float64), indexing="ij")
    proj = rr * np.sin(theta) + cc * np.cos(theta)
    lo, hi = proj.min(), proj.max()
    t = (proj - lo) / (hi - lo) if hi > lo else np.zeros_like(proj)
    img = 32.0 + 192.0 * t
    for _ in range(n_rect):
        h = int(rng.integers(16, 97))
        w = int(rng.integers(16, 97))
        r0 = int(rng.integers(0, max(1, height)))
        c0 = int(rng.integers(0, max(1, width)))
        val = rng.uniform(0.0, 255.0)
        img[r0:r0 + h, c0:c0 + w] = val
    img = img + rng.normal(0.0, noise_sigma, size=img.shape)
    return np.clip(img, 0.0, 255.0)


def checkerboard(height: int, width: int, cell: int = 64,
                 lo: float = 0.0, hi: float = 255.0) -> np.ndarray:
    """Binary checkerboard with `cell`-pixel square cells."""
    r = np.arange(height)[:, None] // cell
    c = np.arange(width)[None, :] // cell
    return np.where((r + c) % 2 == 0, lo, hi).astype(np.float64)


def _fill_polygon(img: np.ndarray, vx: np.ndarray, vy: np.ndarray, val: float) -> None:
    """Even-odd fill of a closed polygon, sampled at integer pixel centres
    (x = column, y = row), restricted to the polygon's bounding box."""
    height, width = img.shape
    c0 = max(0, int(np.floor(vx.min())))
    c1 = min(width, int(np.ceil(vx.max())) + 1)
    r0 = max(0, int(np.floor(vy.min())))
    r1 = min(height, int(np.ceil(vy.max())) + 1)
    if c0 >= c1 or r0 >= r1:
        return
    yy = np.arange(r0, r1, dtype=np.float64)[:, None]
    xx = np.arange(c0, c1, dtype=np.float64)[None, :]
    inside = np.zeros((r1 - r0, c1 - c0), dtype=bool)
    n = len(vx)
    for k in range(n):
        xa, ya = vx[k], vy[k]
        xb, yb = vx[(k + 1) % n], vy[(k + 1) % n]
        if ya == yb:
            continue
        crosses = (ya > yy) != (yb > yy)                   # rows the edge spans
        xcross = xa + (yy - ya) * (xb - xa) / (yb - ya)    # per row
        inside ^= crosses & (xx < xcross)
    region = img[r0:r1, c0:c1]
    region[inside] = val


def edge_rich(height: int, width: int, seed: int, n_poly: int | None = None,
              cell: int = 64, noise_sigma: float = 5.0) -> np.ndarray:
    """Edge-rich image: a 0/255 checkerboard with `cell`-pixel cells, then
    `n_poly` star-shaped polygons (3-8 vertices, centre uniform, radius
    U[32,256], intensity U[0,255]) painted in order, then i.i.d.
    N(0, noise_sigma^2) noise, clipped to [0, 255].

    Default polygon count keeps the density of 32 polygons per 1024^2."""
    rng = _rng(seed)
    if n_poly is None:
        n_poly = max(1, int(round(32.0 * height * width / (1024.0 * 1024.0))))
    img = checkerboard(height, width, cell)
    for _ in range(n_poly):
        nv = int(rng.integers(3, 9))
        cy = rng.uniform(0.0, height)
        cx = rng.uniform(0.0, width)
        radius = rng.uniform(32.0, 256.0)
        ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, size=nv))
        rad = radius * rng.uniform(0.4, 1.0, size=nv)
        val = rng.uniform(0.0, 255.0)
        _fill_polygon(img, cx + rad * np.cos(ang), cy + rad * np.sin(ang), val)
    img = img + rng.normal(0.0, noise_sigma, size=img.shape)
    return np.clip(img, 0.0, 255.0)


@dataclasses.dataclass(frozen=True)
class ImageSpec:
    """One image of a batch: shape, seed and filter parameters."""
    height: int
    width: int
    seed: int
    sigma_s: float
    sigma_r: float

    def image(self) -> np.ndarray:
        return edge_rich(self.height, self.width, self.seed)


def batch_specs(count: int = 64, seed0: int = 4000,
                sides=tuple(range(256, 2049, 128)),
                sigma_s_range=(2.0, 16.0), sigma_r_range=(10.0, 60.0)) -> list[ImageSpec]:
    """Uneven batch: long side uniform over `sides`; square, or 2:1 with
    probability 1/2 in a random orientation; sigma_s and sigma_r uniform."""
    out = []
    for k in range(count):
        rng = _rng(seed0 + k)
        side = int(rng.choice(np.asarray(sides)))
        if rng.uniform() < 0.5:
            h, w = side, side
        elif rng.uniform() < 0.5:
            h, w = side, side // 2
        else:
            h, w = side // 2, side
        out.append(ImageSpec(h, w, seed0 + k,
                             float(rng.uniform(*sigma_s_range)),
                             float(rng.uniform(*sigma_r_range))))
    return out


def diff_batch(batch: int = 8, height: int = 1024, width: int = 1024,
               seed0: int = 5000, target_seed0: int = 5100):
    """Images (edge-rich, seeds seed0+b) and targets (i.i.d. U[0,255],
    seeds target_seed0+b) for a differentiation workload."""
    imgs = np.stack([edge_rich(height, width, seed0 + b) for b in range(batch)])
    tgts = np.stack([_rng(target_seed0 + b).uniform(0.0, 255.0, size=(height, width))
                     for b in range(batch)])
    return imgs, tgts
