"""Seeded synthetic inputs: gridded fields with gaps.

This module holds no arithmetic of the gap-filling method; it only draws the test and benchmark inputs, and it is
the one module that the library's tests and the CPU oracle's tests share.

The paper evaluates on three gridded data sets (Walker lake L = 256, Kaibab plateau L = 2048, Wasatch front
L = 8192; Sec. 3.1, Table 1) with M = 100 masks of uniformly random removal at p = 0.1 .. 0.9 (Sec. 3.2).  Those
data are not available here; the generators below stand in for them:

* ``grf``: a stationary Gaussian random field with exponential covariance exp(-r / xi), drawn by circulant
  embedding on a torus (negative eigenvalues clipped to zero), white noise from PCG64, cropped and standardised;
* ``ns_field``: a non-stationary field: a k x k grid of regions with log-uniform correlation lengths, one GRF per
  region blended by products of edge sigmoids, plus a linear trend and 5 % Gaussian noise;
* ``uniform_mask`` / ``blob_mask``: removal of an exact number of pixels, uniformly or as elliptical cloud-like
  blobs topped up uniformly.
Masks use 1 = observed (sample), 0 = removed (gap).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2212013170
ROLE_FIELD, ROLE_MASK, ROLE_PHILOX, ROLE_HOLDOUT = 0, 1, 2, 3


def seed_for(config: int, role: int) -> int:
    return SEED_BASE + 100 * config + role


def _torus_grf(M0: int, M1: int, xi: float, rng: np.random.Generator) -> np.ndarray:
    """Stationary GRF with covariance exp(-r/xi) on an M0 x M1 torus (circulant embedding)."""
    d0 = np.minimum(np.arange(M0), M0 - np.arange(M0)).astype(np.float64)
    d1 = np.minimum(np.arange(M1), M1 - np.arange(M1)).astype(np.float64)
    r = np.sqrt(d0[:, None] ** 2 + d1[None, :] ** 2)
    cov = np.exp(-r / xi)
    lam = np.fft.rfft2(cov).real
    lam = np.clip(lam, 0.0, None)
    noise = rng.standard_normal((M0, M1))
    f = np.fft.irfft2(np.sqrt(lam) * np.fft.rfft2(noise), s=(M0, M1))
    return f


def grf_aniso(H: int, W: int, xi_x: float, xi_y: float, rng: np.random.Generator) -> np.ndarray:
    """Standardised stationary GRF with geometric anisotropy: covariance exp(-sqrt((dx/xi_x)^2 + (dy/xi_y)^2)),
    circulant embedding on a 2H x 2W torus (negative eigenvalues clipped)."""
    M0, M1 = 2 * H, 2 * W
    d0 = np.minimum(np.arange(M0), M0 - np.arange(M0)).astype(np.float64) / xi_y
    d1 = np.minimum(np.arange(M1), M1 - np.arange(M1)).astype(np.float64) / xi_x
    cov = np.exp(-np.sqrt(d0[:, None] ** 2 + d1[None, :] ** 2))
    lam = np.clip(np.fft.rfft2(cov).real, 0.0, None)
    f = np.fft.irfft2(np.sqrt(lam) * np.fft.rfft2(rng.standard_normal((M0, M1))), s=(M0, M1))[:H, :W]
    return (f - f.mean()) / max(f.std(), 1e-300)


def grf(H: int, W: int, xi: float, rng: np.random.Generator) -> np.ndarray:
    """Standardised stationary GRF on H x W, embedded in a 2H x 2W torus."""
    f = _torus_grf(2 * H, 2 * W, xi, rng)[:H, :W]
    return (f - f.mean()) / max(f.std(), 1e-300)


def _sigmoid(u):
    return 0.5 * (1.0 + np.tanh(0.5 * u))


def ns_field(H: int, W: int, k: int, xi_range, rng: np.random.Generator, noise: float = 0.05) -> np.ndarray:
    """Non-stationary blend of k x k regional GRFs (see module docstring).

    Region r spans [y0, y1) x [x0, x1); its weight is the product of four sigmoids of width side/16 centred on the
    region's edges.  Each regional GRF is drawn on a window that extends the region by half a side on every edge,
    embedded in a torus 4 * xi_max larger than the window.  f = sum_r w_r f_r / sqrt(sum_r w_r^2), then a trend
    alpha (x/W - 1/2) + beta (y/H - 1/2) with alpha, beta ~ U[-1, 1], then noise * N(0, 1).
    """
    lo, hi = float(xi_range[0]), float(xi_range[1])
    ys = np.linspace(0, H, k + 1).round().astype(int)
    xs = np.linspace(0, W, k + 1).round().astype(int)
    num = np.zeros((H, W))
    wsq = np.zeros((H, W))
    pad_t = int(math.ceil(4 * hi))
    for i in range(k):
        for j in range(k):
            y0, y1, x0, x1 = ys[i], ys[i + 1], xs[j], xs[j + 1]
            sh, sw = y1 - y0, x1 - x0
            xi = math.exp(rng.uniform(math.log(lo), math.log(hi)))
            my, mx = max(sh // 2, 1), max(sw // 2, 1)
            wy0, wy1 = max(0, y0 - my), min(H, y1 + my)
            wx0, wx1 = max(0, x0 - mx), min(W, x1 + mx)
            hh, ww = wy1 - wy0, wx1 - wx0
            f = _torus_grf(hh + pad_t, ww + pad_t, xi, rng)[:hh, :ww]
            f = (f - f.mean()) / max(f.std(), 1e-300)
            yy = np.arange(wy0, wy1)[:, None] + 0.5
            xx = np.arange(wx0, wx1)[None, :] + 0.5
            wy_s = max(sh / 16.0, 1e-3)
            wx_s = max(sw / 16.0, 1e-3)
            w = (_sigmoid((yy - y0) / wy_s) * _sigmoid((y1 - yy) / wy_s)
                 * _sigmoid((xx - x0) / wx_s) * _sigmoid((x1 - xx) / wx_s))
            num[wy0:wy1, wx0:wx1] += w * f
            wsq[wy0:wy1, wx0:wx1] += w * w
    out = num / np.sqrt(np.maximum(wsq, 1e-300))
    alpha, beta = rng.uniform(-1.0, 1.0, size=2)
    yy = (np.arange(H)[:, None] + 0.5) / H - 0.5
    xx = (np.arange(W)[None, :] + 0.5) / W - 0.5
    out = out + alpha * xx + beta * yy
    out = out + noise * rng.standard_normal((H, W))
    return out


def uniform_mask(H: int, W: int, n_remove: int, rng: np.random.Generator, base=None) -> np.ndarray:
    """Remove exactly n_remove of the currently observed pixels of `base` (default: all observed)."""
    mask = np.ones((H, W), np.uint8) if base is None else base.copy()
    obs = np.flatnonzero(mask.ravel())
    n_remove = int(min(max(n_remove, 0), obs.size))
    if n_remove:
        pick = rng.choice(obs.size, size=n_remove, replace=False)
        mask.ravel()[obs[pick]] = 0
    return mask


def blob_mask(H: int, W: int, p: float, blob_share: float, rng: np.random.Generator,
              axes=(10.0, 80.0)) -> np.ndarray:
    """Remove round(p H W) pixels: elliptical blobs (semi-axes ~ U[axes], orientation ~ U[0, pi), centre uniform)
    until blob_share of that count is removed, then uniform removal tops up to the total."""
    total = int(round(p * H * W))
    target_blob = int(round(blob_share * total))
    mask = np.ones((H, W), np.uint8)
    removed = 0
    while removed < target_blob:
        a, b = rng.uniform(axes[0], axes[1], size=2)
        th = rng.uniform(0.0, math.pi)
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        R = int(math.ceil(max(a, b))) + 1
        y0, y1 = max(0, int(cy) - R), min(H, int(cy) + R + 1)
        x0, x1 = max(0, int(cx) - R), min(W, int(cx) + R + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        yy = np.arange(y0, y1)[:, None] + 0.5 - cy
        xx = np.arange(x0, x1)[None, :] + 0.5 - cx
        c, s = math.cos(th), math.sin(th)
        u = (xx * c + yy * s) / a
        v = (-xx * s + yy * c) / b
        inside = (u * u + v * v) <= 1.0
        sub = mask[y0:y1, x0:x1]
        newly = inside & (sub == 1)
        k = int(newly.sum())
        if k == 0:
            continue
        if removed + k > total:
            # trim the last blob so that the total is never exceeded
            idx = np.flatnonzero(newly.ravel())[: total - removed]
            flat = sub.ravel().copy()
            flat[idx] = 0
            sub[...] = flat.reshape(sub.shape)
            removed = total
            break
        sub[newly] = 0
        removed += k
    return uniform_mask(H, W, total - removed, rng, base=mask)


@dataclass
class Scene:
    """One gap-filling problem: the true field, the observation mask and the sites that are scored."""
    z_true: np.ndarray            # float32 [H, W]
    mask: np.ndarray              # uint8 [H, W], 1 = observed sample
    eval_mask: np.ndarray         # uint8 [H, W], 1 = scored site (removed pixels, plus any hold-out)
    block: tuple = (32, 32)       # T-block size (lb_h, lb_w)
    meta: dict = field(default_factory=dict)

    @property
    def z_obs(self) -> np.ndarray:
        """The field as the method sees it: removed pixels carry NaN."""
        z = self.z_true.copy()
        z[self.mask == 0] = np.nan
        return z


def config1(scale: int = 1) -> Scene:
    """Plain MPR: 128 x 128 GRF (xi = 8 px), 33 % of pixels removed uniformly, one global temperature."""
    H = W = 128 // scale
    f = grf(H, W, 8.0, np.random.default_rng(seed_for(1, ROLE_FIELD)))
    m = uniform_mask(H, W, int(round(0.33 * H * W)), np.random.default_rng(seed_for(1, ROLE_MASK)))
    return Scene(f.astype(np.float32), m, (1 - m).astype(np.uint8), block=(H, W), meta=dict(config=1))


def config2(H: int = 1024, W: int = 1024) -> Scene:
    """SV-MPR: 1024^2 NS(4, [2, 32]), 50 % missing (half uniform, half blobs), 16 x 16 T-blocks."""
    f = ns_field(H, W, 4, (2.0, 32.0), np.random.default_rng(seed_for(2, ROLE_FIELD)))
    m = blob_mask(H, W, 0.5, 0.5, np.random.default_rng(seed_for(2, ROLE_MASK)))
    return Scene(f.astype(np.float32), m, (1 - m).astype(np.uint8), block=(16, 16), meta=dict(config=2))


def config3(p: float = 0.6, H: int = 4096, W: int = 4096) -> Scene:
    """SV-MPR at scale: 4096^2 NS(8, [2, 64]), gap fraction p, blob-dominated (80 % blobs), 32 x 32 T-blocks."""
    f = ns_field(H, W, 8, (2.0, 64.0), np.random.default_rng(seed_for(3, ROLE_FIELD)))
    m = blob_mask(H, W, p, 0.8, np.random.default_rng([seed_for(3, ROLE_MASK), int(round(p * 1000))]))
    return Scene(f.astype(np.float32), m, (1 - m).astype(np.uint8), block=(32, 32), meta=dict(config=3, p=p))


def _config4_scene(base: int, i: int, side) -> Scene:
    rng = np.random.default_rng([base, i])
    H = int(round(math.exp(rng.uniform(math.log(side[0]), math.log(side[1])))))
    W = int(round(math.exp(rng.uniform(math.log(side[0]), math.log(side[1])))))
    p = float(rng.uniform(0.1, 0.9))
    f = ns_field(H, W, 4, (2.0, 32.0), rng)
    if i % 2 == 0:
        m = uniform_mask(H, W, int(round(p * H * W)), rng)
    else:
        m = blob_mask(H, W, p, 1.0, rng)
    return Scene(f.astype(np.float32), m, (1 - m).astype(np.uint8), block=(16, 16), meta=dict(config=4, index=i, p=p))


def config4_scenes(n: int = 256, side=(64, 2048), base_seed: int | None = None, workers: int = 1):
    """Batched: n scenes, sides log-uniform in [64, 2048] (independently), p ~ U[0.1, 0.9], half uniform and half
    blob removal, NS(4, [2, 32]) fields, 16 x 16 T-blocks.  Scene i depends only on (seed, i), so `workers` > 1
    generates them in parallel processes with identical results."""
    base = seed_for(4, ROLE_FIELD) if base_seed is None else base_seed
    if workers <= 1:
        return [_config4_scene(base, i, side) for i in range(n)]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_config4_scene, [base] * n, range(n), [side] * n))


def config5(H: int = 512, W: int = 512, holdout: float = 0.05) -> Scene:
    """Differentiable SV-MPR: 512^2 NS(4, [2, 32]), 50 % missing, and 5 % of the observed pixels held out: they are
    treated as gaps by the method and scored (eval_mask marks only them)."""
    f = ns_field(H, W, 4, (2.0, 32.0), np.random.default_rng(seed_for(5, ROLE_FIELD)))
    m = blob_mask(H, W, 0.5, 0.5, np.random.default_rng(seed_for(5, ROLE_MASK)))
    obs = np.flatnonzero(m.ravel())
    rng = np.random.default_rng(seed_for(5, ROLE_HOLDOUT))
    k = int(round(holdout * obs.size))
    held = obs[rng.choice(obs.size, size=k, replace=False)]
    ev = np.zeros(H * W, np.uint8)
    ev[held] = 1
    m2 = m.copy().ravel()
    m2[held] = 0
    return Scene(f.astype(np.float32), m2.reshape(H, W), ev.reshape(H, W), block=(32, 32),
                 meta=dict(config=5, n_holdout=k))


def skewed_field(L: int, seed: int, sigma: float = 0.79) -> np.ndarray:
    """Complete L x L field for the validation harness: a lognormal transform exp(sigma g) of a standardised
    non-stationary NS(4, [2, 32]) field g; sigma = 0.79 gives the marginal skewness (e^{s^2} + 2) sqrt(e^{s^2} - 1)
    of about 3.6 that Table 1 lists for the smallest data set."""
    rng = np.random.default_rng(seed)
    g = ns_field(L, L, 4, (2.0, 32.0), rng).astype(np.float64)
    g = (g - g.mean()) / g.std()
    return np.exp(sigma * g).astype(np.float32)


def grf3(D: int, H: int, W: int, xi: float, rng: np.random.Generator) -> np.ndarray:
    """Standardised stationary GRF with covariance exp(-r/xi) on a periodic D x H x W grid (circulant, negative
    eigenvalues clipped): the stand-in field of the 3D lattice."""
    ds = [np.minimum(np.arange(M), M - np.arange(M)).astype(np.float64) for M in (D, H, W)]
    r = np.sqrt(ds[0][:, None, None] ** 2 + ds[1][None, :, None] ** 2 + ds[2][None, None, :] ** 2)
    lam = np.clip(np.fft.rfftn(np.exp(-r / xi)).real, 0.0, None)
    del r
    f = np.fft.irfftn(np.sqrt(lam) * np.fft.rfftn(rng.standard_normal((D, H, W))), s=(D, H, W), axes=(0, 1, 2))
    return ((f - f.mean()) / max(f.std(), 1e-300)).astype(np.float32)


def config3d(L: int = 256, p: float = 0.6):
    """The 3D lattice at the site count of the 4096^2 plane: an L^3 GRF (xi = 8), a fraction p of the sites removed
    uniformly.  Returns (field, mask) as float32 / uint8 [L, L, L]."""
    rng = np.random.default_rng(seed_for(7, ROLE_FIELD))
    f = grf3(L, L, L, 8.0, rng)
    m = (np.random.default_rng(seed_for(7, ROLE_MASK)).random((L, L, L)) >= p).astype(np.uint8)
    return f, m


def random_small(H: int, W: int, p: float, seed: int, xi: float = 4.0) -> Scene:
    """A small GRF scene with uniform removal, for parity tests of ragged shapes."""
    rng = np.random.default_rng(seed)
    f = grf(H, W, xi, rng)
    m = uniform_mask(H, W, int(round(p * H * W)), rng)
    return Scene(f.astype(np.float32), m, (1 - m).astype(np.uint8), block=(8, 8), meta=dict(seed=seed))
