"""Seeded synthetic segmentation inputs.

The paper's test images (noisy grid, cartoon, stripes, RGB fish; Section 4,
Figs. 5-9) are not available, so every workload here is generated from a
seed.  Each generator returns only the *inputs* of the segmentation model of
Section 3 (an image f, a codebook c, and the model parameters Lambda, gamma,
iteration count, number of scales J).  Nothing in this module computes any
part of the method itself (no data term, no transform, no projection): both
the FP64 oracle and the GPU path consume these inputs independently.

All randomness comes from numpy's PCG64 with ``seed = 1000 * config + index``.

Workload classes (standing in for the paper's image classes):

* C0  128x128 gray, 3 piecewise-constant regions bounded by two random
      ellipses, intensities {0.2, 0.5, 0.8}, Gaussian noise sigma 0.1
      (cartoon-like, cf. Fig. 6).  J=2, lambda=0.1, 200 iterations.
* C1  512x512 gray, 4 regions bounded by nested smooth star-shaped contours,
      each filled with its mean plus an oriented sinusoid (period 6-16 px),
      noise sigma 0.05 (curved textures, cf. Fig. 7).  J=3, lambda=0.05,
      500 iterations.
* C2  1024x1024 RGB, 5 labels, curved Voronoi partition (20 seeds), random
      codebook colours in [0,1]^3, noise sigma 0.08 (cf. Figs. 8-9).  J=4,
      300 iterations, the paper's noisy-fish weights (Fig. 9f).
* C3  batch of 64 gray images, sizes 32*{3..24}, 2..6 labels, alternating
      the C0 and C1 generators, J=3, 200 iterations.
* C4  2048x2048 gray, 8 labels with codebook linspace(0,1,8), curved Voronoi
      (32 seeds), regions flat or textured with probability 1/2, noise
      sigma 0.05.  J=4, 300 iterations.

Unless a workload says otherwise gamma = 1 and Lambda = (0, lambda, ..., lambda):
the paper leaves the low-pass unpenalised in every experiment (Figs. 6, 7, 9).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    """Inputs of one segmentation problem (Section 3 model)."""

    name: str
    img: np.ndarray          # [C][N][N] float64 (C = 1 gray or 3 RGB)
    codebook: np.ndarray     # [q][C] float64
    J: int                   # number of shearlet scales
    lam: np.ndarray          # Lambda = (lambda_0, lambda_1..lambda_J), length J+1
    gamma: float             # ADMM penalty
    iters: int               # fixed iteration count
    truth: np.ndarray | None = None   # [N][N] int32 generating label map (for reporting only)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.img.shape[-1])

    @property
    def q(self) -> int:
        return int(self.codebook.shape[0])

    @property
    def channels(self) -> int:
        return int(self.img.shape[0])


def _rng(config: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * config + index))


def _grid(n: int):
    y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    return y, x


def _ellipse_mask(n, rng):
    y, x = _grid(n)
    cy, cx = rng.uniform(0.25 * n, 0.75 * n, size=2)
    ay, ax = rng.uniform(0.1 * n, 0.3 * n, size=2)
    th = rng.uniform(0.0, np.pi)
    dy, dx = y - cy, x - cx
    r1 = (dx * np.cos(th) + dy * np.sin(th)) / ax
    r2 = (-dx * np.sin(th) + dy * np.cos(th)) / ay
    return r1 * r1 + r2 * r2 <= 1.0


def ellipse_labels(n: int, q: int, rng: np.random.Generator) -> np.ndarray:
    """Background label 0, then q-1 random ellipses painted in order with labels 1..q-1."""
    lab = np.zeros((n, n), dtype=np.int32)
    for k in range(1, q):
        lab[_ellipse_mask(n, rng)] = k
    return lab


def star_labels(n: int, q: int, rng: np.random.Generator) -> np.ndarray:
    """q nested regions bounded by smooth star-shaped closed curves
    r(theta) = r0 (1 + sum_{m=2..4} a_m cos(m theta + phi_m)) around a common centre."""
    y, x = _grid(n)
    cy, cx = rng.uniform(0.4 * n, 0.6 * n, size=2)
    r = np.hypot(y - cy, x - cx)
    th = np.arctan2(y - cy, x - cx)
    lab = np.zeros((n, n), dtype=np.int32)
    radii = np.sort(rng.uniform(0.12 * n, 0.45 * n, size=q - 1))[::-1]
    for k, r0 in enumerate(radii, start=1):
        a = rng.uniform(0.03, 0.12, size=3)
        ph = rng.uniform(0.0, 2 * np.pi, size=3)
        rb = r0 * (1.0 + sum(a[i] * np.cos((i + 2) * th + ph[i]) for i in range(3)))
        lab[r <= rb] = k
    return lab


def curved_voronoi_labels(n: int, q: int, seeds: int, rng: np.random.Generator) -> np.ndarray:
    """Voronoi partition with `seeds` sites whose boundaries are curved by a smooth
    displacement field (8 low-frequency sinusoids, amplitude 0.03 n) applied before the
    nearest-site test.  Every label 0..q-1 owns at least one site."""
    y, x = _grid(n)
    sy = rng.uniform(0, n, size=seeds)
    sx = rng.uniform(0, n, size=seeds)
    lab_of_seed = np.concatenate([np.arange(q), rng.integers(0, q, size=seeds - q)])
    rng.shuffle(lab_of_seed)
    dy = np.zeros_like(y)
    dx = np.zeros_like(x)
    amp = 0.03 * n
    for _ in range(8):
        ky, kx = rng.uniform(-3, 3, size=2) * 2 * np.pi / n
        ph1, ph2 = rng.uniform(0, 2 * np.pi, size=2)
        dy += (amp / 8) * np.sin(ky * y + kx * x + ph1) * 2
        dx += (amp / 8) * np.sin(kx * y - ky * x + ph2) * 2
    py, px = y + dy, x + dx
    best = np.full((n, n), np.inf)
    lab = np.zeros((n, n), dtype=np.int32)
    for i in range(seeds):
        d = (py - sy[i]) ** 2 + (px - sx[i]) ** 2
        m = d < best
        best[m] = d[m]
        lab[m] = lab_of_seed[i]
    return lab


def oriented_texture(n: int, lab: np.ndarray, q: int, amp: float, rng: np.random.Generator,
                     textured: np.ndarray | None = None) -> np.ndarray:
    """Per region k: amp * sin(2 pi <x, e_theta> / T + phi), T ~ U[6,16] px, theta ~ U[0, pi)."""
    y, x = _grid(n)
    out = np.zeros((n, n))
    for k in range(q):
        T = rng.uniform(6.0, 16.0)
        th = rng.uniform(0.0, np.pi)
        ph = rng.uniform(0.0, 2 * np.pi)
        if textured is not None and not textured[k]:
            continue
        m = lab == k
        out[m] = amp * np.sin(2 * np.pi * (x[m] * np.cos(th) + y[m] * np.sin(th)) / T + ph)
    return out


def _lam(J: int, lam: float) -> np.ndarray:
    return np.array([0.0] + [lam] * J, dtype=np.float64)


def make_c0(index: int = 0, n: int = 128) -> Workload:
    rng = _rng(0, index)
    q = 3
    levels = np.array([0.2, 0.5, 0.8])
    perm = rng.permutation(q)
    lab = ellipse_labels(n, q, rng)
    img = levels[perm][lab] + rng.normal(0.0, 0.1, size=(n, n))
    return Workload("C0", img[None], levels[:, None].copy(), J=2, lam=_lam(2, 0.1), gamma=1.0,
                    iters=200, truth=perm[lab].astype(np.int32))


def make_c1(index: int = 0, n: int = 512) -> Workload:
    rng = _rng(1, index)
    q = 4
    means = np.array([0.2, 0.4, 0.6, 0.8])
    perm = rng.permutation(q)
    lab = star_labels(n, q, rng)
    img = means[perm][lab] + oriented_texture(n, lab, q, 0.1, rng) + rng.normal(0.0, 0.05, size=(n, n))
    return Workload("C1", img[None], means[:, None].copy(), J=3, lam=_lam(3, 0.05), gamma=1.0,
                    iters=500, truth=perm[lab].astype(np.int32))


def make_c2(index: int = 0, n: int = 1024) -> Workload:
    rng = _rng(2, index)
    q = 5
    cb = rng.uniform(0.0, 1.0, size=(q, 3))
    lab = curved_voronoi_labels(n, q, 20, rng)
    img = np.transpose(cb[lab], (2, 0, 1)) + rng.normal(0.0, 0.08, size=(3, n, n))
    # Weights of the paper's noisy RGB fish run (Fig. 9f): gamma = 4, Lambda = (1/100)(0, .1, .2, .4, 2).
    lam = np.array([0.0, 0.1, 0.2, 0.4, 2.0]) / 100.0
    return Workload("C2", img, cb, J=4, lam=lam, gamma=4.0, iters=300, truth=lab)


def make_c3_image(index: int) -> Workload:
    rng = _rng(3, index)
    n = 32 * int(rng.integers(3, 25))
    q = int(rng.integers(2, 7))
    levels = np.sort(rng.uniform(0.05, 0.95, size=q))
    if index % 2 == 0:
        lab = ellipse_labels(n, q, rng)
        img = levels[lab] + rng.normal(0.0, 0.1, size=(n, n))
    else:
        lab = star_labels(n, q, rng)
        img = levels[lab] + oriented_texture(n, lab, q, 0.1, rng) + rng.normal(0.0, 0.05, size=(n, n))
    lam = np.array([0.0, 0.1, 0.2, 0.4]) / 20.0
    return Workload(f"C3[{index}]", img[None], levels[:, None].copy(), J=3, lam=lam, gamma=1.0,
                    iters=200, truth=lab)


def make_c3(count: int = 64) -> list[Workload]:
    return [make_c3_image(i) for i in range(count)]


def make_c4(index: int = 0, n: int = 2048, q: int = 8) -> Workload:
    """C4; `q` < 8 gives the same image class with q grey levels (a label count the
    oracle can run at 2048^2 in host memory)."""
    rng = _rng(4, index)
    levels = np.linspace(0.0, 1.0, q)
    lab = curved_voronoi_labels(n, q, 32, rng)
    textured = rng.uniform(size=q) < 0.5
    img = levels[lab] + oriented_texture(n, lab, q, 0.1, rng, textured) + rng.normal(0.0, 0.05, size=(n, n))
    lam = np.array([0.0, 0.1, 0.2, 0.4, 0.8]) / 20.0
    return Workload("C4", img[None], levels[:, None].copy(), J=4, lam=lam, gamma=1.0, iters=300, truth=lab)


def make_denoise(count: int = 16, n: int = 1024, sigma: float = 0.1):
    """Denoising inputs: `count` gray cartoon-texture images (curved Voronoi with 24 sites,
    8 grey levels, half of the regions textured as in C1/C4) and their noisy versions with
    N(0, sigma^2) noise.  Returns (clean, noisy), each [count][n][n] float64."""
    clean = np.empty((count, n, n))
    noisy = np.empty((count, n, n))
    for i in range(count):
        rng = _rng(5, i)
        levels = np.linspace(0.0, 1.0, 8)
        lab = curved_voronoi_labels(n, 8, 24, rng)
        textured = rng.uniform(size=8) < 0.5
        clean[i] = levels[lab] + oriented_texture(n, lab, 8, 0.1, rng, textured)
        noisy[i] = clean[i] + rng.normal(0.0, sigma, size=(n, n))
    return clean, noisy


def make_small(n: int, q: int, J: int, channels: int = 1, seed: int = 0, lam: float = 0.1,
               gamma: float = 1.0, iters: int = 20, noise: float = 0.1) -> Workload:
    """Small ellipse workload of any size, for parity tests (seeded by `seed`)."""
    rng = np.random.Generator(np.random.PCG64(900000 + seed))
    lab = ellipse_labels(n, q, rng)
    cb = rng.uniform(0.0, 1.0, size=(q, channels))
    img = np.transpose(cb[lab], (2, 0, 1)) + rng.normal(0.0, noise, size=(channels, n, n))
    return Workload(f"small{n}x{q}J{J}", img, cb, J=J, lam=_lam(J, lam), gamma=gamma, iters=iters, truth=lab)


def random_image(n: int, seed: int, channels: int = 1) -> np.ndarray:
    """Plain N(0,1) test image [C][N][N] (transform tests)."""
    rng = np.random.Generator(np.random.PCG64(700000 + seed))
    return rng.normal(size=(channels, n, n))


def random_data(shape, seed: int) -> np.ndarray:
    """Plain N(0,1) array of any shape (coefficient-domain tests)."""
    rng = np.random.Generator(np.random.PCG64(800000 + seed))
    return rng.normal(size=shape)


CONFIGS = {0: make_c0, 1: make_c1, 2: make_c2, 4: make_c4}


def make_config(i: int, index: int = 0) -> Workload:
    if i == 3:
        return make_c3_image(index)
    return CONFIGS[i](index)
