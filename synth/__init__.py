"""Seeded synthetic inputs shaped like the paper's workloads.

The paper fits Kodak (24 images, 768x512) and DIV2K (x2-downscaled, 408-1020 px sides) with
70 000 Gaussians (Sec. 4.1, Table 1).  Neither dataset is available here, so these generators
stand in for them with images and Gaussian sets of the same shapes and sizes.

This module holds no part of the rendering method: it only draws random numbers.  It is the one
module that both the FP64 oracle tests and the GPU path tests import, so that both sides see the
same inputs.  Every array is produced on the CPU as float32 with ``numpy.random.default_rng``.

Gaussian records follow the 8-parameter layout of the merged-colour Gaussian (Sec. 3.2,
Eq. rasterization4): ``(mu_x, mu_y, l1, l2, l3, c0, c1, c2)`` in pixel units, where
``L = [[l1, 0], [l2, l3]]`` is the Cholesky factor of the covariance (Sec. 3.1, Eq. cholesky).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PARAMS_PER_GAUSSIAN = 8


def gaussians(n: int, height: int, width: int, seed: int, l_lo: float = 1.0,
              l_hi: float = 8.0, l2_sd: float = 0.5) -> np.ndarray:
    """Random Gaussian records, float32 ``[n, 8]``.

    Means are uniform over ``[0, W) x [0, H)``; the Cholesky diagonals ``l1, l3`` are
    ``exp(U(log l_lo, log l_hi))`` pixels; the off-diagonal ``l2`` is ``N(0, l2_sd^2)``; the
    weighted colours are ``U[0, 1]^3``.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((n, PARAMS_PER_GAUSSIAN), dtype=np.float32)
    out[:, 0] = rng.uniform(0.0, width, n)
    out[:, 1] = rng.uniform(0.0, height, n)
    out[:, 2] = np.exp(rng.uniform(math.log(l_lo), math.log(l_hi), n))
    out[:, 3] = rng.normal(0.0, l2_sd, n)
    out[:, 4] = np.exp(rng.uniform(math.log(l_lo), math.log(l_hi), n))
    out[:, 5:8] = rng.uniform(0.0, 1.0, (n, 3))
    # uniform(0, W) can round up to W in float32; keep means inside the half-open frame
    np.minimum(out[:, 0], np.nextafter(np.float32(width), np.float32(0)), out=out[:, 0])
    np.minimum(out[:, 1], np.nextafter(np.float32(height), np.float32(0)), out=out[:, 1])
    return out


def gaussians_rs(n: int, height: int, width: int, seed: int, s_lo: float = 1.2,
                 s_hi: float = 6.0, c_lo: float = -0.5, c_hi: float = 1.0) -> np.ndarray:
    """Random rotation-scale records ``(mu_x, mu_y, s1, s2, theta, c0, c1, c2)``, float32
    ``[n, 8]`` (the covariance factorisation of Sec. 3.1, Eq. RSSR).

    Means are uniform over ``[0, W) x [0, H)``; the scales ``s1, s2`` are
    ``exp(U(log s_lo, log s_hi))`` pixels; the angle is ``U(-pi, pi)``; the weighted colours are
    ``U[c_lo, c_hi]^3``.
    """
    rng = np.random.default_rng(seed)
    p = np.empty((n, PARAMS_PER_GAUSSIAN), np.float32)
    p[:, 0] = rng.uniform(0, width, n)
    p[:, 1] = rng.uniform(0, height, n)
    p[:, 2] = np.exp(rng.uniform(math.log(s_lo), math.log(s_hi), n))
    p[:, 3] = np.exp(rng.uniform(math.log(s_lo), math.log(s_hi), n))
    p[:, 4] = rng.uniform(-math.pi, math.pi, n)
    p[:, 5:8] = rng.uniform(c_lo, c_hi, (n, 3))
    np.minimum(p[:, 0], np.nextafter(np.float32(width), np.float32(0)), out=p[:, 0])
    np.minimum(p[:, 1], np.nextafter(np.float32(height), np.float32(0)), out=p[:, 1])
    return p


@dataclasses.dataclass
class CodecSet:
    """A compressed Gaussian set in the layout of Sec. 3.3 (arrays on the CPU)."""
    mu_bits: np.ndarray     # [N, 2] uint16, binary16 bit patterns of the positions
    codes: np.ndarray       # [N, 3] uint8, b-bit covariance codes
    index: np.ndarray       # [N, M] uint8, residual-VQ indices
    codebooks: np.ndarray   # [M, B, 3] float32
    gamma: np.ndarray       # [3] float32 scales
    beta: np.ndarray        # [3] float32 offsets
    bits: int


def codec_set(n: int, height: int, width: int, seed: int, bits: int = 6, stages: int = 2,
              book: int = 8, rotation_scale: bool = False) -> CodecSet:
    """Random compressed set with the paper's codec settings by default (16-bit positions, 6-bit
    covariance codes, 2 RVQ stages of 8 colours; Sec. 4.1).

    Positions are U[0, W) x U[0, H) drawn in float64 and stored as binary16; codes are uniform
    over [0, 2^bits - 1]; scales and offsets map the codes onto l1, l3 in [1, 8] px and l2 in
    [-1.5, 1.5] (or s1, s2 in [1, 8] px and theta in [-pi, pi]); stage 0 colours are U[0, 1]^3,
    later stages N(0, 0.1^2).
    """
    rng = np.random.default_rng(seed)
    mu = np.stack([rng.uniform(0, width, n), rng.uniform(0, height, n)], axis=1)
    mu16 = mu.astype(np.float16)
    # keep the rounded positions inside the frame
    mu16[:, 0] = np.minimum(mu16[:, 0], np.nextafter(np.float16(width), np.float16(0)))
    mu16[:, 1] = np.minimum(mu16[:, 1], np.nextafter(np.float16(height), np.float16(0)))
    top = (1 << bits) - 1
    codes = rng.integers(0, top + 1, (n, 3)).astype(np.uint8)
    index = rng.integers(0, book, (n, stages)).astype(np.uint8)
    books = np.empty((stages, book, 3), np.float32)
    books[0] = rng.uniform(0, 1, (book, 3))
    if stages > 1:
        books[1:] = rng.normal(0, 0.1, (stages - 1, book, 3))
    if rotation_scale:
        lo, hi = np.array([1.0, 1.0, -math.pi]), np.array([8.0, 8.0, math.pi])
    else:
        lo, hi = np.array([1.0, -1.5, 1.0]), np.array([8.0, 1.5, 8.0])
    gamma = ((hi - lo) / top).astype(np.float32)
    beta = lo.astype(np.float32)
    return CodecSet(mu16.view(np.uint16), codes, index, books, gamma, beta, bits)


def target_sinusoids(height: int, width: int, seed: int) -> np.ndarray:
    """Smooth target: per channel, 1/2 plus 1/16 times a sum of 8 random plane sinusoids.

    Frequencies are U(0.5, 4) cycles per image along each axis and phases U[0, 2pi); the result
    lies in [0, 1].  Float32 ``[H, W, 3]``.
    """
    rng = np.random.default_rng(seed)
    y, x = np.meshgrid(np.arange(height, dtype=np.float64), np.arange(width, dtype=np.float64),
                       indexing="ij")
    img = np.empty((height, width, 3), dtype=np.float64)
    for ch in range(3):
        fx = rng.uniform(0.5, 4.0, 8)
        fy = rng.uniform(0.5, 4.0, 8)
        ph = rng.uniform(0.0, 2.0 * math.pi, 8)
        acc = np.zeros((height, width))
        for j in range(8):
            acc += np.sin(2.0 * math.pi * (fx[j] * x / width + fy[j] * y / height) + ph[j])
        img[:, :, ch] = 0.5 + acc / 16.0
    return img.astype(np.float32)


def _value_noise(height: int, width: int, rng: np.random.Generator) -> np.ndarray:
    acc = np.zeros((height, width))
    total = 0.0
    for octave in range(6):
        spacing = 64 >> octave
        amp = 0.5 ** octave
        gh = height // spacing + 2
        gw = width // spacing + 2
        lattice = rng.uniform(0.0, 1.0, (gh, gw))
        ys = np.arange(height) / spacing
        xs = np.arange(width) / spacing
        y0 = np.floor(ys).astype(np.int64)
        x0 = np.floor(xs).astype(np.int64)
        ty = ys - y0
        tx = xs - x0
        ty = ty * ty * (3.0 - 2.0 * ty)
        tx = tx * tx * (3.0 - 2.0 * tx)
        # smoothstep bilinear interpolation, done separably: along x on the lattice rows, then y
        rows = lattice[:, x0] + (lattice[:, x0 + 1] - lattice[:, x0]) * tx[None, :]
        top = rows[y0]
        acc += amp * (top + (rows[y0 + 1] - top) * ty[:, None])
        total += amp
    return acc / total


def target_noise_rects(height: int, width: int, seed: int, n_rects: int = 32) -> np.ndarray:
    """Textured target: 6-octave value noise per channel plus sharp-edged rectangles.

    Lattice spacings 64, 32, ..., 2 px with amplitudes 0.5^octave and smoothstep bilinear
    interpolation, normalised to [0, 1]; then ``n_rects`` opaque axis-aligned rectangles with
    sides U(2%, 25%) of the image side and colours U[0, 1]^3, painted in order; clipped to
    [0, 1].  Float32 ``[H, W, 3]``.
    """
    rng = np.random.default_rng(seed)
    img = np.stack([_value_noise(height, width, rng) for _ in range(3)], axis=-1)
    for _ in range(n_rects):
        rw = max(1, int(round(rng.uniform(0.02, 0.25) * width)))
        rh = max(1, int(round(rng.uniform(0.02, 0.25) * height)))
        x0 = int(rng.integers(0, max(1, width - rw + 1)))
        y0 = int(rng.integers(0, max(1, height - rh + 1)))
        img[y0:y0 + rh, x0:x0 + rw, :] = rng.uniform(0.0, 1.0, 3)
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def upstream_gradient(height: int, width: int, seed: int) -> np.ndarray:
    """A seeded dL/dimage of unit-order signed values, float32 ``[H, W, 3]``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (height, width, 3)).astype(np.float32)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One image of a workload: its size, Gaussian count and the seeds of its inputs."""
    name: str
    height: int
    width: int
    n: int
    param_seed: int
    target_seed: int
    l_lo: float = 1.0
    l_hi: float = 8.0
    smooth_target: bool = False

    def params(self) -> np.ndarray:
        return gaussians(self.n, self.height, self.width, self.param_seed, self.l_lo, self.l_hi)

    def target(self) -> np.ndarray:
        if self.smooth_target:
            return target_sinusoids(self.height, self.width, self.target_seed)
        return target_noise_rects(self.height, self.width, self.target_seed)


def plain_256(n: int = 2000) -> Workload:
    """One 256x256 image with 2 000 Gaussians and a smooth sinusoid target."""
    return Workload("plain-256x256", 256, 256, n, param_seed=0, target_seed=1,
                    smooth_target=True)


def kodak_like(n: int = 70_000) -> Workload:
    """One 768x512 image (Kodak's size) with 10k, 30k or 70k Gaussians."""
    return Workload(f"kodak-768x512-{n // 1000}k", 512, 768, n, param_seed=2000 + n // 1000,
                    target_seed=200)


def div2k_full(n: int = 100_000) -> Workload:
    """One 2040x1356 image (DIV2K full resolution) with 100k or 300k Gaussians, l in 0.5-32 px."""
    return Workload(f"div2k-2040x1356-{n // 1000}k", 1356, 2040, n, param_seed=3000 + n // 1000,
                    target_seed=300, l_lo=0.5, l_hi=32.0)


def batch_small(count: int = 64) -> list[Workload]:
    """64 images with sides U{128..1024} and N_i = clamp(round(HW * 50000 / 1024^2), 1e3, 5e4)."""
    rng = np.random.default_rng(4)
    out = []
    for i in range(count):
        h = int(rng.integers(128, 1025))
        w = int(rng.integers(128, 1025))
        n = int(min(50_000, max(1_000, round(h * w * 50_000 / 1024 ** 2))))
        out.append(Workload(f"batch64-{i}", h, w, n, param_seed=4000 + i, target_seed=400 + i))
    return out


def batch_large(count: int = 256) -> list[Workload]:
    """256 images with sides U{512..2048} and N_i = clamp(round(HW * 2e5 / 2048^2), 2e4, 2e5)."""
    rng = np.random.default_rng(5)
    out = []
    for i in range(count):
        h = int(rng.integers(512, 2049))
        w = int(rng.integers(512, 2049))
        n = int(min(200_000, max(20_000, round(h * w * 200_000 / 2048 ** 2))))
        out.append(Workload(f"batch256-{i}", h, w, n, param_seed=5000 + i, target_seed=500 + i))
    return out


def _target_of(w: "Workload") -> np.ndarray:
    return w.target()


def targets(workloads: list[Workload], processes: int = 0) -> list[np.ndarray]:
    """Targets of many workloads, generated in worker processes (same values as w.target())."""
    if processes <= 1 or len(workloads) < 4:
        return [w.target() for w in workloads]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(processes) as pool:
        return pool.map(_target_of, workloads, chunksize=1)
