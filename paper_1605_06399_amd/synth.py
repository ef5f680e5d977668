"""Seeded synthetic inputs shared by the kernels' callers and the CPU oracle.

This module draws random numbers and shapes them into images, filter taps and
batch descriptions.  It holds no stencil arithmetic: no convolution, gradient,
response or suppression is computed here, so the GPU path and the oracle share
nothing but the input bits.

Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) in counter form,
``v_i = mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)``, which yields exactly the
sequential generator's outputs and vectorises in numpy.

Streams are keyed by ``seed(config, purpose) = config * 2**32 + purpose`` with
purposes PIXELS=0, TAPS=1, RECTS=2, SIZES=3, TARGET=4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

PIXELS, TAPS, RECTS, SIZES, TARGET = 0, 1, 2, 3, 4


def seed(config: int, purpose: int) -> int:
    return ((config << 32) + purpose) & MASK64


def splitmix64(s: int, n: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+n-1 of the SplitMix64 stream started at state ``s``."""
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(s & MASK64) + i * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform01(s: int, n: int, offset: int = 0) -> np.ndarray:
    """U[0,1) with 24 random bits, exactly representable in float32."""
    v = splitmix64(s, n, offset)
    return ((v >> np.uint64(40)).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def uniform_large(s: int, n: int, lo: float = 0.0, hi: float = 1.0, chunk: int = 1 << 24) -> np.ndarray:
    """Same values as lo + (hi - lo) * uniform01(s, n), generated in chunks to bound host memory."""
    out = np.empty(n, dtype=np.float32)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        u = uniform01(s, b - a, offset=a)
        out[a:b] = u if (lo, hi) == (0.0, 1.0) else (lo + (hi - lo) * u.astype(np.float64)).astype(np.float32)
    return out


def normal(s: int, n: int, std: float = 1.0) -> np.ndarray:
    """N(0, std^2) by Box-Muller in float64 (one normal per pair of draws), rounded to float32."""
    v = splitmix64(s, 2 * n)
    a = v[0::2] >> np.uint64(11)
    b = v[1::2] >> np.uint64(11)
    u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -53          # (0, 1]
    u2 = b.astype(np.float64) * 2.0 ** -53                  # [0, 1)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    return (z * std).astype(np.float32)


def randint(s: int, n: int, lo: int, hi: int, offset: int = 0) -> np.ndarray:
    """Integers uniform on [lo, hi] (inclusive) from the top 32 bits (modulo bias < 2^-20)."""
    v = splitmix64(s, n, offset) >> np.uint64(32)
    return (lo + (v % np.uint64(hi - lo + 1)).astype(np.int64)).astype(np.int64)


# ----------------------------------------------------------------------------- images

def image_uniform(config: int, height: int, width: int, purpose: int = PIXELS) -> np.ndarray:
    """H x W float32 image, pixels U[0,1), row-major with x fastest."""
    return uniform01(seed(config, purpose), height * width).reshape(height, width)


def image_with_rectangles(config: int, height: int, width: int, count: int = 64) -> np.ndarray:
    """U[0,1) noise plus 1.0 inside the union of ``count`` seeded axis-aligned rectangles.

    Per rectangle: x0 = floor(u*W), y0 = floor(u*H), side lengths 16 + floor(u*497)
    (16..512), clipped to the image.
    """
    img = image_uniform(config, height, width).astype(np.float32)
    u = uniform01(seed(config, RECTS), 4 * count).astype(np.float64).reshape(count, 4)
    inside = np.zeros((height, width), dtype=bool)
    for k in range(count):
        x0 = int(u[k, 0] * width)
        y0 = int(u[k, 1] * height)
        w = 16 + int(u[k, 2] * 497)
        h = 16 + int(u[k, 3] * 497)
        inside[y0:min(y0 + h, height), x0:min(x0 + w, width)] = True
    img[inside] += np.float32(1.0)
    return img


def integer_image(config: int, height: int, width: int, hi: int = 255) -> np.ndarray:
    """Integer-valued float32 image on {0..hi}: every partial sum of small integer taps is exact."""
    return randint(seed(config, PIXELS), height * width, 0, hi).reshape(height, width).astype(np.float32)


def volume_uniform(config: int, depth: int, height: int, width: int) -> np.ndarray:
    """D x H x W float32 volume, voxels U[0,1), slices of row-major rows."""
    return uniform01(seed(config, PIXELS), depth * height * width).reshape(depth, height, width)


def u8_image(config: int, height: int, width: int) -> np.ndarray:
    """unsigned char image, bytes uniform on 0..255."""
    return randint(seed(config, PIXELS), height * width, 0, 255).reshape(height, width).astype(np.uint8)


# ----------------------------------------------------------------------------- taps

def gaussian_taps(radius: int, sigma: float) -> np.ndarray:
    """Sampled Gaussian exp(-i^2 / (2 sigma^2)), i = -r..r, normalised to sum 1 in float64, stored float32.
    Radius 0 is the single tap 1."""
    if radius == 0:
        return np.ones(1, dtype=np.float32)
    i = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-(i * i) / (2.0 * sigma * sigma))
    return (g / g.sum()).astype(np.float32)


def normal_taps_normalised(config: int, count: int, stream: int = 0) -> np.ndarray:
    """``count`` taps drawn N(0,1) and divided by their sum.

    A draw whose sum has magnitude below 0.1 is redrawn from the next stream so
    that the division does not blow the taps up.
    """
    k = 0
    while True:
        z = normal(seed(config, TAPS) + 1000 * stream + k, count).astype(np.float64)
        s = z.sum()
        if abs(s) >= 0.1:
            return (z / s).astype(np.float32)
        k += 1


# ----------------------------------------------------------------------------- storage rounding

def to_f16_bits(a: np.ndarray) -> np.ndarray:
    """IEEE binary16 storage bits of a float32 array (round to nearest even)."""
    return np.ascontiguousarray(a, dtype=np.float32).astype(np.float16).view(np.uint16)


def to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """bfloat16 storage bits of a (finite) float32 array, round to nearest even."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    return ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)).astype(np.uint16)


# ----------------------------------------------------------------------------- workloads

@dataclass
class BatchItem:
    width: int
    height: int
    radius: int
    taps: np.ndarray          # float32, 2r+1, used for both passes
    image: np.ndarray         # float32 H x W draw (before storage rounding)


def batch_uneven(config: int = 4, count: int = 256, side_lo: int = 64, side_hi: int = 2048,
                 r_lo: int = 1, r_hi: int = 7, draw_pixels: bool = True) -> list[BatchItem]:
    """Uneven batch: W and H independently uniform on {side_lo..side_hi}, radius uniform on
    {r_lo..r_hi}; each image gets a normalised Gaussian of sigma = r/2 for both passes."""
    s = seed(config, SIZES)
    ws = randint(s, count, side_lo, side_hi, 0)
    hs = randint(s, count, side_lo, side_hi, count)
    rs = randint(s, count, r_lo, r_hi, 2 * count)
    items = []
    off = 0
    for k in range(count):
        w, h, r = int(ws[k]), int(hs[k]), int(rs[k])
        img = (uniform01(seed(config, PIXELS), w * h, off).reshape(h, w) if draw_pixels
               else np.zeros((0, 0), np.float32))
        off += w * h
        items.append(BatchItem(w, h, r, gaussian_taps(r, r / 2.0), img))
    return items


def bank_inputs(config: int = 5, n: int = 32, f: int = 16, h: int = 1024, w: int = 1024,
                radius: int = 4, tap_std: float = 0.1):
    """Filter-bank workload: x [n,1,h,w] U[0,1), filters [f,2r+1,2r+1] N(0, std^2), target [n,f,h,w] U[0,1)."""
    x = uniform_large(seed(config, PIXELS), n * h * w).reshape(n, 1, h, w)
    k = 2 * radius + 1
    wt = normal(seed(config, TAPS), f * k * k, std=tap_std).reshape(f, k, k)
    t = uniform_large(seed(config, TARGET), n * f * h * w).reshape(n, f, h, w)
    return x, wt, t


# ----------------------------------------------------------------------------- named workloads

SWEEP_RADII = (1, 2, 3, 5, 7)


def sweep_image(side: int = 4096) -> np.ndarray:
    """Convolution sweep image: side x side float32, U[0,1)."""
    return image_uniform(2, side, side)


def sweep_taps_sep(r: int):
    """Row and column taps of the sweep's separable filter of radius r: N(0,1) normalised to sum 1."""
    return (normal_taps_normalised(2, 2 * r + 1, stream=10 * r),
            normal_taps_normalised(2, 2 * r + 1, stream=10 * r + 1))


def sweep_taps_2d(r: int) -> np.ndarray:
    n = 2 * r + 1
    return normal_taps_normalised(2, n * n, stream=10 * r + 2).reshape(n, n)


def u8_taps(config: int, radius: int, shift: int) -> np.ndarray:
    """Signed 16-bit fixed-point taps with `shift` fraction bits: a sampled Gaussian
    (sigma = r/2, or 1 for r <= 2) scaled by 2^shift and rounded, plus seeded integer
    noise of up to 2^(shift-4) per tap, so the filter is non-separable and has negative
    taps while its sum stays near 2^shift."""
    n = 2 * radius + 1
    g = gaussian_taps(radius, max(1.0, radius / 2.0)).astype(np.float64) if radius else np.ones(1)
    base = np.rint(np.outer(g, g) * (1 << shift)).astype(np.int64)
    amp = max(1, 1 << max(shift - 4, 0))
    noise = randint(seed(config, TAPS), n * n, -amp, amp).reshape(n, n)
    return np.clip(base + noise, -32768, 32767).astype(np.int16)


U8_SHIFT = 12


def paper_u8_image(side: int = 8192) -> np.ndarray:
    """Non-separable convolution workload of Section 6: side x side unsigned char."""
    return u8_image(6, side, side)


def corner_image(side: int = 8192) -> np.ndarray:
    """Harris workload: side x side U[0,1) noise plus 64 seeded bright rectangles."""
    return image_with_rectangles(3, side, side, 64)


def corner_window() -> np.ndarray:
    """5x5 Gaussian window (sigma 1), as its 5 separable taps."""
    return gaussian_taps(2, 1.0)
