"""Seeded synthetic HDR scenes.

A scene is a radiance field f_c(X, Y) on the reference plane, in photo-electrons
per unit exposure, for the three colour channels.  It stands in for the paper's
high-resolution reference scenes, which are not available: piecewise-smooth
regions separated by straight step edges, with per-channel radiance spanning
six decades (log-uniform over [1e-2, 1e4]).

Recipe: K random lines partition the plane; every cell gets a per-channel base
u_c ~ U(-2, 4) (drawn from a counter-based hash of the cell's side pattern, so
cells are consistent at any sampling density); a global gradient adds
a_c (X/W - 1/2) + b_c (Y/H - 1/2) with a_c, b_c ~ U(-1, 1); the log10 radiance
is clipped to [-2, 4].

This module holds the forward image model only; it contains none of the
reconstruction's arithmetic.
"""
from __future__ import annotations

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def _hash_uniform(key: np.ndarray) -> np.ndarray:
    """Uniform [0, 1) doubles from uint64 keys."""
    return (splitmix64(key) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


class EdgeScene:
    """Piecewise log-smooth radiance field with random step edges."""

    def __init__(self, width: float, height: float, seed: int, n_lines: int | None = None,
                 log_lo: float = -2.0, log_hi: float = 4.0):
        self.width = float(width)
        self.height = float(height)
        self.seed = int(seed)
        rng = np.random.default_rng(np.random.SeedSequence([self.seed, 0]))
        k = n_lines if n_lines is not None else 8 * max(1, int(round(width / 256.0)))
        px = rng.uniform(0.0, width, k)
        py = rng.uniform(0.0, height, k)
        theta = rng.uniform(0.0, np.pi, k)
        self.nx = np.cos(theta)
        self.ny = np.sin(theta)
        self.off = self.nx * px + self.ny * py
        self.grad_a = rng.uniform(-1.0, 1.0, 3)
        self.grad_b = rng.uniform(-1.0, 1.0, 3)
        self.log_lo = log_lo
        self.log_hi = log_hi
        self.salt = np.uint64(rng.integers(0, 2**63, dtype=np.int64))

    def _cell_key(self, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
        key = np.full(X.shape, self.salt, np.uint64)
        with np.errstate(over="ignore"):
            for i in range(self.nx.size):
                side = (self.nx[i] * X + self.ny[i] * Y > self.off[i]).astype(np.uint64)
                key = splitmix64(key ^ (side + np.uint64(2 * i)))
        return key

    def log_radiance(self, X: np.ndarray, Y: np.ndarray, channel) -> np.ndarray:
        """log10 radiance of channel(s) at reference positions (X, Y).

        ``channel`` is an int or an integer array broadcastable to X."""
        X = np.asarray(X, np.float64)
        Y = np.asarray(Y, np.float64)
        ch = np.broadcast_to(np.asarray(channel, np.int64), X.shape)
        key = self._cell_key(X, Y)
        with np.errstate(over="ignore"):
            base = -2.0 + 6.0 * _hash_uniform(key ^ (ch.astype(np.uint64) * np.uint64(0x632BE59BD9B4E019)))
        val = (base + self.grad_a[ch] * (X / self.width - 0.5)
               + self.grad_b[ch] * (Y / self.height - 0.5))
        return np.clip(val, self.log_lo, self.log_hi)

    def radiance(self, X, Y, channel) -> np.ndarray:
        return np.power(10.0, self.log_radiance(X, Y, channel))


class PolynomialScene:
    """Radiance given by a polynomial of degree <= 2 per channel:
    f_c = c0 + c1 X + c2 Y + c3 X^2 + c4 X Y + c5 Y^2 (noise-free test fields)."""

    def __init__(self, coeffs):
        self.coeffs = np.asarray(coeffs, np.float64).reshape(3, 6)

    def radiance(self, X, Y, channel) -> np.ndarray:
        X = np.asarray(X, np.float64)
        Y = np.asarray(Y, np.float64)
        c = self.coeffs[np.broadcast_to(np.asarray(channel, np.int64), X.shape)]
        return (c[..., 0] + c[..., 1] * X + c[..., 2] * Y + c[..., 3] * X * X
                + c[..., 4] * X * Y + c[..., 5] * Y * Y)


class StepScene:
    """Axis-aligned step edge: radiance lo for X < x_edge, hi otherwise (all channels)."""

    def __init__(self, x_edge: float, lo: float, hi: float):
        self.x_edge, self.lo, self.hi = float(x_edge), float(lo), float(hi)

    def radiance(self, X, Y, channel) -> np.ndarray:
        X = np.asarray(X, np.float64)
        return np.where(X < self.x_edge, self.lo, self.hi) + 0.0 * np.asarray(Y, np.float64)
