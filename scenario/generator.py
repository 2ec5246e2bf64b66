"""Synthetic C-RAN scenarios shaped like the paper's association workloads.

The paper never publishes its instances (Sec. IV and V describe them only in
words), so every input here is drawn from a frozen recipe:

* devices uniform in an L x L square, plus optional Gaussian hot spots
  (sigma 150 m) that hold a fixed share of the devices;
* RRHs at the centres of an r x c grid, jittered by up to 25 % of the pitch;
* device traffic lambda_i = exp(N(0, 1)), device marginal a = lambda / sum,
  RRH marginal b_j = 1 / J (the "equal RRH traffic" choice of Sec. IV);
* a 64-bit key that seeds the per-link shadowing hash (the hash itself is
  implemented independently by each consumer from its published definition).

Positions are float32 metres; marginals are float64. Host randomness is numpy
PCG64 seeded with ``1000 * config + instance``. Nothing in this module
computes path loss, rates, costs or any step of the Sinkhorn method.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

# Radio constants of the downlink model of Sec. II-A. The paper leaves them
# open; these values are the frozen reading used by every workload:
# 1 W per RRH, 38 dB loss at 1 m, path-loss exponent 3.5, 10 m minimum
# distance, 8 dB lognormal shadowing, 20 MHz bandwidth, and thermal noise
# kTB = -174 dBm/Hz over 20 MHz.
RADIO = dict(
    tx_power_w=1.0,
    ref_gain=10.0 ** (-3.8),
    pathloss_exp=3.5,
    min_dist_m=10.0,
    shadow_sigma_db=8.0,
    bandwidth_hz=20e6,
    noise_w=10.0 ** ((-174.0 + 10.0 * math.log10(20e6) - 30.0) / 10.0),
)


@dataclass
class Layout:
    """One association instance: who is where and how much traffic they ask."""

    dev_xy: np.ndarray  # (I, 2) float32, metres
    rrh_xy: np.ndarray  # (J, 2) float32, metres
    lam: np.ndarray  # (I,) float64 traffic lambda_i
    a: np.ndarray  # (I,) float64 device marginal, sums to 1
    b: np.ndarray  # (J,) float64 RRH marginal, sums to 1
    shadow_key: int  # uint64 key of the per-link shadowing hash
    side_m: float
    seed: int
    radio: dict = field(default_factory=lambda: dict(RADIO))

    @property
    def I(self) -> int:  # noqa: E743 - paper notation
        return int(self.dev_xy.shape[0])

    @property
    def J(self) -> int:
        return int(self.rrh_xy.shape[0])


# Workload presets (devices, RRHs, square side, hot spots, hot-spot share).
PRESETS = {
    "small_1000x50": dict(I=1000, J=50, side_m=1000.0, hot_spots=0, hot_share=0.0, config=0),
    "cran_20000x400": dict(I=20000, J=400, side_m=5000.0, hot_spots=4, hot_share=0.4, config=1),
    "large_200000x2000": dict(I=200000, J=2000, side_m=15000.0, hot_spots=16, hot_share=0.4, config=2),
}


def grid_shape(J: int) -> tuple[int, int]:
    """Rows x columns of the RRH grid: the largest divisor r of J with
    r <= sqrt(J); if that r is below sqrt(J)/2 (J prime or nearly so) use
    r = floor(sqrt(J)), c = ceil(J / r) and keep the first J cells."""
    if J < 1:
        raise ValueError("J must be >= 1")
    s = math.sqrt(J)
    r = max(d for d in range(1, int(math.isqrt(J)) + 1) if J % d == 0)
    if r < s / 2:
        r = int(math.isqrt(J))
        c = -(-J // r)
    else:
        c = J // r
    return r, c


def _rrh_positions(rng: np.random.Generator, J: int, side: float) -> np.ndarray:
    r, c = grid_shape(J)
    idx = np.arange(J)
    row, col = idx // c, idx % c
    jit = rng.uniform(-0.25, 0.25, size=(J, 2))
    x = (col + 0.5 + jit[:, 0]) * (side / c)
    y = (row + 0.5 + jit[:, 1]) * (side / r)
    return np.stack([x, y], axis=1)


def _device_positions(rng, I, side, hot_spots, hot_share, hot_sigma=150.0):
    n_hot = int(round(hot_share * I)) if hot_spots > 0 else 0
    centres = rng.uniform(0.0, side, size=(hot_spots, 2))
    uni = rng.uniform(0.0, side, size=(I - n_hot, 2))
    parts = [uni]
    for h in range(hot_spots):
        n = n_hot // hot_spots + (1 if h < n_hot % hot_spots else 0)
        pts = rng.normal(centres[h], hot_sigma, size=(n, 2))
        bad = ~((pts >= 0.0) & (pts <= side)).all(axis=1)
        while bad.any():  # resample points that fall outside the square
            pts[bad] = rng.normal(centres[h], hot_sigma, size=(int(bad.sum()), 2))
            bad = ~((pts >= 0.0) & (pts <= side)).all(axis=1)
        parts.append(pts)
    return np.concatenate(parts, axis=0)


def make_layout(I, J, side_m, hot_spots=0, hot_share=0.0, seed=0, radio=None) -> Layout:
    """Draw one instance. Draw order is frozen: shadow key, RRH jitter,
    hot-spot centres, uniform devices, hot-spot devices, lambda."""
    if I < 1 or J < 1:
        raise ValueError("I and J must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    key = int(rng.integers(0, 2**63 - 1, dtype=np.int64)) * 2 + 1
    rrh = _rrh_positions(rng, J, side_m).astype(np.float32)
    dev = _device_positions(rng, I, side_m, hot_spots, hot_share).astype(np.float32)
    lam = np.exp(rng.standard_normal(I))
    a = lam / lam.sum()
    b = np.full(J, 1.0 / J)
    return Layout(dev_xy=np.ascontiguousarray(dev), rrh_xy=np.ascontiguousarray(rrh),
                  lam=lam, a=a, b=b, shadow_key=key & (2**64 - 1), side_m=float(side_m),
                  seed=int(seed), radio=dict(radio or RADIO))


def preset_layout(name: str, instance: int = 0) -> Layout:
    p = PRESETS[name]
    return make_layout(p["I"], p["J"], p["side_m"], p["hot_spots"], p["hot_share"],
                       seed=1000 * p["config"] + instance)


def _log_uniform_int(rng, lo, hi, n):
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi + 1), size=n))).astype(np.int64).clip(lo, hi)


def batch_sizes(n: int, seed: int = 3000, I_range=(500, 20000), J_range=(20, 400)):
    """(I, J) pairs drawn log-uniformly, as for the uneven batched workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Is = _log_uniform_int(rng, I_range[0], I_range[1], n)
    Js = _log_uniform_int(rng, J_range[0], J_range[1], n)
    return [(int(i), int(j)) for i, j in zip(Is, Js)]


def batch_layouts(n: int = 256, seed: int = 3000, side_m: float = 1000.0, sizes=None):
    """Independent uneven instances, each from its own seed (seed + k), with
    the small-workload geometry (uniform devices in a 1 km square)."""
    sizes = sizes if sizes is not None else batch_sizes(n, seed)
    return [make_layout(I, J, side_m, 0, 0.0, seed=seed + k) for k, (I, J) in enumerate(sizes)]


def snapshot_marginals(I: int, B: int, seed: int = 3500) -> np.ndarray:
    """B traffic snapshots over the same devices: lambda resampled per
    snapshot (seed + s) and normalised. Returns (B, I) float64."""
    out = np.empty((B, I))
    for s in range(B):
        rng = np.random.Generator(np.random.PCG64(seed + s))
        lam = np.exp(rng.standard_normal(I))
        out[s] = lam / lam.sum()
    return out


def drift_positions(layout: Layout, steps: int, step_m: float = 5.0, seed: int = 0):
    """Device positions after each of `steps` moves of `step_m` metres in a
    uniform random direction, reflected at the square's walls. Returns a list
    of (I, 2) float32 arrays, the first being the layout's own positions."""
    rng = np.random.Generator(np.random.PCG64(seed))
    side = layout.side_m
    pos = layout.dev_xy.astype(np.float64)
    out = [layout.dev_xy.copy()]
    for _ in range(steps - 1):
        th = rng.uniform(0.0, 2.0 * math.pi, size=layout.I)
        pos = pos + step_m * np.stack([np.cos(th), np.sin(th)], axis=1)
        pos = np.where(pos < 0.0, -pos, pos)
        pos = np.where(pos > side, 2.0 * side - pos, pos)
        out.append(pos.astype(np.float32))
    return out


def poisson_arrivals(rate_hz: float, n: int, seed: int = 4000) -> np.ndarray:
    """Arrival times (s) of a Poisson request stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


def with_positions(layout: Layout, dev_xy: np.ndarray) -> Layout:
    return replace(layout, dev_xy=np.ascontiguousarray(dev_xy, dtype=np.float32))
