"""Writes shadow_rates.txt: rates of the downlink model (Sec. II-A) in layouts
where lognormal shadowing is the only thing that tells the links apart, so
that the rate is a closed form of the shadowing draws alone.

Definitions written out here, independently of the oracle (this script imports
nothing from the repository):

* SplitMix64 output for a 64-bit state x (Steele, Lea & Flood, OOPSLA 2014):
  z = x + 0x9E3779B97F4A7C15, then z ^= z >> 30, z *= 0xBF58476D1CE4E5B9,
  z ^= z >> 27, z *= 0x94D049BB133111EB, z ^= z >> 31 (all mod 2^64). The
  repository pins this mixer separately against the published outputs for
  seed 0 (splitmix64_seed0.txt); the function below is re-checked against
  them before anything is written.
* The per-link draw of the generator recipe: state = key XOR (i 2^32 + j);
  h = SplitMix64(state); u1 = (high 32 bits of h + 1/2) 2^-32,
  u2 = (low 32 bits of h + 1/2) 2^-32; X = sqrt(-2 ln u1) cos(2 pi u2)
  (Box & Muller, 1958).
* Path gain with shadowing: G = K0 max(d, d_min)^-alpha 10^(sigma X / 10),
  sigma in dB.

Layouts: devices at the origin, N RRHs at the first N of (100, 0), (-100, 0),
(0, 100), (0, -100) metres (exactly 100 m away in FP32 too, above d_min), no
noise. Every path-loss factor then cancels in
  SINR_j = G_j / sum_{k != j} G_k = 10^(s X_j) / sum_{k != j} 10^(s X_k),
with s = sigma / 10, and R_j = W log2(1 + SINR_j). With two RRHs this is
SINR_0 = 10^(s (X_0 - X_1)): the sigma / 10 factor and the (u1, u2) mapping
decide the value directly, and the file records, for each row, what a
sigma / 20 slip and swapped hash halves would give instead, to show that
either mistake moves the rate far outside the test tolerance.

Usage: python tests/golden/make_shadow_golden.py  (rewrites shadow_rates.txt)
"""

import math
import os

M64 = (1 << 64) - 1
HERE = os.path.dirname(os.path.abspath(__file__))


def splitmix64(x):
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def draw(key, i, j, swap=False):
    h = splitmix64(key ^ (((i << 32) + j) & M64))
    hi, lo = h >> 32, h & 0xFFFFFFFF
    if swap:
        hi, lo = lo, hi
    u1 = (hi + 0.5) * 2.0 ** -32
    u2 = (lo + 0.5) * 2.0 ** -32
    return h, math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def rates(X, s, W):
    p = [10.0 ** (s * x) for x in X]
    out = []
    for j in range(len(X)):
        interf = sum(p[k] for k in range(len(X)) if k != j)
        out.append(W * math.log2(1.0 + p[j] / interf))
    return out


def check_against_published():
    for ln in open(os.path.join(HERE, "splitmix64_seed0.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        _, state, out = ln.split()
        assert splitmix64(int(state, 16)) == int(out, 16)


CASES = [
    # name, key, device index i, number of equidistant RRHs, sigma dB
    ("pair_s8_k1", 0x0123456789ABCDEF, 0, 2, 8.0),
    ("pair_s8_k1_i7", 0x0123456789ABCDEF, 7, 2, 8.0),
    ("pair_s8_k2_i3", 0xD1B54A32D192ED03, 3, 2, 8.0),
    ("pair_s4_k2_i3", 0xD1B54A32D192ED03, 3, 2, 4.0),
    ("triple_s8_k3_i5", 0x9E3779B97F4A7C15, 5, 3, 8.0),
    ("quad_s8_k4_i100000", 0x0000000100000002, 100000, 4, 8.0),
]
W = 20e6


def main():
    check_against_published()
    lines = [
        "# Rates with shadowing as the only difference between links (Sec. II-A downlink model):",
        "# devices at (0, 0), N RRHs at the first N of (100,0) (-100,0) (0,100) (0,-100) m; K0 = 10^-3.8,",
        "# alpha = 3.5, d_min = 10 m, N0 = 0, P = 1 W, W = 20 MHz;",
        "# SINR_j = 10^(s X_j) / sum_{k != j} 10^(s X_k), s = sigma / 10.",
        "# X_j from h = SplitMix64(key ^ (i 2^32 + j)) through u1 = (hi + 1/2) 2^-32, u2 = (lo + 1/2) 2^-32,",
        "# X = sqrt(-2 ln u1) cos(2 pi u2). Written by make_shadow_golden.py from these definitions alone.",
        "# columns: name key i N sigma | per RRH: h X R | then per RRH the rate with sigma/20 and with swapped halves",
    ]
    for name, key, i, n, sigma in CASES:
        s = sigma / 10.0
        hs, X = zip(*[draw(key, i, j) for j in range(n)])
        R = rates(X, s, W)
        R_slip = rates(X, sigma / 20.0, W)
        R_swap = rates([draw(key, i, j, swap=True)[1] for j in range(n)], s, W)
        for r, a, b in zip(R, R_slip, R_swap):
            assert abs(a - r) > 1e-3 * r and abs(b - r) > 1e-3 * r, name
        cols = [name, f"0x{key:016x}", str(i), str(n), repr(sigma)]
        for h, x, r in zip(hs, X, R):
            cols += [f"0x{h:016x}", repr(x), repr(r)]
        cols += [repr(v) for v in R_slip] + [repr(v) for v in R_swap]
        lines.append(" ".join(cols))
    with open(os.path.join(HERE, "shadow_rates.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
