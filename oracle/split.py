"""Plain CPU oracle for split finding from decrypted histograms.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and nothing in the product
path), like ``oracle.paillier``; it shares no code with the GPU path.

The paper leaves this step to the active party (Sec. III-B: the decrypted
histograms are used by the active party for tree building) without restating
it, so it is XGBoost's exact greedy split criterion over histogram bins
(Chen & Guestrin, KDD 2016, the split-gain equation of Sec. 2.2): for a
node with gradient sum G and Hessian sum H, splitting the bins of feature f
after bin b sends bins 0..b left (sums G_L, H_L) and the rest right, with

    gain = 1/2 [G_L^2 / (H_L + lambda) + G_R^2 / (H_R + lambda)
                - G^2 / (H + lambda)] - gamma.

Readings (the GPU path computes the same IEEE double operations in the same
order, so gains agree bit for bit):
* sums arrive as int64 fixed point with ``frac_bits`` fractional bits; the
  left/right sums are formed exactly in integers and then converted
  (correctly rounded int -> double) and scaled by 2^-frac_bits (exact);
* a split is admissible iff H_L >= min_child_weight, H_R >= min_child_weight,
  H_L + lambda > 0 and H_R + lambda > 0;
* term(g, h) = (g * g) / (h + lambda), gain = 0.5 * ((term_L + term_R) -
  term_P) - gamma, evaluated in that order;
* the best split of a feature is the admissible bin with the largest gain,
  the lowest bin on ties; the best of a node the largest over features, the
  lowest feature on ties; none -> gain -inf, feature and bin -1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple


@dataclass(frozen=True)
class Split:
    gain: float
    feature: int
    bin: int
    g_left: int
    h_left: int


NO_SPLIT = Split(-math.inf, -1, -1, 0, 0)


def term(g: float, h: float, lam: float) -> float:
    return (g * g) / (h + lam)


def split_gain(gl: int, hl: int, g: int, h: int, frac_bits: int, lam: float, gamma: float,
               min_child_weight: float):
    """Gain of one candidate split from exact fixed-point sums, or None when
    the split is not admissible."""
    s = 2.0 ** -frac_bits
    fgl, fhl = float(gl) * s, float(hl) * s
    fgr, fhr = float(g - gl) * s, float(h - hl) * s
    fg, fh = float(g) * s, float(h) * s
    if not (fhl >= min_child_weight and fhr >= min_child_weight and fhl + lam > 0 and fhr + lam > 0):
        return None
    return 0.5 * ((term(fgl, fhl, lam) + term(fgr, fhr, lam)) - term(fg, fh, lam)) - gamma


def best_split_feature(hist_f: Sequence[Sequence[int]], frac_bits: int, lam: float, gamma: float,
                       min_child_weight: float, feature: int = 0) -> Split:
    """hist_f[b] = (G_b, H_b): scan the bins left to right."""
    g = sum(int(x[0]) for x in hist_f)
    h = sum(int(x[1]) for x in hist_f)
    best = NO_SPLIT
    gl = hl = 0
    for b in range(len(hist_f) - 1):
        gl += int(hist_f[b][0])
        hl += int(hist_f[b][1])
        gain = split_gain(gl, hl, g, h, frac_bits, lam, gamma, min_child_weight)
        if gain is not None and gain > best.gain:
            best = Split(gain, feature, b, gl, hl)
    return best


def best_splits(hist: Sequence[Sequence[Sequence[Sequence[int]]]], frac_bits: int, lam: float,
                gamma: float, min_child_weight: float) -> Tuple[List[List[Split]], List[Split]]:
    """hist[node][f][b] = (G, H) -> (per-feature best [node][f], per-node best [node])."""
    per_feat, per_node = [], []
    for node in hist:
        row = [best_split_feature(hf, frac_bits, lam, gamma, min_child_weight, f) for f, hf in enumerate(node)]
        best = NO_SPLIT
        for s in row:
            if s.gain > best.gain:
                best = s
        per_feat.append(row)
        per_node.append(best)
    return per_feat, per_node
