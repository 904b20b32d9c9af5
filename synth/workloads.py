"""Seeded synthetic inputs for the Paillier histogram path.

This module holds input generators only: gradient values, bin indices, tree
node sample sets, random r values below a given modulus, batched job shapes
and request arrival traces.  It holds none of the method's arithmetic (no
encoding, no encryption, no products), so both the GPU path's tests and the
CPU oracle can take their inputs from it.

The paper's datasets (CreditCard, HIGGS, Epsilon; Sec. IV-B) are not used;
these generators produce inputs with the shapes of the workloads the
benchmarks run (sample counts, feature and bin counts, tree depth) and the
value distributions stated with each function.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np


def streams(base_seed: int, k: int = 8) -> List[np.random.Generator]:
    """Independent numpy generators derived from one base seed (the order
    is: key, gradients, bins, r, splits, jobs, arrivals, spare)."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(base_seed).spawn(k)]


def gradients(n_samples: int, rng: np.random.Generator) -> np.ndarray:
    """Logistic-loss gradient pairs, float64 [M, 2]: z ~ N(0, 1),
    p = sigmoid(z), y ~ Bernoulli(0.5), g = p - y, h = p (1 - p)."""
    z = rng.standard_normal(n_samples)
    p = 1.0 / (1.0 + np.exp(-z))
    y = (rng.random(n_samples) < 0.5).astype(np.float64)
    out = np.empty((n_samples, 2), dtype=np.float64)
    out[:, 0] = p - y
    out[:, 1] = p * (1.0 - p)
    return out


def bins_uniform(n_features: int, n_samples: int, n_bins: int,
                 rng: np.random.Generator) -> np.ndarray:
    """uint8 [J, M], each bin index uniform on [0, n_bins)."""
    assert 1 <= n_bins <= 256
    return rng.integers(0, n_bins, size=(n_features, n_samples), dtype=np.uint8)


def zipf_probs(n_bins: int, s: float = 1.1) -> np.ndarray:
    """P(rank k) proportional to k^-s for k = 1..n_bins (truncated Zipf)."""
    w = np.arange(1, n_bins + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def bins_zipf(n_features: int, n_samples: int, n_bins: int, rng: np.random.Generator,
              s: float = 1.1) -> np.ndarray:
    """uint8 [J, M]: per feature, a truncated Zipf(s) over ranks, with the
    rank -> bin assignment a seeded permutation of the bins, so that each
    feature has its own hot bins."""
    assert 1 <= n_bins <= 256
    probs = zipf_probs(n_bins, s)
    out = np.empty((n_features, n_samples), dtype=np.uint8)
    for f in range(n_features):
        perm = rng.permutation(n_bins).astype(np.uint8)
        ranks = rng.choice(n_bins, size=n_samples, p=probs)
        out[f] = perm[ranks]
    return out


def split_node(samples: np.ndarray, rng: np.random.Generator,
               lo: float = 0.2, hi: float = 0.8):
    """Seeded split of a node's sorted sample list: fraction f ~ U(lo, hi);
    left = the first round(f |S|) of a seeded permutation, right = the rest,
    both returned sorted (uint32)."""
    frac = rng.uniform(lo, hi)
    perm = rng.permutation(samples)
    k = int(round(frac * len(samples)))
    return np.sort(perm[:k]).astype(np.uint32), np.sort(perm[k:]).astype(np.uint32)


def tree_levels(n_samples: int, depth: int, rng: np.random.Generator) -> List[List[np.ndarray]]:
    """Node sample sets level by level: level 0 is the root with all samples;
    each node of level d splits into two children of level d + 1.  Returns
    ``depth`` levels (2^depth - 1 nodes in all)."""
    levels = [[np.arange(n_samples, dtype=np.uint32)]]
    for _ in range(1, depth):
        nxt = []
        for node in levels[-1]:
            a, b = split_node(node, rng)
            nxt += [a, b]
        levels.append(nxt)
    return levels


def random_units(n: int, count: int, rng: np.random.Generator) -> List[int]:
    """``count`` integers drawn uniformly from [1, n) with gcd(r, n) = 1
    (explicit r values for encryption); each is 64 bits wider than n before
    the reduction, so the draw is within 2^-64 of uniform."""
    nbytes = (n.bit_length() + 64 + 7) // 8
    out: List[int] = []
    while len(out) < count:
        x = int.from_bytes(rng.bytes(nbytes), "little") % n
        if x and math.gcd(x, n) == 1:
            out.append(x)
    return out


def bins_tables(n_rows: int, n_features: int, bin_choices: Sequence[int], rng: np.random.Generator,
                s: float = 1.1):
    """One Zipf(s) bin table per bin count: {B: uint8 [n_features, n_rows]}."""
    return {int(b): bins_zipf(n_features, n_rows, int(b), rng, s) for b in bin_choices}


def batched_jobs(n_jobs: int, rng: np.random.Generator, pool_rows: int,
                 min_samples: int = 1_000, max_samples: int = 200_000,
                 min_features: int = 8, max_features: int = 128,
                 bin_choices: Sequence[int] = (16, 64, 256)) -> List[dict]:
    """Shapes of uneven tree-node histogram jobs over a pool of ``pool_rows``
    encrypted samples: |S| log-uniform in [min_samples, max_samples] (capped
    at the pool), F uniform on {min_features..max_features}, B uniform over
    ``bin_choices``, a seeded sorted subset of the pool as the node's samples,
    and a seeded window [f0, f0 + F) of the rows of the Zipf table for B (see
    ``bins_tables``, built with max_features rows) as the job's features."""
    jobs = []
    for _ in range(n_jobs):
        m = int(round(math.exp(rng.uniform(math.log(min_samples), math.log(max_samples)))))
        m = min(m, pool_rows)
        f = int(rng.integers(min_features, max_features + 1))
        b = int(rng.choice(np.asarray(bin_choices)))
        idx = np.sort(rng.choice(pool_rows, size=m, replace=False)).astype(np.uint32)
        f0 = int(rng.integers(0, max_features - f + 1))
        jobs.append(dict(sample_idx=idx, n_features=f, n_bins=b, f0=f0))
    return jobs


def poisson_arrivals(n_requests: int, rate_per_s: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (s) of a Poisson process: exponential gaps, mean 1/rate."""
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_requests))
