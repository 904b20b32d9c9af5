"""Process-pool drivers for the oracle -- test infrastructure only.

The arithmetic is exactly ``oracle.paillier``'s; this module only spreads
independent calls (one encryption, one decryption, one feature's histogram)
over worker processes so that tests and the CPU baseline finish in seconds.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor
from typing import List, Optional, Sequence, Tuple

from . import paillier as P


def _enc(args: Tuple[int, int, int]) -> int:
    n, m, r = args
    return P.encrypt(P.PublicKey(n), m, r)


def _dec(args: Tuple[int, int, int]) -> int:
    p, q, c = args
    return P.decrypt(P.PrivateKey(p, q), c)


def _hist_feature(args):
    n, ct, idx, bins_f, n_bins = args
    return P.aggregate(P.PublicKey(n), ct, idx, [bins_f], 1, n_bins)[0]


class _Cycled:
    """Row i of a ciphertext table of R rows is row i mod R (a long sample
    list over a few distinct ciphertexts, for timing)."""

    def __init__(self, rows):
        self.rows = rows

    def __getitem__(self, i):
        return self.rows[i % len(self.rows)]


def _hist_feature_cycled(args):
    n, rows, n_samples, bins_f, n_bins = args
    return P.aggregate(P.PublicKey(n), _Cycled(rows), range(n_samples), [bins_f], 1, n_bins)[0]


# At most 16 worker processes: the host CPU share that goes with one GPU on
# the machines this runs on (os.cpu_count() there counts the whole host).
MAX_WORKERS = 16


def workers(requested: Optional[int] = None) -> int:
    if requested:
        return requested
    return max(1, min(MAX_WORKERS, os.cpu_count() or 1))


def encrypt_many(pk: P.PublicKey, ms: Sequence[int], rs: Sequence[int],
                 processes: Optional[int] = None) -> List[int]:
    jobs = [(pk.n, int(m), int(r)) for m, r in zip(ms, rs)]
    if len(jobs) < 8:
        return [_enc(j) for j in jobs]
    with ProcessPoolExecutor(workers(processes)) as ex:
        return list(ex.map(_enc, jobs, chunksize=max(1, len(jobs) // (4 * workers(processes)))))


def decrypt_many(sk: P.PrivateKey, cs: Sequence[int], processes: Optional[int] = None) -> List[int]:
    jobs = [(sk.p, sk.q, int(c)) for c in cs]
    if len(jobs) < 8:
        return [_dec(j) for j in jobs]
    with ProcessPoolExecutor(workers(processes)) as ex:
        return list(ex.map(_dec, jobs, chunksize=max(1, len(jobs) // (4 * workers(processes)))))


def aggregate_many(pk: P.PublicKey, ct, sample_idx, bins, n_features: int, n_bins: int,
                   processes: Optional[int] = None):
    """Same result as ``paillier.aggregate``, one feature per task."""
    idx = [int(i) for i in sample_idx]
    sub = {i: ct[i] for i in idx}
    jobs = [(pk.n, sub, idx, {i: int(bins[f][i]) for i in idx}, n_bins) for f in range(n_features)]
    with ProcessPoolExecutor(workers(processes)) as ex:
        return list(ex.map(_hist_feature, jobs))


def aggregate_features_cycled(pk: P.PublicKey, rows, n_samples: int, bins_rows, n_bins: int,
                              processes: Optional[int] = None):
    """``paillier.aggregate`` of the node of samples 0 .. n_samples-1, one
    feature per task (bins_rows[k] is feature k's bin row), where sample i
    carries the ciphertext pair rows[i mod len(rows)]."""
    jobs = [(pk.n, [list(r) for r in rows], n_samples, bytes(bytearray(b)), n_bins) for b in bins_rows]
    with ProcessPoolExecutor(workers(processes)) as ex:
        return list(ex.map(_hist_feature_cycled, jobs))
