"""Degenerate inputs across the GPU library: zero-length calls return
success and touch nothing, a single-bin histogram holds the product of
every sample, 256 bins (the maximum) and a one-sample node are exact,
counts that leave a ragged tail in every kernel's grid are exact, and
explicit randomness at the ends of its range or off the unit group gives the
formula's ciphertext."""
import functools
import sys

import numpy as np
import pytest

import oracle.paillier as P
from synth import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def he():
    import torch
    assert torch.cuda.is_available()
    from paper_2504_03909_amd import he as H
    return H


@functools.lru_cache(maxsize=None)
def keys(bits, seed):
    from paper_2504_03909_amd import he as H
    p, q = P.keygen(bits, seed)
    return P.PrivateKey(p, q), H.Key.from_primes(bits, p, q)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_zero_length_calls(he):
    """count = 0 everywhere: success, and the output buffers keep their bytes."""
    import torch
    from paper_2504_03909_amd import ckks
    say("zero-length calls")
    _, k = keys(1024, 1)
    L2 = 2 * k.limbs
    sentinel = torch.full((4, L2), 7, dtype=torch.int32, device="cuda")
    empty_m = torch.empty(0, dtype=torch.int64, device="cuda")
    empty_ct = torch.empty((0, L2), dtype=torch.int32, device="cuda")
    he.encrypt(k, empty_m, seed=1, out=sentinel[:0])
    he.encrypt(k, empty_m, seed=1, public=True, out=sentinel[:0])
    dm, _, ovf = he.decrypt(k, empty_ct)
    assert dm.numel() == 0 and int(host(ovf)[0]) == 0
    he.hist_subtract(k, empty_ct, empty_ct)
    he.ct_mul(k, empty_ct, empty_ct)
    packed, slots = he.pack(k, empty_ct, 3)
    assert packed.shape[0] == 0
    res = he.split_find(torch.empty((0, 3, 4, 2), dtype=torch.int64, device="cuda"))
    assert res["gain"].numel() == 0
    ct8 = he.encrypt(k, torch.arange(16, dtype=torch.int64, device="cuda"), seed=2).view(8, 2, L2)
    (h,) = he.hist_aggregate(k, ct8, [he.Job(torch.empty(0, dtype=torch.int32, device="cuda"),
                                             torch.zeros((2, 8), dtype=torch.uint8, device="cuda"), 5)])
    assert he.limbs_to_ints(host(h)) == [1] * (2 * 5 * 2)   # empty node: every bin is the ciphertext 1
    ctx = ckks.Context(12, 40, 1)
    z = ctx.encode(torch.empty((0, 8), dtype=torch.float64, device="cuda"))
    assert z.shape[0] == 0
    torch.cuda.synchronize()
    assert bool((sentinel == 7).all())


@pytest.mark.parametrize("n_bins", [1, 256])
def test_extreme_bin_counts(he, n_bins):
    """B = 1: every sample lands in the one bin; B = 256: the maximum.
    Decrypted sums exact, sampled slots bit-exact in closed form."""
    import torch
    say(f"bins={n_bins}")
    sk, k = keys(1024, 1)
    pk = sk.public
    M, J, r_seed = 1501, 3, 31
    s = W.streams(40 + n_bins)
    g = W.gradients(M, s[1])
    bins = (np.zeros((J, M), dtype=np.uint8) if n_bins == 1 else W.bins_uniform(J, M, n_bins, s[2]))
    m = np.array([[P.encode(float(x)) for x in row] for row in g], dtype=np.int64)
    ct = he.encrypt(k, dev(m.reshape(-1)), seed=r_seed).view(M, 2, -1)
    (hist,) = he.hist_aggregate(k, ct, [he.Job(torch.arange(M, dtype=torch.int32, device="cuda"), dev(bins),
                                               n_bins)])
    dm = host(he.decrypt(k, hist)[0])
    for f in range(J):
        for t in range(2):
            want = np.zeros(n_bins, dtype=np.int64)
            np.add.at(want, bins[f].astype(np.int64), m[:, t])
            assert np.array_equal(dm[f, :, t], want)
    h = host(hist)
    f, b, t = 1, int(bins[1][0]), 0
    members = np.nonzero(bins[f] == b)[0]
    rp = 1
    for i in members:
        rp = rp * P.seeded_r(pk.n, 1024, r_seed, 2 * int(i) + t) % pk.n
    assert he.limbs_to_ints(h[f, b, t][None])[0] == P.encrypt(pk, int(m[members, t].sum()), rp)


def test_single_sample_node_is_its_ciphertext(he):
    import torch
    say("one-sample node")
    _, k = keys(2048, 2)
    M = 40
    s = W.streams(50)
    g = W.gradients(M, s[1])
    bins = W.bins_uniform(4, M, 16, s[2])
    ct = he.encrypt(k, he.encode(dev(g.reshape(-1))), seed=3).view(M, 2, -1)
    i = 17
    (hist,) = he.hist_aggregate(k, ct, [he.Job(torch.tensor([i], dtype=torch.int32, device="cuda"), dev(bins), 16)])
    h, c = host(hist), host(ct)
    for f in range(4):
        for b in range(16):
            for t in range(2):
                want = c[i, t] if b == bins[f][i] else None
                got = he.limbs_to_ints(h[f, b, t][None])[0]
                assert got == (he.limbs_to_ints(want[None])[0] if want is not None else 1)


@pytest.mark.parametrize("count", [1, 15, 16, 17, 63, 65, 4097])
def test_ragged_counts_encrypt_decrypt(he, count):
    """Counts around the group and block sizes of every exponentiation kernel
    (4-, 8- and 16-lane groups are picked by size): E then D is the identity
    and the ciphertexts match the oracle on sampled indices."""
    say(f"ragged count={count}")
    sk, k = keys(1024, 1)
    pk = sk.public
    rng = np.random.default_rng(count)
    m = rng.integers(-(1 << 62), 1 << 62, size=count, dtype=np.int64)
    ct = he.encrypt(k, dev(m), seed=count)
    back = host(he.decrypt(k, ct)[0])
    assert np.array_equal(back, m)
    got = he.limbs_to_ints(host(ct))
    for i in sorted({0, count // 2, count - 1}):
        assert got[i] == P.encrypt(pk, int(m[i]), P.seeded_r(pk.n, 1024, count, i))


@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
@pytest.mark.parametrize("public", [False, True])
def test_encrypt_degenerate_r(he, bits, seed, public):
    """Explicit r at the ends of its range and off the unit group: 1, 2,
    n - 1, n + 1 and 2^(32 L) - 1 (only r mod n matters), and r = p, q, 2p,
    n - p (0 mod p or mod q: the exponentiation bases are 0, the ciphertext
    is not a unit).  Both the CRT and the public-key path give the formula's
    value (1 + m n) r^n mod n^2, bit for bit."""
    sk, k = keys(bits, seed)
    n, p, q = sk.public.n, sk.p, sk.q
    rs = [1, 2, n - 1, n + 1, (1 << (32 * k.limbs)) - 1, p, q, 2 * p, n - p]
    ms = [0, 5, -3, 1 << 40, -(1 << 62), 7, -7, 0, 123456789]
    say(f"degenerate r {bits} public={public}")
    ct = he.encrypt(k, dev(np.array(ms, dtype=np.int64)), r=dev(he.ints_to_limbs(rs, k.limbs)), public=public)
    got = he.limbs_to_ints(host(ct))
    want = [P.encrypt(sk.public, m, r) for m, r in zip(ms, rs)]
    assert got == want


@pytest.mark.parametrize("form", [0, 1])
def test_out_of_range_rows_and_bins_are_skipped_and_counted(he, form):
    """Device data the library cannot trust: node rows at or past the resident
    row count and bin values at or past n_bins.  Such (sample, feature) pairs
    join no bin and are counted into the job's n_bad; every other bin equals
    the oracle's aggregation of the valid pairs, bit for bit."""
    import torch
    say(f"out-of-range rows and bins form={form}")
    sk, k = keys(1024, 1)
    pk = sk.public
    R, J, B, r_seed = 300, 3, 12, 77
    s = W.streams(61)
    g = W.gradients(R, s[1])
    m = np.array([[P.encode(float(x)) for x in row] for row in g], dtype=np.int64)
    bins = W.bins_uniform(J, R, B, s[2])
    rng = np.random.default_rng(61)
    bins[0, rng.choice(R, 20, replace=False)] = B          # first value past the range
    bins[1, rng.choice(R, 9, replace=False)] = 255         # the largest byte
    # rows: every resident row but four, and in their place rows past the end
    # (R, R + 1, a large value, the largest uint32); the node keeps n_samples
    # <= rows, which the host checks
    bad_rows = np.array([R, R + 1, 1 << 30, (1 << 32) - 1], dtype=np.uint64)
    dropped = rng.choice(R, len(bad_rows), replace=False)
    kept = np.setdiff1d(np.arange(R, dtype=np.uint64), dropped.astype(np.uint64))
    idx = np.concatenate([kept, bad_rows])
    rng.shuffle(idx)
    idx32 = idx.astype(np.uint32).view(np.int32)
    ct = he.encrypt(k, dev(m.reshape(-1)), seed=r_seed).view(R, 2, -1)
    ctin = he.to_mont(k, ct) if form == 1 else ct
    n_bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    job = he.Job(dev(idx32), dev(bins), B, n_bad=n_bad)
    (hist,) = he.hist_aggregate(k, ctin, [job], form=form, chunk=16)
    got = he.limbs_to_ints(host(hist))
    keep = np.zeros(R, dtype=bool)
    keep[kept.astype(np.int64)] = True
    want_bad = J * len(bad_rows) + int(np.sum(keep & (bins[0] >= B))) + int(np.sum(keep & (bins[1] >= B)))
    assert int(host(n_bad)[0]) == want_bad
    cts = he.limbs_to_ints(host(ct))
    rows_ct = [[cts[2 * i], cts[2 * i + 1]] for i in range(R)]
    for f in range(J):
        # the oracle's histogram of feature f over the pairs the library keeps
        valid = [int(i) for i in kept if bins[f][i] < B]
        want = P.aggregate(pk, rows_ct, valid, bins[f:f + 1], 1, B)
        assert [got[(f * B + b) * 2 + t] for b in range(B) for t in range(2)] == \
            [want[0][b][t] for b in range(B) for t in range(2)], f
    # and the decrypted histogram equals the plaintext sums of the valid pairs
    dm = host(he.decrypt(k, hist)[0])
    for f in range(J):
        ok = (bins[f] < B) & keep
        for t in range(2):
            ref = np.zeros(B, dtype=np.int64)
            np.add.at(ref, bins[f][ok].astype(np.int64), m[ok, t])
            assert np.array_equal(dm[f, :, t], ref)
