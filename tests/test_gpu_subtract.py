"""GPU parity of encrypted histogram subtraction (parent times the inverse
of a child mod n^2) and of ciphertext products / re-randomisation against the
oracle, and of the sibling tree mode against direct aggregation of every node.  Expected ciphertexts come from the
oracle's ``subtract``; for histograms, from the identity that the parent's
product divided by one child's is the other child's product."""
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


@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
@pytest.mark.parametrize("count,batch", [(1, 0), (6, 1), (37, 4), (300, 0), (300, 64), (1000, 7)])
def test_subtract_bit_exact(he, bits, seed, count, batch):
    say(f"subtract {bits} count={count} batch={batch}")
    sk, k = keys(bits, seed)
    pk = sk.public
    n2 = pk.n2
    rng = np.random.default_rng(count * 31 + batch + bits)
    num = W.random_units(n2, count, rng)
    den = W.random_units(n2, count, rng)
    edge = [(1, 1), (n2 - 1, n2 - 1), (5, n2 - 1), (1, pk.n + 1), (n2 - 2, 2)]
    for i, (x, y) in enumerate(edge[:count]):
        num[i], den[i] = x, y
    out = he.hist_subtract(k, dev(he.ints_to_limbs(num, 2 * k.limbs)), dev(he.ints_to_limbs(den, 2 * k.limbs)),
                           batch=batch)
    assert he.limbs_to_ints(host(out)) == [P.subtract(pk, x, y) for x, y in zip(num, den)]


@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
def test_subtract_non_units_flagged(he, bits, seed):
    """Non-units in the divisor (never ciphertexts) give 0 and are counted;
    every other element of their batch is still exact."""
    import torch
    say(f"subtract non-units {bits}")
    sk, k = keys(bits, seed)
    pk = sk.public
    n2 = pk.n2
    rng = np.random.default_rng(3)
    count = 22
    num = W.random_units(n2, count, rng)
    den = W.random_units(n2, count, rng)
    bad = {2: 0, 9: sk.p * 12345 % n2, 13: pk.n, 19: sk.q * sk.q}
    for i, v in bad.items():
        den[i] = v
    nb = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = he.hist_subtract(k, dev(he.ints_to_limbs(num, 2 * k.limbs)), dev(he.ints_to_limbs(den, 2 * k.limbs)),
                           batch=4, n_bad=nb)
    got = he.limbs_to_ints(host(out))
    for i in range(count):
        assert got[i] == (0 if i in bad else P.subtract(pk, num[i], den[i])), i
    assert int(host(nb)[0]) == len(bad)


def test_subtract_rejects_overlap(he):
    import torch
    _, k = keys(1024, 1)
    a = torch.ones((10, 2 * k.limbs), dtype=torch.int32, device="cuda")
    b = torch.ones_like(a)
    with pytest.raises(he.HEError):
        he.hist_subtract(k, a, b, out=a)
    with pytest.raises(he.HEError):
        he.hist_subtract(k, a, b, out=b)
    he.hist_subtract(k, a, b, out=torch.empty_like(a))  # disjoint: accepted


def test_subtract_batches_agree_at_level_size(he):
    """65,536 elements (a tree level's sibling slots at 2048 bits): the
    automatic batch and explicit batches give identical results, and sampled
    elements match the oracle."""
    import torch
    say("subtract 65536 elements, 2048-bit")
    sk, k = keys(2048, 2)
    pk = sk.public
    n2 = pk.n2
    count = 65536
    rng = np.random.default_rng(17)
    base_num = W.random_units(n2, 256, rng)
    base_den = W.random_units(n2, 256, rng)
    perm = rng.integers(0, 256, size=(2, count))
    num_l = he.ints_to_limbs(base_num, 2 * k.limbs)[perm[0]]
    den_l = he.ints_to_limbs(base_den, 2 * k.limbs)[perm[1]]
    num, den = dev(num_l), dev(den_l)
    auto = he.hist_subtract(k, num, den)
    for batch in (1, 33):
        assert torch.equal(he.hist_subtract(k, num, den, batch=batch), auto), batch
    got = host(auto)
    for i in rng.choice(count, size=200, replace=False):
        want = P.subtract(pk, base_num[perm[0, i]], base_den[perm[1, i]])
        assert he.limbs_to_ints(got[i][None])[0] == want


def test_sibling_tree_equals_direct(he):
    """1024-bit key, 6,000 samples, 8 features x 32 Zipf bins, depth-5 tree:
    sibling mode (batched and captured) equals one direct aggregation per
    node bit for bit, and decrypts to the oracle's sums."""
    import torch
    from paper_2504_03909_amd import pipeline
    say("sibling tree depth 5, 1024-bit")
    bits, M, J, K, r_seed = 1024, 6000, 8, 32, 77
    sk, k = keys(bits, 1)
    s = W.streams(9)
    g = W.gradients(M, s[1])
    bins = W.bins_zipf(J, M, K, s[2])
    levels = W.tree_levels(M, 5, s[4])
    res = pipeline.encrypt_gradients(k, dev(g), r_seed)
    bins_d = dev(bins)
    lv_d = [[dev(n.view(np.int32)) for n in lvl] for lvl in levels]
    direct = pipeline.aggregate_levels(res, lv_d, bins_d, K, mode="per_node")
    for mode in ("sibling", "sibling_graph"):
        sib = pipeline.aggregate_levels(res, lv_d, bins_d, K, mode=mode)
        for la, lb in zip(direct.hists, sib.hists):
            for a, b in zip(la, lb):
                assert torch.equal(a, b), mode
    dec = pipeline.decrypt_levels(k, sib)
    m = np.array([[P.encode(float(x)) for x in row] for row in g], dtype=np.int64)
    for lvl, dl in zip(levels, dec):
        for node, dm in zip(lvl, dl):
            dmh = host(dm)
            idx = node.astype(np.int64)
            for f in range(J):
                want = np.stack([np.bincount(bins[f][idx], weights=m[idx, t].astype(np.float64), minlength=K)
                                 for t in range(2)], axis=-1)
                assert np.array_equal(dmh[f], np.rint(want).astype(np.int64))


@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
@pytest.mark.parametrize("count", [1, 37, 1000])
def test_ct_mul_bit_exact(he, bits, seed, count):
    say(f"ct_mul {bits} count={count}")
    sk, k = keys(bits, seed)
    pk = sk.public
    rng = np.random.default_rng(count + bits + 1)
    a = W.random_units(pk.n2, count, rng)
    b = W.random_units(pk.n2, count, rng)
    a[0], b[0] = 1, pk.n2 - 1
    da, db = dev(he.ints_to_limbs(a, 2 * k.limbs)), dev(he.ints_to_limbs(b, 2 * k.limbs))
    got = he.limbs_to_ints(host(he.ct_mul(k, da, db)))
    assert got == [P.add(pk, x, y) for x, y in zip(a, b)]
    he.ct_mul(k, da, db, out=da)  # in place
    assert he.limbs_to_ints(host(da)) == got


def test_rerandomize_histogram_public_key(he):
    """A passive party (public key only) re-randomises an encrypted histogram:
    every ciphertext changes, equals the oracle's c E(0; r') for the seeded
    r', and decrypts to the same sums."""
    import torch
    say("rerandomize histogram, public key")
    sk, k = keys(1024, 1)
    pk = sk.public
    kpub = he.Key.public(1024, pk.n)
    rng = np.random.default_rng(8)
    count = 300
    ms = [int(x) for x in rng.integers(-(1 << 40), 1 << 40, size=count)]
    rs = W.random_units(pk.n, count, rng)
    cts = [P.encrypt(pk, m, r) for m, r in zip(ms, rs)]
    h = dev(he.ints_to_limbs(cts, 2 * k.limbs)).view(30, 10, -1)
    hr = he.rerandomize(kpub, h, seed=4242, offset=5)
    got = he.limbs_to_ints(host(hr))
    want = [P.rerandomize(pk, c, P.seeded_r(pk.n, 1024, 4242, 5 + i)) for i, c in enumerate(cts)]
    assert got == want and all(g != c for g, c in zip(got, cts))
    dm, _, _ = he.decrypt(k, hr)
    assert host(dm).reshape(-1).tolist() == ms


def test_shard_partials_combine_to_whole(he):
    """The combine step of sample sharding: histograms of two disjoint sample
    shards, multiplied slot by slot, equal the histogram of all samples."""
    import torch
    say("shard partial histograms combine")
    sk, k = keys(2048, 2)
    s = W.streams(21)
    M, J, K = 30000, 16, 64
    g = W.gradients(M, s[1])
    bins = dev(W.bins_zipf(J, M, K, s[2]))
    ct = he.encrypt(k, he.encode(dev(g.reshape(-1))), seed=8).view(M, 2, -1)
    perm = np.random.default_rng(3).permutation(M)
    a = np.sort(perm[: M // 3]).astype(np.int32)
    b = np.sort(perm[M // 3:]).astype(np.int32)
    (ha,) = he.hist_aggregate(k, ct, [he.Job(dev(a), bins, K)])
    (hb,) = he.hist_aggregate(k, ct, [he.Job(dev(b), bins, K)])
    (hall,) = he.hist_aggregate(k, ct, [he.Job(torch.arange(M, dtype=torch.int32, device="cuda"), bins, K)])
    assert torch.equal(he.ct_mul(k, ha, hb), hall)
