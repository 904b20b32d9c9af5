"""GPU parity of the gfx950 Paillier path against the CPU oracle.

Every expected value comes from ``oracle/`` on the same seeded inputs (from
``synth``); the HIP library is called through its C ABI binding.  Ciphertexts
and histograms must match bit for bit, decrypted values exactly.
"""
import functools
import sys

import numpy as np
import pytest

import oracle.paillier as P
from oracle import pool
from synth import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def he():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2504_03909_amd import he as H
    return H


@functools.lru_cache(maxsize=None)
def oracle_key(bits, seed):
    p, q = P.keygen(bits, seed)
    return P.PrivateKey(p, q)


@functools.lru_cache(maxsize=None)
def gpu_key(bits, seed):
    from paper_2504_03909_amd import he as H
    sk = oracle_key(bits, seed)
    return H.Key.from_primes(bits, sk.p, sk.q)


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ------------------------------------------------------------- keys
@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
def test_keygen_matches_oracle(he, bits, seed):
    say(f"keygen {bits} seed={seed}")
    k = he.Key.generate(bits, seed)
    n, p, q = k.export()
    sk = oracle_key(bits, seed)
    assert (p, q) == (sk.p, sk.q) and n == sk.p * sk.q


def test_public_key_refuses_decrypt(he):
    import torch
    sk = oracle_key(1024, 1)
    k = he.Key.public(1024, sk.public.n)
    assert not k.has_private
    ct = torch.zeros((1, 64), dtype=torch.int32, device="cuda")
    with pytest.raises(he.HEError) as e:
        he.decrypt(k, ct)
    assert e.value.code == he.HE_ERR_NOPRIV


# ---------------------------------------------------------- encoding
def test_encode_bit_exact(he):
    say("encode")
    rng = np.random.default_rng(3)
    g = W.gradients(5000, rng).reshape(-1)
    s = 2.0 ** -32
    g = np.concatenate([g, [0.5 * s, 1.5 * s, 2.5 * s, -1.5 * s, -0.5 * s, 1.0, -1.0, 0.0, 2.0 ** 30, -(2.0 ** 30)]])
    m = host(he.encode(dev(g)))
    assert m.tolist() == [P.encode(x) for x in g]


def test_encode_out_of_range_flagged(he):
    import torch
    bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    x = dev(np.array([1.0, 2.0 ** 40, -(2.0 ** 31), float("nan"), 2.0 ** 31 - 2.0 ** -20]))
    m = host(he.encode(x, n_bad=bad))
    lo = np.iinfo(np.int64).min
    assert m.tolist() == [1 << 32, lo, lo, lo, (1 << 63) - (1 << 12)]
    assert int(host(bad)[0]) == 3


# ---------------------------------------------------------- encryption
def plaintexts(n, rng):
    """Encoded gradients plus the edge plaintexts."""
    g = W.gradients(n, rng).reshape(-1)
    ms = [P.encode(x) for x in g]
    edge = [0, 1, -1, (1 << 32) - 1, -((1 << 32) - 1), (1 << 63) - 1, -(1 << 63)]
    return ms[: max(0, 2 * n - len(edge))] + edge


@pytest.mark.parametrize("bits,seed,count", [(1024, 1, 2000), (1024, 1, 37), (2048, 2, 96)])
@pytest.mark.parametrize("path", ["crt", "public"])
def test_encrypt_explicit_r_bit_exact(he, bits, seed, count, path):
    say(f"encrypt explicit r {bits} count={count} path={path}")
    sk = oracle_key(bits, seed)
    pk = sk.public
    rng = np.random.default_rng(count + bits)
    ms = plaintexts(count // 2 + 4, rng)[:count]
    rs = W.random_units(pk.n, len(ms), rng)
    k = gpu_key(bits, seed)
    ct = he.encrypt(k, dev(np.array(ms, dtype=np.int64)), r=dev(he.ints_to_limbs(rs, k.limbs)),
                    public=(path == "public"))
    got = he.limbs_to_ints(host(ct))
    want = pool.encrypt_many(pk, ms, rs)
    assert got == want


@pytest.mark.parametrize("bits,seed,count,offset", [(1024, 1, 2000, 0), (1024, 1, 19, 12345), (2048, 2, 64, 7)])
@pytest.mark.parametrize("path", ["crt", "public"])
def test_encrypt_seeded_r_bit_exact(he, bits, seed, count, offset, path):
    say(f"encrypt seeded r {bits} count={count} path={path}")
    sk = oracle_key(bits, seed)
    pk = sk.public
    rng = np.random.default_rng(count)
    ms = plaintexts(count // 2 + 4, rng)[:count]
    r_seed = 0xC0FFEE + count
    rs = [P.seeded_r(pk.n, bits, r_seed, offset + i) for i in range(count)]
    k = gpu_key(bits, seed)
    ct = he.encrypt(k, dev(np.array(ms, dtype=np.int64)), seed=r_seed, offset=offset,
                    public=(path == "public"))
    assert he.limbs_to_ints(host(ct)) == pool.encrypt_many(pk, ms, rs)


@pytest.mark.parametrize("bits,seed,count,offset", [(1024, 1, 1500, 3), (2048, 2, 77, 0)])
def test_obfuscated_encryption_bit_exact(he, bits, seed, count, offset):
    """Obfuscators r^n mod n^2 (the oracle's encryption of 0 with r), and
    encryption with them, equal the oracle's E(m; r) for the seeded r."""
    say(f"obfuscated encryption {bits} count={count}")
    sk = oracle_key(bits, seed)
    pk = sk.public
    rng = np.random.default_rng(count + 5)
    ms = plaintexts(count // 2 + 4, rng)[:count]
    r_seed = 0xBEEF + count
    rs = [P.seeded_r(pk.n, bits, r_seed, offset + i) for i in range(count)]
    k = gpu_key(bits, seed)
    rho = he.obfuscators(k, count, seed=r_seed, offset=offset)
    pick = rng.choice(count, size=min(count, 64), replace=False)
    got_rho = he.limbs_to_ints(host(rho))
    want_rho = pool.encrypt_many(pk, [0] * len(pick), [rs[i] for i in pick])
    assert [got_rho[i] for i in pick] == want_rho
    ct = he.encrypt_obfuscated(k, dev(np.array(ms, dtype=np.int64)), rho)
    assert he.limbs_to_ints(host(ct)) == pool.encrypt_many(pk, ms, rs)
    # explicit r, and the result written over the obfuscators
    rx = W.random_units(pk.n, 40, rng)
    rho2 = he.obfuscators(k, 40, r=dev(he.ints_to_limbs(rx, k.limbs)))
    m2 = dev(np.array(ms[:40], dtype=np.int64))
    he.encrypt_obfuscated(k, m2, rho2, out=rho2)
    assert he.limbs_to_ints(host(rho2)) == pool.encrypt_many(pk, ms[:40], rx)


def _group_counts(cus):
    """Encryption counts that make the group-width rule of the CRT kernels
    (narrowest group, 2 lanes only for the mod-p kernel, whose launch still
    gives every SIMD two waves: 2 * ceil(count / (64 / G)) >= 8 * CUs) pick
    each width: mod-p kernel 2, 4, 8, 16 and lift / decryption 4, 4, 8, 16."""
    need = 8 * cus
    return [int(32 * need / 2) + 7, int(16 * need / 2) + 5, int(8 * need / 2) + 3, 1000]


def test_exponentiation_group_widths(he):
    """Encryption and decryption at counts that run the radix-2^29
    exponentiations at every group width (2, 4, 8 and 16 lanes): sampled
    ciphertexts bit-exact against the oracle, every decryption exact."""
    import torch
    bits = 2048
    sk = oracle_key(bits, 2)
    pk = sk.public
    k = gpu_key(bits, 2)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    rng = np.random.default_rng(31)
    for count in _group_counts(cus):
        say(f"group widths: {count} encryptions")
        m = rng.integers(-(1 << 62), 1 << 62, size=count, dtype=np.int64)
        ct = he.encrypt(k, dev(m), seed=77)
        dm, _, ovf = he.decrypt(k, ct)
        assert host(dm).tolist() == m.tolist()
        assert int(host(ovf)[0]) == 0
        pick = rng.choice(count, size=6, replace=False)
        got = he.limbs_to_ints(host(ct)[pick])
        want = pool.encrypt_many(pk, [int(m[i]) % pk.n for i in pick],
                                 [P.seeded_r(pk.n, bits, 77, int(i)) for i in pick])
        assert got == want


def test_untuned_default_shapes_exact(he):
    """32,768 encryptions and decryptions at the untuned default shapes --
    at 2048 bits the lift's and decryption's 4,096 units take two rounds at
    three or at two waves per SIMD, so the default runs two -- equal the
    same work at pinned own-occupancy shapes: every decryption equals its
    plaintext and sampled ciphertexts equal the oracle's."""
    import torch
    bits, n = 2048, 32768
    sk = oracle_key(bits, 2)
    pk = sk.public
    k = gpu_key(bits, 2)
    say(f"untuned default shapes, {n} encryptions and decryptions")
    rng = np.random.default_rng(95)
    m = rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    ct = he.encrypt(k, dev(m), seed=13)
    dm, raw, ovf = he.decrypt(k, ct, raw=True)
    assert host(dm).tolist() == m.tolist() and int(host(ovf)[0]) == 0
    pick = [0, 1, n // 3, n - 17, n - 1]
    want = pool.encrypt_many(pk, [int(m[i]) % pk.n for i in pick], [P.seeded_r(pk.n, bits, 13, i) for i in pick])
    assert he.limbs_to_ints(host(ct)[pick]) == want
    for kind, lanes in (("mod_p", 2), ("lift", 4), ("decrypt", 4)):
        he.crt_set_shape(k, kind, n, lanes, 0, 0)
    assert torch.equal(he.encrypt(k, dev(m), seed=13), ct)
    dm2, raw2, _ = he.decrypt(k, ct, raw=True)
    assert torch.equal(dm2, dm) and torch.equal(raw2, raw)


@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
def test_constant_time_exponentiations(he, bits, seed):
    """With the key's constant-time table reads on, CRT encryption (every
    group width) and decryption give the same ciphertexts and plaintexts as
    the default path, and sampled ciphertexts equal the oracle's."""
    import torch
    say(f"constant-time exponentiations {bits}")
    sk = oracle_key(bits, seed)
    pk = sk.public
    ref = gpu_key(bits, seed)
    k = he.Key.from_primes(bits, sk.p, sk.q)
    k.set_constant_time(True)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    counts = _group_counts(cus) if bits == 2048 else [1000, 37]
    rng = np.random.default_rng(bits + 7)
    for count in counts:
        say(f"constant-time {bits}: {count} encryptions")
        m = rng.integers(-(1 << 62), 1 << 62, size=count, dtype=np.int64)
        ct = he.encrypt(k, dev(m), seed=91)
        assert torch.equal(ct, he.encrypt(ref, dev(m), seed=91))
        dm, raw, _ = he.decrypt(k, ct, raw=True)
        dm_ref, raw_ref, _ = he.decrypt(ref, ct, raw=True)
        assert torch.equal(dm, dm_ref) and torch.equal(raw, raw_ref)
        assert host(dm).tolist() == m.tolist()
        pick = rng.choice(count, size=4, replace=False)
        want = pool.encrypt_many(pk, [int(m[i]) % pk.n for i in pick],
                                 [P.seeded_r(pk.n, bits, 91, int(i)) for i in pick])
        assert he.limbs_to_ints(host(ct)[pick]) == want
    k.close()


def test_crt_autotune_keeps_results(he):
    """The exponentiation autotuner picks a built shape for each kind, and
    encryption and decryption at the tuned shapes stay exact: sampled
    ciphertexts equal the oracle's, every decryption equals its plaintext."""
    bits = 2048
    sk = oracle_key(bits, 2)
    pk = sk.public
    k = gpu_key(bits, 2)
    enc_count, dec_count = 5003, 3001
    say(f"crt autotune {enc_count}/{dec_count}")
    tuned = he.crt_autotune(k, enc_count, dec_count)
    for kind, (lanes, waves, tail, ms) in tuned.items():
        assert lanes in (2, 4, 8, 16) and waves in (0, 2, 3) and ms > 0, (kind, lanes, waves, ms)
        assert tail == 0 or (tail in (4, 8, 16) and tail > lanes), (kind, lanes, tail)
    assert tuned["lift"][0] != 2 and tuned["decrypt"][0] != 2
    rng = np.random.default_rng(77)
    m = rng.integers(-(1 << 62), 1 << 62, size=enc_count, dtype=np.int64)
    ct = he.encrypt(k, dev(m), seed=5)
    dm, _, ovf = he.decrypt(k, ct[:dec_count])
    assert host(dm).tolist() == m[:dec_count].tolist() and int(host(ovf)[0]) == 0
    pick = rng.choice(enc_count, size=5, replace=False)
    want = pool.encrypt_many(pk, [int(m[i]) % pk.n for i in pick],
                             [P.seeded_r(pk.n, bits, 5, int(i)) for i in pick])
    assert he.limbs_to_ints(host(ct)[pick]) == want


def test_last_round_launch_exact(he):
    """Encryption and decryption with the last partial round of each
    exponentiation in a launch of its own (pinned shapes with tail lanes)
    stay exact: every decryption equals its plaintext, and sampled
    ciphertexts, across the range and densely in its last few percent
    (where the second launch works), equal the oracle's.  Bad pins are
    refused."""
    bits, n = 2048, 200_000
    sk = oracle_key(bits, 2)
    pk = sk.public
    k = gpu_key(bits, 2)
    say(f"pinned split launches, {n} encryptions and decryptions")
    he.crt_set_shape(k, "mod_p", n, 2, 0, 8)
    he.crt_set_shape(k, "lift", n, 4, 0, 16)
    he.crt_set_shape(k, "decrypt", n, 4, 0, 8)
    rng = np.random.default_rng(91)
    m = rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    ct = he.encrypt(k, dev(m), seed=9)
    dm, _, ovf = he.decrypt(k, ct)
    assert host(dm).tolist() == m.tolist() and int(host(ovf)[0]) == 0
    pick = sorted(set(rng.choice(n, size=40, replace=False).tolist()) | set(range(n - 4000, n, 151))
                  | set(range(n - 24, n)))
    want = pool.encrypt_many(pk, [int(m[i]) % pk.n for i in pick], [P.seeded_r(pk.n, bits, 9, i) for i in pick])
    assert he.limbs_to_ints(host(ct)[pick]) == want
    for bad in (("lift", 2, 0, 0), ("mod_p", 4, 0, 4), ("decrypt", 4, 1, 0), ("mod_p", 3, 0, 0)):
        with pytest.raises(he.HEError):
            he.crt_set_shape(k, bad[0], n, *bad[1:])


def test_public_key_path_pinned_shapes_equal_crt(he):
    """The public-key path (r mod n^2, the exponentiation by n in the
    exponentiation kernel over pairs of ciphertexts, the product with
    1 + m n) at pinned shapes -- 16 lanes, and 8 lanes with the last partial
    round at 16 -- on an odd count equals the CRT path's ciphertexts for the
    same seeded r, which equal the oracle's; a key holding n only takes the
    same path.  Widths that are not built are refused."""
    import torch
    bits, n = 2048, 60_001
    sk = oracle_key(bits, 2)
    pk = sk.public
    k = gpu_key(bits, 2)
    kp = he.Key.public(bits, pk.n)
    say(f"public path, pinned shapes, {n} encryptions")
    rng = np.random.default_rng(93)
    m = rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    want = he.encrypt(k, dev(m), seed=11)
    pick = [0, 1, n // 2, n - 2, n - 1]
    assert he.limbs_to_ints(host(want)[pick]) == pool.encrypt_many(
        pk, [int(m[i]) % pk.n for i in pick], [P.seeded_r(pk.n, bits, 11, i) for i in pick])
    for lanes, tail in ((16, 0), (8, 16)):
        he.crt_set_shape(k, "public", n, lanes, 0, tail)
        he.crt_set_shape(kp, "public", n, lanes, 0, tail)
        assert torch.equal(he.encrypt(k, dev(m), seed=11, public=True), want), (lanes, tail)
        assert torch.equal(he.encrypt(kp, dev(m), seed=11), want), (lanes, tail)
    for bad in ((4, 0, 0), (8, 0, 8), (16, 1, 0)):
        with pytest.raises(he.HEError):
            he.crt_set_shape(k, "public", n, *bad)


# ---------------------------------------------------------- decryption
@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
def test_decrypt_exact(he, bits, seed):
    say(f"decrypt {bits}")
    sk = oracle_key(bits, seed)
    pk = sk.public
    rng = np.random.default_rng(bits)
    ms = plaintexts(40, rng)
    # near the decode boundary and outside int64
    big = [(pk.n - 1) // 2, (pk.n + 1) // 2, 1 << 63, -(1 << 63) - 1, 1 << 200]
    rs = W.random_units(pk.n, len(ms) + len(big), rng)
    cts = pool.encrypt_many(pk, ms + big, rs)
    k = gpu_key(bits, seed)
    m, raw, ovf = he.decrypt(k, dev(he.ints_to_limbs(cts, 2 * k.limbs)), raw=True)
    m, raw = host(m), he.limbs_to_ints(host(raw))
    assert raw == [x % pk.n for x in ms + big]
    assert m[: len(ms)].tolist() == ms
    i64 = np.iinfo(np.int64)
    assert m[len(ms):].tolist() == [i64.max, i64.min, i64.max, i64.min, i64.max]
    assert int(host(ovf)[0]) == 5


def test_decrypt_unit_ciphertext_is_zero(he):
    # The empty-bin value 1 decrypts to 0.
    k = gpu_key(2048, 2)
    ct = np.zeros((3, 2 * k.limbs), dtype=np.int32)
    ct[:, 0] = 1
    m, _, _ = he.decrypt(k, dev(ct))
    assert host(m).tolist() == [0, 0, 0]


# ---------------------------------------------------------- aggregation
def c1_inputs(M=1000, J=8, K=32, seed=0):
    s = W.streams(seed)
    g = W.gradients(M, s[1])
    bins = W.bins_uniform(J, M, K, s[2])
    return g, bins


@functools.lru_cache(maxsize=None)
def c1_oracle(bits=1024, kseed=1, M=1000, J=8, K=32):
    sk = oracle_key(bits, kseed)
    pk = sk.public
    g, bins = c1_inputs(M, J, K)
    m = [[P.encode(a), P.encode(b)] for a, b in g]
    r_seed = 77
    rs = [P.seeded_r(pk.n, bits, r_seed, i) for i in range(2 * M)]
    flat = pool.encrypt_many(pk, [v for row in m for v in row], rs)
    ct = [[flat[2 * i], flat[2 * i + 1]] for i in range(M)]
    return m, ct, rs, r_seed, bins


def test_c1_full_path_bit_exact(he):
    """1024-bit key, 1000 samples, 8 features x 32 uniform bins, root node:
    GPU encode -> encrypt (seeded r) -> histogram -> decrypt, against the
    oracle at every stage."""
    say("c1 full path")
    import torch
    bits, M, J, K = 1024, 1000, 8, 32
    sk = oracle_key(bits, 1)
    pk = sk.public
    m, ct_o, rs, r_seed, bins = c1_oracle()
    g, _ = c1_inputs(M, J, K)
    k = gpu_key(bits, 1)
    mg = he.encode(dev(g.reshape(-1)))
    assert host(mg).tolist() == [v for row in m for v in row]
    ct = he.encrypt(k, mg, seed=r_seed).view(M, 2, 2 * k.limbs)
    assert he.limbs_to_ints(host(ct)) == [v for row in ct_o for v in row]
    idx = np.arange(M, dtype=np.uint32)
    job = he.Job(dev(idx.view(np.int32)), dev(bins), K)
    (hist,) = he.hist_aggregate(k, ct, [job])
    want = pool.aggregate_many(pk, ct_o, idx, bins, J, K)
    got = he.limbs_to_ints(host(hist))
    assert got == [want[f][b][t] for f in range(J) for b in range(K) for t in range(2)]
    dm, _, ovf = he.decrypt(k, hist)
    plain = P.plaintext_histogram(m, idx, bins, J, K)
    assert host(dm).reshape(-1).tolist() == [plain[f][b][t] for f in range(J) for b in range(K) for t in range(2)]
    assert int(host(ovf)[0]) == 0
    # resident Montgomery form gives the same histogram
    ctm = he.to_mont(k, ct)
    (hist2,) = he.hist_aggregate(k, ctm, [he.Job(dev(idx.view(np.int32)), dev(bins), K)], form=he.HE_FORM_MONT)
    assert torch.equal(hist, hist2)
    assert torch.equal(he.from_mont(k, ctm), ct)


@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
def test_montgomery_form_definition(he, bits, seed):
    """he_to_mont is x R' mod n^2 with R' = 2^(29 s), s the histogram
    kernels' 29-bit limb count (144 at 2048 bits, 80 at 1024 bits with their
    16-lane groups), canonical in the 2L-limb layout; he_from_mont inverts it
    (checked with Python integers, including 0, 1 and n^2 - 1)."""
    sk = oracle_key(bits, seed)
    n2 = sk.public.n * sk.public.n
    k = gpu_key(bits, seed)
    s = {1024: 80, 2048: 144}[bits]
    R = pow(2, 29 * s, n2)
    rng = np.random.default_rng(3)
    xs = [0, 1, n2 - 1] + [int.from_bytes(rng.bytes(bits // 4), "little") % n2 for _ in range(61)]
    ct = dev(he.ints_to_limbs(xs, 2 * k.limbs))
    say(f"montgomery form {bits}")
    got = he.limbs_to_ints(host(he.to_mont(k, ct)))
    assert got == [x * R % n2 for x in xs]
    back = he.limbs_to_ints(host(he.from_mont(k, he.to_mont(k, ct))))
    assert back == xs


@pytest.mark.parametrize("chunk", [1, 2, 3, 7, 64, 5000])
def test_hist_independent_of_chunking_order_and_batching(he, chunk):
    """Subsets (ragged sizes, empty bins, an empty node, a single sample) in
    one batch equal the oracle histograms, for any chunk length and order."""
    say(f"hist chunk={chunk}")
    import torch
    bits, M, J, K = 1024, 1000, 8, 32
    sk = oracle_key(bits, 1)
    pk = sk.public
    m, ct_o, _, r_seed, bins = c1_oracle()
    k = gpu_key(bits, 1)
    ct = dev(he.ints_to_limbs([v for row in ct_o for v in row], 2 * k.limbs)).view(M, 2, 2 * k.limbs)
    rng = np.random.default_rng(chunk)
    subsets = [np.sort(rng.choice(M, size=s, replace=False)).astype(np.uint32) for s in (513, 1, 0, 77, 1000)]
    subsets[3] = rng.permutation(subsets[3]).astype(np.uint32)  # any order
    kbins = [K, 5, 3, 256, 17]
    jb = []
    for s, kb in zip(subsets, kbins):
        b = (bins.astype(np.int64) % kb).astype(np.uint8)
        if kb == 256:
            b = rng.integers(0, 256, size=bins.shape, dtype=np.uint8)
        jb.append(b)
    jobs = [he.Job(dev(s.view(np.int32)), dev(b), kb) for s, b, kb in zip(subsets, jb, kbins)]
    hists = he.hist_aggregate(k, ct, jobs, chunk=chunk)
    for s, b, kb, h in zip(subsets, jb, kbins, hists):
        want = P.aggregate(pk, ct_o, s, b, J, kb)
        got = he.limbs_to_ints(host(h))
        assert got == [want[f][x][t] for f in range(J) for x in range(kb) for t in range(2)]
    # each job alone gives the same bits as in the batch
    for s, b, kb, h in zip(subsets, jb, kbins, hists):
        (alone,) = he.hist_aggregate(k, ct, [he.Job(dev(s.view(np.int32)), dev(b), kb)], chunk=chunk)
        assert torch.equal(alone, h)


# ---------------------------------------------------------- 2048-bit, GPU scale
def test_c2_scale_sampled_parity(he):
    """2048-bit key, 100,000 samples, 32 features x 256 Zipf(1.1) bins, root
    node: sampled ciphertexts bit-exact, sampled histogram slots bit-exact via
    the closed form prod E(m_i; r_i) = E(sum m_i; prod r_i), and every
    decrypted histogram slot equal to the oracle's plaintext sum."""
    say("c2 scale")
    bits, M, J, K = 2048, 100_000, 32, 256
    sk = oracle_key(bits, 2)
    pk = sk.public
    s = W.streams(1)
    g = W.gradients(M, s[1])
    bins = W.bins_zipf(J, M, K, s[2])
    r_seed = 2024
    k = gpu_key(bits, 2)
    mg = he.encode(dev(g.reshape(-1)))
    m = host(mg).reshape(M, 2)
    ct = he.encrypt(k, mg, seed=r_seed).view(M, 2, 2 * k.limbs)
    idx = np.arange(M, dtype=np.uint32)
    (hist,) = he.hist_aggregate(k, ct, [he.Job(dev(idx.view(np.int32)), dev(bins), K)])
    dm, _, ovf = he.decrypt(k, hist)
    dm = host(dm).reshape(J, K, 2)
    # plaintext sums from the oracle's own encoding
    mo = np.array([[P.encode(a), P.encode(b)] for a, b in g], dtype=np.int64)
    assert np.array_equal(m, mo)
    for f in range(J):
        for t in range(2):
            ref = np.zeros(K, dtype=np.int64)
            np.add.at(ref, bins[f].astype(np.int64), mo[:, t])
            assert dm[f, :, t].tolist() == ref.tolist()
    assert int(host(ovf)[0]) == 0
    # sampled ciphertexts
    rng = np.random.default_rng(9)
    pick = rng.choice(2 * M, size=48, replace=False)
    cth = host(ct).reshape(2 * M, -1)
    got = he.limbs_to_ints(cth[pick])
    want = pool.encrypt_many(pk, [int(mo.reshape(-1)[i]) for i in pick],
                             [P.seeded_r(pk.n, bits, r_seed, int(i)) for i in pick])
    assert got == want
    # sampled histogram slots: hot, cold and one empty if present
    hh = host(hist).reshape(J, K, 2, -1)
    counts = np.stack([np.bincount(bins[f], minlength=K) for f in range(J)])
    f0 = 3
    order = np.argsort(counts[f0])
    slots = [(f0, int(order[-1]), 0), (f0, int(order[-1]), 1), (f0, int(order[len(order) // 2]), 0),
             (11, int(np.argsort(counts[11])[0]), 1)]
    for f, b, t in slots:
        members = np.nonzero(bins[f] == b)[0]
        rp = 1
        for i in members:
            rp = rp * P.seeded_r(pk.n, bits, r_seed, 2 * int(i) + t) % pk.n
        want = P.encrypt(pk, int(mo[members, t].sum()), rp) if len(members) else 1
        assert he.limbs_to_ints(hh[f, b, t][None])[0] == want
