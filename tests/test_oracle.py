"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: a published reference output,
a brute-force enumeration on a toy key, a closed form of Paillier's algebra,
an independent route to the same value (CRT decryption, numpy sums), or a
number-theoretic fact (known primes and pseudoprimes).
"""
import functools
import math
import os
import random

import numpy as np
import pytest

import oracle.paillier as P
from synth import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@functools.lru_cache(maxsize=None)
def real_key(bits: int, seed: int):
    p, q = P.keygen(bits, seed)
    return P.PrivateKey(p, q)


# ---------------------------------------------------------------- SplitMix64
def test_splitmix64_matches_published_outputs():
    rows = []
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(int(x) for x in line.split()))
    assert len(rows) == 8
    for seed, idx, val in rows:
        assert P.splitmix64_word(seed, idx) == val


def test_seeded_r_assembles_published_words():
    # 128-bit modulus -> 3 words per r; r_0 uses stream outputs 0, 1, 2 and
    # r_1 uses outputs 3, 4 (plus 5).  The words are the published values.
    n = (1 << 127) + 45  # odd, 128 bits
    w = [6457827717110365317, 3203168211198807973, 9817491932198370423]
    x = w[0] + (w[1] << 64) + (w[2] << 128)
    assert P.words_per_r(128) == 3
    assert P.seeded_r(n, 128, 1234567, 0) == x % n
    r1 = P.seeded_r(n, 128, 1234567, 1)
    low = 4593380528125082431 + (16408922859458223821 << 64)
    assert r1 == (low + (P.splitmix64_word(1234567, 5) << 128)) % n



def test_prime_candidate_assembles_published_words():
    # Candidate 0 of p (stream counter 0) at 128 bits takes two words, low
    # word first: published outputs 0 and 1 of seed 1234567,
    #   0x599ed017fb08fc85 (6457827717110365317) and
    #   0x2c73f08458540fa5 (3203168211198807973);
    # forcing bits 127, 126 and 0 turns the high word into 0xec73f08458540fa5
    # (the low word is already odd).
    assert P.prime_candidate(1234567, 0, 0, 128) == 0xEC73F08458540FA5_599ED017FB08FC85
    # Candidate 1 starts two words later: outputs 2 and 3,
    #   0x883ebce5a3f27c77 and 0x3fbef740e9177b3f -> high word 0xffbef740e9177b3f.
    assert P.prime_candidate(1234567, 0, 1, 128) == 0xFFBEF740E9177B3F_883EBCE5A3F27C77
    # A 64-bit candidate is one word: output 4, 0xe3b8346708cb5ecd, with
    # bits 63, 62 and 0 forced -> 0xe3b8346708cb5ecd (all three already set).
    assert P.prime_candidate(1234567, 0, 4, 64) == 0xE3B8346708CB5ECD

# ---------------------------------------------------------- toy-key brute force
TOY = P.PrivateKey(11, 13)


def toy_table():
    pk = TOY.public
    n = pk.n
    units = [r for r in range(1, n) if math.gcd(r, n) == 1]
    return {(m, r): P.encrypt(pk, m, r) for m in range(n) for r in units}, units


def test_toy_encryption_is_bijection_onto_units_mod_n2():
    # Paillier's E: Z_n x Z_n^* -> Z_{n^2}^* is a bijection (n = 143:
    # 143 * 120 = 17160 = phi(143^2) distinct ciphertexts).
    table, units = toy_table()
    n2 = TOY.public.n2
    vals = set(table.values())
    assert len(units) == 120
    assert len(vals) == len(table) == 17160
    assert vals == {c for c in range(1, n2) if math.gcd(c, n2) == 1}


def test_toy_decrypt_inverts_every_ciphertext():
    table, _ = toy_table()
    for (m, _r), c in table.items():
        assert P.decrypt(TOY, c) == m


def test_toy_mu_lambda():
    # lambda = lcm(10, 12) = 60; with g = n + 1, L(g^lambda) = lambda mod n
    # so mu = 60^-1 mod 143 (brute force over Z_143).
    assert TOY.lam == 60
    assert [x for x in range(143) if 60 * x % 143 == 1] == [TOY.mu]


# ----------------------------------------------------------------- closed forms
@pytest.mark.parametrize("bits,seed", [(256, 3), (1024, 1)])
def test_encrypt_closed_form_binomial(bits, seed):
    # (1 + n)^m = 1 + m n (mod n^2): the binomial theorem kills every term
    # with n^2.  So E(m; r) = (1 + m n) r^n mod n^2.
    sk = real_key(bits, seed)
    pk = sk.public
    rng = random.Random(7)
    for _ in range(20):
        m = rng.randrange(-(1 << 63), 1 << 63)
        r = rng.randrange(1, pk.n)
        expect = (1 + (m % pk.n) * pk.n) * pow(r, pk.n, pk.n2) % pk.n2
        assert P.encrypt(pk, m, r) == expect


@pytest.mark.parametrize("bits,seed", [(256, 3), (1024, 1)])
def test_homomorphic_product_is_encryption_of_sum(bits, seed):
    # E(a; r1) E(b; r2) = E(a + b; r1 r2) mod n^2, bit for bit.
    sk = real_key(bits, seed)
    pk = sk.public
    rng = random.Random(11)
    for _ in range(20):
        a, b = rng.randrange(-(1 << 40), 1 << 40), rng.randrange(-(1 << 40), 1 << 40)
        r1, r2 = rng.randrange(1, pk.n), rng.randrange(1, pk.n)
        lhs = P.add(pk, P.encrypt(pk, a, r1), P.encrypt(pk, b, r2))
        assert lhs == P.encrypt(pk, a + b, r1 * r2 % pk.n)
        assert P.decode(P.decrypt(sk, lhs), pk.n) == a + b


def test_toy_subtract_inverts_every_unit():
    # For every unit c mod 143^2, subtract(1, c) is the c' with c c' = 1,
    # found here by search over the unit group for a sample of c.
    pk = TOY.public
    n2 = pk.n2
    units = [c for c in range(1, n2) if math.gcd(c, n2) == 1]
    for c in units:
        assert P.subtract(pk, 1, c) * c % n2 == 1
    for c in units[::997]:
        assert [x for x in units if x * c % n2 == 1] == [P.subtract(pk, 1, c)]
    for bad in (0, 11, 13 * 5, 143):
        with pytest.raises(ValueError):
            P.subtract(pk, 1, bad)


@pytest.mark.parametrize("bits,seed", [(256, 3), (1024, 1)])
def test_subtract_closed_form(bits, seed):
    # E(a; r1) / E(b; r2) = E(a - b; r1 r2^-1 mod n), bit for bit, and it
    # decrypts to a - b; dividing a product by one factor gives the other.
    sk = real_key(bits, seed)
    pk = sk.public
    rng = random.Random(13)
    for _ in range(20):
        a, b = rng.randrange(-(1 << 40), 1 << 40), rng.randrange(-(1 << 40), 1 << 40)
        r1, r2 = rng.randrange(1, pk.n), rng.randrange(1, pk.n)
        c1, c2 = P.encrypt(pk, a, r1), P.encrypt(pk, b, r2)
        d = P.subtract(pk, c1, c2)
        # r2^-1 mod n from the extended Euclidean identity u r2 + v n = 1
        u, v, x0, x1 = r2, pk.n, 1, 0
        while v:
            qq = u // v
            u, v, x0, x1 = v, u - qq * v, x1, x0 - qq * x1
        assert u == 1
        assert d == P.encrypt(pk, a - b, r1 * (x0 % pk.n) % pk.n)
        assert P.decode(P.decrypt(sk, d), pk.n) == a - b
        assert P.subtract(pk, P.add(pk, c1, c2), c2) == c1


@pytest.mark.parametrize("bits,seed", [(256, 3), (1024, 1)])
def test_rerandomize_closed_form(bits, seed):
    # E(m; r1) E(0; r) = E(m; r1 r): same plaintext, randomness multiplied.
    sk = real_key(bits, seed)
    pk = sk.public
    rng = random.Random(17)
    for _ in range(10):
        m = rng.randrange(-(1 << 50), 1 << 50)
        r1, r = rng.randrange(1, pk.n), rng.randrange(1, pk.n)
        c = P.rerandomize(pk, P.encrypt(pk, m, r1), r)
        assert c == P.encrypt(pk, m, r1 * r % pk.n)
        assert P.decode(P.decrypt(sk, c), pk.n) == m


@pytest.mark.parametrize("bits,seed", [(256, 3), (1024, 1)])
def test_pack_closed_form_and_roundtrip(bits, seed):
    # pack(E(m_j; r_j)) = E(sum_j 2^(64 j) (m_j + 2^63); prod_j r_j^(2^(64 j))),
    # and the slots of its decryption are the m_j (slot values at the edges of
    # the signed 64-bit range included).
    sk = real_key(bits, seed)
    pk = sk.public
    rng = random.Random(23)
    max_slots = (bits - 1) // 64
    for slots in (1, 2, max_slots):
        ms = [rng.randrange(-(1 << 63), 1 << 63) for _ in range(slots)]
        ms[0] = -(1 << 63)
        ms[-1] = (1 << 63) - 1
        rs = [rng.randrange(1, pk.n) for _ in range(slots)]
        c = P.pack(pk, [P.encrypt(pk, m, r) for m, r in zip(ms, rs)])
        plain = sum((m + (1 << 63)) << (64 * j) for j, m in enumerate(ms))
        rp = 1
        for j, r in enumerate(rs):
            rp = rp * pow(r, 1 << (64 * j), pk.n) % pk.n
        assert c == P.encrypt(pk, plain, rp)
        assert P.unpack(P.decrypt(sk, c), slots) == ms


def test_subtract_histograms_gives_sibling():
    # A parent node's samples split into two children: the parent's encrypted
    # histogram divided by one child's equals the other child's, slot by slot.
    sk = real_key(256, 3)
    pk = sk.public
    rng = np.random.default_rng(5)
    M, F, B = 60, 3, 5
    rs = W.random_units(pk.n, 2 * M, rng)
    ct = [[P.encrypt(pk, int(rng.integers(-1000, 1000)), rs[2 * i + t]) for t in range(2)] for i in range(M)]
    bins = rng.integers(0, B, size=(F, M)).tolist()
    parent = rng.choice(M, size=40, replace=False)
    left = parent[rng.random(40) < 0.4]
    right = np.setdiff1d(parent, left)
    hp = P.aggregate(pk, ct, parent, bins, F, B)
    hl = P.aggregate(pk, ct, left, bins, F, B)
    hr = P.aggregate(pk, ct, right, bins, F, B)
    for f in range(F):
        for b in range(B):
            for t in range(2):
                assert P.subtract(pk, hp[f][b][t], hl[f][b][t]) == hr[f][b][t]


@pytest.mark.parametrize("bits,seed", [(256, 3), (1024, 1)])
def test_decrypt_equals_crt_decryption(bits, seed):
    # Independent route: per prime, m_p = L_p(c^(p-1) mod p^2) h_p mod p with
    # h_p = L_p(g^(p-1) mod p^2)^-1 mod p, then the CRT.
    sk = real_key(bits, seed)
    pk = sk.public
    p, q, n = sk.p, sk.q, pk.n
    g = n + 1

    def half(c, a):
        h = pow((pow(g, a - 1, a * a) - 1) // a, -1, a)
        return (pow(c % (a * a), a - 1, a * a) - 1) // a * h % a

    rng = random.Random(13)
    for _ in range(10):
        m, r = rng.randrange(n), rng.randrange(1, n)
        c = P.encrypt(pk, m, r)
        mp, mq = half(c, p), half(c, q)
        crt = (mq + q * ((mp - mq) * pow(q, -1, p) % p)) % n
        assert P.decrypt(sk, c) == crt == m


@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
def test_decrypt_edge_plaintexts(bits, seed):
    sk = real_key(bits, seed)
    pk = sk.public
    n = pk.n
    edge = [0, 1, -1, (1 << 32) - 1, -((1 << 32) - 1), (1 << 63) - 1, -(1 << 63), (1 << 52), -(1 << 52)]
    r = 0x1234567890ABCDEF1234567 % n
    for m in edge:
        c = P.encrypt(pk, m, r)
        assert P.decode(P.decrypt(sk, c), n) == m
    # decode boundary: (n - 1) / 2 is the largest positive value.
    assert P.decode((n - 1) // 2, n) == (n - 1) // 2
    assert P.decode((n + 1) // 2, n) == -((n - 1) // 2)
    assert P.decode(n - 1, n) == -1


# ------------------------------------------------------------------- keygen
def test_primality_matches_trial_division_below_20000():
    def brute(x):
        return x >= 2 and all(x % d for d in range(2, int(x ** 0.5) + 1))
    for x in range(20000):
        assert P.is_probable_prime(x) == brute(x), x


def test_primality_known_large_cases():
    for e in (521, 607, 1279):  # Mersenne primes
        assert P.is_probable_prime((1 << e) - 1)
    # Carmichael numbers and strong pseudoprimes to base 2 are composite.
    for c in (561, 1105, 1729, 2465, 2821, 6601, 8911, 41041, 825265, 321197185,
              2047, 3277, 4033, 4681, 8321, 3215031751, 3825123056546413051):
        assert not P.is_probable_prime(c)
    assert not P.is_probable_prime(((1 << 521) - 1) * ((1 << 607) - 1))
    assert not P.is_probable_prime((1 << 523) - 1)  # 523 is prime, M523 is not


@pytest.mark.parametrize("bits,seed", [(1024, 1), (1024, 5), (2048, 2)])
def test_keygen_properties(bits, seed):
    sk = real_key(bits, seed)
    p, q = sk.p, sk.q
    for x in (p, q):
        assert x.bit_length() == bits // 2 and (x >> (bits // 2 - 2)) == 3 and x & 1
        assert pow(2, x - 1, x) == 1 and pow(3, x - 1, x) == 1
    assert p != q and (p * q).bit_length() == bits
    assert math.gcd(p * q, (p - 1) * (q - 1)) == 1
    # p is the first prime candidate of its stream.
    a = 0
    while not P.is_probable_prime(P.prime_candidate(seed, 0, a, bits // 2)):
        a += 1
    assert P.prime_candidate(seed, 0, a, bits // 2) == p


# ----------------------------------------------------------------- encoding
def test_encode_round_half_even_and_sign():
    s = 2.0 ** -32
    assert P.encode(0.5 * s) == 0
    assert P.encode(1.5 * s) == 2
    assert P.encode(2.5 * s) == 2
    assert P.encode(-1.5 * s) == -2
    assert P.encode(-0.5 * s) == 0
    assert P.encode(1.0) == 1 << 32
    assert P.encode(-0.25) == -(1 << 30)
    assert P.encode(0.3) == int(np.rint(0.3 * 2 ** 32))
    xs = np.random.default_rng(0).standard_normal(1000)
    assert [P.encode(x) for x in xs] == [int(v) for v in np.rint(xs * 2.0 ** 32)]


def test_to_plaintext_and_decode_roundtrip():
    n = real_key(1024, 1).public.n
    for m in (0, 5, -5, (1 << 63) - 1, -(1 << 63)):
        s = P.to_plaintext(m, n)
        assert 0 <= s < n and P.decode(s, n) == m


# -------------------------------------------------------------- aggregation
def test_aggregate_matches_closed_form_and_plaintext_sums():
    sk = real_key(256, 3)
    pk = sk.public
    rng = np.random.default_rng(5)
    M, J, K = 200, 3, 8
    g = W.gradients(M, rng)
    m = [[P.encode(a), P.encode(b)] for a, b in g]
    bins = W.bins_uniform(J, M, K, rng)
    bins[0, :] = np.where(bins[0] == 3, 4, bins[0])  # leave bin 3 of feature 0 empty
    rs = W.random_units(pk.n, 2 * M, rng)
    ct = [[P.encrypt(pk, m[i][t], rs[2 * i + t]) for t in range(2)] for i in range(M)]
    idx = np.sort(rng.choice(M, size=150, replace=False))
    hist = P.aggregate(pk, ct, idx, bins, J, K)
    plain = P.plaintext_histogram(m, idx, bins, J, K)
    # numpy route for the plaintext sums
    mm = np.array(m, dtype=np.int64)
    for f in range(J):
        for t in range(2):
            ref = np.zeros(K, dtype=np.int64)
            np.add.at(ref, bins[f][idx].astype(np.int64), mm[idx, t])
            assert [plain[f][b][t] for b in range(K)] == ref.tolist()
    for f in range(J):
        for b in range(K):
            members = [i for i in idx if bins[f][i] == b]
            for t in range(2):
                rprod = 1
                for i in members:
                    rprod = rprod * rs[2 * i + t] % pk.n
                # closed form: product of E(m_i; r_i) = E(sum m_i; prod r_i)
                assert hist[f][b][t] == P.encrypt(pk, plain[f][b][t], rprod)
                assert P.decode(P.decrypt(sk, hist[f][b][t]), pk.n) == plain[f][b][t]
    assert hist[0][3] == [1, 1] and plain[0][3] == [0, 0]


def test_limb_roundtrip():
    x = (1 << 4095) + 12345
    limbs = P.to_limbs(x, 128)
    assert limbs[0] == 12345 and limbs[127] == 1 << 31
    assert P.from_limbs(limbs) == x


# ------------------------------------------------------------ split finding
def test_split_gain_hand_values():
    from oracle import split as S
    # G_L = 2, H_L = 1, G_R = -2, H_R = 1, lambda = 1: 1/2 (4/2 + 4/2 - 0/3) = 2
    one = 1 << 32
    assert S.split_gain(2 * one, one, 0, 2 * one, 32, 1.0, 0.0, 0.0) == 2.0
    # gamma is subtracted once; lambda = 0 and H_L = 0 is not admissible
    assert S.split_gain(2 * one, one, 0, 2 * one, 32, 1.0, 0.5, 0.0) == 1.5
    assert S.split_gain(one, 0, one, one, 32, 0.0, 0.0, 0.0) is None
    # min_child_weight
    assert S.split_gain(one, one, 2 * one, 3 * one, 32, 1.0, 0.0, 1.5) is None


def test_split_from_samples_brute_force():
    # Against the definition over samples: for every candidate bin, sum the
    # samples with bin <= b directly (no running sums) and take the argmax.
    from oracle import split as S
    rng = np.random.default_rng(21)
    n, F, B = 400, 5, 12
    g = rng.integers(-(1 << 33), 1 << 33, size=n)
    h = rng.integers(0, 1 << 32, size=n)
    bins = rng.integers(0, B, size=(F, n))
    hist = [[(int(g[bins[f] == b].sum()), int(h[bins[f] == b].sum())) for b in range(B)] for f in range(F)]
    per_feat, per_node = S.best_splits([hist], 32, 1.0, 0.0, 0.25)
    G, H = int(g.sum()), int(h.sum())
    best_all = (-math.inf, -1, -1)
    for f in range(F):
        best = (-math.inf, -1)
        for b in range(B - 1):
            left = bins[f] <= b
            gl, hl = int(g[left].sum()), int(h[left].sum())
            s = 2.0 ** -32
            if hl * s >= 0.25 and (H - hl) * s >= 0.25:
                val = 0.5 * (((gl * s) ** 2 / (hl * s + 1) + ((G - gl) * s) ** 2 / ((H - hl) * s + 1))
                             - (G * s) ** 2 / (H * s + 1))
                if val > best[0]:
                    best = (val, b)
        assert per_feat[0][f].bin == best[1]
        assert per_feat[0][f].gain == pytest.approx(best[0], rel=1e-12)
        if best[0] > best_all[0]:
            best_all = (best[0], f, best[1])
    assert (per_node[0].feature, per_node[0].bin) == best_all[1:]


def test_split_planted_boundary():
    # Samples in bins < 5 have g = -1, the rest g = +1 (h = 1): the best split
    # of that feature is after bin 4, with G_L = -(count of bins < 5).
    from oracle import split as S
    rng = np.random.default_rng(3)
    bins = rng.integers(0, 16, size=1000)
    one = 1 << 32
    hist = [(int(((bins == b) * (-1 if b < 5 else 1)).sum()) * one, int((bins == b).sum()) * one)
            for b in range(16)]
    s = S.best_split_feature(hist, 32, 1.0, 0.0, 1.0)
    assert s.bin == 4 and s.g_left == -int((bins < 5).sum()) * one
    assert S.best_split_feature(hist[:1], 32, 1.0, 0.0, 1.0) == S.NO_SPLIT
