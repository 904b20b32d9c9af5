"""Pins of the CKKS oracle (oracle/ckks.py) against facts that do not come
from it: schoolbook negacyclic products, trial-division primality, the
closed-form encoding of a constant vector, encode/decode round trips within
the rounding bound, the exact noise identity of decryption, and the moments
of the samplers."""
import math
import random

import numpy as np
import pytest

import oracle.ckks as C


def trial_prime(q):
    if q < 2 or q % 2 == 0:
        return q == 2
    d = 3
    while d * d <= q:
        if q % d == 0:
            return False
        d += 2
    return True


@pytest.mark.parametrize("log_n", [6, 12, 14])
def test_ntt_primes(log_n):
    n = 1 << log_n
    ps = C.ntt_primes(n)
    assert len(ps) == 3 and ps == sorted(ps, reverse=True)
    for q in ps:
        assert q < 1 << 30 and q % (2 * n) == 1 and trial_prime(q)
    # nothing skipped: no other prime = 1 mod 2N between the smallest and 2^30
    between = [q for q in range(ps[-1], 1 << 30, 2 * n) if trial_prime(q)]
    assert sorted(between, reverse=True) == ps


def test_ring_mul_matches_schoolbook():
    rng = random.Random(3)
    n, q = 64, C.ntt_primes(64)[0]
    for _ in range(5):
        a = [rng.randrange(q) for _ in range(n)]
        b = [rng.randrange(q) for _ in range(n)]
        want = [x % q for x in C.negacyclic_int(a, b)]
        assert C.ring_mul(a, b, q) == want
    # X * X^(N-1) = X^N = -1
    x = [0] * n
    x[1] = 1
    y = [0] * n
    y[n - 1] = 1
    assert C.ring_mul(x, y, q) == [q - 1] + [0] * (n - 1)


def test_rns_roundtrip():
    p = C.Params(6, 20)
    rng = random.Random(4)
    Q = p.modulus
    vals = [rng.randrange(-(Q // 2) + 1, Q // 2) for _ in range(p.n)]
    assert C.from_rns(C.to_rns(vals, p.primes), p.primes) == vals


def test_encode_constant_closed_form():
    # m(X) = Delta c is the constant polynomial with m(zeta^e) = Delta c at
    # every evaluation point.
    p = C.Params(8, 30)
    m = C.encode([1.25] * (p.n // 2), p)
    assert m[0] == int(1.25 * 2 ** 30) and all(x == 0 for x in m[1:])


@pytest.mark.parametrize("log_n", [8, 12])
def test_encode_decode_roundtrip(log_n):
    p = C.Params(log_n, 40)
    rng = np.random.default_rng(log_n)
    z = rng.normal(0, 1000, size=p.n // 2)
    m = C.encode(z, p)
    back = C.decode(m, p, p.n // 2)
    # rounding each coefficient moves every slot by at most N/2 / Delta
    assert np.max(np.abs(back - z)) <= (p.n / 2) / 2 ** 40 + 1e-9


def test_samplers_moments():
    seed = 99
    t = C.ternary(seed, 0, 60000)
    assert set(t) == {-1, 0, 1}
    for v in (-1, 0, 1):
        assert abs(t.count(v) / 60000 - 1 / 3) < 0.01
    e = np.array(C.cbd(seed, 1 << 20, 60000))
    assert e.min() >= -21 and e.max() <= 21
    assert abs(e.mean()) < 0.05 and abs(e.var() - 10.5) < 0.3



# Published SplitMix64 outputs 0..4 of seed 1234567 (tests/golden/splitmix64.txt).
W1234567 = (0x599ED017FB08FC85, 0x2C73F08458540FA5, 0x883EBCE5A3F27C77, 0x3FBEF740E9177B3F,
            0xE3B8346708CB5ECD)


def test_samplers_assemble_published_words():
    # ternary = word mod 3 - 1: the words are 0, 1, 0, 1, 2 mod 3.
    assert C.ternary(1234567, 0, 5) == [-1, 0, -1, 0, 1]
    assert C.ternary(1234567, 2, 3) == [-1, 0, 1]          # the counter base shifts the words
    # centered binomial = popcount(bits 0..20) - popcount(bits 21..41):
    #   word 0: 0x08fc85 (10 ones) - 0x00bfd8 (11) = -1
    #   word 1: 0x140fa5 (10)      - 0x0422c2 (6)  =  4
    #   word 2: 0x127c77 (13)      - 0x072d1f (12) =  1
    #   word 3: 0x177b3f (16)      - 0x1a0748 (8)  =  8
    #   word 4: 0x0b5ecd (13)      - 0x033846 (8)  =  5
    assert C.cbd(1234567, 0, 5) == [-1, 4, 1, 8, 5]
    assert C.cbd(1234567, 3, 2) == [8, 5]
    # uniform mod q = word mod q, here q = 1073479681 (a 30-bit prime that is
    # 1 mod 2^15)
    assert C.uniform(1234567, 0, 5, 1073479681) == [977752849, 627650537, 407729945, 553364867, 106535843]
    assert C.uniform(1234567, 1, 1, 1000003) == [W1234567[1] % 1000003]


def test_encryption_randomness_counter_layout():
    # Ciphertext t of a call takes u, e0, e1 from counters (offset + t) 3N +
    # [0, N), [N, 2N), [2N, 3N).  With N = 1 the three come from single words:
    # t = 0 -> words 0, 1, 2; t = 1 -> words 3, 4, 5.
    p1 = C.Params(0, 30)
    u, e0, e1 = C.enc_randomness(p1, 1234567, 0)
    assert (u, e0, e1) == ([-1], [4], [1])
    u, e0, _ = C.enc_randomness(p1, 1234567, 1)
    assert (u, e0) == ([0], [5])
    # N = 2, t = 0: u from words 0, 1; e0 from words 2, 3; e1 from word 4 onwards.
    u, e0, e1 = C.enc_randomness(C.Params(1, 30), 1234567, 0)
    assert u == [-1, 0] and e0 == [1, 8] and e1[0] == 5

def test_decrypt_is_message_plus_exact_noise():
    p = C.Params(7, 20)
    keys = C.keygen(p, 5)
    rng = random.Random(6)
    m = [rng.randrange(-(1 << 40), 1 << 40) for _ in range(p.n)]
    ct = C.encrypt(keys, C.to_rns(m, p.primes), seed=77, index=3)
    dec = C.from_rns(C.decrypt(keys, ct), p.primes)
    assert [d - x for d, x in zip(dec, m)] == C.fresh_noise(p, 5, 77, 3)
    # addition: messages and noises add
    m2 = [rng.randrange(-(1 << 40), 1 << 40) for _ in range(p.n)]
    ct2 = C.encrypt(keys, C.to_rns(m2, p.primes), seed=77, index=4)
    dec2 = C.from_rns(C.decrypt(keys, C.add(ct, ct2, p.primes)), p.primes)
    n1, n2 = C.fresh_noise(p, 5, 77, 3), C.fresh_noise(p, 5, 77, 4)
    assert dec2 == [a + b + x + y for a, b, x, y in zip(m, m2, n1, n2)]
    # the noise is small: |e0 + e1 s + e u| <= 21 (2N + 1)
    assert max(abs(x) for x in n1) <= 21 * (2 * p.n + 1)
