"""Plain CPU oracle for the secure horizontal path: CKKS encryption of local
gradient histograms, ciphertext addition, decryption.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and nothing in the product
path; it shares no code with the GPU path (no NTT, no FFT: ring products are
exact integer products by Kronecker substitution, the canonical embedding is
summed term by term).

The paper (Sec. III-A, III-C) picks CKKS (Cheon, Kim, Kim, Song, ASIACRYPT
2017) for horizontal federated XGBoost -- each client encrypts its local G/H
histogram vectors, the server adds the ciphertexts, clients decrypt the
global histogram -- without restating the scheme or fixing parameters.  The
textbook scheme restricted to what that needs (public-key encryption,
addition, decryption), with these readings:

* ring R_Q = Z_Q[X]/(X^N + 1), N = 2^log_n, Q = q_0 q_1 q_2 with the three
  largest primes below 2^30 that are 1 mod 2N (RNS; coefficient j of a
  polynomial is kept as its residues mod each q_i);
* encoding of n <= N/2 real values z (padded with zeros to N/2): the
  polynomial m with m(zeta^(5^k)) = Delta z_k for k < N/2, zeta = e^(i pi/N),
  i.e. m_j = (2/N) Re(sum_k Delta z_k zeta^(-5^k j)), rounded to integers
  (round half to even); decoding evaluates m(zeta^(5^k)) / Delta;
* keys from a seed: s ternary, a uniform mod each q_i, e from the centered
  binomial distribution with eta = 21 (variance 10.5, close to the usual
  sigma = 3.2 Gaussian); b = -a s + e;
* encryption of m with randomness (u ternary, e0, e1 centered binomial):
  c = (b u + e0 + m, a u + e1); decryption c0 + c1 s; addition
  coefficient-wise;
* the randomness is drawn from the SplitMix64 word stream (the published
  generator, implemented again here): ternary = word mod 3 - 1, centered
  binomial = popcount of the low 21 bits minus popcount of the next 21,
  uniform mod q = word mod q; counters: key s at [0, N), key e at
  [2^40, 2^40 + N), key a for prime i at [2^41 + i N, ...); ciphertext t of a
  call with offset o: u, e0, e1 at (o + t) 3N + [0, N), + N, + 2N.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

from .paillier import is_probable_prime, splitmix64_word

N_PRIMES = 3
PRIME_BITS = 30
ETA = 21
KEY_E_BASE = 1 << 40
KEY_A_BASE = 1 << 41


def ntt_primes(n: int, count: int = N_PRIMES, bits: int = PRIME_BITS) -> List[int]:
    """The `count` largest primes below 2^bits that are 1 mod 2n, descending."""
    out = []
    q = ((1 << bits) - 1) // (2 * n) * (2 * n) + 1
    while len(out) < count:
        if q < (1 << bits) and is_probable_prime(q):
            out.append(q)
        q -= 2 * n
    return out


@dataclass(frozen=True)
class Params:
    log_n: int
    scale_bits: int

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def primes(self) -> List[int]:
        return ntt_primes(self.n)

    @property
    def modulus(self) -> int:
        return math.prod(self.primes)


# ------------------------------------------------------------ sampling
def ternary(seed: int, base: int, n: int) -> List[int]:
    return [splitmix64_word(seed, base + j) % 3 - 1 for j in range(n)]


def cbd(seed: int, base: int, n: int) -> List[int]:
    out = []
    for j in range(n):
        w = splitmix64_word(seed, base + j)
        out.append(bin(w & ((1 << ETA) - 1)).count("1") - bin((w >> ETA) & ((1 << ETA) - 1)).count("1"))
    return out


def uniform(seed: int, base: int, n: int, q: int) -> List[int]:
    return [splitmix64_word(seed, base + j) % q for j in range(n)]


# ------------------------------------------------------------ ring arithmetic
def ring_mul(a: Sequence[int], b: Sequence[int], q: int) -> List[int]:
    """a b mod (X^N + 1, q) for coefficients in [0, q): the full integer
    product by Kronecker substitution (each coefficient in a byte-aligned
    slot wide enough for every convolution sum, the whole polynomial one big
    integer), then the upper half folded back with a minus sign."""
    n = len(a)
    width = (2 * q.bit_length() + n.bit_length() + 8) // 8      # bytes per slot
    A = int.from_bytes(b"".join(int(x).to_bytes(width, "little") for x in a), "little")
    B = int.from_bytes(b"".join(int(x).to_bytes(width, "little") for x in b), "little")
    raw = (A * B).to_bytes(2 * n * width, "little")
    full = [int.from_bytes(raw[k * width:(k + 1) * width], "little") for k in range(2 * n)]
    return [(full[k] - full[k + n]) % q for k in range(n)]


def ring_mul_rns(a: Sequence[Sequence[int]], b: Sequence[Sequence[int]], primes: Sequence[int]):
    return [ring_mul(x, y, q) for x, y, q in zip(a, b, primes)]


def to_rns(coeffs: Sequence[int], primes: Sequence[int]) -> List[List[int]]:
    return [[int(c) % q for c in coeffs] for q in primes]


def from_rns(res: Sequence[Sequence[int]], primes: Sequence[int]) -> List[int]:
    """Centered integers in (-Q/2, Q/2] from residues, by the CRT."""
    Q = math.prod(primes)
    out = []
    for j in range(len(res[0])):
        x = 0
        for r, q in zip(res, primes):
            Mi = Q // q
            x += int(r[j]) * Mi * pow(Mi, -1, q)
        x %= Q
        out.append(x - Q if x > Q // 2 else x)
    return out


# ------------------------------------------------------------ encoding
def _angles(log_n: int):
    n = 1 << log_n
    two_n = 2 * n
    e = np.array([pow(5, k, two_n) for k in range(n // 2)], dtype=np.int64)
    return n, two_n, e


def encode(z: Sequence[float], params: Params) -> List[int]:
    """Integer coefficients of the encoding of z (len(z) <= N/2)."""
    n, two_n, e = _angles(params.log_n)
    zz = np.zeros(n // 2, dtype=np.complex128)
    zz[: len(z)] = np.asarray(z, dtype=np.float64) * float(2 ** params.scale_bits)
    out = np.empty(n, dtype=np.float64)
    step = 256
    for j0 in range(0, n, step):
        j = np.arange(j0, min(n, j0 + step), dtype=np.int64)
        ex = (e[None, :] * j[:, None]) % two_n               # exact exponent mod 2N
        w = np.exp(-1j * np.pi * ex / n)
        out[j0:j0 + len(j)] = (2.0 / n) * np.real(w @ zz)
    return [int(x) for x in np.rint(out)]


def decode(m: Sequence[int], params: Params, count: int) -> np.ndarray:
    """z_k = m(zeta^(5^k)) / Delta for k < count (real parts)."""
    n, two_n, e = _angles(params.log_n)
    mm = np.asarray([float(x) for x in m], dtype=np.float64)
    out = np.empty(count, dtype=np.float64)
    j = np.arange(n, dtype=np.int64)
    step = 128
    for k0 in range(0, count, step):
        k = np.arange(k0, min(count, k0 + step))
        ex = (e[k][:, None] * j[None, :]) % two_n
        out[k0:k0 + len(k)] = np.real(np.exp(1j * np.pi * ex / n) @ mm)
    return out / float(2 ** params.scale_bits)


# ------------------------------------------------------------ scheme
@dataclass
class Keys:
    params: Params
    s: List[int]                 # ternary, as integers
    a: List[List[int]]           # [prime][N]
    b: List[List[int]]


def keygen(params: Params, seed: int) -> Keys:
    n, primes = params.n, params.primes
    s = ternary(seed, 0, n)
    e = cbd(seed, KEY_E_BASE, n)
    a = [uniform(seed, KEY_A_BASE + i * n, n, q) for i, q in enumerate(primes)]
    s_r = to_rns(s, primes)
    a_s = ring_mul_rns(a, s_r, primes)
    b = [[(-x + ee) % q for x, ee in zip(row, e)] for row, q in zip(a_s, primes)]
    return Keys(params, s, a, b)


def enc_randomness(params: Params, seed: int, index: int):
    n = params.n
    base = index * 3 * n
    return ternary(seed, base, n), cbd(seed, base + n, n), cbd(seed, base + 2 * n, n)


def encrypt(keys: Keys, m_rns: Sequence[Sequence[int]], seed: int, index: int):
    """(c0, c1), each [prime][N] residues."""
    primes = keys.params.primes
    u, e0, e1 = enc_randomness(keys.params, seed, index)
    u_r = to_rns(u, primes)
    bu = ring_mul_rns(keys.b, u_r, primes)
    au = ring_mul_rns(keys.a, u_r, primes)
    c0 = [[(x + y + int(mm)) % q for x, y, mm in zip(row, e0, mrow)] for row, mrow, q in zip(bu, m_rns, primes)]
    c1 = [[(x + y) % q for x, y in zip(row, e1)] for row, q in zip(au, primes)]
    return c0, c1


def add(ct1, ct2, primes):
    return tuple([[(x + y) % q for x, y in zip(r1, r2)] for r1, r2, q in zip(p1, p2, primes)]
                 for p1, p2 in zip(ct1, ct2))


def decrypt(keys: Keys, ct) -> List[List[int]]:
    """c0 + c1 s, residues [prime][N]."""
    primes = keys.params.primes
    c1s = ring_mul_rns(ct[1], to_rns(keys.s, primes), primes)
    return [[(x + y) % q for x, y in zip(r0, r1)] for r0, r1, q in zip(ct[0], c1s, primes)]


def negacyclic_int(a: Sequence[int], b: Sequence[int]) -> List[int]:
    """a b in Z[X]/(X^N + 1) over the integers (small operands), schoolbook."""
    n = len(a)
    out = [0] * n
    for i, x in enumerate(a):
        if x == 0:
            continue
        for j, y in enumerate(b):
            k = i + j
            if k < n:
                out[k] += x * y
            else:
                out[k - n] -= x * y
    return out


def fresh_noise(params: Params, key_seed: int, seed: int, index: int) -> List[int]:
    """e0 + e1 s + e u over the integers for ciphertext `index` of a call
    with `seed` under the keys of `key_seed`: decrypt(encrypt(m)) - m."""
    n = params.n
    s = ternary(key_seed, 0, n)
    e = cbd(key_seed, KEY_E_BASE, n)
    u, e0, e1 = enc_randomness(params, seed, index)
    e1s = negacyclic_int(e1, s)
    eu = negacyclic_int(e, u)
    return [x + y + z for x, y, z in zip(e0, e1s, eu)]
