"""Plain CPU Paillier oracle for the secure vertical federated XGBoost hot path.

TEST INFRASTRUCTURE ONLY.  This module is the correctness reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(the HIP library and its Python binding) never calls it and never falls back
to it.  It shares no code with the GPU path: all arithmetic here is Python's
arbitrary-precision ``int`` (``pow``, ``%``, ``//``), with no Montgomery
form, no CRT and no limbs.

What the paper fixes (Xu et al., "Secure Federated XGBoost with
CUDA-accelerated Homomorphic Encryption via NVIDIA FLARE"):

* Sec. III-B (Secure Vertical): the active party encrypts the per-sample
  gradients g and h, each passive party accumulates the ciphertexts into
  per-(feature, bin) histograms according to its own feature binning, and the
  active party decrypts the returned cumulative histograms.
* Sec. III-C (Encryption with proper HE schemes): every g and every h is
  encrypted as a single number (2M encryptions for M samples), the scheme is
  Paillier, and histogram accumulation is encrypted addition.

The paper cites Paillier (EUROCRYPT 1999) without restating it, so the scheme
below is the textbook one: with n = p q and g = n + 1,
E(m; r) = g^m r^n mod n^2, D(c) = L(c^lambda mod n^2) mu mod n with
L(u) = (u - 1) / n, lambda = lcm(p - 1, q - 1), mu = L(g^lambda mod n^2)^-1
mod n; encrypted addition is the product of ciphertexts mod n^2, and
encrypted subtraction (a node's histogram "minus" one child's, for the
sibling) multiplies by the inverse mod n^2.

Readings where the paper is silent:
key sizes 1024/2048 bits with p, q of exactly half the bits (top two bits set);
fixed-point encoding rint(x * 2^32) with round-half-even and negatives taken
mod n; r drawn from a counter-based SplitMix64 word stream reduced mod n;
empty histogram bins hold the ciphertext 1; decryption returns m in [0, n)
and the signed decode maps m >= (n + 1) / 2 to m - n.

Every function is pinned by ``tests/test_oracle.py`` against facts that do
not come from this module (toy-key brute force, closed forms, published
SplitMix64 outputs, exact plaintext sums).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Iterable, List, Sequence, Tuple

MASK64 = (1 << 64) - 1
SPLITMIX_GAMMA = 0x9E3779B97F4A7C15  # golden-ratio increment of SplitMix64

# Domain offsets of the keygen word stream: p candidates start at counter 0,
# q candidates at 2^48, so the two never overlap.
KEYGEN_STREAM_BASE = (0, 1 << 48)
MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59,
            61, 67, 71, 73, 79, 83, 89, 97, 101, 103, 107, 109, 113, 127, 131,
            137, 139, 149, 151, 157, 163, 167, 173)  # 40 Miller-Rabin rounds
SMALL_PRIMES = tuple(x for x in range(3, 2000) if all(x % d for d in range(2, int(x ** 0.5) + 1)))
FIXED_POINT_BITS = 32


# --------------------------------------------------------------------------
# Counter-based word stream (SplitMix64; Steele, Lea & Flood, OOPSLA 2014).
# --------------------------------------------------------------------------
def splitmix64_word(seed: int, index: int) -> int:
    """The ``index``-th (0-based) output of SplitMix64 started from state
    ``seed``: the state after index+1 increments by the golden-ratio gamma,
    passed through the published 64-bit finaliser."""
    z = (seed + (index + 1) * SPLITMIX_GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def words_per_r(n_bits: int) -> int:
    """Number of 64-bit words per random r: n_bits + 64 bits, so the
    reduction mod n is within 2^-64 of uniform."""
    return n_bits // 64 + 1


def seeded_r(n: int, n_bits: int, seed: int, index: int) -> int:
    """r for ciphertext ``index`` of a seeded stream: the little-endian
    integer made of words_per_r consecutive stream words, reduced mod n.
    (Paillier draws r uniformly from Z_n^*; the paper only says randomness is
    used, so this counter-based form is the reading.)"""
    w = words_per_r(n_bits)
    x = 0
    for j in range(w):
        x |= splitmix64_word(seed, index * w + j) << (64 * j)
    return x % n


# --------------------------------------------------------------------------
# Key generation.
# --------------------------------------------------------------------------
def is_probable_prime(x: int) -> bool:
    """Trial division by the odd primes below 2000, then Miller-Rabin with the
    first 40 prime bases."""
    if x < 2:
        return False
    if x in (2, 3):
        return True
    if x % 2 == 0:
        return False
    for sp in SMALL_PRIMES:
        if x == sp:
            return True
        if x % sp == 0:
            return False
    d, s = x - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in MR_BASES:
        if a % x == 0:
            continue
        y = pow(a, d, x)
        if y == 1 or y == x - 1:
            continue
        for _ in range(s - 1):
            y = y * y % x
            if y == x - 1:
                break
        else:
            return False
    return True


def prime_candidate(seed: int, which: int, attempt: int, bits: int) -> int:
    """Candidate ``attempt`` for prime ``which`` (0 = p, 1 = q): bits/64 stream
    words little-endian, with the top two bits and the low bit set."""
    nw = bits // 64
    base = KEYGEN_STREAM_BASE[which] + attempt * nw
    x = 0
    for j in range(nw):
        x |= splitmix64_word(seed, base + j) << (64 * j)
    x |= (3 << (bits - 2)) | 1
    return x


def keygen(n_bits: int, seed: int) -> Tuple[int, int]:
    """Deterministic primes (p, q) for a key of ``n_bits`` bits: the first
    candidate of each stream that passes the primality test; q must differ
    from p and satisfy gcd(pq, (p-1)(q-1)) = 1."""
    if n_bits % 128:
        raise ValueError("n_bits must be a multiple of 128")
    half = n_bits // 2
    a = 0
    while True:
        p = prime_candidate(seed, 0, a, half)
        a += 1
        if is_probable_prime(p):
            break
    a = 0
    while True:
        q = prime_candidate(seed, 1, a, half)
        a += 1
        if q != p and is_probable_prime(q) and math.gcd(p * q, (p - 1) * (q - 1)) == 1:
            break
    return p, q


@dataclass(frozen=True)
class PublicKey:
    n: int

    @property
    def n2(self) -> int:
        return self.n * self.n

    @property
    def g(self) -> int:
        return self.n + 1

    @property
    def bits(self) -> int:
        return self.n.bit_length()


@dataclass(frozen=True)
class PrivateKey:
    p: int
    q: int

    @property
    def public(self) -> PublicKey:
        return PublicKey(self.p * self.q)

    @property
    def lam(self) -> int:
        """lambda = lcm(p - 1, q - 1)."""
        return (self.p - 1) * (self.q - 1) // math.gcd(self.p - 1, self.q - 1)

    @property
    def mu(self) -> int:
        """mu = L(g^lambda mod n^2)^-1 mod n."""
        pk = self.public
        return pow(L(pow(pk.g, self.lam, pk.n2), pk.n), -1, pk.n)


def L(u: int, n: int) -> int:
    """Paillier's L function, an exact division: (u - 1) / n."""
    assert (u - 1) % n == 0
    return (u - 1) // n


# --------------------------------------------------------------------------
# Fixed-point encoding of g and h.
# --------------------------------------------------------------------------
def encode(x: float, bits: int = FIXED_POINT_BITS) -> int:
    """Signed fixed-point integer rint(x * 2^bits), ties to even (Python's
    round on a float).  x * 2^bits is exact in binary64."""
    return round(float(x) * (1 << bits))


def to_plaintext(m: int, n: int) -> int:
    """Signed integer -> Paillier plaintext in [0, n)."""
    return m % n


def decode(s: int, n: int) -> int:
    """Plaintext in [0, n) -> signed integer: s >= (n + 1) / 2 means s - n."""
    return s - n if s >= (n + 1) // 2 else s


# --------------------------------------------------------------------------
# Encryption, encrypted addition, decryption (textbook Paillier).
# --------------------------------------------------------------------------
def encrypt(pk: PublicKey, m: int, r: int) -> int:
    """E(m; r) = g^m r^n mod n^2 with g = n + 1; m is reduced mod n."""
    n2 = pk.n2
    return pow(pk.g, m % pk.n, n2) * pow(r, pk.n, n2) % n2


def add(pk: PublicKey, c1: int, c2: int) -> int:
    """Encrypted addition: the product of two ciphertexts mod n^2."""
    return c1 * c2 % pk.n2


def rerandomize(pk: PublicKey, c: int, r: int) -> int:
    """c times a fresh encryption of 0 (r' = r): the same plaintext under
    randomness multiplied by r."""
    return add(pk, c, encrypt(pk, 0, r))


def subtract(pk: PublicKey, c1: int, c2: int) -> int:
    """Encrypted subtraction: c1 times the inverse of c2 mod n^2, an
    encryption of m1 - m2 (the inverse of E(m; r) is E(-m; r^-1)).  Raises
    ValueError when c2 is not a unit mod n^2."""
    return c1 * pow(c2, -1, pk.n2) % pk.n2


PACK_SLOT_BITS = 64


def pack_offset(slots: int) -> int:
    """K = sum over slots j of 2^(64 j + 63): shifts every slot's signed
    value into [0, 2^64)."""
    return sum(1 << (PACK_SLOT_BITS * j + PACK_SLOT_BITS - 1) for j in range(slots))


def pack(pk: PublicKey, cts: Sequence[int]) -> int:
    """Several ciphertexts folded into one with the public key: the product
    of c_j^(2^(64 j)) and of g^K = 1 + K n, an encryption of
    sum_j 2^(64 j) (m_j + 2^63).  Needs 64 len(cts) < log2 n."""
    n2 = pk.n2
    acc = 1
    for j, c in enumerate(cts):
        acc = acc * pow(c, 1 << (PACK_SLOT_BITS * j), n2) % n2
    return acc * (1 + pack_offset(len(cts)) * pk.n) % n2


def unpack(m: int, slots: int) -> List[int]:
    """The slot values of a decrypted packed plaintext m in [0, n)."""
    out = []
    for j in range(slots):
        field = (m >> (PACK_SLOT_BITS * j)) & ((1 << PACK_SLOT_BITS) - 1)
        out.append(field - (1 << (PACK_SLOT_BITS - 1)))
    return out


def decrypt(sk: PrivateKey, c: int) -> int:
    """D(c) = L(c^lambda mod n^2) * mu mod n, a plaintext in [0, n)."""
    pk = sk.public
    return L(pow(c, sk.lam, pk.n2), pk.n) * sk.mu % pk.n


def aggregate(pk: PublicKey, ct: Sequence[Sequence[int]], sample_idx: Iterable[int],
              bins: Sequence[Sequence[int]], n_features: int, n_bins: int) -> List[List[List[int]]]:
    """Encrypted histogram of one tree node (Sec. III-B): for every feature f,
    bin b and slot t (0 = g, 1 = h), the product mod n^2 of ct[i][t] over the
    node's samples i whose feature-f bin is b.  An empty bin holds 1, the
    empty product."""
    hist = [[[1, 1] for _ in range(n_bins)] for _ in range(n_features)]
    idx = list(sample_idx)
    for f in range(n_features):
        for i in idx:
            b = bins[f][i]
            for t in range(2):
                hist[f][b][t] = add(pk, hist[f][b][t], ct[i][t])
    return hist


def plaintext_histogram(m: Sequence[Sequence[int]], sample_idx: Iterable[int],
                        bins: Sequence[Sequence[int]], n_features: int,
                        n_bins: int) -> List[List[List[int]]]:
    """The histogram the active party should recover: exact integer sums of
    the encoded g and h over the same index sets."""
    hist = [[[0, 0] for _ in range(n_bins)] for _ in range(n_features)]
    idx = list(sample_idx)
    for f in range(n_features):
        for i in idx:
            b = bins[f][i]
            hist[f][b][0] += m[i][0]
            hist[f][b][1] += m[i][1]
    return hist


# --------------------------------------------------------------------------
# Limb conversion (the canonical little-endian u32 buffer layout).
# --------------------------------------------------------------------------
def to_limbs(x: int, n_limbs: int) -> List[int]:
    """x as ``n_limbs`` little-endian 32-bit words."""
    assert 0 <= x < (1 << (32 * n_limbs))
    return [(x >> (32 * i)) & 0xFFFFFFFF for i in range(n_limbs)]


def from_limbs(words: Iterable[int]) -> int:
    x = 0
    for i, w in enumerate(words):
        x |= (int(w) & 0xFFFFFFFF) << (32 * i)
    return x
