// Host-side multiprecision integers for key setup: everything the device
// kernels need precomputed per key (Montgomery constants, CRT constants,
// exponents) and the seeded prime search.  Not on the hot path.
//
// Representation: little-endian std::vector<uint32_t>, normalised so that the
// top limb is non-zero (zero is the empty vector).
#pragma once
#include <stdint.h>

#include <algorithm>
#include <stdexcept>
#include <vector>

namespace hebn {

using Limbs = std::vector<uint32_t>;

inline void norm(Limbs &a) {
  while (!a.empty() && a.back() == 0) a.pop_back();
}
inline Limbs from_u64(uint64_t v) {
  Limbs r{(uint32_t)v, (uint32_t)(v >> 32)};
  norm(r);
  return r;
}
inline Limbs from_words(const uint32_t *w, size_t n) {
  Limbs r(w, w + n);
  norm(r);
  return r;
}
inline bool is_zero(const Limbs &a) { return a.empty(); }
inline bool is_odd(const Limbs &a) { return !a.empty() && (a[0] & 1); }
inline size_t bit_length(const Limbs &a) {
  if (a.empty()) return 0;
  return 32 * (a.size() - 1) + (32 - __builtin_clz(a.back()));
}
inline int bit(const Limbs &a, size_t i) {
  size_t w = i / 32;
  return w < a.size() ? (a[w] >> (i % 32)) & 1 : 0;
}
// Copies a into exactly n limbs (zero padded); throws if it does not fit.
inline void to_words(const Limbs &a, uint32_t *out, size_t n) {
  if (a.size() > n) throw std::runtime_error("value does not fit");
  std::fill(out, out + n, 0u);
  std::copy(a.begin(), a.end(), out);
}
inline Limbs padded(const Limbs &a, size_t n) {
  Limbs r(n, 0u);
  to_words(a, r.data(), n);
  return r;
}

inline int cmp(const Limbs &a, const Limbs &b) {
  if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
  for (size_t i = a.size(); i-- > 0;)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}

inline Limbs add(const Limbs &a, const Limbs &b) {
  const Limbs &x = a.size() >= b.size() ? a : b;
  const Limbs &y = a.size() >= b.size() ? b : a;
  Limbs r(x.size() + 1, 0u);
  uint64_t c = 0;
  for (size_t i = 0; i < x.size(); ++i) {
    c += (uint64_t)x[i] + (i < y.size() ? y[i] : 0u);
    r[i] = (uint32_t)c;
    c >>= 32;
  }
  r[x.size()] = (uint32_t)c;
  norm(r);
  return r;
}

// a - b, requires a >= b.
inline Limbs sub(const Limbs &a, const Limbs &b) {
  if (cmp(a, b) < 0) throw std::runtime_error("negative difference");
  Limbs r(a.size(), 0u);
  int64_t br = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    int64_t d = (int64_t)a[i] - (i < b.size() ? b[i] : 0u) - br;
    br = d < 0;
    r[i] = (uint32_t)(d + (br ? (1LL << 32) : 0));
  }
  norm(r);
  return r;
}

inline Limbs mul(const Limbs &a, const Limbs &b) {
  if (a.empty() || b.empty()) return {};
  Limbs r(a.size() + b.size(), 0u);
  for (size_t i = 0; i < a.size(); ++i) {
    uint64_t c = 0;
    for (size_t j = 0; j < b.size(); ++j) {
      c += (uint64_t)a[i] * b[j] + r[i + j];
      r[i + j] = (uint32_t)c;
      c >>= 32;
    }
    r[i + b.size()] = (uint32_t)c;
  }
  norm(r);
  return r;
}

inline Limbs shl(const Limbs &a, size_t s) {
  if (a.empty()) return {};
  size_t w = s / 32, b = s % 32;
  Limbs r(a.size() + w + 1, 0u);
  for (size_t i = 0; i < a.size(); ++i) {
    r[i + w] |= a[i] << b;
    if (b) r[i + w + 1] |= a[i] >> (32 - b);
  }
  norm(r);
  return r;
}

// Low `bits` bits of a (a mod 2^bits).
inline Limbs low_bits(const Limbs &a, size_t bits) {
  size_t w = (bits + 31) / 32;
  Limbs r(a.begin(), a.begin() + std::min(w, a.size()));
  if (bits % 32 && r.size() == w) r[w - 1] &= (1u << (bits % 32)) - 1;
  norm(r);
  return r;
}

// Knuth, TAOCP vol. 2, 4.3.1 Algorithm D: quotient and remainder of a / b.
inline void divmod(const Limbs &a, const Limbs &b, Limbs *q, Limbs *r) {
  if (b.empty()) throw std::runtime_error("division by zero");
  if (cmp(a, b) < 0) {
    if (q) q->clear();
    if (r) *r = a;
    return;
  }
  if (b.size() == 1) {
    Limbs qq(a.size(), 0u);
    uint64_t rem = 0;
    for (size_t i = a.size(); i-- > 0;) {
      uint64_t cur = (rem << 32) | a[i];
      qq[i] = (uint32_t)(cur / b[0]);
      rem = cur % b[0];
    }
    norm(qq);
    if (q) *q = qq;
    if (r) *r = from_u64(rem);
    return;
  }
  const size_t n = b.size(), m = a.size() - n;
  const int s = __builtin_clz(b.back());
  Limbs v(n, 0u), u(a.size() + 1, 0u);
  for (size_t i = n; i-- > 0;) v[i] = (b[i] << s) | (s && i ? b[i - 1] >> (32 - s) : 0u);
  u[a.size()] = s ? a.back() >> (32 - s) : 0u;
  for (size_t i = a.size(); i-- > 0;) u[i] = (a[i] << s) | (s && i ? a[i - 1] >> (32 - s) : 0u);
  Limbs qq(m + 1, 0u);
  for (size_t j = m + 1; j-- > 0;) {
    uint64_t num = ((uint64_t)u[j + n] << 32) | u[j + n - 1];
    uint64_t qhat = num / v[n - 1], rhat = num % v[n - 1];
    while (qhat >= (1ULL << 32) || qhat * v[n - 2] > ((rhat << 32) | u[j + n - 2])) {
      --qhat;
      rhat += v[n - 1];
      if (rhat >= (1ULL << 32)) break;
    }
    int64_t borrow = 0;
    uint64_t carry = 0;
    for (size_t i = 0; i < n; ++i) {
      uint64_t p = qhat * v[i] + carry;
      carry = p >> 32;
      int64_t t = (int64_t)u[i + j] - (int64_t)(uint32_t)p - borrow;
      borrow = t < 0;
      u[i + j] = (uint32_t)t;
    }
    int64_t t = (int64_t)u[j + n] - (int64_t)carry - borrow;
    borrow = t < 0;
    u[j + n] = (uint32_t)t;
    if (borrow) {  // qhat was one too large: add v back
      --qhat;
      uint64_t c = 0;
      for (size_t i = 0; i < n; ++i) {
        c += (uint64_t)u[i + j] + v[i];
        u[i + j] = (uint32_t)c;
        c >>= 32;
      }
      u[j + n] += (uint32_t)c;
    }
    qq[j] = (uint32_t)qhat;
  }
  norm(qq);
  if (q) *q = qq;
  if (r) {
    Limbs rr(n, 0u);
    for (size_t i = 0; i < n; ++i) rr[i] = (u[i] >> s) | (s && i + 1 <= n ? (uint32_t)((uint64_t)u[i + 1] << (32 - s)) : 0u);
    norm(rr);
    *r = rr;
  }
}

inline Limbs mod(const Limbs &a, const Limbs &m) {
  Limbs r;
  divmod(a, m, nullptr, &r);
  return r;
}
inline Limbs mulmod(const Limbs &a, const Limbs &b, const Limbs &m) { return mod(mul(a, b), m); }

inline Limbs powmod(const Limbs &base, const Limbs &e, const Limbs &m) {
  Limbs r = mod(from_u64(1), m), b = mod(base, m);
  for (size_t i = bit_length(e); i-- > 0;) {
    r = mulmod(r, r, m);
    if (bit(e, i)) r = mulmod(r, b, m);
  }
  return r;
}

inline Limbs gcd(Limbs a, Limbs b) {
  while (!b.empty()) {
    Limbs r = mod(a, b);
    a = std::move(b);
    b = std::move(r);
  }
  return a;
}

// Inverse of a modulo m (gcd(a, m) = 1) by the extended Euclidean algorithm
// with non-negative coefficients tracked modulo m.
inline Limbs invmod(const Limbs &a, const Limbs &m) {
  Limbs r0 = m, r1 = mod(a, m), t0, t1 = from_u64(1);
  while (!r1.empty()) {
    Limbs q, r2;
    divmod(r0, r1, &q, &r2);
    // t2 = t0 - q t1 (mod m)
    Limbs qt = mod(mul(q, t1), m);
    Limbs t2 = cmp(t0, qt) >= 0 ? sub(t0, qt) : sub(add(t0, m), qt);
    r0 = std::move(r1);
    r1 = std::move(r2);
    t0 = std::move(t1);
    t1 = std::move(t2);
  }
  if (cmp(r0, from_u64(1)) != 0) throw std::runtime_error("not invertible");
  return t0;
}

// -m^-1 mod 2^32 for odd m (Newton iteration).
inline uint32_t neg_inv32(uint32_t m0) {
  uint32_t x = m0;  // correct to 3 bits
  for (int i = 0; i < 5; ++i) x *= 2u - m0 * x;
  return 0u - x;
}

// m^-1 mod 2^bits for odd m (Newton iteration on big integers).
inline Limbs inv_pow2(const Limbs &m, size_t bits) {
  Limbs x = from_u64(1);
  size_t prec = 1;
  while (prec < bits) {
    prec = std::min(2 * prec, bits);
    // x = x (2 - m x) mod 2^prec
    Limbs mx = low_bits(mul(low_bits(m, prec), x), prec);
    Limbs two_minus = sub(shl(from_u64(1), prec + 1), mx);  // 2^(prec+1) - mx >= 0
    x = low_bits(mul(x, add(two_minus, from_u64(2))), prec);
    // (2^(prec+1) + 2 - mx) = 2 - mx mod 2^prec
  }
  return low_bits(x, bits);
}

// ------------------------------------------------------------------ keygen
inline uint64_t splitmix64_word(uint64_t seed, uint64_t index) {
  uint64_t z = seed + (index + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

inline const std::vector<uint32_t> &small_odd_primes() {
  static std::vector<uint32_t> ps = [] {
    std::vector<uint32_t> v;
    for (uint32_t x = 3; x < 2000; x += 2) {
      bool pr = true;
      for (uint32_t d = 3; d * d <= x; d += 2)
        if (x % d == 0) { pr = false; break; }
      if (pr) v.push_back(x);
    }
    return v;
  }();
  return ps;
}

inline uint32_t mod_small(const Limbs &a, uint32_t d) {
  uint64_t r = 0;
  for (size_t i = a.size(); i-- > 0;) r = ((r << 32) | a[i]) % d;
  return (uint32_t)r;
}

inline bool is_probable_prime(const Limbs &x) {
  static const uint32_t bases[40] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43,
                                     47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97, 101, 103,
                                     107, 109, 113, 127, 131, 137, 139, 149, 151, 157, 163,
                                     167, 173};
  if (bit_length(x) <= 32) {
    uint32_t v = x.empty() ? 0 : x[0];
    if (v < 2) return false;
    for (uint32_t d = 2; (uint64_t)d * d <= v; ++d)
      if (v % d == 0) return false;
    return true;
  }
  if (!is_odd(x)) return false;
  for (uint32_t p : small_odd_primes())
    if (mod_small(x, p) == 0) return false;
  Limbs xm1 = sub(x, from_u64(1)), d = xm1;
  size_t s = 0;
  while (!is_odd(d)) {
    d = Limbs(d);
    // shift right by one bit
    for (size_t i = 0; i < d.size(); ++i) d[i] = (d[i] >> 1) | (i + 1 < d.size() ? d[i + 1] << 31 : 0u);
    norm(d);
    ++s;
  }
  for (uint32_t a : bases) {
    Limbs y = powmod(from_u64(a), d, x);
    if (cmp(y, from_u64(1)) == 0 || cmp(y, xm1) == 0) continue;
    bool ok = false;
    for (size_t k = 1; k < s; ++k) {
      y = mulmod(y, y, x);
      if (cmp(y, xm1) == 0) { ok = true; break; }
    }
    if (!ok) return false;
  }
  return true;
}

inline Limbs prime_candidate(uint64_t seed, int which, uint64_t attempt, uint32_t bits) {
  const uint32_t nw = bits / 64;
  const uint64_t base = (which ? (1ULL << 48) : 0ULL) + attempt * nw;
  Limbs x(2 * nw, 0u);
  for (uint32_t j = 0; j < nw; ++j) {
    uint64_t w = splitmix64_word(seed, base + j);
    x[2 * j] = (uint32_t)w;
    x[2 * j + 1] = (uint32_t)(w >> 32);
  }
  x[0] |= 1u;
  x[(bits - 1) / 32] |= 3u << ((bits - 2) % 32);
  norm(x);
  return x;
}

}  // namespace hebn
