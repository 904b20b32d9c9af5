// Host-side derivation of every per-key constant the kernels read, laid out
// in one blob of 32-bit limbs (uploaded once per key).  Host only; no HIP.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "hostbn.hpp"
#include "radix29.hpp"

namespace hekey {

using hebn::Limbs;
constexpr int kWindowBits = 5;

struct Blob {
  std::vector<uint32_t> words;
  // Appends x as exactly `limbs` limbs (plus `pad` zero limbs), 16-byte
  // aligned; returns the offset in limbs.
  size_t put(const Limbs &x, size_t limbs, size_t pad = 0) {
    const size_t off = words.size();
    words.resize(off + limbs + pad, 0u);
    hebn::to_words(x, words.data() + off, limbs);
    words.resize((words.size() + 3) & ~size_t(3), 0u);
    return off;
  }
  // Appends x as exactly `limbs` limbs of 29 bits (one per 32-bit word),
  // 16-byte aligned; throws if it does not fit.
  size_t put29(const Limbs &x, size_t limbs) {
    if (hebn::bit_length(x) > he29::kBits * limbs) throw std::runtime_error("value exceeds 29-bit limbs");
    const size_t off = words.size();
    words.resize(off + limbs, 0u);
    for (size_t i = 0; i < limbs; ++i) {
      uint32_t v = 0;
      for (int k = 0; k < he29::kBits; ++k) v |= (uint32_t)hebn::bit(x, he29::kBits * i + k) << k;
      words[off + i] = v;
    }
    words.resize((words.size() + 3) & ~size_t(3), 0u);
    return off;
  }
};

struct ModOff {  // Montgomery modulus N of S limbs, R = 2^(32 S)
  size_t N, R1, R2, R3, R4;
  uint32_t ninv;
  // radix-2^29 form per variant: N, R mod N and R^2 mod N with R = 2^(29 S29)
  size_t N29[he29::kVariants], R1_29[he29::kVariants], R2_29[he29::kVariants];
};
struct ExpOff {
  size_t e;
  int nwin;
  size_t ops;  // sliding-window schedule (see sliding_schedule)
  int nops;
};

// Sliding-window schedule of e >= 1 with windows of up to kSlideBits bits
// whose lowest bit is 1 (Koc 1995, left to right): the first op loads the
// odd power x^(2 k + 1) of its window (k in bits 0..7); every later op is
// `nsq` squarings (bits 8..31) and then a multiplication by the odd power
// of its window, or no multiplication when k = kSlideNoMul (the trailing
// zero bits).  Evaluating e' = 2 k0 + 1, then e' = e' 2^nsq + (2 k + 1) per
// op rebuilds e.  Empty for e = 0.
constexpr int kSlideBits = 6;
constexpr uint32_t kSlideNoMul = 0xFF;
inline std::vector<uint32_t> sliding_schedule(const Limbs &e) {
  std::vector<uint32_t> ops;
  int i = (int)hebn::bit_length(e) - 1;
  uint32_t pend = 0;
  bool first = true;
  while (i >= 0) {
    if (!hebn::bit(e, (size_t)i)) {
      ++pend;
      --i;
      continue;
    }
    int j = std::max(i - kSlideBits + 1, 0);
    while (!hebn::bit(e, (size_t)j)) ++j;
    uint32_t val = 0;
    for (int b = i; b >= j; --b) val = (val << 1) | (uint32_t)hebn::bit(e, (size_t)b);
    const uint32_t k = (val - 1) >> 1;
    ops.push_back(first ? k : (((pend + (uint32_t)(i - j + 1)) << 8) | k));
    first = false;
    pend = 0;
    i = j - 1;
  }
  if (pend) ops.push_back((pend << 8) | kSlideNoMul);
  return ops;
}
struct PrimeOff {
  ModOff P, P2;
  ExpOff e_enc, e_lift, e_dec;
  size_t QR_P, PR_P2, Pinv, hR_P;
};
struct KeyConsts {
  Blob blob;
  ModOff n, n2;
  ExpOff e_n;
  size_t nR_n2 = 0, half = 0;
  PrimeOff pr[2]{};
  size_t Cq = 0, q2R_n2 = 0, qinv_p = 0, qR_n = 0;
};

inline Limbs pow2(size_t e) { return hebn::shl(hebn::from_u64(1), e); }

inline ModOff put_mod(Blob &b, const Limbs &N, size_t S) {
  ModOff m;
  const Limbs R1 = hebn::mod(pow2(32 * S), N);
  const Limbs R2 = hebn::mulmod(R1, R1, N);
  const Limbs R3 = hebn::mulmod(R2, R1, N);
  const Limbs R4 = hebn::mulmod(R3, R1, N);
  m.N = b.put(N, S);
  m.R1 = b.put(R1, S);
  m.R2 = b.put(R2, S);
  m.R3 = b.put(R3, S);
  m.R4 = b.put(R4, S);
  m.ninv = hebn::neg_inv32(N[0]);
  for (int v = 0; v < he29::kVariants; ++v) {
    const size_t S29 = (size_t)he29::limbs((int)S, v);
    const Limbs Q1 = hebn::mod(pow2(he29::kBits * S29), N);
    m.N29[v] = b.put29(N, S29);
    m.R1_29[v] = b.put29(Q1, S29);
    m.R2_29[v] = b.put29(hebn::mulmod(Q1, Q1, N), S29);
  }
  return m;
}

inline ExpOff put_exp(Blob &b, const Limbs &e, size_t limbs) {
  ExpOff x;
  x.e = b.put(e, limbs, 1);
  const size_t bits = std::max<size_t>(hebn::bit_length(e), 1);
  x.nwin = (int)((bits + kWindowBits - 1) / kWindowBits);
  const std::vector<uint32_t> ops = sliding_schedule(e);
  x.nops = (int)ops.size();
  x.ops = b.words.size();
  b.words.insert(b.words.end(), ops.begin(), ops.end());
  b.words.resize((b.words.size() + 3) & ~size_t(3), 0u);
  return x;
}

// Constants of prime P (other prime Q) for the CRT paths; S_P limbs per prime.
inline PrimeOff put_prime(Blob &b, const Limbs &P, const Limbs &Q, const Limbs &n, size_t SP) {
  PrimeOff o;
  const Limbs one = hebn::from_u64(1);
  const Limbs P2 = hebn::mul(P, P);
  o.P = put_mod(b, P, SP);
  o.P2 = put_mod(b, P2, 2 * SP);
  const Limbs Pm1 = hebn::sub(P, one);
  o.e_enc = put_exp(b, hebn::mod(Q, Pm1), SP);
  o.e_lift = put_exp(b, P, SP);
  o.e_dec = put_exp(b, Pm1, SP);
  const Limbs RP = hebn::mod(pow2(32 * SP), P);
  const Limbs RP2 = hebn::mod(pow2(64 * SP), P2);
  o.QR_P = b.put(hebn::mulmod(Q, RP, P), SP);
  o.PR_P2 = b.put(hebn::mulmod(P, RP2, P2), 2 * SP);
  o.Pinv = b.put(hebn::inv_pow2(P, 32 * SP), SP);
  // h_P = L_P(g^(P-1) mod P^2)^-1 mod P with g = n + 1, L_P(x) = (x - 1) / P
  const Limbs gp = hebn::powmod(hebn::add(n, one), Pm1, P2);
  Limbs Lp;
  hebn::divmod(hebn::sub(gp, one), P, &Lp, nullptr);
  o.hR_P = b.put(hebn::mulmod(hebn::invmod(Lp, P), RP, P), SP);
  return o;
}

// All constants of a key of n_bits bits (L = n_bits / 32 limbs of n).
inline KeyConsts derive(uint32_t n_bits, const Limbs &n, const Limbs &p, const Limbs &q, bool priv) {
  KeyConsts k;
  const size_t L = n_bits / 32, SP = L / 2;
  const Limbs one = hebn::from_u64(1);
  const Limbs n2 = hebn::mul(n, n);
  Blob &b = k.blob;
  k.n = put_mod(b, n, L);
  k.n2 = put_mod(b, n2, 2 * L);
  k.e_n = put_exp(b, n, L);
  const Limbs Rn2 = hebn::mod(pow2(64 * L), n2);
  const Limbs Rn = hebn::mod(pow2(32 * L), n);
  k.nR_n2 = b.put(hebn::mulmod(n, Rn2, n2), 2 * L);
  Limbs h = hebn::add(n, one);  // (n + 1) / 2
  for (size_t i = 0; i < h.size(); ++i) h[i] = (h[i] >> 1) | (i + 1 < h.size() ? h[i + 1] << 31 : 0u);
  hebn::norm(h);
  k.half = b.put(h, L);
  if (priv) {
    k.pr[0] = put_prime(b, p, q, n, SP);
    k.pr[1] = put_prime(b, q, p, n, SP);
    const Limbs p2 = hebn::mul(p, p), q2 = hebn::mul(q, q);
    const Limbs Rp2 = hebn::mod(pow2(32 * L), p2);
    k.Cq = b.put(hebn::mulmod(hebn::invmod(q2, p2), Rp2, p2), L);
    k.q2R_n2 = b.put(hebn::mulmod(q2, Rn2, n2), 2 * L);
    k.qinv_p = b.put(hebn::invmod(q, p), SP);
    k.qR_n = b.put(hebn::mulmod(q, Rn, n), L);
  }
  return k;
}

}  // namespace hekey
