// Wave-cooperative multiprecision Montgomery arithmetic for gfx950.
//
// One big integer of S = 16 K little-endian 32-bit limbs lives in a "group"
// of 16 consecutive lanes (one DPP row): lane l holds limbs l*K .. l*K+K-1 in
// VGPRs.  A wave64 therefore works on four independent integers at once, and
// every cross-lane step of the arithmetic is a DPP row operation (shift by one
// lane, broadcast of lane 0 or 15 of the row) or one wave-wide ballot.
//
// Montgomery product (CIOS: for each limb a_i of the multiplier, add a_i * b,
// pick the quotient digit that clears the lowest limb, add q * N, shift down
// one limb).  The multiplier's limbs are read from LDS with one address per
// group, so the 16 lanes get a broadcast; the multiplicand b and the modulus
// N stay in registers.  Carries between lanes are deferred: each lane keeps a
// small pending word for the column just above its limbs, which the shift
// hands to the lane's own top limb on the next step, so no step waits on a
// cross-lane carry chain.  The final carry resolution and the conditional
// subtraction use a ballot carry-lookahead over the 16 lanes.
//
// Every function here must be called by all 64 lanes of the wave (ballots and
// DPP read all of them); callers predicate results, never control flow.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace he {

constexpr int kGroupLanes = 16;
constexpr int kGroupsPerWave = 4;
constexpr int kWindow = 5;                 // fixed-window exponentiation width
constexpr int kTable = 1 << kWindow;       // entries per window table

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t glane() { return __lane_id() & 15u; }

// ---- DPP row operations (rows of 16 lanes) --------------------------------
// row_newbcast:0 / :15 -- every lane of the row reads lane 0 / lane 15.
__device__ __forceinline__ uint32_t bcast_first(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t bcast_last(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x15F, 0xF, 0xF, false);
}
// row_shl:1 -- lane l reads lane l+1 of its row; lane 15 reads 0.
__device__ __forceinline__ uint32_t from_next(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x101, 0xF, 0xF, true);
}
// row_shr:1 -- lane l reads lane l-1 of its row; lane 0 reads 0.
__device__ __forceinline__ uint32_t from_prev(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
}

// Carry lookahead across the 16 lanes of every row at once.  gen: the lane
// produces a carry by itself; prop: the lane passes an incoming carry on
// (all its limbs are at their maximum).  Returns the carry into this lane.
// Lane 15 neither sends to the next row nor is allowed to chain into it.
__device__ __forceinline__ bool carry_in(bool gen, bool prop) {
  constexpr uint64_t kRowTop = 0x8000800080008000ull;
  const uint64_t g = __builtin_amdgcn_ballot_w64(gen) & ~kRowTop;
  const uint64_t p = __builtin_amdgcn_ballot_w64(prop) & ~kRowTop;
  const uint64_t c = ((g << 1) + p) ^ p;
  return (c >> lane_id()) & 1ull;
}

// True in every lane of a row iff `v` is true in any lane of the row.
__device__ __forceinline__ bool row_any(bool v) {
  const uint64_t b = __builtin_amdgcn_ballot_w64(v);
  return ((b >> (lane_id() & 48u)) & 0xFFFFull) != 0;
}

// ---- register <-> memory ----------------------------------------------------
template <int K>
__device__ __forceinline__ void ld(uint32_t (&x)[K], const uint32_t *p) {
  p += glane() * K;
  if constexpr (K % 4 == 0) {
#pragma unroll
    for (int j = 0; j < K; j += 4) {
      uint4 v = *reinterpret_cast<const uint4 *>(p + j);
      x[j] = v.x; x[j + 1] = v.y; x[j + 2] = v.z; x[j + 3] = v.w;
    }
  } else if constexpr (K == 2) {
    uint2 v = *reinterpret_cast<const uint2 *>(p);
    x[0] = v.x; x[1] = v.y;
  } else {
    x[0] = p[0];
  }
}
template <int K>
__device__ __forceinline__ void st(uint32_t *p, const uint32_t (&x)[K]) {
  p += glane() * K;
  if constexpr (K % 4 == 0) {
#pragma unroll
    for (int j = 0; j < K; j += 4)
      *reinterpret_cast<uint4 *>(p + j) = make_uint4(x[j], x[j + 1], x[j + 2], x[j + 3]);
  } else if constexpr (K == 2) {
    *reinterpret_cast<uint2 *>(p) = make_uint2(x[0], x[1]);
  } else {
    p[0] = x[0];
  }
}
template <int K>
__device__ __forceinline__ void set_zero(uint32_t (&x)[K]) {
#pragma unroll
  for (int j = 0; j < K; ++j) x[j] = 0;
}
template <int K>
__device__ __forceinline__ void set_small(uint32_t (&x)[K], uint32_t v) {
  set_zero(x);
  if (glane() == 0) x[0] = v;
}
template <int K>
__device__ __forceinline__ void copy(uint32_t (&d)[K], const uint32_t (&s)[K]) {
#pragma unroll
  for (int j = 0; j < K; ++j) d[j] = s[j];
}
template <int K>
__device__ __forceinline__ void select(uint32_t (&d)[K], bool c, const uint32_t (&a)[K],
                                       const uint32_t (&b)[K]) {
#pragma unroll
  for (int j = 0; j < K; ++j) d[j] = c ? a[j] : b[j];
}

// ---- modulus context --------------------------------------------------------
template <int K>
struct Mod {
  uint32_t n[K];   // this lane's limbs of N
  uint32_t ninv;   // -N^-1 mod 2^32
};
template <int K>
__device__ __forceinline__ Mod<K> load_mod(const uint32_t *N, uint32_t ninv) {
  Mod<K> m;
  ld<K>(m.n, N);
  m.ninv = ninv;
  return m;
}

// ---- carry resolution and reduction ----------------------------------------
// Turns the redundant accumulator (limbs + pending word per lane; lane 15's
// pending word is the top limb S) into plain limbs; returns the top word in
// lane 15 (0 or 1 for a Montgomery result below 2N < 2^(32S+1)).
template <int K>
__device__ __forceinline__ uint32_t resolve(uint32_t (&t)[K], uint32_t pc) {
  const uint32_t in = from_prev(pc);
  unsigned c;
  t[0] = __builtin_addc(t[0], in, 0u, &c);
#pragma unroll
  for (int j = 1; j < K; ++j) t[j] = __builtin_addc(t[j], 0u, c, &c);
  const bool gen = c;
  bool prop = true;
#pragma unroll
  for (int j = 0; j < K; ++j) prop = prop && (t[j] == 0xFFFFFFFFu);
  unsigned c2 = carry_in(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) t[j] = __builtin_addc(t[j], 0u, c2, &c2);
  return pc + (uint32_t)gen + c2;
}

// If top:t >= N then t -= N (t < 2N on entry).  Result in [0, N).
template <int K>
__device__ __forceinline__ void cond_sub(uint32_t (&t)[K], uint32_t top, const Mod<K> &M) {
  uint32_t d[K];
  unsigned b;
  d[0] = __builtin_subc(t[0], M.n[0], 0u, &b);
#pragma unroll
  for (int j = 1; j < K; ++j) d[j] = __builtin_subc(t[j], M.n[j], b, &b);
  const bool gen = b;
  bool prop = true;
#pragma unroll
  for (int j = 0; j < K; ++j) prop = prop && (d[j] == 0u);
  unsigned b2 = carry_in(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) d[j] = __builtin_subc(d[j], 0u, b2, &b2);
  const bool borrow_out = gen || b2;
  const bool ge = bcast_last((top != 0u || !borrow_out) ? 1u : 0u) != 0u;
  select(t, ge, d, t);
}

// ---- Montgomery product -----------------------------------------------------
// One CIOS step for multiplier limb ai.
template <int K>
__device__ __forceinline__ void mont_step(uint32_t (&acc)[K], uint32_t &pc, uint32_t ai,
                                          const uint32_t (&b)[K], const Mod<K> &M) {
  uint64_t x[K];
#pragma unroll
  for (int j = 0; j < K; ++j) x[j] = (uint64_t)ai * b[j] + acc[j];
  uint32_t u[K];
  unsigned c = 0;
  u[0] = (uint32_t)x[0];
#pragma unroll
  for (int j = 1; j < K; ++j) u[j] = __builtin_addc((uint32_t)x[j], (uint32_t)(x[j - 1] >> 32), c, &c);
  const uint32_t top1 = (uint32_t)(x[K - 1] >> 32) + c;
  const uint32_t q = bcast_first(u[0] * M.ninv);
  uint64_t y[K];
#pragma unroll
  for (int j = 0; j < K; ++j) y[j] = (uint64_t)q * M.n[j] + u[j];
  uint32_t v[K];
  unsigned c2 = 0;
  v[0] = (uint32_t)y[0];
#pragma unroll
  for (int j = 1; j < K; ++j) v[j] = __builtin_addc((uint32_t)y[j], (uint32_t)(y[j - 1] >> 32), c2, &c2);
  const uint32_t top2 = (uint32_t)(y[K - 1] >> 32) + c2;
  const uint32_t nb = from_next(v[0]);
  const uint64_t s = (uint64_t)nb + top1 + top2 + pc;
#pragma unroll
  for (int j = 0; j + 1 < K; ++j) acc[j] = v[j + 1];
  acc[K - 1] = (uint32_t)s;
  pc = (uint32_t)(s >> 32);
}

template <int K>
__device__ __forceinline__ void lds_limbs(uint32_t (&a)[K], const uint32_t *p) {
  if constexpr (K % 4 == 0) {
#pragma unroll
    for (int j = 0; j < K; j += 4) {
      uint4 v = *reinterpret_cast<const uint4 *>(p + j);
      a[j] = v.x; a[j + 1] = v.y; a[j + 2] = v.z; a[j + 3] = v.w;
    }
  } else if constexpr (K == 2) {
    uint2 v = *reinterpret_cast<const uint2 *>(p);
    a[0] = v.x; a[1] = v.y;
  } else {
    a[0] = p[0];
  }
}

// t = a * b * 2^(-32 S) mod N with a taken from this group's LDS copy
// (S limbs, a < 2^(32 S)) and b < N in registers.  t may alias b.
template <int K>
__device__ __forceinline__ void mont_mul_lds(uint32_t (&t)[K], const uint32_t *a_lds,
                                             const uint32_t (&b)[K], const Mod<K> &M) {
  uint32_t acc[K];
  set_zero(acc);
  uint32_t pc = 0;
#pragma unroll 1
  for (int i0 = 0; i0 < kGroupLanes * K; i0 += K) {
    uint32_t av[K];
    lds_limbs<K>(av, a_lds + i0);
#pragma unroll
    for (int s = 0; s < K; ++s) mont_step<K>(acc, pc, av[s], b, M);
  }
  const uint32_t top = resolve<K>(acc, pc);
  cond_sub<K>(acc, top, M);
  copy(t, acc);
}

// t = a * b * 2^(-32 S) mod N, both operands in registers; `lds` is this
// group's S-limb scratch row.  t may alias a or b.
template <int K>
__device__ __forceinline__ void mont_mul(uint32_t (&t)[K], const uint32_t (&a)[K],
                                         const uint32_t (&b)[K], const Mod<K> &M, uint32_t *lds) {
  st<K>(lds, a);
  __builtin_amdgcn_wave_barrier();
  mont_mul_lds<K>(t, lds, b, M);
  __builtin_amdgcn_wave_barrier();
}

// ---- modular add / sub --------------------------------------------------------
// t = x + y mod N for x, y < N.
template <int K>
__device__ __forceinline__ void add_mod(uint32_t (&t)[K], const uint32_t (&x)[K],
                                        const uint32_t (&y)[K], const Mod<K> &M) {
  unsigned c;
  t[0] = __builtin_addc(x[0], y[0], 0u, &c);
#pragma unroll
  for (int j = 1; j < K; ++j) t[j] = __builtin_addc(x[j], y[j], c, &c);
  const bool gen = c;
  bool prop = true;
#pragma unroll
  for (int j = 0; j < K; ++j) prop = prop && (t[j] == 0xFFFFFFFFu);
  unsigned c2 = carry_in(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) t[j] = __builtin_addc(t[j], 0u, c2, &c2);
  const uint32_t top = (uint32_t)gen + c2;  // meaningful in lane 15
  cond_sub<K>(t, top, M);
}

// t = x + y (no reduction); returns the carry out of the top (lane 15).
template <int K>
__device__ __forceinline__ uint32_t add_plain(uint32_t (&t)[K], const uint32_t (&x)[K],
                                              const uint32_t (&y)[K]) {
  unsigned c;
  t[0] = __builtin_addc(x[0], y[0], 0u, &c);
#pragma unroll
  for (int j = 1; j < K; ++j) t[j] = __builtin_addc(x[j], y[j], c, &c);
  const bool gen = c;
  bool prop = true;
#pragma unroll
  for (int j = 0; j < K; ++j) prop = prop && (t[j] == 0xFFFFFFFFu);
  unsigned c2 = carry_in(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) t[j] = __builtin_addc(t[j], 0u, c2, &c2);
  return (uint32_t)gen + c2;
}

// t = x - y (mod 2^(32S)); returns true in lane 15 iff x < y.
template <int K>
__device__ __forceinline__ bool sub_plain(uint32_t (&t)[K], const uint32_t (&x)[K],
                                          const uint32_t (&y)[K]) {
  unsigned b;
  t[0] = __builtin_subc(x[0], y[0], 0u, &b);
#pragma unroll
  for (int j = 1; j < K; ++j) t[j] = __builtin_subc(x[j], y[j], b, &b);
  const bool gen = b;
  bool prop = true;
#pragma unroll
  for (int j = 0; j < K; ++j) prop = prop && (t[j] == 0u);
  unsigned b2 = carry_in(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) t[j] = __builtin_subc(t[j], 0u, b2, &b2);
  return gen || b2;
}

// t = x - y mod N for x, y < N.
template <int K>
__device__ __forceinline__ void sub_mod(uint32_t (&t)[K], const uint32_t (&x)[K],
                                        const uint32_t (&y)[K], const Mod<K> &M) {
  const bool neg = bcast_last(sub_plain<K>(t, x, y) ? 1u : 0u) != 0u;
  uint32_t w[K];
  add_plain<K>(w, t, M.n);
  select(t, neg, w, t);
}

// ---- low-half product ----------------------------------------------------------
// t = a * b mod 2^(32 S), with a from this group's LDS copy and b in registers.
// (Used for the exact division x / P = x * P^-1 mod 2^(32 S) when P | x.)
template <int K>
__device__ __forceinline__ void mul_lo_lds(uint32_t (&t)[K], const uint32_t *a_lds,
                                           const uint32_t (&b)[K]) {
  uint32_t acc[K], bs[K];
  set_zero(acc);
  copy(bs, b);
  uint32_t cin = 0;  // pending carry into this lane's lowest column
#pragma unroll 1
  for (int i0 = 0; i0 < kGroupLanes * K; i0 += K) {
    uint32_t av[K];
    lds_limbs<K>(av, a_lds + i0);
#pragma unroll
    for (int s = 0; s < K; ++s) {
      // acc += a_i * (b << 32 i): bs holds b shifted up by i limbs.
      uint64_t x[K];
      x[0] = (uint64_t)av[s] * bs[0] + ((uint64_t)acc[0] + cin);
#pragma unroll
      for (int j = 1; j < K; ++j) x[j] = (uint64_t)av[s] * bs[j] + acc[j];
      unsigned c = 0;
      acc[0] = (uint32_t)x[0];
#pragma unroll
      for (int j = 1; j < K; ++j) acc[j] = __builtin_addc((uint32_t)x[j], (uint32_t)(x[j - 1] >> 32), c, &c);
      const uint32_t top = (uint32_t)(x[K - 1] >> 32) + c;
      cin = from_prev(top);
      // shift bs up by one limb for the next multiplier limb
      const uint32_t down = from_prev(bs[K - 1]);
#pragma unroll
      for (int j = K - 1; j > 0; --j) bs[j] = bs[j - 1];
      bs[0] = down;
    }
  }
  // fold the last pending carries in (anything past limb S-1 is dropped)
  unsigned c;
  acc[0] = __builtin_addc(acc[0], cin, 0u, &c);
#pragma unroll
  for (int j = 1; j < K; ++j) acc[j] = __builtin_addc(acc[j], 0u, c, &c);
  const bool gen = c;
  bool prop = true;
#pragma unroll
  for (int j = 0; j < K; ++j) prop = prop && (acc[j] == 0xFFFFFFFFu);
  unsigned c2 = carry_in(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) acc[j] = __builtin_addc(acc[j], 0u, c2, &c2);
  copy(t, acc);
}

// ---- fixed-window exponentiation ----------------------------------------------
// Window digit w (bits 5w .. 5w+4) of an exponent stored as limbs with one
// zero limb of padding.  The exponent is the same for the whole wave, so this
// is scalar work.
__device__ __forceinline__ uint32_t exp_digit(const uint32_t *e, int w) {
  const int bit = kWindow * w;
  const uint64_t v = (uint64_t)e[bit >> 5] | ((uint64_t)e[(bit >> 5) + 1] << 32);
  return (uint32_t)(v >> (bit & 31)) & (kTable - 1);
}

// x <- x^e mod N in Montgomery form (x is the Montgomery form of the base,
// one = R mod N).  Left-to-right fixed 5-bit windows over `nwin` windows; a
// multiplication by the table entry is done for every window, zero digits
// included, so the sequence of operations does not depend on the exponent.
// `tab` is this group's table: kTable entries of S limbs in global memory.
template <int K>
__device__ __forceinline__ void mont_pow(uint32_t (&x)[K], const uint32_t *e, int nwin,
                                         uint32_t *tab, const uint32_t (&one)[K],
                                         const Mod<K> &M, uint32_t *lds) {
  constexpr int S = kGroupLanes * K;
  st<K>(tab, one);
  st<K>(tab + S, x);
  uint32_t cur[K];
  copy(cur, x);
#pragma unroll 1
  for (int d = 2; d < kTable; ++d) {
    mont_mul<K>(cur, cur, x, M, lds);
    st<K>(tab + d * S, cur);
  }
  __threadfence_block();
  ld<K>(cur, tab + exp_digit(e, nwin - 1) * S);
#pragma unroll 1
  for (int w = nwin - 2; w >= 0; --w) {
    uint32_t tb[K];
    ld<K>(tb, tab + exp_digit(e, w) * S);
#pragma unroll 1
    for (int s = 0; s < kWindow; ++s) mont_mul<K>(cur, cur, cur, M, lds);
    mont_mul<K>(cur, cur, tb, M, lds);
  }
  copy(x, cur);
}

// Moves an integer between limb layouts through this group's LDS row:
// src has 16*KS limbs (KS per lane), dst gets 16*KD limbs (KD per lane); the
// limbs are taken starting at `first` and limbs beyond the source are zero.
template <int KS, int KD>
__device__ __forceinline__ void relayout(uint32_t (&dst)[KD], const uint32_t (&src)[KS],
                                         uint32_t *lds, int first = 0) {
  constexpr int SS = kGroupLanes * KS;
  st<KS>(lds, src);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < KD; ++j) {
    const int idx = first + (int)glane() * KD + j;
    dst[j] = idx < SS ? lds[idx] : 0u;
  }
  __builtin_amdgcn_wave_barrier();
}

// ---- SplitMix64 counter-based words ------------------------------------------
// The index-th output of SplitMix64 (Steele, Lea & Flood 2014) started from
// state `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t index) {
  uint64_t z = seed + (index + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace he
