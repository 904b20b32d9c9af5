// Wave-cooperative multiprecision Montgomery arithmetic for gfx950.
//
// One big integer of S = G K little-endian 32-bit limbs lives in a "group" of
// G consecutive lanes (G = 16: one DPP row; G = 8: half a row; G = 4: one
// quad; G = 2: half a quad): lane l of the group holds limbs l*K .. l*K+K-1
// in VGPRs.  A wave64
// works on 64/G independent integers at once, and every cross-lane step of the
// arithmetic is a DPP operation (shift by one lane, broadcast of the group's
// first or last lane) or one wave-wide ballot.  Smaller groups give each lane
// more limbs, which amortises the per-step cross-lane work over more
// multiply-adds; larger groups keep more integers' worth of registers free.
//
// Montgomery product (CIOS: for each limb a_i of the multiplier, add a_i * b,
// pick the quotient digit that clears the lowest limb, add q * N, shift down
// one limb).  The multiplier's limbs are read from LDS with one address per
// group, so the lanes of a group get a broadcast; the multiplicand b and the modulus
// N stay in registers.  The accumulator is kept as per-column 64-bit words
// with overflow counters (see "column accumulators" below), so a product costs
// one multiply-add and one carry add, and only the lowest column is folded per
// step; no step waits on a cross-lane carry chain.  The final carry
// resolution and the conditional subtraction use a ballot carry-lookahead over
// the lanes of the group.
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
// The lane's index in its group.  Opaque to the optimiser (an empty volatile
// asm), so that addresses derived from it are recomputed where they are used
// instead of being hoisted out of the persistent loops, where the kernels
// have no registers to keep them and would spill them.
template <int G = 16>
__device__ __forceinline__ uint32_t glane() {
  uint32_t l = __lane_id() & (G - 1u);
  asm volatile("" : "+v"(l));
  return l;
}

// ---- DPP group operations -------------------------------------------------
// Every lane of the group reads the group's first / last lane.
//   G = 16: row_newbcast:0 / :15;  G = 8: row_newbcast:0 on banks 0-1 and :8
//   on banks 2-3 (resp. :7 / :15);  G = 4: quad_perm [0,0,0,0] / [3,3,3,3];
//   G = 2: quad_perm [0,0,2,2] / [1,1,3,3].
// Full row and bank masks with every lane reading a valid source lane write
// every lane, so these use mov_dpp (no "old" value to set up first).
template <int G = 16>
__device__ __forceinline__ uint32_t bcast_first(uint32_t v) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16, "group width");
  if constexpr (G == 16) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x150, 0xF, 0xF, false);
  } else if constexpr (G == 8) {
    const int t = __builtin_amdgcn_update_dpp(0, (int)v, 0x150, 0xF, 0x3, false);
    return (uint32_t)__builtin_amdgcn_update_dpp(t, (int)v, 0x158, 0xF, 0xC, false);
  } else if constexpr (G == 4) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x00, 0xF, 0xF, false);
  } else {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xA0, 0xF, 0xF, false);  // quad_perm [0,0,2,2]
  }
}
template <int G = 16>
__device__ __forceinline__ uint32_t bcast_last(uint32_t v) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16, "group width");
  if constexpr (G == 16) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x15F, 0xF, 0xF, false);
  } else if constexpr (G == 8) {
    const int t = __builtin_amdgcn_update_dpp(0, (int)v, 0x157, 0xF, 0x3, false);
    return (uint32_t)__builtin_amdgcn_update_dpp(t, (int)v, 0x15F, 0xF, 0xC, false);
  } else if constexpr (G == 4) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xFF, 0xF, 0xF, false);
  } else {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xF5, 0xF, 0xF, false);  // quad_perm [1,1,3,3]
  }
}
// Lane l reads lane l+1 of its group; the group's last lane reads 0
// (row_shl:1 with bound_ctrl, which writes 0 where the source is outside the
// row; for G < 16 the lane that would read across a group edge inside the
// row is cleared).
template <int G = 16>
__device__ __forceinline__ uint32_t from_next(uint32_t v) {
  const uint32_t t = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x101, 0xF, 0xF, true);
  if constexpr (G == 16) return t;
  else return glane<G>() == G - 1 ? 0u : t;
}
// Lane l reads lane l+1 of its group, the group's last lane reads the group's
// first lane (G = 2: quad_perm [1,0,3,2]; G = 4: quad_perm [1,2,3,0]; G = 16:
// row_ror:15).  Used for the one-limb shift of a Montgomery step, where the
// first lane's value is the cleared lowest column and therefore 0, so this
// equals from_next without the edge fix-up.  G = 8 has no 8-lane rotation; it
// uses row_shl:1, whose group-edge lane reads the next group's first lane,
// which in this use holds zero as well (every group clears its own lowest
// column), and the row's last lane reads 0 (bound_ctrl).
template <int G = 16>
__device__ __forceinline__ uint32_t rotate_next(uint32_t v) {
  if constexpr (G == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
  else if constexpr (G == 4) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x39, 0xF, 0xF, false);
  else if constexpr (G == 16) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x12F, 0xF, 0xF, false);
  else return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x101, 0xF, 0xF, true);
}
// Lane l reads lane l-1 of its group; the group's first lane reads 0 (row_shr:1).
template <int G = 16>
__device__ __forceinline__ uint32_t from_prev(uint32_t v) {
  const uint32_t t = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x111, 0xF, 0xF, true);
  if constexpr (G == 16) return t;
  else return glane<G>() == 0 ? 0u : t;
}

template <int G>
constexpr uint64_t group_top_mask() {
  return G == 16 ? 0x8000800080008000ull
                 : (G == 8 ? 0x8080808080808080ull : (G == 4 ? 0x8888888888888888ull : 0xAAAAAAAAAAAAAAAAull));
}

// Carry lookahead across the lanes of every group at once.  gen: the lane
// produces a carry by itself; prop: the lane passes an incoming carry on
// (all its limbs are at their maximum).  Returns the carry into this lane.
// A group's last lane neither sends to the next group nor chains into it.
template <int G = 16>
__device__ __forceinline__ bool carry_in(bool gen, bool prop) {
  constexpr uint64_t kTop = group_top_mask<G>();
  const uint64_t g = __builtin_amdgcn_ballot_w64(gen) & ~kTop;
  const uint64_t p = __builtin_amdgcn_ballot_w64(prop) & ~kTop;
  const uint64_t c = ((g << 1) + p) ^ p;
  return (c >> lane_id()) & 1ull;
}

// True in every lane of a group iff `v` is true in any lane of the group.
template <int G = 16>
__device__ __forceinline__ bool row_any(bool v) {
  const uint64_t b = __builtin_amdgcn_ballot_w64(v);
  return ((b >> (lane_id() & ~(uint32_t)(G - 1))) & ((1ull << G) - 1)) != 0;
}

// ---- register <-> memory ----------------------------------------------------
template <int K, int G = 16>
__device__ __forceinline__ void ld(uint32_t (&x)[K], const uint32_t *p) {
  p += glane<G>() * K;
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
template <int K, int G = 16>
__device__ __forceinline__ void st(uint32_t *p, const uint32_t (&x)[K]) {
  p += glane<G>() * K;
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
template <int K, int G = 16>
__device__ __forceinline__ void set_zero(uint32_t (&x)[K]) {
#pragma unroll
  for (int j = 0; j < K; ++j) x[j] = 0;
}
template <int K, int G = 16>
__device__ __forceinline__ void set_small(uint32_t (&x)[K], uint32_t v) {
  set_zero(x);
  if (glane<G>() == 0) x[0] = v;
}
template <int K, int G = 16>
__device__ __forceinline__ void copy(uint32_t (&d)[K], const uint32_t (&s)[K]) {
#pragma unroll
  for (int j = 0; j < K; ++j) d[j] = s[j];
}
template <int K, int G = 16>
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
template <int K, int G = 16>
__device__ __forceinline__ Mod<K> load_mod(const uint32_t *N, uint32_t ninv) {
  Mod<K> m;
  ld<K, G>(m.n, N);
  m.ninv = ninv;
  return m;
}

// ---- carry resolution and reduction ----------------------------------------
// If top:t >= N then t -= N (t < 2N on entry, top = bits at and above limb S,
// meaningful in the group's last lane).  Result in [0, N).
template <int K, int G = 16>
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
  unsigned b2 = carry_in<G>(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) d[j] = __builtin_subc(d[j], 0u, b2, &b2);
  const bool borrow_out = gen || b2;
  const bool ge = bcast_last<G>((top != 0u || !borrow_out) ? 1u : 0u) != 0u;
  select(t, ge, d, t);
}

// ---- column accumulators ------------------------------------------------------
// The Montgomery accumulator is kept per column as a 64-bit word C plus an
// overflow word O: column c holds V_c = C_c + O_c 2^64 and the accumulator is
// sum_c V_c 2^(32 c).  A product a*b is added to a column by one
// v_mad_u64_u32 (64-bit addend = C, carry-out into a lane mask) and one
// v_addc_co_u32 of that mask into O, so no product needs its high half moved
// to the next column.  The compiler does not form the mad carry-out from C++,
// hence the inline assembly; the K mads come before their K carry adds so
// every carry mask is read at least K-1 VALU instructions after it is written
// (an s_nop covers K <= 2).

// C[j] += a * b[j], O[j] += carry, for 4 columns.
__device__ __forceinline__ void mac4(uint64_t &c0, uint64_t &c1, uint64_t &c2, uint64_t &c3,
                                     uint32_t &o0, uint32_t &o1, uint32_t &o2, uint32_t &o3,
                                     uint32_t a, uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3) {
  uint64_t k0, k1, k2, k3;
  asm("v_mad_u64_u32 %0, %8, %12, %13, %0\n\t"
      "v_mad_u64_u32 %1, %9, %12, %14, %1\n\t"
      "v_mad_u64_u32 %2, %10, %12, %15, %2\n\t"
      "v_mad_u64_u32 %3, %11, %12, %16, %3\n\t"
      "v_addc_co_u32_e64 %4, %8, %4, 0, %8\n\t"
      "v_addc_co_u32_e64 %5, %9, %5, 0, %9\n\t"
      "v_addc_co_u32_e64 %6, %10, %6, 0, %10\n\t"
      "v_addc_co_u32_e64 %7, %11, %7, 0, %11"
      : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3), "+v"(o0), "+v"(o1), "+v"(o2), "+v"(o3),
        "=&s"(k0), "=&s"(k1), "=&s"(k2), "=&s"(k3)
      : "v"(a), "v"(b0), "v"(b1), "v"(b2), "v"(b3));
}
__device__ __forceinline__ void mac2(uint64_t &c0, uint64_t &c1, uint32_t &o0, uint32_t &o1,
                                     uint32_t a, uint32_t b0, uint32_t b1) {
  uint64_t k0, k1;
  asm("v_mad_u64_u32 %0, %4, %6, %7, %0\n\t"
      "v_mad_u64_u32 %1, %5, %6, %8, %1\n\t"
      "s_nop 1\n\t"
      "v_addc_co_u32_e64 %2, %4, %2, 0, %4\n\t"
      "v_addc_co_u32_e64 %3, %5, %3, 0, %5"
      : "+v"(c0), "+v"(c1), "+v"(o0), "+v"(o1), "=&s"(k0), "=&s"(k1)
      : "v"(a), "v"(b0), "v"(b1));
}
__device__ __forceinline__ void mac1(uint64_t &c0, uint32_t &o0, uint32_t a, uint32_t b0) {
  uint64_t k0;
  asm("v_mad_u64_u32 %0, %2, %3, %4, %0\n\t"
      "s_nop 2\n\t"
      "v_addc_co_u32_e64 %1, %2, %1, 0, %2"
      : "+v"(c0), "+v"(o0), "=&s"(k0)
      : "v"(a), "v"(b0));
}

template <int K, int G = 16>
__device__ __forceinline__ void row_mac(uint64_t (&C)[K], uint32_t (&O)[K], uint32_t a,
                                        const uint32_t (&b)[K]) {
  if constexpr (K == 1) {
    mac1(C[0], O[0], a, b[0]);
  } else if constexpr (K == 2) {
    mac2(C[0], C[1], O[0], O[1], a, b[0], b[1]);
  } else {
    static_assert(K % 4 == 0, "K must be 1, 2 or a multiple of 4");
#pragma unroll
    for (int j = 0; j < K; j += 4)
      mac4(C[j], C[j + 1], C[j + 2], C[j + 3], O[j], O[j + 1], O[j + 2], O[j + 3], a, b[j], b[j + 1],
           b[j + 2], b[j + 3]);
  }
}

// Low 32 bits of x * y through the full-rate multiplier.
__device__ __forceinline__ uint32_t mul_lo32(uint32_t x, uint32_t y) {
  uint64_t r, k;
  asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(r), "=s"(k) : "v"(x), "v"(y));
  return (uint32_t)r;
}

// One CIOS step for multiplier limb ai: add ai*b, pick q that clears the
// lowest column, add q*N, divide by 2^32.  The division moves the upper part
// (high word and overflow) of column 0 into column 1 -- the same weight after
// the shift -- and hands the low word of column 0 to the previous lane, whose
// new top column it becomes (lane 0's low word is zero and is dropped).
template <int K, int G = 16>
__device__ __forceinline__ void mont_step(uint64_t (&C)[K], uint32_t (&O)[K], uint32_t ai,
                                          const uint32_t (&b)[K], const Mod<K> &M) {
  row_mac<K>(C, O, ai, b);
  const uint32_t q = bcast_first<G>(mul_lo32((uint32_t)C[0], M.ninv));
  row_mac<K>(C, O, q, M.n);
  const uint32_t lo0 = (uint32_t)C[0], hi0 = (uint32_t)(C[0] >> 32);
  const uint32_t nb = rotate_next<G>(lo0);
  if constexpr (K == 1) {
    // the lane's new column = low word from the next lane + own upper part
    unsigned c;
    const uint32_t l = __builtin_addc(hi0, nb, 0u, &c);
    const uint32_t h = __builtin_addc(O[0], 0u, c, &c);
    C[0] = ((uint64_t)h << 32) | l;
    O[0] = c;
  } else {
    unsigned c;
    const uint32_t l1 = __builtin_addc((uint32_t)C[1], hi0, 0u, &c);
    const uint32_t h1 = __builtin_addc((uint32_t)(C[1] >> 32), O[0], c, &c);
    const uint32_t o1 = O[1] + c;
    C[0] = ((uint64_t)h1 << 32) | l1;
    O[0] = o1;
#pragma unroll
    for (int j = 1; j + 1 < K; ++j) {
      C[j] = C[j + 1];
      O[j] = O[j + 1];
    }
    C[K - 1] = nb;
    O[K - 1] = 0;
  }
}

// Turns the column accumulators into plain limbs t (columns 0..S-1 of the
// group) and returns, in the group's last lane, the part at and above limb S.
template <int K, int G = 16>
__device__ __forceinline__ uint32_t resolve(uint32_t (&t)[K], const uint64_t (&C)[K],
                                            const uint32_t (&O)[K]) {
  // Column c receives lo(C_c), hi(C_{c-1}) and O_{c-2}; the terms of the
  // lane's lowest columns come from the previous lane(s).
  const uint32_t in_hi = from_prev<G>((uint32_t)(C[K - 1] >> 32));
  const uint32_t in_o1 = from_prev<G>(O[K - 1]);
  const uint32_t in_o2 = K >= 2 ? from_prev<G>(O[K >= 2 ? K - 2 : 0]) : from_prev<G>(in_o1);
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t h = j >= 1 ? (uint32_t)(C[j >= 1 ? j - 1 : 0] >> 32) : in_hi;
    const uint32_t o = j >= 2 ? O[j >= 2 ? j - 2 : 0] : (j == 1 ? in_o1 : in_o2);
    const uint64_t s = (uint64_t)(uint32_t)C[j] + h + o + carry;
    t[j] = (uint32_t)s;
    carry = (uint32_t)(s >> 32);
  }
  // the lane's carry (at most 3) goes to the next lane's lowest limb
  const uint32_t cin = from_prev<G>(carry);
  unsigned c;
  t[0] = __builtin_addc(t[0], cin, 0u, &c);
#pragma unroll
  for (int j = 1; j < K; ++j) t[j] = __builtin_addc(t[j], 0u, c, &c);
  const bool gen = c;
  bool prop = true;
#pragma unroll
  for (int j = 0; j < K; ++j) prop = prop && (t[j] == 0xFFFFFFFFu);
  unsigned c2 = carry_in<G>(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) t[j] = __builtin_addc(t[j], 0u, c2, &c2);
  // last lane: everything at and above limb S.  The result is below 2N < 2^(32S+1),
  // so this is 0 or 1; any nonzero part counts.
  const uint32_t top_hi = (uint32_t)(C[K - 1] >> 32);
  const uint32_t top_o2 = K >= 2 ? O[K >= 2 ? K - 2 : 0] : in_o1;
  return (top_hi | top_o2 | O[K - 1]) != 0u ? 1u : (carry + (uint32_t)gen + c2);
}

template <int K, int G = 16>
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
template <int K, int G = 16>
__device__ __forceinline__ void mont_mul_lds(uint32_t (&t)[K], const uint32_t *a_lds,
                                             const uint32_t (&b)[K], const Mod<K> &M) {
  uint64_t C[K];
  uint32_t O[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    C[j] = 0;
    O[j] = 0;
  }
  // U steps per loop iteration (at least 8, and two full rotations of the
  // lane's columns while that fits in registers) so the loop-carried
  // registers rotate back less often.
  constexpr int U = K >= 8 ? K : (K >= 4 ? 2 * K : 8);
  static_assert((G * K) % U == 0, "unroll must divide S");
#pragma unroll 1
  for (int i0 = 0; i0 < G * K; i0 += U) {
    uint32_t av[U];
#pragma unroll
    for (int h = 0; h < U; h += 4) {
      const uint4 v = *reinterpret_cast<const uint4 *>(a_lds + i0 + h);
      av[h] = v.x; av[h + 1] = v.y; av[h + 2] = v.z; av[h + 3] = v.w;
    }
#pragma unroll
    for (int s = 0; s < U; ++s) mont_step<K, G>(C, O, av[s], b, M);
  }
  uint32_t r[K];
  const uint32_t top = resolve<K, G>(r, C, O);
  cond_sub<K, G>(r, top, M);
  copy(t, r);
}

// t = a * b * 2^(-32 S) mod N, both operands in registers; `lds` is this
// group's S-limb scratch row.  t may alias a or b.
template <int K, int G = 16>
__device__ __forceinline__ void mont_mul(uint32_t (&t)[K], const uint32_t (&a)[K],
                                         const uint32_t (&b)[K], const Mod<K> &M, uint32_t *lds) {
  st<K, G>(lds, a);
  __builtin_amdgcn_wave_barrier();
  mont_mul_lds<K, G>(t, lds, b, M);
  __builtin_amdgcn_wave_barrier();
}

// ---- modular add / sub --------------------------------------------------------
// t = x + y mod N for x, y < N.
template <int K, int G = 16>
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
  unsigned c2 = carry_in<G>(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) t[j] = __builtin_addc(t[j], 0u, c2, &c2);
  const uint32_t top = (uint32_t)gen + c2;  // meaningful in the last lane
  cond_sub<K, G>(t, top, M);
}

// t = x + y (no reduction); returns the carry out of the top (last lane).
template <int K, int G = 16>
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
  unsigned c2 = carry_in<G>(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) t[j] = __builtin_addc(t[j], 0u, c2, &c2);
  return (uint32_t)gen + c2;
}

// t = x - y (mod 2^(32S)); returns true in the last lane iff x < y.
template <int K, int G = 16>
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
  unsigned b2 = carry_in<G>(gen, prop);
#pragma unroll
  for (int j = 0; j < K; ++j) t[j] = __builtin_subc(t[j], 0u, b2, &b2);
  return gen || b2;
}

// t = x - y mod N for x, y < N.
template <int K, int G = 16>
__device__ __forceinline__ void sub_mod(uint32_t (&t)[K], const uint32_t (&x)[K],
                                        const uint32_t (&y)[K], const Mod<K> &M) {
  const bool neg = bcast_last<G>(sub_plain<K, G>(t, x, y) ? 1u : 0u) != 0u;
  uint32_t w[K];
  add_plain<K, G>(w, t, M.n);
  select(t, neg, w, t);
}

// ---- shifts and tests ----------------------------------------------------------
__device__ __forceinline__ bool wave_any(bool v) { return __builtin_amdgcn_ballot_w64(v) != 0ull; }

// Group-uniform: x == 0.
template <int K, int G = 16>
__device__ __forceinline__ bool is_zero(const uint32_t (&x)[K]) {
  bool nz = false;
#pragma unroll
  for (int j = 0; j < K; ++j) nz = nz || x[j] != 0u;
  return !row_any<G>(nz);
}
// Group-uniform: x == 1.
template <int K, int G = 16>
__device__ __forceinline__ bool is_one(const uint32_t (&x)[K]) {
  bool bad = false;
#pragma unroll
  for (int j = 0; j < K; ++j) bad = bad || x[j] != ((j == 0 && glane<G>() == 0) ? 1u : 0u);
  return !row_any<G>(bad);
}
// (hi:lo) >> t for 0 <= t <= 32 (v_alignbit_b32; written out, the 64-bit
// form gets turned into unaligned loads from a stack copy of the array).
__device__ __forceinline__ uint32_t funnel_r(uint32_t hi, uint32_t lo, uint32_t t) {
  return t >= 32u ? hi : __builtin_amdgcn_alignbit(hi, lo, t);
}
// x >>= t for 0 <= t <= 32 (group-uniform t); the bits entering at the top
// come from `top` (read in the group's last lane).
template <int K, int G = 16>
__device__ __forceinline__ void shr_bits(uint32_t (&x)[K], uint32_t t, uint32_t top = 0u) {
  uint32_t hi = from_next<G>(x[0]);
  if (glane<G>() == G - 1) hi = top;
#pragma unroll
  for (int j = 0; j + 1 < K; ++j) x[j] = funnel_r(x[j + 1], x[j], t);
  x[K - 1] = funnel_r(hi, x[K - 1], t);
}
// x <<= t for 0 <= t <= 32 (group-uniform t); bits above limb S are dropped.
template <int K, int G = 16>
__device__ __forceinline__ void shl_bits(uint32_t (&x)[K], uint32_t t) {
  const uint32_t lo = from_prev<G>(x[K - 1]);
  if (t == 0u) return;
#pragma unroll
  for (int j = K - 1; j > 0; --j) x[j] = __builtin_amdgcn_alignbit(x[j], x[j - 1], 32u - t);
  x[0] = __builtin_amdgcn_alignbit(x[0], lo, 32u - t);
}
// If z: x >>= 32 (resp. x <<= 32, dropping the top limb).
template <int K, int G = 16>
__device__ __forceinline__ void shr_limb_if(uint32_t (&x)[K], bool z) {
  const uint32_t hi = from_next<G>(x[0]);
#pragma unroll
  for (int j = 0; j + 1 < K; ++j) x[j] = z ? x[j + 1] : x[j];
  x[K - 1] = z ? hi : x[K - 1];
}
template <int K, int G = 16>
__device__ __forceinline__ void shl_limb_if(uint32_t (&x)[K], bool z) {
  const uint32_t lo = from_prev<G>(x[K - 1]);
#pragma unroll
  for (int j = K - 1; j > 0; --j) x[j] = z ? x[j - 1] : x[j];
  x[0] = z ? lo : x[0];
}
// Trailing zero bits of the group's lowest limb (0 if that limb is 0).
template <int G = 16>
__device__ __forceinline__ uint32_t low_ctz(uint32_t x0) {
  const uint32_t lo = bcast_first<G>(x0);
  return lo ? (uint32_t)__builtin_ctz(lo) : 0u;
}

// ---- inversion --------------------------------------------------------------------
// Kaliski's almost-inverse ("The Montgomery inverse and its applications",
// IEEE Trans. Computers 1995), phase one, for odd N and 0 < y < N:
// x = y^-1 2^k mod N.  The state u, v, r, s keeps u s + v r = N,
// y s = v 2^k and y r = -u 2^k (mod N); each step subtracts the smaller of
// the odd pair u, v from the larger and shifts every trailing zero of the
// difference out at once (doubling r or s as often), so log2(u v) drops by at
// least one per step and the loop ends within 2 log2 N + 1 steps with u = v =
// gcd(y, N).  When that gcd is 1, x = N - r.  Nothing here is secret (the
// operands are public ciphertexts), so the running time may depend on them.
// Returns (group-uniform) whether y was invertible; `active` false skips the
// group (it still takes part in the wave's cross-lane steps).
template <int K, int G = 16>
__device__ __forceinline__ bool almost_inverse(uint32_t (&x)[K], uint32_t &k, const uint32_t (&y)[K],
                                               const Mod<K> &M, bool active) {
  uint32_t u[K], v[K], r[K], s[K];
  copy(u, M.n);
  copy(v, y);
  set_zero(r);
  set_small<K, G>(s, 1u);
  k = 0;
  bool live = active && !is_zero<K, G>(y);
  bool met = false;  // the loop ended with u == v
  // make v odd: while r = 0, halving v only adds to k
  while (wave_any(live && bcast_first<G>(v[0]) == 0u)) {
    const bool z = live && bcast_first<G>(v[0]) == 0u;
    shr_limb_if<K, G>(v, z);
    k += z ? 32u : 0u;
  }
  {
    const uint32_t t = live ? low_ctz<G>(v[0]) : 0u;
    shr_bits<K, G>(v, t);
    k += t;
  }
  constexpr int kCap = 2 * 32 * G * K + 2;
#pragma unroll 1
  for (int it = 0; it < kCap; ++it) {
    if (!wave_any(live)) break;
    // d = |u - v|: the larger of the odd pair minus the smaller
    uint32_t d[K];
    const bool lt = bcast_last<G>(sub_plain<K, G>(d, u, v) ? 1u : 0u) != 0u;  // u < v
    {
      uint32_t e[K];
      sub_plain<K, G>(e, v, u);
      select(d, lt, e, d);
    }
    const bool eq = is_zero<K, G>(d);
    met = met || (live && eq);
    live = live && !eq;
    // the larger one's coefficient gains the other's (p); the other's is
    // doubled once per bit shifted out of d (q)
    uint32_t p[K], q[K];
    select(p, lt, s, r);
    select(q, lt, r, s);
    add_plain<K, G>(p, p, q);
    while (wave_any(live && bcast_first<G>(d[0]) == 0u)) {
      const bool z = live && bcast_first<G>(d[0]) == 0u;
      shr_limb_if<K, G>(d, z);
      shl_limb_if<K, G>(q, z);
      k += z ? 32u : 0u;
    }
    const uint32_t t = live ? low_ctz<G>(d[0]) : 0u;
    shr_bits<K, G>(d, t);
    shl_bits<K, G>(q, t);
    k += t;
    const bool lu = live && !lt, lv = live && lt;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      u[j] = lu ? d[j] : u[j];
      v[j] = lv ? d[j] : v[j];
      r[j] = lu ? p[j] : (lv ? q[j] : r[j]);
      s[j] = lu ? q[j] : (lv ? p[j] : s[j]);
    }
  }
  sub_plain<K, G>(x, M.n, r);
  return met && is_one<K, G>(u);
}

// x <- x 2^-k mod N for x < N (group-uniform k): up to 32 bits per step,
// x = (x + q N) / 2^j with q = -x N^-1 mod 2^j, which stays below N.
template <int K, int G = 16>
__device__ __forceinline__ void div_pow2(uint32_t (&x)[K], uint32_t k, const Mod<K> &M) {
#pragma unroll 1
  for (;;) {
    const bool act = k > 0u;
    if (!wave_any(act)) break;
    const uint32_t j = k >= 32u ? 32u : k;
    const uint32_t mask = j >= 32u ? 0xFFFFFFFFu : ((1u << j) - 1u);
    const uint32_t q = act ? (bcast_first<G>(mul_lo32(x[0], M.ninv)) & mask) : 0u;
    uint32_t t[K];
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const uint64_t w = (uint64_t)q * M.n[i] + x[i] + c;
      t[i] = (uint32_t)w;
      c = (uint32_t)(w >> 32);
    }
    // the lane's carry word goes into the next lane's lowest limb
    const uint32_t cin = from_prev<G>(c);
    unsigned b;
    t[0] = __builtin_addc(t[0], cin, 0u, &b);
#pragma unroll
    for (int i = 1; i < K; ++i) t[i] = __builtin_addc(t[i], 0u, b, &b);
    const bool gen = b;
    bool prop = true;
#pragma unroll
    for (int i = 0; i < K; ++i) prop = prop && (t[i] == 0xFFFFFFFFu);
    unsigned b2 = carry_in<G>(gen, prop);
#pragma unroll
    for (int i = 0; i < K; ++i) t[i] = __builtin_addc(t[i], 0u, b2, &b2);
    const uint32_t top = c + (uint32_t)gen + b2;  // x + q N < 2^j N: one word above limb S
    shr_bits<K, G>(t, j, top);
    select(x, act, t, x);
    k -= act ? j : 0u;
  }
}

// J = y^-1 R mod N (R = 2^(32 S), i.e. the Montgomery form of y^-1) for
// 0 < y < N coprime to N; returns false (group-uniform) otherwise.  R2 points
// to R^2 mod N (S limbs).
template <int K, int G = 16>
__device__ __forceinline__ bool mont_inverse(uint32_t (&J)[K], const uint32_t (&y)[K], const Mod<K> &M,
                                             const uint32_t *R2, uint32_t *lds, bool active) {
  uint32_t k;
  const bool ok = almost_inverse<K, G>(J, k, y, M, active);
  div_pow2<K, G>(J, ok ? k : 0u, M);
  uint32_t r2[K];
  ld<K, G>(r2, R2);
  mont_mul<K, G>(J, J, r2, M, lds);
  return ok;
}

// ---- low-half product ----------------------------------------------------------
// t = a * b mod 2^(32 S), with a from this group's LDS copy and b in registers.
// (Used for the exact division x / P = x * P^-1 mod 2^(32 S) when P | x.)
template <int K, int G = 16>
__device__ __forceinline__ void mul_lo_lds(uint32_t (&t)[K], const uint32_t *a_lds,
                                           const uint32_t (&b)[K]) {
  uint32_t acc[K], bs[K];
  set_zero(acc);
  copy(bs, b);
  uint32_t cin = 0;  // pending carry into this lane's lowest column
#pragma unroll 1
  for (int i0 = 0; i0 < G * K; i0 += K) {
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
      cin = from_prev<G>(top);
      // shift bs up by one limb for the next multiplier limb
      const uint32_t down = from_prev<G>(bs[K - 1]);
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
  unsigned c2 = carry_in<G>(gen, prop);
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

// Moves an integer between limb layouts through this group's LDS row:
// src has G*KS limbs (KS per lane), dst gets G*KD limbs (KD per lane); the
// limbs are taken starting at `first` and limbs beyond the source are zero.
template <int KS, int KD, int G = 16>
__device__ __forceinline__ void relayout(uint32_t (&dst)[KD], const uint32_t (&src)[KS],
                                         uint32_t *lds, int first = 0) {
  constexpr int SS = G * KS;
  st<KS, G>(lds, src);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < KD; ++j) {
    const int idx = first + (int)glane<G>() * KD + j;
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
