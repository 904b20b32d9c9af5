// Radix-2^29 Montgomery arithmetic for gfx950: the modular exponentiations
// and the histogram products (group layout as in mont.hpp: G lanes per
// integer, lane l holding limbs l*K .. l*K+K-1).
//
// With 29-bit limbs every partial product is below 2^58, and a 64-bit column
// accumulator can absorb every product a column receives while it lives in
// one lane: a column enters the lane's top below 2^29, takes two products
// (a_i b_j and q_i n_j, each below 2^58 (1 + 2^-20) for limbs up to
// 2^29 + 2^8) in each of the K steps it takes to reach the lane's bottom,
// plus one fold carry below 2^36, and is then folded, so it stays below
// 2^64 for K <= 31.  A product is one
// v_mad_u64_u32 and nothing else; the 32-bit-limb code in mont.hpp needs a
// second instruction per product for the carry out of the 64-bit column.
// The price is 29/32 of the bits per limb (about 1.1x the limbs and steps).
//
// The fold of a step: q_i = c_0 (-N^-1) mod 2^29 clears the low 29 bits of
// the group's lowest column; every lane then passes the low 29 bits of its
// lowest column down to the previous lane's new top column (lane 0 passes
// zero) and adds the rest (c_0 >> 29) to its next column, which has that
// weight after the shift.
//
// Between products an integer is "settled": limbs below 2^29 except each
// lane's second limb, below 2^29 + 2^8 (one carry pass inside the lane, the
// lane's carry added to the next lane's lowest limb).  With R = 2^(29 S29) >
// 4N, operands below 2N give a product below 2N, so there is no conditional
// subtraction until the exponentiation ends.
//
// Every function must be called by all 64 lanes of the wave.
#pragma once
#include "mont.hpp"
#include "radix29.hpp"

#include <type_traits>

namespace he {

constexpr uint32_t kMask29 = (1u << he29::kBits) - 1u;

// f(integral_constant<I>), ..., f(integral_constant<N-1>): a loop whose index
// is a compile-time constant in the body.
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <int K>
struct Mod29 {
  uint32_t n[K];  // this lane's 29-bit limbs of N
  uint32_t ninv;  // -N^-1 mod 2^29
  uint32_t mask;  // 2^29 - 1, held in a VGPR for the masked DPP moves
};

// Lane-local K words at lane offset glane * K (64-bit accesses for even K).
template <int K, int G>
__device__ __forceinline__ void ld29(uint32_t (&x)[K], const uint32_t *p) {
  p += glane<G>() * K;
  if constexpr (K % 4 == 0) {
#pragma unroll
    for (int j = 0; j < K; j += 4) {
      const uint4 v = *reinterpret_cast<const uint4 *>(p + j);
      x[j] = v.x; x[j + 1] = v.y; x[j + 2] = v.z; x[j + 3] = v.w;
    }
  } else if constexpr (K % 2 == 0) {
#pragma unroll
    for (int j = 0; j < K; j += 2) {
      const uint2 v = *reinterpret_cast<const uint2 *>(p + j);
      x[j] = v.x; x[j + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) x[j] = p[j];
  }
}
template <int K, int G>
__device__ __forceinline__ void st29(uint32_t *p, const uint32_t (&x)[K]) {
  p += glane<G>() * K;
  if constexpr (K % 4 == 0) {
#pragma unroll
    for (int j = 0; j < K; j += 4)
      *reinterpret_cast<uint4 *>(p + j) = make_uint4(x[j], x[j + 1], x[j + 2], x[j + 3]);
  } else if constexpr (K % 2 == 0) {
#pragma unroll
    for (int j = 0; j < K; j += 2) *reinterpret_cast<uint2 *>(p + j) = make_uint2(x[j], x[j + 1]);
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) p[j] = x[j];
  }
}

template <int K, int G>
__device__ __forceinline__ Mod29<K> load_mod29(const DMod &D) {
  Mod29<K> m;
  ld29<K, G>(m.n, D.N29[he29::variant(G)]);
  m.ninv = D.ninv & kMask29;
  m.mask = kMask29;
  return m;
}


// x from the group's first lane (resp. the next lane, the last lane reading
// the first), masked to 29 bits, in one v_and_b32_dpp (two, each writing one
// half of the row, for the 8-lane broadcast; the 8-lane hand-down uses
// row_shl:1, see rotate_next).  The s_nop gives the DPP read of x the two
// wait states it needs after the VALU write of x; it costs this wave an issue
// cycle, not a VALU slot.
template <int G>
__device__ __forceinline__ uint32_t bcast_first_m29(uint32_t x, uint32_t mask) {
  uint32_t r;
  if constexpr (G == 2)
    asm("s_nop 1\n\tv_and_b32_dpp %0, %1, %2 quad_perm:[0,0,2,2] row_mask:0xf bank_mask:0xf"
        : "=v"(r) : "v"(x), "v"(mask));
  else if constexpr (G == 4)
    asm("s_nop 1\n\tv_and_b32_dpp %0, %1, %2 quad_perm:[0,0,0,0] row_mask:0xf bank_mask:0xf"
        : "=v"(r) : "v"(x), "v"(mask));
  else if constexpr (G == 16)
    asm("s_nop 1\n\tv_and_b32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf"
        : "=v"(r) : "v"(x), "v"(mask));
  else
    asm("s_nop 1\n\tv_and_b32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0x3\n\t"
        "v_and_b32_dpp %0, %1, %2 row_newbcast:8 row_mask:0xf bank_mask:0xc"
        : "=&v"(r) : "v"(x), "v"(mask));
  return r;
}
template <int G>
__device__ __forceinline__ uint32_t rotate_next_m29(uint32_t x, uint32_t mask) {
  uint32_t r;
  if constexpr (G == 2)
    asm("s_nop 1\n\tv_and_b32_dpp %0, %1, %2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf"
        : "=v"(r) : "v"(x), "v"(mask));
  else if constexpr (G == 4)
    asm("s_nop 1\n\tv_and_b32_dpp %0, %1, %2 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf"
        : "=v"(r) : "v"(x), "v"(mask));
  else if constexpr (G == 16)
    asm("s_nop 1\n\tv_and_b32_dpp %0, %1, %2 row_ror:15 row_mask:0xf bank_mask:0xf"
        : "=v"(r) : "v"(x), "v"(mask));
  else
    asm("s_nop 1\n\tv_and_b32_dpp %0, %1, %2 row_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=v"(r) : "v"(x), "v"(mask));
  return r;
}

// One step for multiplier limb ai (see the header comment).  The lane's new
// top column (the low 29 bits handed down by the next lane) is kept in `top`
// and enters the next step as the addend of that column's first
// multiply-add, so no register copy places it; C[K-1] is stale between steps.
template <int K, int G>
__device__ __forceinline__ void step29(uint64_t (&C)[K], uint32_t &top, uint32_t ai, const uint32_t (&b)[K],
                                       const Mod29<K> &M) {
  static_assert(K >= 2 && K <= 31, "column bound needs 2 <= K <= 31");
#pragma unroll
  for (int j = 0; j + 1 < K; ++j) C[j] += (uint64_t)ai * b[j];
  C[K - 1] = (uint64_t)top + (uint64_t)ai * b[K - 1];
  const uint32_t q = bcast_first_m29<G>(mul_lo32((uint32_t)C[0], M.ninv), M.mask);
#pragma unroll
  for (int j = 0; j < K; ++j) C[j] += (uint64_t)q * M.n[j];
  top = rotate_next_m29<G>((uint32_t)C[0], M.mask);
  C[1] += C[0] >> he29::kBits;
#pragma unroll
  for (int j = 0; j + 1 < K; ++j) C[j] = C[j + 1];
  // The sums are opaque from one step to the next (an empty asm per column,
  // no instruction), so the compiler keeps one accumulator per column instead
  // of reassociating several steps' products into extra registers.
#pragma unroll
  for (int j = 0; j + 1 < K; ++j) asm("" : "+v"(C[j]));
  asm("" : "+v"(top));
}

// t = a b R'^-1 mod N (settled, below 2N) with a (settled, below 2N) in this
// group's LDS row and b (settled, below 2N) in registers.  t may alias b.
template <int K, int G>
__device__ __forceinline__ void mm29_lds(uint32_t (&t)[K], const uint32_t *a_lds, const uint32_t (&b)[K],
                                         const Mod29<K> &M) {
  constexpr int S = G * K;
  constexpr int U = K % 2 == 0 ? K : 2 * K;  // steps per loop iteration (even: 64-bit LDS reads)
  static_assert(S % U == 0, "unroll must divide the limb count");
  uint64_t C[K];
  uint32_t top = 0;
#pragma unroll
  for (int j = 0; j + 1 < K; ++j) C[j] = 0;
#pragma unroll 1
  for (int i0 = 0; i0 < S; i0 += U) {
    // multiplier limbs two at a time, read right before their steps
    uint2 v;
    static_for<0, U>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      if constexpr (s % 2 == 0) v = *reinterpret_cast<const uint2 *>(a_lds + i0 + s);
      step29<K, G>(C, top, s % 2 == 0 ? v.x : v.y, b, M);
    });
  }
  C[K - 1] = top;
  // settle: one carry pass in the lane, the lane's carry (below 2^36) into
  // the next lane's lowest limb; the group's top carry is zero (result < 2N)
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint64_t s = C[j] + c;
    t[j] = (uint32_t)s & kMask29;
    c = s >> he29::kBits;
  }
  const uint32_t cl = from_prev<G>((uint32_t)c), ch = from_prev<G>((uint32_t)(c >> 32));
  const uint64_t s0 = (uint64_t)t[0] + (((uint64_t)ch << 32) | cl);
  t[0] = (uint32_t)s0 & kMask29;
  t[1] += (uint32_t)(s0 >> he29::kBits);
}

// Squaring.  The products a_i a_j of a square pair up (a_i a_j = a_j a_i),
// and the pair's doubled product 2 a_i a_j can join its column (i + j) in
// either of its two steps: at step i it is the multiply-add of position j,
// at step j that of position i, and both positions hold column i + j then.
// Each step keeps about half of its positions, the same local indices in
// every lane so that the kept multiply-adds are ordinary lane-uniform
// instructions: for local indices x = i mod K and y = j mod K with x != y,
// step i keeps position j when y - x mod K lies in [1, K/2) (for even K
// also when it equals K/2 and x < K/2); this is a tournament on the K local
// indices, so exactly one of the pair's two steps keeps it.  Positions with
// y = x (the square a_i^2 and the pairs of limbs at the same local index of
// different lanes) are kept at every step with a per-lane multiplier: 2 a_i
// in the lanes above the step's own lane (j > i), a_i in its own lane
// (j = i) and 0 below (those pairs were taken at step j < i).  A column is
// complete when its reduction step comes, since both steps of each of its
// pairs are at most its index.  A kept doubled product is below 2^59 (1 +
// 2^-20), so a column still stays below 2^64 for K <= 21.
//
// The multipliers come from LDS: the group's row holds a (S29 words) and
// right after it 2a; the per-lane multiplier of the diagonal position is
// read from the 2a row, the a row or a block-shared row of zeros, chosen
// per lane once for every K steps, so a step costs no extra VALU work.
template <int K>
__host__ __device__ constexpr bool sq_keeps(int x, int y) {
  const int d = ((y - x) % K + K) % K;
  return K % 2 ? (d >= 1 && d <= (K - 1) / 2) : ((d >= 1 && d < K / 2) || (d == K / 2 && x < K / 2));
}

// One squaring step for multiplier limb a_i (i mod K = X): a2 = 2 a_i for the
// kept pair positions, ad = this lane's multiplier at local index X.
template <int K, int G, int X>
__device__ __forceinline__ void sqstep29(uint64_t (&C)[K], uint32_t &top, uint32_t a2, uint32_t ad,
                                         const uint32_t (&b)[K], const Mod29<K> &M) {
  static_assert(K >= 2 && K <= 21, "column bound of the squaring needs 2 <= K <= 21");
  static_for<0, K>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    const uint64_t base = j == K - 1 ? (uint64_t)top : C[j];
    if constexpr (j == X)
      C[j] = base + (uint64_t)ad * b[j];
    else if constexpr (sq_keeps<K>(X, j))
      C[j] = base + (uint64_t)a2 * b[j];
    else
      C[j] = base;
  });
  const uint32_t q = bcast_first_m29<G>(mul_lo32((uint32_t)C[0], M.ninv), M.mask);
#pragma unroll
  for (int j = 0; j < K; ++j) C[j] += (uint64_t)q * M.n[j];
  top = rotate_next_m29<G>((uint32_t)C[0], M.mask);
  C[1] += C[0] >> he29::kBits;
#pragma unroll
  for (int j = 0; j + 1 < K; ++j) C[j] = C[j + 1];
#pragma unroll
  for (int j = 0; j + 1 < K; ++j) asm("" : "+v"(C[j]));
  asm("" : "+v"(top));
}

// t = a^2 R'^-1 mod N (settled, below 2N) with a (settled, below 2N) in
// registers (b), in this group's LDS row (lds[0, S29)) and doubled right
// after it (lds[S29, 2 S29)); `zeros`: S29 zero words in the same LDS array
// as the row.  t may alias b.
template <int K, int G>
__device__ __forceinline__ void sq29_lds(uint32_t (&t)[K], const uint32_t *lds, const uint32_t (&b)[K],
                                         const uint32_t *zeros, const Mod29<K> &M) {
  constexpr int S = G * K;
  constexpr int U = K % 2 == 0 ? K : 2 * K;  // steps per loop iteration, a multiple of K
  static_assert(S % U == 0, "unroll must divide the limb count");
  const int gl = (int)glane<G>();
  const uint32_t *row2 = lds + S;
  const int zoff = (int)(zeros - lds);  // same LDS array: an integer offset keeps the loads in LDS
  uint64_t C[K];
  uint32_t top = 0;
#pragma unroll
  for (int j = 0; j + 1 < K; ++j) C[j] = 0;
#pragma unroll 1
  for (int i0 = 0; i0 < S; i0 += U) {
    uint2 v2, vd;
    const uint32_t *dsel = nullptr;
    static_for<0, U>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      if constexpr (s % K == 0) {
        const int ls = i0 / K + s / K;  // lane holding limbs i0 + s .. i0 + s + K - 1
        dsel = lds + (gl > ls ? S : (gl == ls ? 0 : zoff));
      }
      if constexpr (s % 2 == 0) v2 = *reinterpret_cast<const uint2 *>(row2 + i0 + s);
      // the diagonal multipliers two at a time while both steps share a lane
      // block (even K), else one at a time
      if constexpr (K % 2 == 0 && s % 2 == 0) vd = *reinterpret_cast<const uint2 *>(dsel + i0 + s);
      if constexpr (K % 2 != 0) vd.x = dsel[i0 + s];
      const uint32_t ad = K % 2 != 0 || s % 2 == 0 ? vd.x : vd.y;
      sqstep29<K, G, s % K>(C, top, s % 2 == 0 ? v2.x : v2.y, ad, b, M);
    });
  }
  C[K - 1] = top;
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint64_t s = C[j] + c;
    t[j] = (uint32_t)s & kMask29;
    c = s >> he29::kBits;
  }
  const uint32_t cl = from_prev<G>((uint32_t)c), ch = from_prev<G>((uint32_t)(c >> 32));
  const uint64_t s0 = (uint64_t)t[0] + (((uint64_t)ch << 32) | cl);
  t[0] = (uint32_t)s0 & kMask29;
  t[1] += (uint32_t)(s0 >> he29::kBits);
}

// Fills the block-shared zero words the squaring reads (n words); every
// thread of the block must call it before any leaves.
__device__ __forceinline__ void zero_lds(uint32_t *z, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) z[t] = 0u;
  __syncthreads();
}

// t = a^2 R'^-1 mod N, a in registers; `lds`: this group's row of at least
// 2 S29 words; `zeros`: S29 zero words in the row's LDS array.  t may alias a.
template <int K, int G>
__device__ __forceinline__ void sq29(uint32_t (&t)[K], const uint32_t (&a)[K], const Mod29<K> &M, uint32_t *lds,
                                     const uint32_t *zeros) {
  constexpr int S = G * K;
  uint32_t d[K];
#pragma unroll
  for (int j = 0; j < K; ++j) d[j] = a[j] << 1;
  st29<K, G>(lds, a);
  st29<K, G>(lds + S, d);
  __builtin_amdgcn_wave_barrier();
  sq29_lds<K, G>(t, lds, a, zeros, M);
  __builtin_amdgcn_wave_barrier();
}

// t = a b R'^-1 mod N, both operands in registers; `lds` is this group's row
// (at least S29 words).  t may alias a or b.
template <int K, int G>
__device__ __forceinline__ void mm29(uint32_t (&t)[K], const uint32_t (&a)[K], const uint32_t (&b)[K],
                                     const Mod29<K> &M, uint32_t *lds) {
  st29<K, G>(lds, a);
  __builtin_amdgcn_wave_barrier();
  mm29_lds<K, G>(t, lds, b, M);
  __builtin_amdgcn_wave_barrier();
}

// t = a b R'^-1 mod N with a read from global memory (this lane's K words
// at a + glane * K) into the LDS row and b in registers.  t may alias b.
// Nothing of a stays in registers across the product.
template <int K, int G>
__device__ __forceinline__ void mm29_mem(uint32_t (&t)[K], const uint32_t *a, const uint32_t (&b)[K],
                                         const Mod29<K> &M, uint32_t *lds) {
  uint32_t v[K];
  ld29<K, G>(v, a);
  mm29<K, G>(t, v, b, M, lds);
}

// Settled t below 2N -> exact 29-bit limbs of t mod N.  One carry pass in
// the lane (every carry is 0 or 1: only the second limb can exceed 2^29), a
// ballot carry-lookahead across the group, then d = t - N the same way (in
// the lane, then a borrow lookahead); t is replaced by d unless the
// subtraction borrows out of the group's top limb.
template <int K, int G>
__device__ __forceinline__ void canon29(uint32_t (&t)[K], const Mod29<K> &M) {
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t s = t[j] + c;
    t[j] = s & kMask29;
    c = s >> he29::kBits;
  }
  bool prop = true;
#pragma unroll
  for (int j = 0; j < K; ++j) prop = prop && t[j] == kMask29;
  uint32_t ci = carry_in<G>(c != 0u, prop) ? 1u : 0u;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t s = t[j] + ci;
    t[j] = s & kMask29;
    ci = s >> he29::kBits;
  }
  uint32_t d[K];
  uint32_t b = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t s = t[j] - M.n[j] - b;
    d[j] = s & kMask29;
    b = s >> 31;
  }
  bool zprop = true;
#pragma unroll
  for (int j = 0; j < K; ++j) zprop = zprop && d[j] == 0u;
  uint32_t bi = carry_in<G>(b != 0u, zprop) ? 1u : 0u;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t s = d[j] - bi;
    d[j] = s & kMask29;
    bi = s >> 31;
  }
  const bool neg = bcast_last<G>((b | bi) != 0u ? 1u : 0u) != 0u;
  select(t, neg, t, d);
}

// 32-bit limbs (K32 per lane, value below 2^(29 S29)) -> 29-bit limbs.
template <int K32, int K, int G>
__device__ __forceinline__ void to29(uint32_t (&t)[K], const uint32_t (&x)[K32], uint32_t *lds) {
  constexpr int S32 = G * K32;
  st<K32, G>(lds, x);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t bit = he29::kBits * (glane<G>() * K + j);
    const uint32_t w = bit >> 5;
    const uint32_t lo = w < S32 ? lds[w] : 0u;
    const uint32_t hi = w + 1 < S32 ? lds[w + 1] : 0u;
    t[j] = __builtin_amdgcn_alignbit(hi, lo, bit & 31u) & kMask29;
  }
  __builtin_amdgcn_wave_barrier();
}

// Exact 29-bit limbs -> 32-bit limbs (K32 per lane; bits beyond dropped).
template <int K, int K32, int G>
__device__ __forceinline__ void to32(uint32_t (&x)[K32], const uint32_t (&t)[K], uint32_t *lds) {
  constexpr int S = G * K;
  st29<K, G>(lds, t);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < K32; ++j) {
    const uint32_t bit = 32u * (glane<G>() * K32 + j);
    const uint32_t k0 = bit / he29::kBits, o = bit % he29::kBits;
    const uint64_t l0 = k0 < S ? lds[k0] : 0u;
    const uint64_t l1 = k0 + 1 < S ? lds[k0 + 1] : 0u;
    const uint64_t l2 = k0 + 2 < S ? lds[k0 + 2] : 0u;
    const uint64_t v = l0 | (l1 << he29::kBits) | (l2 << (2 * he29::kBits));
    x[j] = (uint32_t)(v >> o);
  }
  __builtin_amdgcn_wave_barrier();
}

// This group's window-table entry `digit` into registers.  With ct (the
// exponent is secret) every entry is read and the wanted one kept by a mask,
// so the addresses the table reads touch do not depend on the digit; the
// digit goes through a VGPR so that the selection is data, never control.
template <int K, int G>
__device__ __forceinline__ void tab_entry(uint32_t (&v)[K], const uint32_t *tab, uint32_t digit, bool ct) {
  constexpr int S29 = G * K;
  if (!ct) {
    ld29<K, G>(v, tab + digit * S29);
    return;
  }
  uint32_t dv = digit;
  asm volatile("" : "+v"(dv));
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0u;
#pragma unroll 1
  for (uint32_t j = 0; j < (uint32_t)kTable; ++j) {
    uint32_t t[K];
    ld29<K, G>(t, tab + j * S29);
    const uint32_t m = dv == j ? 0xFFFFFFFFu : 0u;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] |= t[k] & m;
  }
}

// x <- x^e mod N for canonical x < N in 32-bit limbs (K32 per lane), result
// canonical, in the radix-2^29 Montgomery domain.  Two schedules, neither
// with a branch on the exponent's bits inside the arithmetic:
//  * ct (the exponent is secret and its table reads must not reveal it):
//    left-to-right fixed 5-bit windows over E.nwin windows, a table of the
//    powers x^0 .. x^31, a multiplication by the table entry for every
//    window, zero digits included, and every entry read for each window
//    (tab_entry), so neither the operations nor the addresses depend on e;
//  * otherwise: E's sliding-window schedule (windows of up to 6 bits ending
//    in a 1 bit; keysetup.hpp), a table of the odd powers x, x^3 .. x^63
//    built with x^2, and per op its squarings and one multiplication by the
//    odd power its window names: about 146 multiplications per 1024-bit
//    exponent instead of 204, with as many squarings.  The schedule is
//    fixed per key and the same for the whole wave.
// `tab`: this group's table, kTable + 1 entries of S29 words in global
// memory; `lds`: this group's row of at least max(G K32, 2 S29) words;
// `zeros`: S29 zero words in the row's LDS array (see sq29).
template <int K32, int G>
__device__ __forceinline__ void pow29(uint32_t (&x)[K32], const DExp &E, uint32_t *tab, const DMod &D,
                                      uint32_t *lds, const uint32_t *zeros, bool ct) {
  constexpr int S29 = he29::limbs_for_group(G * K32, G);
  constexpr int K = S29 / G;
  constexpr int v = he29::variant(G);
  const Mod29<K> M = load_mod29<K, G>(D);
  uint32_t cur[K];
  {
    uint32_t c[K];
    to29<K32, K, G>(cur, x, lds);
    ld29<K, G>(c, D.R2_29[v]);
    mm29<K, G>(cur, cur, c, M, lds);  // Montgomery form of x
  }
  if (ct) {
    {
      uint32_t c[K];
      ld29<K, G>(c, D.R1_29[v]);  // Montgomery form of 1
      st29<K, G>(tab, c);
      st29<K, G>(tab + S29, cur);
    }
    // table entries d = x^d; the multiplier x comes back from the table so
    // that only the running power is held in registers
#pragma unroll 1
    for (int d = 2; d < kTable; ++d) {
      mm29_mem<K, G>(cur, tab + S29, cur, M, lds);
      st29<K, G>(tab + d * S29, cur);
    }
    __threadfence_block();
    tab_entry<K, G>(cur, tab, exp_digit(E.e, E.nwin - 1), true);
#pragma unroll 1
    for (int w = E.nwin - 2; w >= 0; --w) {
#pragma unroll 1
      for (int s = 0; s < kWindow; ++s) sq29<K, G>(cur, cur, M, lds, zeros);
      uint32_t t[K];
      tab_entry<K, G>(t, tab, exp_digit(E.e, w), true);
      mm29<K, G>(cur, t, cur, M, lds);
    }
  } else {
    // odd powers: entry k = x^(2k+1); x^2 in entry kTable, read back as
    // the multiplier of each step
    st29<K, G>(tab, cur);
    sq29<K, G>(cur, cur, M, lds, zeros);
    st29<K, G>(tab + kTable * S29, cur);
    ld29<K, G>(cur, tab);
#pragma unroll 1
    for (int k = 1; k < kTable; ++k) {
      mm29_mem<K, G>(cur, tab + kTable * S29, cur, M, lds);
      st29<K, G>(tab + k * S29, cur);
    }
    __threadfence_block();
    if (E.nops == 0) {
      ld29<K, G>(cur, D.R1_29[v]);  // x^0
    } else {
      ld29<K, G>(cur, tab + (E.ops[0] & 0xFFu) * S29);
#pragma unroll 1
      for (int t = 1; t < E.nops; ++t) {
        const uint32_t op = E.ops[t];
        const uint32_t k = op & 0xFFu;
#pragma unroll 1
        for (uint32_t s = op >> 8; s > 0; --s) sq29<K, G>(cur, cur, M, lds, zeros);
        if (k < (uint32_t)kTable) mm29_mem<K, G>(cur, tab + k * S29, cur, M, lds);
      }
    }
  }
  // leave the Montgomery domain: cur R'^-1 (a product with 1, at most N)
  {
    uint32_t one[K];
    set_small<K, G>(one, 1u);
    mm29<K, G>(cur, cur, one, M, lds);
  }
  canon29<K, G>(cur, M);
  to32<K, K32, G>(x, cur, lds);
}

}  // namespace he
