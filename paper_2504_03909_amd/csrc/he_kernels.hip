// gfx950 kernels of the Paillier histogram path: fixed-point encoding,
// encryption (CRT and public-key), Montgomery conversion, histogram
// aggregation (bucketing + chunked ciphertext products) and CRT decryption.
//
// Layout conventions: one big integer per 16-lane group (see mont.hpp);
// 256-thread blocks = 4 waves = 16 groups; every group owns one LDS row.
// Kernels keep all 64 lanes of a wave active until they return; groups with
// no work compute on a valid dummy item and do not store.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <tuple>

#include "he_internal.hpp"
#include "hist_bucket.hpp"
#include "mont.hpp"
#include "mont29.hpp"

namespace he {

static_assert(kWindow == kWindowBits, "window width mismatch");

// ------------------------------------------------------------- small helpers
// Limb t of a little-endian buffer of `nl` limbs, zero past the end.
template <int K, int G = 16>
__device__ __forceinline__ void ld_part(uint32_t (&x)[K], const uint32_t *p, int nl) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int t = (int)glane<G>() * K + j;
    x[j] = t < nl ? p[t] : 0u;
  }
}

// x = v mod N for a signed 64-bit v (|v| < N).
template <int K, int G = 16>
__device__ __forceinline__ void signed_mod(uint32_t (&x)[K], int64_t v, const uint32_t (&N)[K]) {
  const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
  uint32_t a[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int t = (int)glane<G>() * K + j;
    a[j] = t == 0 ? (uint32_t)mag : (t == 1 ? (uint32_t)(mag >> 32) : 0u);
  }
  if (v < 0) {
    uint32_t d[K];
    sub_plain<K, G>(d, N, a);
    copy(x, d);
  } else {
    copy(x, a);
  }
}

// x += 1 (no reduction).
template <int K, int G = 16>
__device__ __forceinline__ void add_one(uint32_t (&x)[K]) {
  uint32_t one[K];
  set_small<K, G>(one, 1u);
  add_plain<K, G>(x, x, one);
}

// Limbs [first, first + G K) of the seeded stream integer
// X = sum_j w(seed, base + j) 2^(64 j), each lane taking its K limbs;
// limbs at or past `nl` are zero.
template <int K, int G = 16>
__device__ __forceinline__ void seeded_limbs(uint32_t (&x)[K], uint64_t seed, uint64_t base,
                                             int first, int nl) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int t = first + (int)glane<G>() * K + j;
    const uint64_t w = splitmix64(seed, base + (uint64_t)(t >> 1));
    x[j] = t < nl ? (uint32_t)((t & 1) ? (w >> 32) : w) : 0u;
  }
}

// The wave's index in its block, as a wave-uniform (scalar) value: what the
// persistent loops derive from it (unit index, prime, modulus and exponent
// pointers) then lives in SGPRs.
__device__ __forceinline__ uint32_t wave_in_block() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// The next work unit for this wave: one atomic add by the wave's first lane,
// its result made wave-uniform.
__device__ __forceinline__ uint64_t claim_unit(uint32_t *next) {
  uint32_t v = 0;
  if (lane_id() == 0) v = atomicAdd(next, 1u);
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint32_t group_in_wave() { return (threadIdx.x >> 4) & 3u; }

// ------------------------------------------------------------------- encode
__global__ void k_encode(const double *__restrict__ x, uint64_t count, uint32_t frac_bits,
                         int64_t *__restrict__ m, uint32_t *__restrict__ n_bad) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const double v = ldexp(x[i], (int)frac_bits);  // exact scaling by a power of two
    if (!(fabs(v) < 9223372036854775808.0)) {
      m[i] = INT64_MIN;
      if (n_bad) atomicAdd(n_bad, 1u);
    } else {
      m[i] = (int64_t)rint(v);  // round to nearest, ties to even
    }
  }
}

// ----------------------------------------------------- private-key exponentiation
// k_pow: x_u <- x_u^(e_P) mod M_P for units u = (ciphertext i, prime P), the
// radix-2^29 exponentiation alone (the products around it run in the 16-lane
// kernels below, so this kernel holds nothing but the exponentiation's own
// state).  Unit (i, w) reads in_limbs limbs at in + (2 i + w) in_stride
// (zero-extended to S32) and writes S32 canonical limbs at
// out + (2 i + w) out_stride.  Work unit = (prime, 64/G consecutive
// ciphertexts), so the modulus and exponent are the same for the whole wave.
// CT: constant-time window-table reads.  At most 3 waves per SIMD: the
// 18-limb-per-lane shapes need about 168 VGPRs to run their step loops
// without spills (at 128, for 4 waves, the loops spill and run 25% slower).
// With `next` (a counter zeroed before the launch) the waves claim units as
// they finish them, so they end together; without, wave w takes units w,
// w + waves, ...
struct PowArgs {
  DMod mod[2];
  DExp exp[2];
  const uint32_t *in;
  uint32_t *out;
  uint32_t in_stride, in_limbs, out_stride;
  uint64_t count;
  uint32_t *tabs;
  uint32_t *next;
};

template <int S32, int G, bool CT>
__global__ __launch_bounds__(kBlockThreads, 3) void k_pow(PowArgs a) {
  constexpr int K32 = S32 / G, NG = 64 / G, GB = kBlockThreads / G;
  constexpr int S29 = he29::limbs_for_group(S32, G), ROW = 2 * S29 > S32 ? 2 * S29 : S32;
  __shared__ __align__(16) uint32_t lds_all[GB * ROW + S29];
  uint32_t *const zeros = lds_all + GB * ROW;
  zero_lds(zeros, S29);
  const uint32_t g = (threadIdx.x & 63u) / G;
  uint32_t *lds = lds_all + (threadIdx.x / G) * ROW;
  const uint64_t gw = (uint64_t)blockIdx.x * 4 + wave_in_block();
  const uint64_t nw = (uint64_t)gridDim.x * 4;
  uint32_t *tab = a.tabs + (gw * NG + g) * (uint64_t)((kTable + 1) * S29);
  const uint64_t nunits = 2 * ((a.count + NG - 1) / NG);
  for (uint64_t qd = a.next ? claim_unit(a.next) : gw; qd < nunits; qd = a.next ? claim_unit(a.next) : qd + nw) {
    const int which = (int)(qd & 1);
    uint64_t i = (qd >> 1) * NG + g;
    const bool valid = i < a.count;
    if (!valid) i = a.count - 1;
    const uint64_t u = i * 2 + which;
    uint32_t x[K32];
    ld_part<K32, G>(x, a.in + u * a.in_stride, (int)a.in_limbs);
    pow29<K32, G>(x, a.exp[which], tab, a.mod[which], lds, zeros, CT);
    if (valid) st<K32, G>(a.out + u * a.out_stride, x);
  }
}

// ----------------------------------------------------------- CRT encryption
// For each (ciphertext i, prime P):
//   c_P = (1 + m n) r^n mod P^2,  r^n mod P^2 = (r^(Q mod (P-1)) mod P)^P mod P^2
// (x -> x^P mod P^2 depends only on x mod P), and 1 + m n = 1 + P (m Q mod P)
// mod P^2.  k_enc_r reduces r mod P, k_pow computes t = r^(Q mod (P-1)) mod P
// (mod-P arithmetic, 2-lane groups for large counts) and then omega = t^P mod
// P^2 (4-lane groups), and k_enc_crt_b forms c_P = omega (1 + P (m Q mod P))
// and combines c_p, c_q by the CRT.

// r mod P for each (ciphertext i, prime P) into tq[2 i + P] (S_P limbs): r's
// S_P-limb words w_k (two for an explicit r, three for the seeded one), each
// times R^k mod P by a Montgomery product with R^(k+1) mod P, summed.  One
// 16-lane group per (i, P).
template <int KP>
__global__ __launch_bounds__(kBlockThreads) void k_enc_r(DKey key, uint64_t count, const uint32_t *__restrict__ r,
                                                        uint64_t seed, uint64_t roff, uint32_t *__restrict__ tq) {
  constexpr int SP = 16 * KP, L = 32 * KP;
  __shared__ __align__(16) uint32_t lds_all[16 * SP];
  const uint32_t gi = wave_in_block() * 4 + group_in_wave();
  uint32_t *lds = lds_all + gi * SP;
  uint64_t u = (uint64_t)blockIdx.x * 16 + gi;
  const bool valid = u < 2 * count;
  if (!valid) u = 2 * count - 1;
  const uint64_t i = u >> 1;
  const DPrime &P = key.pr[u & 1];
  const Mod<KP> Mp = load_mod<KP>(P.P.N, P.P.ninv);
  const uint64_t W = (uint64_t)SP + 1;  // stream words per r
  const uint64_t base = (roff + i) * W;
  const int words = r ? 2 : 3;
  uint32_t x[KP], t[KP], c[KP];
  set_zero(x);
#pragma unroll 1
  for (int k = 0; k < words; ++k) {
    if (r)
      ld<KP>(t, r + i * L + k * SP);
    else
      seeded_limbs<KP>(t, seed, base, k * SP, 2 * SP + 2);
    ld<KP>(c, k == 0 ? P.P.R1 : (k == 1 ? P.P.R2 : P.P.R3));
    mont_mul<KP>(t, t, c, Mp, lds);
    add_mod<KP>(x, x, t, Mp);
  }
  if (valid) st<KP>(tq + u * SP, x);
}

// c_P = omega_P (1 + P (m Q mod P)) mod P^2 for both primes, then
// c = c_q + q^2 ((c_p - c_q) (q^2)^-1 mod p^2), the CRT to mod n^2.  One
// 16-lane group per ciphertext.
template <int KP>
__global__ __launch_bounds__(kBlockThreads) void k_enc_crt_b(DKey key, const int64_t *__restrict__ m,
                                                            const uint32_t *__restrict__ cpq, uint64_t count,
                                                            uint32_t *__restrict__ ct) {
  constexpr int KP2 = 2 * KP, KN2 = 4 * KP, SP2 = 32 * KP, SN2 = 64 * KP;
  __shared__ __align__(16) uint32_t lds_all[16 * SN2];
  const uint32_t gi = wave_in_block() * 4 + group_in_wave();
  uint32_t *lds = lds_all + gi * SN2;
  uint64_t i = (uint64_t)blockIdx.x * 16 + gi;
  const bool valid = i < count;
  if (!valid) i = count - 1;
  const int64_t mi = m ? m[i] : 0;
  uint32_t cw[2][KP2];
#pragma unroll 1
  for (int which = 0; which < 2; ++which) {
    const DPrime &P = key.pr[which];
    uint32_t w[KP2], f[KP2], c2[KP2];
    ld<KP2>(w, cpq + (i * 2 + which) * SP2);  // omega = t^P mod P^2
    {
      // u = (m mod P) Q mod P, then f = 1 + m n mod P^2 = 1 + P u
      const Mod<KP> Mp = load_mod<KP>(P.P.N, P.P.ninv);
      uint32_t uu[KP], c[KP];
      signed_mod<KP>(uu, mi, Mp.n);
      ld<KP>(c, P.QR_P);
      mont_mul<KP>(uu, uu, c, Mp, lds);
      relayout<KP, KP2>(f, uu, lds);
    }
    const Mod<KP2> M2 = load_mod<KP2>(P.P2.N, P.P2.ninv);
    ld<KP2>(c2, P.PR_P2);
    mont_mul<KP2>(f, f, c2, M2, lds);
    add_one<KP2>(f);
    ld<KP2>(c2, P.P2.R2);
    mont_mul<KP2>(f, f, c2, M2, lds);  // Montgomery form of f
    mont_mul<KP2>(cw[which], w, f, M2, lds);  // the Montgomery factor of f cancels
  }
  const DPrime &Pp = key.pr[0];
  const Mod<KP2> M2 = load_mod<KP2>(Pp.P2.N, Pp.P2.ninv);
  uint32_t c[KP2], a[KP2], b[KP2];
  ld<KP2>(c, key.Cq);
  mont_mul<KP2>(a, cw[0], c, M2, lds);
  mont_mul<KP2>(b, cw[1], c, M2, lds);
  sub_mod<KP2>(a, a, b, M2);
  const Mod<KN2> Mn2 = load_mod<KN2>(key.n2.N, key.n2.ninv);
  uint32_t u[KN2], cq4[KN2], k4[KN2];
  relayout<KP2, KN2>(u, a, lds);
  relayout<KP2, KN2>(cq4, cw[1], lds);
  ld<KN2>(k4, key.q2R_n2);
  mont_mul<KN2>(u, u, k4, Mn2, lds);
  add_plain<KN2>(u, u, cq4);
  if (valid) st<KN2>(ct + i * SN2, u);
}

// ------------------------------------------------------ public-key encryption
// c = (1 + (m mod n) n) r^n mod n^2 by one exponentiation mod n^2, in three
// launches like the CRT path: k_pub_pre reduces r mod n^2 (the seeded X of
// L + 2 limbs is used as is: r^n mod n^2 depends only on r mod n), k_pow
// raises it to n (its units of both "primes" are n^2 and n, so a unit pair
// covers two consecutive ciphertexts), k_pub_post multiplies by 1 + (m mod
// n) n.  One 16-lane group per ciphertext in the light kernels.  x has
// count + (count & 1) rows: an odd count's last row is repeated, so the
// exponentiation's last unit pair reads and writes a row of its own.
template <int KP>
__global__ __launch_bounds__(kBlockThreads) void k_pub_pre(DKey key, uint64_t count, const uint32_t *__restrict__ r,
                                                          uint64_t seed, uint64_t roff, uint32_t *__restrict__ x) {
  constexpr int KN2 = 4 * KP, SN2 = 64 * KP, L = 32 * KP;
  __shared__ __align__(16) uint32_t lds_all[16 * SN2];
  const uint32_t gi = wave_in_block() * 4 + group_in_wave();
  uint32_t *lds = lds_all + gi * SN2;
  const uint64_t rows = count + (count & 1);
  uint64_t row = (uint64_t)blockIdx.x * 16 + gi;
  const bool valid = row < rows;
  if (!valid) row = rows - 1;
  const uint64_t i = row < count ? row : count - 1;
  const uint64_t W = (uint64_t)L / 2 + 1;
  const Mod<KN2> M = load_mod<KN2>(key.n2.N, key.n2.ninv);
  uint32_t v[KN2], c[KN2];
  if (r)
    ld_part<KN2>(v, r + i * L, L);
  else
    seeded_limbs<KN2>(v, seed, (roff + i) * W, 0, L + 2);
  // v mod n^2: a Montgomery product with R^2 gives v R, one with 1 leaves
  // the Montgomery domain
  ld<KN2>(c, key.n2.R2);
  mont_mul<KN2>(v, v, c, M, lds);
  set_small(c, 1u);
  mont_mul<KN2>(v, v, c, M, lds);
  if (valid) st<KN2>(x + row * SN2, v);
}

template <int KP>
__global__ __launch_bounds__(kBlockThreads) void k_pub_post(DKey key, const int64_t *__restrict__ m, uint64_t count,
                                                           const uint32_t *__restrict__ x, uint32_t *__restrict__ ct) {
  constexpr int KN2 = 4 * KP, SN2 = 64 * KP, L = 32 * KP;
  __shared__ __align__(16) uint32_t lds_all[16 * SN2];
  const uint32_t gi = wave_in_block() * 4 + group_in_wave();
  uint32_t *lds = lds_all + gi * SN2;
  uint64_t i = (uint64_t)blockIdx.x * 16 + gi;
  const bool valid = i < count;
  if (!valid) i = count - 1;
  const Mod<KN2> M = load_mod<KN2>(key.n2.N, key.n2.ninv);
  uint32_t v[KN2], c[KN2], f[KN2];
  ld<KN2>(v, x + i * SN2);
  // f = 1 + (m mod n) n, exact (< n^2), in Montgomery form
  ld_part<KN2>(c, key.n.N, L);
  signed_mod<KN2>(f, m ? m[i] : 0, c);
  ld<KN2>(c, key.nR_n2);
  mont_mul<KN2>(f, f, c, M, lds);
  add_one<KN2>(f);
  ld<KN2>(c, key.n2.R2);
  mont_mul<KN2>(f, f, c, M, lds);
  mont_mul<KN2>(v, v, f, M, lds);
  if (valid) st<KN2>(ct + i * SN2, v);
}

// ------------------------------------------------ obfuscated encryption
// ct = (1 + (m mod n) n) rho mod n^2 with a precomputed obfuscator
// rho = r^n mod n^2 (canonical).  Since (1 + m n) rho = rho + n (m rho) and
// n x mod n^2 = n (x mod n), ct = rho + n t mod n^2 with t = m rho mod n:
// three products mod n (rho R mod n from rho's halves, then times m) and
// one mod n^2 (n t), instead of three mod n^2.
template <int KP>
__global__ __launch_bounds__(kBlockThreads) void k_enc_obf(DKey key, const int64_t *__restrict__ m,
                                                          uint64_t count, const uint32_t *rho,
                                                          uint32_t *ct) {
  constexpr int KN = 2 * KP, KN2 = 4 * KP, SN2 = 64 * KP, L = 32 * KP;
  __shared__ __align__(16) uint32_t lds_all[16 * SN2];
  const uint32_t gi = wave_in_block() * 4 + group_in_wave();
  uint32_t *lds = lds_all + gi * SN2;
  uint64_t i = (uint64_t)blockIdx.x * 16 + gi;
  const bool valid = i < count;
  if (!valid) i = count - 1;
  uint32_t t2[KN2];
  {
    // t = m rho mod n: s = rho0 R + rho1 R^2 = rho R (mod n) from the halves
    // rho = rho0 + rho1 R (R = 2^(32 L)), then t = s (m mod n) R^-1
    const Mod<KN> Mn = load_mod<KN>(key.n.N, key.n.ninv);
    uint32_t a[KN], b[KN], c[KN];
    ld<KN>(a, rho + i * SN2);
    ld<KN>(c, key.n.R2);
    mont_mul<KN>(a, a, c, Mn, lds);
    ld<KN>(b, rho + i * SN2 + L);
    ld<KN>(c, key.n.R3);
    mont_mul<KN>(b, b, c, Mn, lds);
    add_mod<KN>(a, a, b, Mn);
    signed_mod<KN>(b, m[i], Mn.n);
    mont_mul<KN>(a, a, b, Mn, lds);
    relayout<KN, KN2>(t2, a, lds);
  }
  // ct = rho + n t mod n^2 (n t by one product with n R' mod n^2)
  const Mod<KN2> M = load_mod<KN2>(key.n2.N, key.n2.ninv);
  uint32_t x[KN2], c[KN2];
  ld<KN2>(c, key.nR_n2);
  mont_mul<KN2>(t2, t2, c, M, lds);
  ld<KN2>(x, rho + i * SN2);
  add_mod<KN2>(x, x, t2, M);
  if (valid) st<KN2>(ct + i * SN2, x);
}

// ------------------------------------------------------ ciphertext division
// out[i] = num[i] den[i]^-1 mod n^2, i.e. an encryption of m_num - m_den.
// Montgomery's batch-inversion trick per group of `batch` consecutive
// elements: prefix products Q_j = Q_(j-1) a_j R^-1 (Q_0 = a_0, stored in
// `out`), one inversion J = Q_last^-1 R, then backwards a_j^-1 R =
// J Q_(j-1) R^-1 and J <- J a_j R^-1 = Q_(j-1)^-1 R -- four Montgomery
// products per element plus one inversion per batch.  A batch whose product
// is not invertible is redone element by element; elements whose den is
// not a unit mod n^2 get 0 and are counted into *n_bad.
template <int KP>
__global__ __launch_bounds__(kBlockThreads) void k_ct_div(DKey key, const uint32_t *__restrict__ num,
                                                         const uint32_t *__restrict__ den, uint64_t count,
                                                         uint32_t batch, uint32_t *__restrict__ out,
                                                         uint32_t *__restrict__ n_bad) {
  constexpr int KN2 = 4 * KP, SN2 = 64 * KP;
  __shared__ __align__(16) uint32_t lds_all[16 * SN2];
  const uint32_t gi = wave_in_block() * 4 + group_in_wave();
  uint32_t *lds = lds_all + gi * SN2;
  const uint64_t first = ((uint64_t)blockIdx.x * 16 + gi) * batch;
  const uint32_t len = first < count ? (uint32_t)min((uint64_t)batch, count - first) : 0u;
  const Mod<KN2> M = load_mod<KN2>(key.n2.N, key.n2.ninv);

  // forward: prefix products
  uint32_t Q[KN2], a[KN2], t[KN2];
  set_zero(Q);
  set_zero(a);
  if (len) {
    ld<KN2>(Q, den + first * SN2);
    st<KN2>(out + first * SN2, Q);
  }
#pragma unroll 1
  for (uint32_t j = 1; j < batch; ++j) {
    const bool v = j < len;
    if (v) ld<KN2>(a, den + (first + j) * SN2);
    mont_mul<KN2>(t, Q, a, M, lds);
    select(Q, v, t, Q);
    if (v) st<KN2>(out + (first + j) * SN2, Q);
  }

  uint32_t J[KN2];
  const bool ok = mont_inverse<KN2>(J, Q, M, key.n2.R2, lds, len > 0u);

  // backward
  uint32_t p[KN2], ainv[KN2];
  set_zero(p);
#pragma unroll 1
  for (uint32_t j = batch; j-- > 0u;) {
    const bool v = ok && j < len;
    if (j > 0u) {
      if (v) ld<KN2>(t, out + (first + j - 1) * SN2);
      mont_mul<KN2>(ainv, J, t, M, lds);
      if (v) ld<KN2>(a, den + (first + j) * SN2);
      mont_mul<KN2>(t, J, a, M, lds);
      select(J, v, t, J);
    } else {
      copy(ainv, J);
    }
    if (v) ld<KN2>(p, num + (first + j) * SN2);
    mont_mul<KN2>(p, p, ainv, M, lds);
    if (v) st<KN2>(out + (first + j) * SN2, p);
  }

  // element-by-element retry for batches that held a non-unit
  const bool retry = len > 0u && !ok;
  if (wave_any(retry)) {
#pragma unroll 1
    for (uint32_t j = 0; j < batch; ++j) {
      const bool v = retry && j < len;
      if (v) {
        ld<KN2>(a, den + (first + j) * SN2);
        ld<KN2>(p, num + (first + j) * SN2);
      }
      const bool ok1 = mont_inverse<KN2>(J, a, M, key.n2.R2, lds, v);
      mont_mul<KN2>(p, p, J, M, lds);
      if (!ok1) set_zero(p);
      if (v) st<KN2>(out + (first + j) * SN2, p);
      if (v && !ok1 && glane() == 0 && n_bad) atomicAdd(n_bad, 1u);
    }
  }
}

// ------------------------------------------------------ split finding
// Best split per (node, feature) and per node from decrypted histograms:
// exact int64 prefix sums over the bins, XGBoost's gain in IEEE double with
// no contraction (every operation rounded as written), the largest gain with
// the lowest bin, then the lowest feature, on ties.  One block per node; each
// wave takes every fourth feature, lane l holds bins 4l .. 4l + 3.
struct SplitCand {
  double gain;
  int32_t feature, bin;
  int64_t gl, hl;
};

__device__ __forceinline__ bool split_better(const SplitCand &a, const SplitCand &b, bool by_feature) {
  if (a.gain > b.gain) return true;
  if (a.gain < b.gain || a.bin < 0) return false;
  if (b.bin < 0) return true;
  return by_feature ? a.feature < b.feature : a.bin < b.bin;
}

__device__ __forceinline__ SplitCand shfl_xor_cand(const SplitCand &c, int m) {
  SplitCand o;
  o.gain = __shfl_xor(c.gain, m, 64);
  o.feature = __shfl_xor(c.feature, m, 64);
  o.bin = __shfl_xor(c.bin, m, 64);
  o.gl = __shfl_xor(c.gl, m, 64);
  o.hl = __shfl_xor(c.hl, m, 64);
  return o;
}

__device__ __forceinline__ double split_term(double g, double h, double lam) {
#pragma clang fp contract(off)
  return (g * g) / (h + lam);
}

__global__ __launch_bounds__(kBlockThreads) void k_split(const int64_t *hist, const int64_t *minus, uint32_t F,
                                                        uint32_t B, double scale, double lam, double gamma,
                                                        double mcw, int64_t *derived, SplitCand *out_feat,
                                                        SplitCand *out_node) {
#pragma clang fp contract(off)
  __shared__ SplitCand waves[kBlockThreads / 64];
  const uint64_t node = blockIdx.x;
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const SplitCand none = {-__builtin_inf(), -1, -1, 0, 0};
  SplitCand best = none;
  for (uint32_t f = w; f < F; f += kBlockThreads / 64) {
    const uint64_t base = (node * F + f) * (uint64_t)B * 2;
    int64_t g[4], h[4], sg = 0, sh = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t b = lane * 4 + k;
      g[k] = h[k] = 0;
      if (b < B) {
        g[k] = hist[base + 2 * b];
        h[k] = hist[base + 2 * b + 1];
        if (minus) {
          g[k] -= minus[base + 2 * b];
          h[k] -= minus[base + 2 * b + 1];
        }
        if (derived) {
          derived[base + 2 * b] = g[k];
          derived[base + 2 * b + 1] = h[k];
        }
      }
      sg += g[k];
      sh += h[k];
    }
    // inclusive scan of the lane sums over the wave
    int64_t pg = sg, ph = sh;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t tg = __shfl_up(pg, d, 64), th = __shfl_up(ph, d, 64);
      if ((int)lane >= d) {
        pg += tg;
        ph += th;
      }
    }
    const int64_t G = __shfl(pg, 63, 64), H = __shfl(ph, 63, 64);
    const double fg = (double)G * scale, fh = (double)H * scale;
    const double tp = split_term(fg, fh, lam);
    int64_t gl = pg - sg, hl = ph - sh;
    SplitCand c = none;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t b = lane * 4 + k;
      gl += g[k];
      hl += h[k];
      if (b + 1 < B) {
        const double fgl = (double)gl * scale, fhl = (double)hl * scale;
        const double fgr = (double)(G - gl) * scale, fhr = (double)(H - hl) * scale;
        if (fhl >= mcw && fhr >= mcw && fhl + lam > 0.0 && fhr + lam > 0.0) {
          const double gain = 0.5 * ((split_term(fgl, fhl, lam) + split_term(fgr, fhr, lam)) - tp) - gamma;
          if (gain > c.gain) c = {gain, (int32_t)f, (int32_t)b, gl, hl};
        }
      }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      const SplitCand o = shfl_xor_cand(c, m);
      if (split_better(o, c, false)) c = o;
    }
    if (lane == 0 && out_feat) out_feat[node * F + f] = c;
    if (split_better(c, best, true)) best = c;
  }
  if (lane == 0) waves[w] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    SplitCand b = waves[0];
    for (uint32_t i = 1; i < kBlockThreads / 64; ++i)
      if (split_better(waves[i], b, true)) b = waves[i];
    out_node[node] = b;
  }
}

// ------------------------------------------------ ciphertext products
// out[i] = a[i] b[i] mod n^2 (canonical in and out): the encrypted sum of two
// ciphertext arrays.  MM(a, b) = a b R^-1, then MM(., R^2) = a b.
template <int KP>
__global__ __launch_bounds__(kBlockThreads) void k_ct_mul(DKey key, const uint32_t *a, const uint32_t *b,
                                                         uint64_t count, uint32_t *out) {
  constexpr int KN2 = 4 * KP, SN2 = 64 * KP;
  __shared__ __align__(16) uint32_t lds_all[16 * SN2];
  const uint32_t gi = wave_in_block() * 4 + group_in_wave();
  uint32_t *lds = lds_all + gi * SN2;
  uint64_t i = (uint64_t)blockIdx.x * 16 + gi;
  const bool valid = i < count;
  if (!valid) i = count - 1;
  const Mod<KN2> M = load_mod<KN2>(key.n2.N, key.n2.ninv);
  uint32_t x[KN2], y[KN2];
  ld<KN2>(x, a + i * SN2);
  ld<KN2>(y, b + i * SN2);
  mont_mul<KN2>(x, x, y, M, lds);
  ld<KN2>(y, key.n2.R2);
  mont_mul<KN2>(x, x, y, M, lds);
  if (valid) st<KN2>(out + i * SN2, x);
}

// ------------------------------------------------------ packing
// Folds `slots` consecutive ciphertexts into one (public key only):
// prod_j c_j^(2^(64 j)) (1 + K n) mod n^2 with K = sum_j 2^(64 j + 63), an
// encryption of sum_j 2^(64 j) (m_j + 2^63), by Horner's rule from the top
// slot down (64 squarings per slot) in Montgomery form.  The last packed
// ciphertext may hold fewer slots; the wave's loops run over `slots` and its
// missing slots multiply by one.
template <int KP>
__global__ __launch_bounds__(kBlockThreads) void k_pack(DKey key, const uint32_t *__restrict__ ct, uint64_t count,
                                                       uint32_t slots, uint32_t *__restrict__ packed) {
  constexpr int KN2 = 4 * KP, SN2 = 64 * KP;
  constexpr int S29 = he29::limbs_for_group(SN2, 16), K = S29 / 16, ROW = 2 * S29 > SN2 ? 2 * S29 : SN2;
  constexpr int v = he29::variant(16);
  __shared__ __align__(16) uint32_t lds_all[16 * ROW + S29];
  uint32_t *const zeros = lds_all + 16 * ROW;
  zero_lds(zeros, S29);
  const uint32_t gi = wave_in_block() * 4 + group_in_wave();
  uint32_t *lds = lds_all + gi * ROW;
  const uint64_t n_packed = (count + slots - 1) / slots;
  uint64_t p = (uint64_t)blockIdx.x * 16 + gi;
  const bool valid = p < n_packed;
  if (!valid) p = n_packed - 1;
  const uint64_t first = p * slots;
  const uint32_t my_slots = (uint32_t)min((uint64_t)slots, count - first);
  const Mod29<K> M = load_mod29<K, 16>(key.n2);
  const uint32_t *one29 = key.n2.R1_29[v], *r2_29 = key.n2.R2_29[v];
  // radix-2^29 Montgomery form of slot ciphertext j: x R'^2 R'^-1 = x R'; a
  // slot this packed ciphertext does not have gets R' R' R'^-1 = R', the
  // Montgomery one (its row read is the packed ciphertext's first, in bounds)
  auto slot_mont = [&](uint32_t (&y)[K], uint32_t j, bool have) {
    uint32_t x[KN2], c[K];
    ld<KN2>(x, ct + (first + (have ? j : 0u)) * SN2);
    to29<KN2, K, 16>(y, x, lds);
    if (!have) ld29<K, 16>(y, one29);
    ld29<K, 16>(c, have ? r2_29 : one29);
    mm29<K, 16>(y, y, c, M, lds);
  };
  uint32_t acc[K];
  // top slot; a shorter (last) packed ciphertext starts from the one
  slot_mont(acc, slots - 1, my_slots == slots);
#pragma unroll 1
  for (uint32_t j = slots - 1; j-- > 0;) {
#pragma unroll 1
    for (int t = 0; t < 64; ++t) sq29<K, 16>(acc, acc, M, lds, zeros);
    uint32_t y[K];
    slot_mont(y, j, j < my_slots);
    mm29<K, 16>(acc, y, acc, M, lds);
  }
  // f = 1 + K n: K has bit 31 of every odd limb below 2 my_slots
  uint32_t f[KN2];
  {
    const Mod<KN2> M32 = load_mod<KN2>(key.n2.N, key.n2.ninv);
    uint32_t c[KN2];
#pragma unroll
    for (int i = 0; i < KN2; ++i) {
      const uint32_t idx = glane() * KN2 + i;
      f[i] = ((idx & 1u) && (idx >> 1) < my_slots) ? 0x80000000u : 0u;
    }
    ld<KN2>(c, key.nR_n2);
    mont_mul<KN2>(f, f, c, M32, lds);  // K n mod n^2
    add_one<KN2>(f);
  }
  // acc f R'^-1 leaves the Montgomery form
  uint32_t f29[K];
  to29<KN2, K, 16>(f29, f, lds);
  mm29<K, 16>(acc, f29, acc, M, lds);
  canon29<K, 16>(acc, M);
  uint32_t out[KN2];
  to32<K, KN2, 16>(out, acc, lds);
  if (valid) st<KN2>(packed + p * SN2, out);
}

// Slot values of decrypted packed plaintexts raw[n_packed][L]: value i is
// the 64-bit field (i mod slots) of plaintext i / slots, minus 2^63.  A
// plaintext with bits above its last slot (a slot sum outside the signed
// 64-bit range at the top, or a negative total) is counted into *n_overflow.
__global__ void k_unpack(const uint32_t *__restrict__ raw, uint64_t count, uint32_t slots, uint32_t L,
                         int64_t *__restrict__ m, uint32_t *__restrict__ n_overflow) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t p = i / slots;
  const uint32_t j = (uint32_t)(i - p * slots);
  const uint32_t my_slots = (uint32_t)min((uint64_t)slots, count - p * slots);
  const uint32_t *w = raw + p * L;
  const uint64_t v = (uint64_t)w[2 * j] | ((uint64_t)w[2 * j + 1] << 32);
  m[i] = (int64_t)(v ^ 0x8000000000000000ull);
  if (j == my_slots - 1 && n_overflow) {
    bool high = false;
    for (uint32_t k = 2 * my_slots; k < L; ++k) high = high || w[k] != 0u;
    if (high) atomicAdd(n_overflow, 1u);
  }
}

// ------------------------------------------------------ Montgomery conversion
// x -> x R' mod n^2 (to_mont) or x R'^-1 mod n^2, R' the radix-2^29 factor of
// the histogram kernels' G-lane groups; canonical 32-bit limbs in and out.
template <int KP, int G>
__global__ __launch_bounds__(kBlockThreads) void k_mont_convert(DKey key, const uint32_t *in, uint64_t count,
                                                               uint32_t *out, int to_mont) {
  constexpr int SN2 = 64 * KP, K32 = SN2 / G, GB = kBlockThreads / G;
  constexpr int S29 = he29::limbs_for_group(SN2, G), K = S29 / G, ROW = S29 > SN2 ? S29 : SN2;
  __shared__ __align__(16) uint32_t lds_all[GB * ROW];
  uint32_t *lds = lds_all + (threadIdx.x / G) * ROW;
  uint64_t i = (uint64_t)blockIdx.x * GB + threadIdx.x / G;
  const bool valid = i < count;
  if (!valid) i = count - 1;
  const Mod29<K> M = load_mod29<K, G>(key.n2);
  uint32_t x[K32], t[K], c[K];
  ld<K32, G>(x, in + i * SN2);
  to29<K32, K, G>(t, x, lds);
  if (to_mont)
    ld29<K, G>(c, key.n2.R2_29[he29::variant(G)]);
  else
    set_small<K, G>(c, 1u);
  mm29<K, G>(t, t, c, M, lds);
  canon29<K, G>(t, M);
  to32<K, K32, G>(x, t, lds);
  if (valid) st<K32, G>(out + i * SN2, x);
}

// -------------------------------------------------------------- decryption
// For (ciphertext i, prime P): x = c^(P-1) mod P^2 (k_pow), then
// m_P = ((x - 1) / P) h_P mod P, and Garner's combination of m_p, m_q.
// k_dec_pre: c mod P^2 for both primes into xpq[2 i + P] (S_P2 limbs):
// c mod P^2 = c0 + c1 R' mod P^2 (halves c0, c1; R' = 2^(32 S_P2)), each half
// by a Montgomery product with R' resp. R'^2.  One 16-lane group per (i, P).
template <int KP>
__global__ __launch_bounds__(kBlockThreads) void k_dec_pre(DKey key, const uint32_t *__restrict__ ct, uint64_t count,
                                                          uint32_t *__restrict__ xpq) {
  constexpr int KP2 = 2 * KP, SP2 = 32 * KP, SN2 = 64 * KP;
  __shared__ __align__(16) uint32_t lds_all[16 * SP2];
  const uint32_t gi = wave_in_block() * 4 + group_in_wave();
  uint32_t *lds = lds_all + gi * SP2;
  uint64_t u = (uint64_t)blockIdx.x * 16 + gi;
  const bool valid = u < 2 * count;
  if (!valid) u = 2 * count - 1;
  const uint64_t i = u >> 1;
  const DPrime &P = key.pr[u & 1];
  const Mod<KP2> M2 = load_mod<KP2>(P.P2.N, P.P2.ninv);
  uint32_t x[KP2], y[KP2], c[KP2];
  ld<KP2>(x, ct + i * SN2);
  ld<KP2>(y, ct + i * SN2 + SP2);
  ld<KP2>(c, P.P2.R1);
  mont_mul<KP2>(x, x, c, M2, lds);
  ld<KP2>(c, P.P2.R2);
  mont_mul<KP2>(y, y, c, M2, lds);
  add_mod<KP2>(x, x, y, M2);
  if (valid) st<KP2>(xpq + u * SP2, x);
}

// m_P = ((x_P - 1) / P) h_P mod P from x_P = c^(P-1) mod P^2 (exact
// division: (x - 1) P^-1 mod 2^(32 S_P), a low-half product), then
// m = m_q + q ((m_p - m_q) q^-1 mod p) and the signed decode.
template <int KP>
__global__ __launch_bounds__(kBlockThreads) void k_dec_b(DKey key, const uint32_t *__restrict__ xpq,
                                                        uint64_t count, int64_t *__restrict__ mout,
                                                        uint32_t *__restrict__ raw,
                                                        uint32_t *__restrict__ n_overflow) {
  constexpr int KN = 2 * KP, KP2 = 2 * KP, SP2 = 32 * KP, SN = 32 * KP;
  __shared__ __align__(16) uint32_t lds_all[16 * SN];
  const uint32_t gi = wave_in_block() * 4 + group_in_wave();
  uint32_t *lds = lds_all + gi * SN;
  uint64_t i = (uint64_t)blockIdx.x * 16 + gi;
  const bool valid = i < count;
  if (!valid) i = count - 1;
  uint32_t mpq[2][KP];
#pragma unroll 1
  for (int which = 0; which < 2; ++which) {
    const DPrime &P = key.pr[which];
    uint32_t x[KP2], one[KP2], lo[KP], k[KP], c[KP];
    ld<KP2>(x, xpq + (i * 2 + which) * SP2);  // canonical, = 1 mod P
    set_small<KP2>(one, 1u);
    sub_plain<KP2>(x, x, one);                 // x - 1 = k P
    relayout<KP2, KP>(lo, x, lds);
    ld<KP>(c, P.Pinv);
    st<KP>(lds, lo);
    __builtin_amdgcn_wave_barrier();
    mul_lo_lds<KP>(k, lds, c);
    __builtin_amdgcn_wave_barrier();
    const Mod<KP> Mp = load_mod<KP>(P.P.N, P.P.ninv);
    ld<KP>(c, P.hR_P);
    mont_mul<KP>(mpq[which], k, c, Mp, lds);
  }
  const DPrime &Pp = key.pr[0];
  const Mod<KP> Mp = load_mod<KP>(Pp.P.N, Pp.P.ninv);
  uint32_t mp[KP], mq[KP], c[KP];
  copy(mp, mpq[0]);
  copy(mq, mpq[1]);
  ld<KP>(c, Pp.P.R2);
  mont_mul<KP>(mp, mp, c, Mp, lds);
  uint32_t mqr[KP];
  mont_mul<KP>(mqr, mq, c, Mp, lds);
  sub_mod<KP>(mp, mp, mqr, Mp);
  ld<KP>(c, key.qinv_p);
  mont_mul<KP>(mp, mp, c, Mp, lds);  // u = (m_p - m_q) q^-1 mod p
  const Mod<KN> Mn = load_mod<KN>(key.n.N, key.n.ninv);
  uint32_t u[KN], v[KN], cn[KN];
  relayout<KP, KN>(u, mp, lds);
  relayout<KP, KN>(v, mq, lds);
  ld<KN>(cn, key.qR_n);
  mont_mul<KN>(u, u, cn, Mn, lds);  // q u (exact, < n)
  add_plain<KN>(u, u, v);           // m in [0, n)
  if (raw && valid) st<KN>(raw + i * SN, u);
  // signed decode: m >= (n + 1) / 2 means m - n
  ld<KN>(cn, key.half);
  const bool below_half = bcast_last(sub_plain<KN>(v, u, cn) ? 1u : 0u) != 0u;
  uint32_t mag[KN];
  sub_plain<KN>(mag, Mn.n, u);
  select(mag, below_half, u, mag);
  bool high = false;
#pragma unroll
  for (int j = 0; j < KN; ++j) high = high || ((glane() * KN + j) >= 2 && mag[j] != 0u);
  high = row_any(high);
  const uint64_t lo64 = (uint64_t)bcast_first(mag[0]) | ((uint64_t)bcast_first(mag[1]) << 32);
  int64_t val;
  bool ovf;
  if (below_half) {
    ovf = high || (lo64 >> 63);
    val = ovf ? INT64_MAX : (int64_t)lo64;
  } else {
    ovf = high || lo64 > (1ull << 63);
    val = ovf ? INT64_MIN : (int64_t)((uint64_t)0 - lo64);
  }
  if (valid && glane() == 0) {
    mout[i] = val;
    if (ovf && n_overflow) atomicAdd(n_overflow, 1u);
  }
}

// ------------------------------------------------------------ histograms
__global__ void k_fill(uint32_t *p, uint64_t n, uint32_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

constexpr int kJobsPerSetup = 24;
struct JobPack {
  DJob j[kJobsPerSetup];
};
__global__ void k_job_setup(JobPack pack, uint32_t n, DJob *dst) {
  if (threadIdx.x < n) dst[threadIdx.x] = pack.j[threadIdx.x];
}

__device__ __forceinline__ uint32_t find_job_by_blk(const DJob *jobs, uint32_t n_jobs, uint64_t blk) {
  uint32_t j = 0;
  while (j + 1 < n_jobs && jobs[j + 1].blk_off <= blk) ++j;
  return j;
}
__device__ __forceinline__ uint32_t find_job_by_f(const DJob *jobs, uint32_t n_jobs, uint64_t f) {
  uint32_t j = 0;
  while (j + 1 < n_jobs && jobs[j + 1].f_off <= f) ++j;
  return j;
}
__device__ __forceinline__ uint32_t find_job_by_fb(const DJob *jobs, uint32_t n_jobs, uint64_t e) {
  uint32_t j = 0;
  while (j + 1 < n_jobs && jobs[j + 1].fb_off <= e) ++j;
  return j;
}

// Bin counts of one (job, feature, sample block) into counts[fb].  Samples
// whose row is not resident or whose bin is out of range are skipped and
// counted into the job's n_bad (bucket_sample).
__global__ __launch_bounds__(256) void k_hist_count(HistWs ws) {
  __shared__ uint32_t h[256];
  __shared__ uint32_t nbad;
  const uint64_t blk = blockIdx.x;
  const uint32_t jn = find_job_by_blk(ws.jobs, ws.n_jobs, blk);
  const DJob J = ws.jobs[jn];
  uint32_t f;
  uint64_t s0, s1;
  bucket_block(blk - J.blk_off, J.nblk, J.n, kSampleBlock, f, s0, s1);
  h[threadIdx.x] = 0;
  if (threadIdx.x == 0) nbad = 0;
  __syncthreads();
  const uint8_t *bf = J.bins + (uint64_t)f * J.ld;
  for (uint64_t s = s0 + threadIdx.x; s < s1; s += 256) {
    uint32_t row, bin;
    if (bucket_sample(J.idx, bf, ws.rows, J.B, s, row, bin))
      atomicAdd(&h[bin], 1u);
    else
      atomicAdd(&nbad, 1u);
  }
  __syncthreads();
  if (threadIdx.x < J.B && h[threadIdx.x])
    atomicAdd(&ws.counts[J.fb_off + (uint64_t)f * J.B + threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x == 0 && nbad && J.n_bad) atomicAdd(J.n_bad, nbad);
}

// Per (job, feature): exclusive scan of the bin counts (the bins' sample runs
// in bin order), chunk counts per bin and their local prefix, taken over the
// bins in decreasing order of their counts (ties: lower bin first), so that
// consecutive work items have about the same length and the waves that take
// several items at once pad little; ftot = chunks of this feature; border =
// the feature's bins in that order (k_hist_final's entry order).
__global__ __launch_bounds__(256) void k_hist_scan(HistWs ws) {
  __shared__ uint32_t sc[256], sh[256], cn[256];
  const uint64_t jf = blockIdx.x;
  const uint32_t jn = find_job_by_f(ws.jobs, ws.n_jobs, jf);
  const DJob J = ws.jobs[jn];
  const uint32_t f = (uint32_t)(jf - J.f_off);
  const uint64_t e = J.fb_off + (uint64_t)f * J.B + threadIdx.x;
  const uint32_t t = threadIdx.x;
  const uint32_t cnt = t < J.B ? ws.counts[e] : 0u;
  const uint32_t nch = (cnt + ws.chunk - 1) / ws.chunk;
  cn[t] = cnt;
  __syncthreads();
  // this bin's place in the item order (bins past J.B keep their own index,
  // which no bin below J.B takes)
  uint32_t rank = t;
  if (t < J.B) {
    rank = 0;
    for (uint32_t b = 0; b < J.B; ++b) {
      const uint32_t c = cn[b];
      rank += (c > cnt || (c == cnt && b < t)) ? 1u : 0u;
    }
  }
  sc[t] = cnt;
  sh[rank] = nch;
  __syncthreads();
  for (uint32_t d = 1; d < 256; d <<= 1) {  // inclusive Hillis-Steele scans
    const uint32_t a = t >= d ? sc[t - d] : 0u, b = t >= d ? sh[t - d] : 0u;
    __syncthreads();
    sc[t] += a;
    sh[t] += b;
    __syncthreads();
  }
  if (t < J.B) {
    ws.offs[e] = sc[t] - cnt;
    ws.cursor[e] = sc[t] - cnt;
    ws.fch[e] = nch;
    ws.fitem[e] = sh[rank] - nch;  // local; made global by k_hist_items
    ws.border[e - t + rank] = t;   // the bins in rank order, for the final kernel
  }
  if (t == 255) ws.ftot[jf] = sh[255];
}

// Exclusive scan of ftot over all (job, feature) pairs; total item count.
__global__ __launch_bounds__(1024) void k_hist_base(HistWs ws) {
  __shared__ uint32_t s[1024];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint64_t b0 = 0; b0 < ws.total_f; b0 += 1024) {
    const uint64_t i = b0 + threadIdx.x;
    const uint32_t v = i < ws.total_f ? ws.ftot[i] : 0u;
    s[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
      const uint32_t a = threadIdx.x >= d ? s[threadIdx.x - d] : 0u;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < ws.total_f) ws.fbase[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *ws.n_items = carry;
    *ws.next = 0;  // k_hist_chunk's work counter
  }
}

// Items of one (job, feature): every bin's sample run split into its nch
// chunks of equal length (to one sample), each at most `chunk` samples.
__global__ __launch_bounds__(256) void k_hist_items(HistWs ws) {
  const uint64_t jf = blockIdx.x;
  const uint32_t jn = find_job_by_f(ws.jobs, ws.n_jobs, jf);
  const DJob J = ws.jobs[jn];
  const uint32_t f = (uint32_t)(jf - J.f_off);
  const uint32_t b = threadIdx.x;
  if (b >= J.B) return;
  const uint64_t e = J.fb_off + (uint64_t)f * J.B + b;
  const uint32_t first = ws.fbase[jf] + ws.fitem[e];
  ws.fitem[e] = first;
  const uint32_t nch = ws.fch[e], cnt = ws.counts[e];
  const uint64_t start = J.perm_off + (uint64_t)f * J.n + ws.offs[e];
  for (uint32_t c = 0; c < nch; ++c) {
    const uint32_t lo = (uint32_t)((uint64_t)c * cnt / nch), hi = (uint32_t)((uint64_t)(c + 1) * cnt / nch);
    HistItem it;
    it.start = start + lo;
    it.len = hi - lo;
    it.pad = 0;
    ws.items[first + c] = it;
  }
}

// Scatter of sample rows into per-(feature, bin) runs of perm, skipping the
// samples k_hist_count skipped (bucket_sample), so each run receives exactly
// the samples counted for its bin.
__global__ __launch_bounds__(256) void k_hist_scatter(HistWs ws) {
  __shared__ uint32_t h[256], base[256];
  const uint64_t blk = blockIdx.x;
  const uint32_t jn = find_job_by_blk(ws.jobs, ws.n_jobs, blk);
  const DJob J = ws.jobs[jn];
  uint32_t f;
  uint64_t s0, s1;
  bucket_block(blk - J.blk_off, J.nblk, J.n, kSampleBlock, f, s0, s1);
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint8_t *bf = J.bins + (uint64_t)f * J.ld;
  constexpr int kPer = kSampleBlock / 256;
  uint32_t rows[kPer], bn[kPer], rk[kPer];
  bool ok[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint64_t s = s0 + threadIdx.x + (uint64_t)k * 256;
    ok[k] = s < s1 && bucket_sample(J.idx, bf, ws.rows, J.B, s, rows[k], bn[k]);
    if (ok[k]) rk[k] = atomicAdd(&h[bn[k]], 1u);
  }
  __syncthreads();
  const uint64_t e0 = J.fb_off + (uint64_t)f * J.B;
  if (threadIdx.x < J.B && h[threadIdx.x]) base[threadIdx.x] = atomicAdd(&ws.cursor[e0 + threadIdx.x], h[threadIdx.x]);
  __syncthreads();
  uint32_t *pf = ws.perm + J.perm_off + (uint64_t)f * J.n;
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (ok[k]) pf[bucket_slot(base[bn[k]], rk[k])] = rows[k];
}

// Product of the ciphertexts of one item (chunk) per (item, slot), in
// groups of G lanes (GW = 64 / G groups per wave; bit 0 of a group's index is
// the slot g/h).  With split 2 an item is taken by four groups: bit 1 of the
// group index picks the first or second half of the chunk, the halves are
// combined at the end, and a wave takes GW / 4 items.  With split 1 a wave
// takes GW / 2 items, one group per (item, slot).  The gathered rows are in
// the radix-2^29 Montgomery form x R' mod n^2 (32-bit limbs); each is moved
// to 29-bit limbs through the group's LDS row and multiplied into the
// accumulator, which stays in 29-bit limbs; partials are stored settled in
// 29-bit limbs (S29 words).  Every loop bound is the maximum over the wave's
// items, so the cross-lane steps of the arithmetic always run on the whole
// wave.
template <int KP, int G>
__global__ __launch_bounds__(kBlockThreads, G == 16 ? kHistWaves : 3) void k_hist_chunk(DKey key,
                                                                                    const uint32_t *__restrict__ ctm,
                                                                      HistWs ws) {
  constexpr int S = 64 * KP, K32 = S / G, GW = 64 / G;
  constexpr int S29 = he29::limbs_for_group(S, G), K = S29 / G, ROW = S29 > S ? S29 : S;
  __shared__ __align__(16) uint32_t lds_all[(kBlockThreads / 64) * GW * ROW];
  const uint32_t g = (threadIdx.x & 63u) / G;
  const uint32_t wrow = wave_in_block() * GW;
  uint32_t *lds = lds_all + (wrow + g) * ROW;
  const uint32_t slot = g & 1u;
  const bool split = ws.split == 2;
  const uint32_t half = (g >> 1) & 1u;
  const Mod29<K> M = load_mod29<K, G>(key.n2);
  const uint32_t *one29 = key.n2.R1_29[he29::variant(G)];  // Montgomery form of 1
  const uint64_t n_items = *ws.n_items;
  const uint64_t per_wave = split ? GW / 4 : GW / 2;
  // wave units (per_wave consecutive items) are claimed from a counter, so a
  // wave that finishes early takes the next unit and the waves end together
  // to within about one unit; the items come longest first within each
  // feature
  for (uint64_t w0 = claim_unit(ws.next) * per_wave; w0 < n_items; w0 = claim_unit(ws.next) * per_wave) {
    // this group's sample run and the wave-wide trip count
    const uint64_t it = w0 + (split ? (g >> 2) : (g >> 1));
    const bool valid = it < n_items;
    const HistItem item = ws.items[valid ? it : n_items - 1];
    uint32_t trip = 0;
    for (uint64_t w = w0; w < w0 + per_wave && w < n_items; ++w) {
      const uint32_t l = ws.items[w].len;
      trip = max(trip, split ? (l + 1) >> 1 : l);
    }
    uint64_t start;
    uint32_t my_len;
    if (split) {
      const uint32_t len_lo = (item.len + 1) >> 1;
      my_len = valid ? (half ? item.len >> 1 : len_lo) : 0u;
      start = item.start + (half ? len_lo : 0u);
    } else {
      my_len = valid ? item.len : 0u;
      start = item.start;
    }
    const uint32_t *pp = ws.perm + start;
    // a group with nothing (more) to do reads row 0 (in bounds) and takes
    // the Montgomery one in its place
    const uint32_t last = my_len ? my_len - 1 : 0u;
    const uint32_t *base = ctm + (uint64_t)slot * S;
    uint32_t acc[K];
    {
      uint32_t x[K32];
      ld<K32, G>(x, base + (my_len ? (uint64_t)pp[0] * 2 * S : 0));
      to29<K32, K, G>(acc, x, lds);
      uint32_t one[K];
      ld29<K, G>(one, one29);
      select(acc, my_len != 0u, acc, one);
    }
    // the row of each product is loaded at the top of its iteration (no
    // prefetch: the registers go to the columns; the other waves of the SIMD
    // cover the gather)
#pragma unroll 1
    for (uint32_t k = 1; k < trip; ++k) {
      // past the end of this group's run the multiplier is the Montgomery
      // form of 1, so the product leaves the accumulator's value as it is
      uint32_t x[K32], a[K];
      ld<K32, G>(x, base + (my_len ? (uint64_t)pp[min(k, last)] * 2 * S : 0));
      to29<K32, K, G>(a, x, lds);
      if (k >= my_len) ld29<K, G>(a, one29);
      mm29<K, G>(acc, a, acc, M, lds);
    }
    if (split) {
      // combine the two halves
      st29<K, G>(lds, acc);
      __builtin_amdgcn_wave_barrier();
      uint32_t other[K];
      ld29<K, G>(other, lds_all + (wrow + (g ^ 2u)) * ROW);
      __builtin_amdgcn_wave_barrier();
      mm29<K, G>(acc, acc, other, M, lds);
      if (half == 0 && valid) st29<K, G>(ws.partials + (it * 2 + slot) * S29, acc);
    } else if (valid) {
      st29<K, G>(ws.partials + (it * 2 + slot) * S29, acc);
    }
    if (ws.mm_count && glane<G>() == 0) {
      // products joining two real partials (the algorithm's count) and
      // products this group executed, masked padding included
      uint64_t real = my_len ? my_len - 1 : 0, done = trip ? trip - 1 : 0;
      if (split) {
        done += 1;
        real += (half == 0 && my_len >= 1 && item.len >= 2) ? 1 : 0;
      }
      atomicAdd(&ws.mm_count[0], (unsigned long long)real);
      atomicAdd(&ws.mm_count[1], (unsigned long long)done);
    }
  }
}

// Out of Montgomery form (a product with 1), exact, back to 32-bit limbs;
// stored by the groups with `store`.
template <int G, int K, int K32>
__device__ __forceinline__ void final_out(uint32_t (&acc)[K], const Mod29<K> &M, uint32_t *lds, uint32_t *dst,
                                          bool store) {
  uint32_t one[K];
  set_small<K, G>(one, 1u);
  mm29<K, G>(acc, acc, one, M, lds);
  canon29<K, G>(acc, M);
  uint32_t y[K32];
  to32<K, K32, G>(y, acc, lds);
  if (store) st<K32, G>(dst, y);
}

// Ranks (within a feature, by decreasing bin count) that k_hist_final takes
// one per block; higher ranks go one per wave, four to a block.
constexpr uint32_t kFinalSolo = 8;

// Final product over the chunks of one (job, feature, bin), conversion out of
// Montgomery form, and the store into the job's histogram.  A block takes
// one rank of one (job, feature) among the first kFinalSolo ranks, else four
// consecutive ranks, one per wave; the units go rank-major over all
// (job, feature) pairs, so the heaviest bins start first.
//  * A block's own entry: its 16 groups are (slot g/h) x (8 runs); the
//    entry's nch partials are cut into P runs of equal length (to one), P
//    the largest power of two that is at most 8 and at most nch / 2, each
//    run's product is one group's chain (about nch / P products instead of
//    nch / 2), and the P products are joined in log2(P) levels through LDS.
//  * A wave's entry: its 4 groups are (slot) x (first or second half of the
//    partials), the halves joined at the end.
template <int KP, int G>
__global__ __launch_bounds__(kBlockThreads, 4) void k_hist_final(DKey key, HistWs ws) {
  static_assert(G == 16, "four groups per wave: two slots x two parts");
  constexpr int S = 64 * KP, K32 = S / G, GW = 64 / G, kWaves = kBlockThreads / 64, kParts = 2 * kWaves;
  constexpr int S29 = he29::limbs_for_group(S, G), K = S29 / G, ROW = S29 > S ? S29 : S;
  __shared__ __align__(16) uint32_t lds_all[kWaves * GW * ROW];
  const uint32_t wv = wave_in_block();
  const uint32_t g = (threadIdx.x & 63u) / G;
  uint32_t *lds = lds_all + (wv * GW + g) * ROW;
  const uint32_t slot = g & 1u, half = g >> 1, part = 2 * wv + half;
  const Mod29<K> M = load_mod29<K, G>(key.n2);
  const uint32_t *one29 = key.n2.R1_29[he29::variant(G)];  // Montgomery form of 1
  const uint64_t solo = ws.total_f * kFinalSolo;
  const uint64_t units = solo + ws.total_f * ((256 - kFinalSolo) / kWaves);  // ranks past a job's bins are skipped
  for (uint64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const bool whole = u < solo;  // block-uniform
    const uint64_t v = whole ? u : u - solo;
    const uint64_t jf = v % ws.total_f;
    const uint32_t r = whole ? (uint32_t)(v / ws.total_f) : kFinalSolo + kWaves * (uint32_t)(v / ws.total_f) + wv;
    const DJob J = ws.jobs[find_job_by_f(ws.jobs, ws.n_jobs, jf)];
    if (whole && r >= J.B) continue;  // block-uniform
    const uint64_t fb_f = (jf - J.f_off) * J.B;  // the feature's first entry within the job
    if (whole) {
      const uint32_t bin = ws.border[J.fb_off + fb_f + r];
      const uint64_t e = J.fb_off + fb_f + bin;
      const uint32_t nch = ws.fch[e], first = ws.fitem[e];
      uint32_t P = 1;
      while (P < (uint32_t)kParts && 4 * P <= nch) P *= 2;
      const bool mine = part < P;
      const uint32_t lo = mine ? (uint32_t)((uint64_t)part * nch / P) : 0u;
      const uint32_t len = mine ? (uint32_t)((uint64_t)(part + 1) * nch / P) - lo : 0u;
      const uint32_t maxlen = (nch + P - 1) / P;
      const bool wave_on = 2 * wv < P;  // wave-uniform: the wave holds a run
      uint64_t done = 0;
      uint32_t acc[K];
      if (wave_on) {
        // past this group's run the multiplier is the Montgomery form of 1;
        // each partial is loaded one product ahead of its use
        const uint64_t p0 = (uint64_t)first + lo;
        uint32_t b[K], nb[K];
        ld29<K, G>(acc, len ? ws.partials + (p0 * 2 + slot) * S29 : one29);
        ld29<K, G>(nb, 1 < len ? ws.partials + ((p0 + 1) * 2 + slot) * S29 : one29);
#pragma unroll 1
        for (uint32_t k = 1; k < maxlen; ++k) {
#pragma unroll
          for (int j = 0; j < K; ++j) b[j] = nb[j];
          if (k + 1 < maxlen) ld29<K, G>(nb, k + 1 < len ? ws.partials + ((p0 + k + 1) * 2 + slot) * S29 : one29);
          mm29<K, G>(acc, b, acc, M, lds);
        }
        done += maxlen ? maxlen - 1 : 0;
      }
      // level d joins run p with run p + d for p a multiple of 2d; only the
      // even runs (half 0 of a wave) ever join, so a wave joins or not as a
      // whole
      for (uint32_t d = 1; d < P; d <<= 1) {  // block-uniform
        if (wave_on) st29<K, G>(lds, acc);
        __syncthreads();
        const bool wave_join = (2 * wv) % (2 * d) == 0 && 2 * wv + d < P;
        uint32_t other[K];
        if (wave_join) {
          const uint32_t q = part + d;  // in range for the joining (even) runs
          const uint32_t qr = half == 0 ? (q >> 1) * GW + ((q & 1u) << 1 | slot) : wv * GW + g;
          ld29<K, G>(other, lds_all + qr * ROW);
        }
        __syncthreads();
        if (wave_join) {
          uint32_t t[K];
          mm29<K, G>(t, acc, other, M, lds);
          select(acc, half == 0, t, acc);
          ++done;
        }
      }
      if (wv == 0) {
        final_out<G, K, K32>(acc, M, lds, J.hist + ((fb_f + bin) * 2 + slot) * S, half == 0);
        ++done;
      }
      if (ws.mm_count && glane<G>() == 0) {
        if (wave_on) atomicAdd(&ws.mm_count[1], (unsigned long long)done);
        if (wv == 0 && half == 0) {
          atomicAdd(&ws.mm_count[0], (unsigned long long)(nch ? nch - 1 : 0));
          atomicAdd(&ws.mm_count[2], 1ull);
        }
      }
      __syncthreads();  // the rows are reused by the block's next unit
    } else if (r < J.B) {  // wave-uniform
      const uint32_t bin = ws.border[J.fb_off + fb_f + r];
      const uint64_t e = J.fb_off + fb_f + bin;
      const uint32_t nch = ws.fch[e], first = ws.fitem[e];
      const uint32_t n_lo = (nch + 1) >> 1, n_hi = nch >> 1;
      const uint32_t my_n = half ? n_hi : n_lo;
      const uint64_t p0 = (uint64_t)first + (half ? n_lo : 0u);
      uint32_t acc[K], b[K], nb[K];
      ld29<K, G>(acc, my_n ? ws.partials + (p0 * 2 + slot) * S29 : one29);
      ld29<K, G>(nb, 1 < my_n ? ws.partials + ((p0 + 1) * 2 + slot) * S29 : one29);
#pragma unroll 1
      for (uint32_t k = 1; k < n_lo; ++k) {
#pragma unroll
        for (int j = 0; j < K; ++j) b[j] = nb[j];
        if (k + 1 < n_lo) ld29<K, G>(nb, k + 1 < my_n ? ws.partials + ((p0 + k + 1) * 2 + slot) * S29 : one29);
        mm29<K, G>(acc, b, acc, M, lds);
      }
      if (n_hi) {  // wave-uniform: join the halves
        st29<K, G>(lds, acc);
        __builtin_amdgcn_wave_barrier();
        uint32_t other[K];
        ld29<K, G>(other, lds_all + (wv * GW + (g ^ 2u)) * ROW);
        __builtin_amdgcn_wave_barrier();
        uint32_t t[K];
        mm29<K, G>(t, acc, other, M, lds);
        select(acc, half == 0, t, acc);
      }
      final_out<G, K, K32>(acc, M, lds, J.hist + ((fb_f + bin) * 2 + slot) * S, half == 0);
      if (ws.mm_count && glane<G>() == 0) {
        const uint64_t done = (n_lo ? n_lo - 1 : 0) + (n_hi ? 1 : 0) + 1;
        atomicAdd(&ws.mm_count[1], (unsigned long long)done);
        if (half == 0) {
          atomicAdd(&ws.mm_count[0], (unsigned long long)(nch ? nch - 1 : 0));
          atomicAdd(&ws.mm_count[2], 1ull);
        }
      }
    }
  }
}

// ------------------------------------------------ integer multiply probe
// Independent 32x32->64 multiply-adds, 8 chains per lane, for the measured
// peak of the VALU integer multiplier (the roofline denominator).
__global__ __launch_bounds__(256) void k_probe_mul(uint64_t iters, uint32_t *sink) {
  uint64_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5,
           a6 = a0 + 6, a7 = a0 + 7;
  uint32_t x = 0x9E3779B9u ^ blockIdx.x, y = 0x85EBCA6Bu + threadIdx.x;
  for (uint64_t i = 0; i < iters; ++i) {
    a0 = (uint64_t)x * y + a0;
    a1 = (uint64_t)x * (y + 1) + a1;
    a2 = (uint64_t)x * (y + 2) + a2;
    a3 = (uint64_t)x * (y + 3) + a3;
    a4 = (uint64_t)x * (y + 4) + a4;
    a5 = (uint64_t)x * (y + 5) + a5;
    a6 = (uint64_t)x * (y + 6) + a6;
    a7 = (uint64_t)x * (y + 7) + a7;
    x = (uint32_t)a0;
  }
  const uint64_t s = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
  if (s == 0x123456789ull) sink[0] = (uint32_t)s;  // keeps the chains alive
}

// ================================================================ launchers
static inline uint32_t blocks_for(uint64_t n, uint64_t per) { return (uint32_t)((n + per - 1) / per); }

hipError_t launch_encode(const double *x, uint64_t count, uint32_t frac_bits, int64_t *m,
                         uint32_t *n_bad, hipStream_t s) {
  if (!count) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(blocks_for(count, 256), 65536);
  hipLaunchKernelGGL(k_encode, dim3(grid), dim3(256), 0, s, x, count, frac_bits, m, n_bad);
  return hipGetLastError();
}

// k_pow at (S32, G, CT), as a function pointer for the generic launch.
template <int S32, int G>
static const void *pow_fn(bool ct) {
  return ct ? (const void *)k_pow<S32, G, true> : (const void *)k_pow<S32, G, false>;
}
static const void *pow_kernel(int S32, int G, bool ct) {
  switch (S32) {
    case 16:
      return G == 2 ? pow_fn<16, 2>(ct) : G == 4 ? pow_fn<16, 4>(ct) : G == 8 ? pow_fn<16, 8>(ct) : pow_fn<16, 16>(ct);
    case 32:
      return G == 2 ? pow_fn<32, 2>(ct) : G == 4 ? pow_fn<32, 4>(ct) : G == 8 ? pow_fn<32, 8>(ct) : pow_fn<32, 16>(ct);
    case 64:  // 2-lane groups would exceed the column bound of the radix-2^29 products
      return G == 4 ? pow_fn<64, 4>(ct) : G == 8 ? pow_fn<64, 8>(ct) : pow_fn<64, 16>(ct);
    default:  // 128: the public exponent n mod n^2 at 2048-bit keys, never secret
      return G == 8 ? (const void *)k_pow<128, 8, false> : (const void *)k_pow<128, 16, false>;
  }
}
bool pow_shape_valid(int S32, int G) {
  return (G == 2 || G == 4 || G == 8 || G == 16) &&
         (S32 == 16 || S32 == 32 || (S32 == 64 && G != 2) || (S32 == 128 && G >= 8));
}

// Modulus and exponent of an exponentiation per prime: kind 4
// r^(Q mod (P-1)) mod P, kind 0 t^P mod P^2, kind 2 c^(P-1) mod P^2; kind 1
// (public key) x^n mod n^2 for both.
static PowArgs pow_args(const DKey &k, int kind, const uint32_t *in, uint32_t in_stride, uint32_t in_limbs,
                        uint32_t *out, uint32_t out_stride, uint64_t count, uint32_t *tabs) {
  PowArgs a{};
  for (int w = 0; w < 2; ++w) {
    if (kind == 1) {
      a.mod[w] = k.n2;
      a.exp[w] = k.e_n;
      continue;
    }
    const DPrime &P = k.pr[w];
    a.mod[w] = kind == 4 ? P.P : P.P2;
    a.exp[w] = kind == 4 ? P.e_enc : (kind == 0 ? P.e_lift : P.e_dec);
  }
  a.in = in;
  a.in_stride = in_stride;
  a.in_limbs = in_limbs;
  a.out = out;
  a.out_stride = out_stride;
  a.count = count;
  a.tabs = tabs;
  return a;
}

static hipError_t launch_pow(int S32, bool ct, PowArgs a, const PowLaunch &l, hipStream_t s) {
  if (!pow_shape_valid(S32, l.G)) return hipErrorInvalidValue;
  void *args[] = {&a};
  return hipLaunchKernel(pow_kernel(S32, l.G, ct), dim3(l.grid), dim3(kBlockThreads), args, l.dyn, s);
}

// The plan's launches over a.count ciphertexts: the first main_count at
// p.main, the rest at p.tail (in and out advanced by the units before them,
// two per ciphertext), each with its work counter in p.ctr when given
// (cleared here, in stream order).
static hipError_t launch_pow_plan(int S32, bool ct, PowArgs a, const PowPlan &p, hipStream_t s) {
  const uint64_t count = a.count;
  const uint64_t mc = p.tail.G ? std::min(p.main_count, count) : count;
  if (p.ctr) {
    const hipError_t e = launch_fill(p.ctr, 2, 0u, s);
    if (e != hipSuccess) return e;
  }
  if (mc) {
    PowArgs am = a;
    am.count = mc;
    am.next = p.ctr;
    const hipError_t e = launch_pow(S32, ct, am, p.main, s);
    if (e != hipSuccess) return e;
  }
  if (mc < count) {
    PowArgs at = a;
    at.in += mc * 2 * a.in_stride;
    at.out += mc * 2 * a.out_stride;
    at.count = count - mc;
    at.next = p.ctr ? p.ctr + 1 : nullptr;
    return launch_pow(S32, ct, at, p.tail, s);
  }
  return hipSuccess;
}

hipError_t launch_pow_kind(int KP, const DKey &k, int kind, const uint32_t *in, uint32_t in_stride,
                           uint32_t in_limbs, uint32_t *out, uint32_t out_stride, uint64_t count, uint32_t *tab,
                           const PowPlan &p, hipStream_t s) {
  if (!count) return hipSuccess;
  const int S32 = kind == 4 ? 16 * KP : (kind == 1 ? 64 * KP : 32 * KP);
  return launch_pow_plan(S32, k.ct != 0, pow_args(k, kind, in, in_stride, in_limbs, out, out_stride, count, tab), p,
                         s);
}

hipError_t launch_enc_r(int KP, const DKey &k, uint64_t count, const uint32_t *r, uint64_t seed, uint64_t roff,
                        uint32_t *tq, hipStream_t s) {
  if (!count) return hipSuccess;
  if (KP == 1)
    hipLaunchKernelGGL(k_enc_r<1>, dim3(blocks_for(2 * count, 16)), dim3(kBlockThreads), 0, s, k, count, r, seed,
                       roff, tq);
  else
    hipLaunchKernelGGL(k_enc_r<2>, dim3(blocks_for(2 * count, 16)), dim3(kBlockThreads), 0, s, k, count, r, seed,
                       roff, tq);
  return hipGetLastError();
}

hipError_t launch_dec_pre(int KP, const DKey &k, const uint32_t *ct, uint64_t count, uint32_t *xpq, hipStream_t s) {
  if (!count) return hipSuccess;
  if (KP == 1)
    hipLaunchKernelGGL(k_dec_pre<1>, dim3(blocks_for(2 * count, 16)), dim3(kBlockThreads), 0, s, k, ct, count, xpq);
  else
    hipLaunchKernelGGL(k_dec_pre<2>, dim3(blocks_for(2 * count, 16)), dim3(kBlockThreads), 0, s, k, ct, count, xpq);
  return hipGetLastError();
}

template <int KP>
static hipError_t enc_crt(const DKey &k, const int64_t *m, uint64_t count, const uint32_t *r, uint64_t seed,
                          uint64_t roff, uint32_t *tq, uint32_t *cpq, uint32_t *ct, uint32_t *tab,
                          const PowPlan &p1, const PowPlan &p2, hipStream_t s) {
  constexpr int SP = 16 * KP, SP2 = 32 * KP;
  hipLaunchKernelGGL(k_enc_r<KP>, dim3(blocks_for(2 * count, 16)), dim3(kBlockThreads), 0, s, k, count, r, seed,
                     roff, tq);
  hipError_t e = launch_pow_plan(SP, k.ct != 0, pow_args(k, 4, tq, SP, SP, tq, SP, count, tab), p1, s);
  if (e != hipSuccess) return e;
  e = launch_pow_plan(SP2, k.ct != 0, pow_args(k, 0, tq, SP, SP, cpq, SP2, count, tab), p2, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_enc_crt_b<KP>, dim3(blocks_for(count, 16)), dim3(kBlockThreads), 0, s, k, m,
                     (const uint32_t *)cpq, count, ct);
  return hipGetLastError();
}
hipError_t launch_enc_crt(int KP, const DKey &k, const int64_t *m, uint64_t count, const uint32_t *r, uint64_t seed,
                          uint64_t roff, uint32_t *tq, uint32_t *cpq, uint32_t *ct, uint32_t *tab,
                          const PowPlan &p1, const PowPlan &p2, hipStream_t s) {
  if (!count) return hipSuccess;
  return KP == 1 ? enc_crt<1>(k, m, count, r, seed, roff, tq, cpq, ct, tab, p1, p2, s)
                 : enc_crt<2>(k, m, count, r, seed, roff, tq, cpq, ct, tab, p1, p2, s);
}

template <int KP>
static hipError_t enc_pub(const DKey &k, const int64_t *m, uint64_t count, const uint32_t *r, uint64_t seed,
                          uint64_t roff, uint32_t *x, uint32_t *ct, uint32_t *tab, const PowPlan &p, hipStream_t s) {
  constexpr int SN2 = 64 * KP;
  hipLaunchKernelGGL(k_pub_pre<KP>, dim3(blocks_for(count + (count & 1), 16)), dim3(kBlockThreads), 0, s, k, count,
                     r, seed, roff, x);
  const hipError_t e = launch_pow_plan(SN2, false, pow_args(k, 1, x, SN2, SN2, x, SN2, (count + 1) / 2, tab), p, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pub_post<KP>, dim3(blocks_for(count, 16)), dim3(kBlockThreads), 0, s, k, m, count,
                     (const uint32_t *)x, ct);
  return hipGetLastError();
}
hipError_t launch_enc_pub(int KP, const DKey &k, const int64_t *m, uint64_t count, const uint32_t *r, uint64_t seed,
                          uint64_t roff, uint32_t *x, uint32_t *ct, uint32_t *tab, const PowPlan &p, hipStream_t s) {
  if (!count) return hipSuccess;
  return KP == 1 ? enc_pub<1>(k, m, count, r, seed, roff, x, ct, tab, p, s)
                 : enc_pub<2>(k, m, count, r, seed, roff, x, ct, tab, p, s);
}

hipError_t launch_enc_obf(int KP, const DKey &k, const int64_t *m, uint64_t count, const uint32_t *rho,
                          uint32_t *ct, hipStream_t s) {
  if (!count) return hipSuccess;
  const dim3 grid(blocks_for(count, 16));
  if (KP == 1)
    hipLaunchKernelGGL(k_enc_obf<1>, grid, dim3(kBlockThreads), 0, s, k, m, count, rho, ct);
  else
    hipLaunchKernelGGL(k_enc_obf<2>, grid, dim3(kBlockThreads), 0, s, k, m, count, rho, ct);
  return hipGetLastError();
}

hipError_t launch_ct_div(int KP, const DKey &k, const uint32_t *num, const uint32_t *den, uint64_t count,
                         uint32_t batch, uint32_t *out, uint32_t *n_bad, hipStream_t s) {
  if (!count) return hipSuccess;
  const uint64_t groups = (count + batch - 1) / batch;
  const dim3 grid(blocks_for(groups, 16));
  if (KP == 1)
    hipLaunchKernelGGL(k_ct_div<1>, grid, dim3(kBlockThreads), 0, s, k, num, den, count, batch, out, n_bad);
  else
    hipLaunchKernelGGL(k_ct_div<2>, grid, dim3(kBlockThreads), 0, s, k, num, den, count, batch, out, n_bad);
  return hipGetLastError();
}

hipError_t launch_split(const int64_t *hist, const int64_t *minus, uint32_t nodes, uint32_t F, uint32_t B,
                        double scale, double lam, double gamma, double mcw, int64_t *derived, void *out_feat,
                        void *out_node, hipStream_t s) {
  if (!nodes) return hipSuccess;
  hipLaunchKernelGGL(k_split, dim3(nodes), dim3(kBlockThreads), 0, s, hist, minus, F, B, scale, lam, gamma, mcw,
                     derived, (SplitCand *)out_feat, (SplitCand *)out_node);
  return hipGetLastError();
}

hipError_t launch_ct_mul(int KP, const DKey &k, const uint32_t *a, const uint32_t *b, uint64_t count,
                         uint32_t *out, hipStream_t s) {
  if (!count) return hipSuccess;
  const dim3 grid(blocks_for(count, 16));
  if (KP == 1)
    hipLaunchKernelGGL(k_ct_mul<1>, grid, dim3(kBlockThreads), 0, s, k, a, b, count, out);
  else
    hipLaunchKernelGGL(k_ct_mul<2>, grid, dim3(kBlockThreads), 0, s, k, a, b, count, out);
  return hipGetLastError();
}

hipError_t launch_pack(int KP, const DKey &k, const uint32_t *ct, uint64_t count, uint32_t slots,
                       uint32_t *packed, hipStream_t s) {
  if (!count) return hipSuccess;
  const dim3 grid(blocks_for((count + slots - 1) / slots, 16));
  if (KP == 1)
    hipLaunchKernelGGL(k_pack<1>, grid, dim3(kBlockThreads), 0, s, k, ct, count, slots, packed);
  else
    hipLaunchKernelGGL(k_pack<2>, grid, dim3(kBlockThreads), 0, s, k, ct, count, slots, packed);
  return hipGetLastError();
}

hipError_t launch_unpack(const uint32_t *raw, uint64_t count, uint32_t slots, uint32_t L, int64_t *m,
                         uint32_t *n_overflow, hipStream_t s) {
  if (!count) return hipSuccess;
  hipLaunchKernelGGL(k_unpack, dim3(blocks_for(count, 256)), dim3(256), 0, s, raw, count, slots, L, m, n_overflow);
  return hipGetLastError();
}

uint32_t pack_slots(int n_bits, uint64_t count) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 1;
  }
  // enough packed ciphertexts for one 16-lane group per wave slot of a
  // wave per SIMD; beyond that, as many slots as the plaintext holds
  const uint64_t groups = (uint64_t)cus * 4 * 4;
  const uint64_t s = (count + groups - 1) / groups;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(s, (uint64_t)(n_bits - 1) / 64));
}

hipError_t launch_mont_convert(int KP, const DKey &k, const uint32_t *in, uint64_t count,
                               uint32_t *out, bool to_mont, hipStream_t s) {
  if (!count) return hipSuccess;
  const dim3 grid(blocks_for(count, kBlockThreads / kHistGroup));
  if (KP == 1)
    hipLaunchKernelGGL((k_mont_convert<1, kHistGroup>), grid, dim3(kBlockThreads), 0, s, k, in, count, out,
                       (int)to_mont);
  else
    hipLaunchKernelGGL((k_mont_convert<2, kHistGroup>), grid, dim3(kBlockThreads), 0, s, k, in, count, out,
                       (int)to_mont);
  return hipGetLastError();
}

template <int KP>
static hipError_t dec(const DKey &k, const uint32_t *ct, uint64_t count, uint32_t *xpq, int64_t *m,
                      uint32_t *raw, uint32_t *n_overflow, uint32_t *tab, const PowPlan &p, hipStream_t s) {
  constexpr int SP2 = 32 * KP;
  hipLaunchKernelGGL(k_dec_pre<KP>, dim3(blocks_for(2 * count, 16)), dim3(kBlockThreads), 0, s, k, ct, count, xpq);
  hipError_t e = launch_pow_plan(SP2, k.ct != 0, pow_args(k, 2, xpq, SP2, SP2, xpq, SP2, count, tab), p, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dec_b<KP>, dim3(blocks_for(count, 16)), dim3(kBlockThreads), 0, s, k,
                     (const uint32_t *)xpq, count, m, raw, n_overflow);
  return hipGetLastError();
}
hipError_t launch_dec(int KP, const DKey &k, const uint32_t *ct, uint64_t count, uint32_t *xpq,
                      int64_t *m, uint32_t *raw, uint32_t *n_overflow, uint32_t *tab, const PowPlan &p,
                      hipStream_t s) {
  if (!count) return hipSuccess;
  return KP == 1 ? dec<1>(k, ct, count, xpq, m, raw, n_overflow, tab, p, s)
                 : dec<2>(k, ct, count, xpq, m, raw, n_overflow, tab, p, s);
}

hipError_t launch_fill(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
  if (!n) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(blocks_for(n, 256), 4096);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

template <int KP>
static hipError_t hist(const DKey &k, const uint32_t *ctm, const DJob *host_jobs, const HistWs &ws,
                       const HistLaunch &l, hipStream_t s) {
  hipError_t e = launch_fill(ws.counts, ws.total_fb, 0u, s);
  if (e != hipSuccess) return e;
  for (uint32_t j0 = 0; j0 < ws.n_jobs; j0 += kJobsPerSetup) {
    JobPack pack;
    const uint32_t n = std::min<uint32_t>(kJobsPerSetup, ws.n_jobs - j0);
    for (uint32_t j = 0; j < n; ++j) pack.j[j] = host_jobs[j0 + j];
    hipLaunchKernelGGL(k_job_setup, dim3(1), dim3(64), 0, s, pack, n, ws.jobs + j0);
  }
  if (ws.total_blocks)
    hipLaunchKernelGGL(k_hist_count, dim3((uint32_t)ws.total_blocks), dim3(256), 0, s, ws);
  hipLaunchKernelGGL(k_hist_scan, dim3((uint32_t)ws.total_f), dim3(256), 0, s, ws);
  hipLaunchKernelGGL(k_hist_base, dim3(1), dim3(1024), 0, s, ws);
  hipLaunchKernelGGL(k_hist_items, dim3((uint32_t)ws.total_f), dim3(256), 0, s, ws);
  if (ws.total_blocks)
    hipLaunchKernelGGL(k_hist_scatter, dim3((uint32_t)ws.total_blocks), dim3(256), 0, s, ws);
  bool narrow = false;
  if constexpr (KP == 2) {
    if (l.G == 8) {
      hipLaunchKernelGGL((k_hist_chunk<KP, 8>), dim3(l.grid), dim3(kBlockThreads), l.dyn, s, k, ctm, ws);
      narrow = true;
    }
  }
  if (!narrow)
    hipLaunchKernelGGL((k_hist_chunk<KP, kHistGroup>), dim3(l.grid), dim3(kBlockThreads), l.dyn, s, k, ctm, ws);
  const uint64_t final_units = ws.total_f * (kFinalSolo + (256 - kFinalSolo) / 4);
  const uint32_t fgrid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(final_units, 1u << 20));
  hipLaunchKernelGGL((k_hist_final<KP, kHistGroup>), dim3(fgrid), dim3(kBlockThreads), 0, s, k, ws);
  return hipGetLastError();
}
hipError_t launch_hist(int KP, const DKey &k, const uint32_t *ctm, const DJob *host_jobs,
                       const HistWs &ws, const HistLaunch &l, hipStream_t s) {
  if (!hist_shape_valid(KP, l.G)) return hipErrorInvalidValue;
  return KP == 1 ? hist<1>(k, ctm, host_jobs, ws, l, s) : hist<2>(k, ctm, host_jobs, ws, l, s);
}

hipError_t launch_probe_mul(uint64_t iters, uint32_t grid, uint32_t *sink, hipStream_t s) {
  hipLaunchKernelGGL(k_probe_mul, dim3(grid), dim3(256), 0, s, iters, sink);
  return hipGetLastError();
}


// Elements per inversion batch of k_ct_div: enough groups for about two
// waves per SIMD, each group then chains as many elements as needed.
uint32_t ct_div_batch(uint64_t count) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 1;
  }
  const uint64_t groups = (uint64_t)cus * 4 * 2 * 4;
  return (uint32_t)std::max<uint64_t>(1, (count + groups - 1) / groups);
}

static int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 1;
  }
  return cus;
}

// Resident blocks of k_pow<S32, G> on the device with `dyn` bytes of dynamic LDS.
uint32_t pow_resident_blocks(int S32, int G, uint32_t dyn) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, uint32_t>, uint32_t> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({S32, G, dyn});
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (!pow_shape_valid(S32, G) ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pow_kernel(S32, G, false), kBlockThreads, dyn) !=
          hipSuccess ||
      nb < 1)
    nb = 1;
  const uint32_t r = (uint32_t)(nb * device_cus());
  cache[{S32, G, dyn}] = r;
  return r;
}

// Dynamic LDS that makes at most `waves` blocks of `fn` fit a compute unit
// (0 if its own occupancy `natural` is already at most that).
static uint32_t cap_dyn_lds(const void *fn, int natural, int waves) {
  if (waves <= 0 || natural <= waves) return 0;
  int dev = 0, lds_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      lds_cu <= 0)
    return 0;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, fn) != hipSuccess) return 0;
  const int64_t per_block = lds_cu / (waves + 1) + 1;
  const int64_t dyn = per_block - (int64_t)fa.sharedSizeBytes;
  return dyn > 0 ? (uint32_t)((dyn + 255) / 256 * 256) : 0u;
}

// Dynamic LDS that caps k_pow<S32, G> at `waves` blocks (= waves per SIMD)
// per compute unit: enough that waves + 1 blocks do not fit.  0 when waves
// is 0 or the kernel's own occupancy is at most `waves`.
uint32_t pow_dyn_lds(int S32, int G, int waves) {
  if (waves <= 0 || !pow_shape_valid(S32, G)) return 0;
  return cap_dyn_lds(pow_kernel(S32, G, false), (int)(pow_resident_blocks(S32, G, 0) / (uint32_t)device_cus()),
                     waves);
}

// Histogram product kernel shapes: 16-lane groups, or 8-lane groups where
// their Montgomery form is the 16-lane one (2048-bit keys: S29 = 144 for
// both; at 1024 bits the 8-lane R' differs).
bool hist_shape_valid(int KP, int G) { return G == 16 || (G == 8 && KP == 2); }
static const void *hist_kernel(int KP, int G) {
  if (KP == 2 && G == 8) return (const void *)k_hist_chunk<2, 8>;
  return KP == 1 ? (const void *)k_hist_chunk<1, kHistGroup> : (const void *)k_hist_chunk<2, kHistGroup>;
}
uint32_t hist_resident_blocks(int KP, int G, uint32_t dyn) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, uint32_t>, uint32_t> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({KP, G, dyn});
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (!hist_shape_valid(KP, G) ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, hist_kernel(KP, G), kBlockThreads, dyn) != hipSuccess ||
      nb < 1)
    nb = 1;
  const uint32_t r = (uint32_t)(nb * device_cus());
  cache[{KP, G, dyn}] = r;
  return r;
}
uint32_t hist_dyn_lds(int KP, int G, int waves) {
  if (waves <= 0 || !hist_shape_valid(KP, G)) return 0;
  return cap_dyn_lds(hist_kernel(KP, G), (int)(hist_resident_blocks(KP, G, 0) / (uint32_t)device_cus()), waves);
}

uint64_t table_bytes_per_block(int KP, int kind, int G) {
  // limbs of the modulus the kernel's exponentiation tables work in
  // (radix-2^29 limbs): mod P (kind 4), mod P^2 (0, 2), mod n^2 (1)
  const uint64_t S = (uint64_t)he29::limbs_for_group(kind == 1 ? 64 * KP : (kind == 4 ? 16 * KP : 32 * KP), G);
  return (uint64_t)(kBlockThreads / G) * (kTable + 1) * S * sizeof(uint32_t);
}

// Group width for an exponentiation (kind 4 mod P, 0 lift, 2 decryption, 1
// public key) over `count` units pairs: the narrowest built group (more
// limbs per lane, less cross-lane work per product) whose launch still gives
// every SIMD at least two waves; below that, wider groups buy parallelism.
int pick_group(int KP, int kind, uint64_t count) {
  const int S32 = kind == 4 ? 16 * KP : (kind == 1 ? 64 * KP : 32 * KP);
  const uint64_t need = 2ull * 4 * (uint64_t)device_cus();  // two waves on each of the 4 SIMDs per CU
  for (int G : {2, 4, 8}) {
    if (!pow_shape_valid(S32, G) || (G == 2 && kind != 4)) continue;  // 2 lanes: the mod-P exponentiation only
    const uint64_t waves = 2 * ((count + 64 / G - 1) / (64 / G));
    if (waves >= need) return G;
  }
  return 16;
}

}  // namespace he
