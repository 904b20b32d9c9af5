// CKKS for the secure horizontal path (clients encrypt local G/H histogram
// vectors, the server adds ciphertexts, clients decrypt the global
// histogram): public-key encryption, addition and decryption over
// R_Q = Z_Q[X]/(X^N + 1) in RNS form (three primes q_i < 2^30, q_i = 1 mod
// 2N), with the canonical-embedding encoding.  Everything runs in the
// kernels below; the host part builds the per-prime tables and the keys.
//
// Layouts: a polynomial is uint32 [L][N] residues (prime-major); a
// ciphertext is [2][L][N] (c0 then c1), coefficient domain.  Keys stay on
// the device in the NTT domain and in Montgomery form (times 2^32 mod q).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/he.h"
#include "../../include/he_ckks.h"
#include "mont.hpp"

namespace {

constexpr int kL = 3;            // RNS primes
constexpr int kPrimeBits = 30;
constexpr int kEta = 21;         // centered binomial parameter
constexpr uint64_t kKeyEBase = 1ull << 40;
constexpr uint64_t kKeyABase = 1ull << 41;
constexpr int kNttThreads = 1024;
constexpr int kFftThreads = 1024;

struct Prime {
  uint32_t q, qinv;       // qinv = -q^-1 mod 2^32
  uint32_t r2;            // 2^64 mod q (into Montgomery form)
  uint32_t ninv, ninv_s;  // N^-1 mod q and its Shoup companion
};

struct Tables {
  Prime p[kL];
  const uint32_t *psi;    // [L][N] psi^bitrev(i)
  const uint32_t *psi_s;  // Shoup companions floor(w 2^32 / q)
  const uint32_t *ipsi;   // [L][N] psi^-bitrev(i)
  const uint32_t *ipsi_s;
};

// ---- modular helpers (q < 2^30) -------------------------------------------
__device__ __forceinline__ uint32_t add_q(uint32_t a, uint32_t b, uint32_t q) {
  const uint32_t s = a + b;
  return s >= q ? s - q : s;
}
__device__ __forceinline__ uint32_t sub_q(uint32_t a, uint32_t b, uint32_t q) {
  return a >= b ? a - b : a + q - b;
}
// x w mod q with the precomputed ws = floor(w 2^32 / q) (Shoup).
__device__ __forceinline__ uint32_t mul_shoup(uint32_t x, uint32_t w, uint32_t ws, uint32_t q) {
  const uint32_t hi = __umulhi(x, ws);
  const uint32_t r = x * w - hi * q;  // in [0, 2q)
  return r >= q ? r - q : r;
}
// a b 2^-32 mod q (Montgomery), a, b < q.
__device__ __forceinline__ uint32_t mont_q(uint32_t a, uint32_t b, uint32_t q, uint32_t qinv) {
  const uint64_t t = (uint64_t)a * b;
  const uint32_t m = (uint32_t)t * qinv;
  const uint32_t r = (uint32_t)((t + (uint64_t)m * q) >> 32);
  return r >= q ? r - q : r;
}
__device__ __forceinline__ uint32_t to_residue(int64_t v, uint32_t q) {
  const int64_t r = v % (int64_t)q;
  return (uint32_t)(r < 0 ? r + q : r);
}

// ---- sampling ---------------------------------------------------------------
// kind 0: ternary (word mod 3 - 1); 1: centered binomial (popcount of bits
// 0..20 minus popcount of bits 21..41); 2: uniform mod q_i, with the counter
// base advanced by i N for prime i.  out: [polys][L][N]; poly p uses counter
// base + p * stride.
__global__ void k_sample(int kind, uint64_t seed, uint64_t base, uint64_t stride, uint32_t n, uint32_t polys,
                         Tables T, uint32_t *out) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)polys * n) return;
  const uint64_t p = idx / n, j = idx % n;
  uint32_t *o = out + p * kL * n + j;
  if (kind == 2) {
    for (int i = 0; i < kL; ++i)
      o[(uint64_t)i * n] = (uint32_t)(he::splitmix64(seed, base + p * stride + (uint64_t)i * n + j) % T.p[i].q);
    return;
  }
  const uint64_t w = he::splitmix64(seed, base + p * stride + j);
  int64_t v;
  if (kind == 0) {
    v = (int64_t)(w % 3) - 1;
  } else {
    const uint32_t mask = (1u << kEta) - 1u;
    v = (int64_t)__popc((uint32_t)w & mask) - (int64_t)__popc((uint32_t)(w >> kEta) & mask);
  }
  for (int i = 0; i < kL; ++i) o[(uint64_t)i * n] = to_residue(v, T.p[i].q);
}

// ---- negacyclic NTT ------------------------------------------------------------
// One block per (polynomial, prime), the polynomial in LDS.  Forward:
// Cooley-Tukey with psi powers in bit-reversed order (natural order in,
// bit-reversed out); inverse: Gentleman-Sande with inverse powers, then
// N^-1 (Longa & Naehrig, CANS 2016, Algorithms 1 and 2).
// Block b works on polynomial b / L, prime b % L; polynomials are `sin` and
// `sout` words apart in the input and output.
__global__ __launch_bounds__(kNttThreads) void k_ntt(const uint32_t *in, uint64_t sin, uint32_t *out, uint64_t sout,
                                                     uint32_t n, uint32_t log_n, Tables T, int inverse) {
  extern __shared__ uint32_t a[];
  const uint32_t i = blockIdx.x % kL;
  const uint64_t p = blockIdx.x / kL;
  const uint32_t *x = in + p * sin + (uint64_t)i * n;
  uint32_t *y = out + p * sout + (uint64_t)i * n;
  const uint32_t q = T.p[i].q;
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) a[j] = x[j];
  __syncthreads();
  const uint32_t half = n >> 1;
  if (!inverse) {
    const uint32_t *w = T.psi + (uint64_t)i * n, *ws = T.psi_s + (uint64_t)i * n;
    for (uint32_t m = 1, t = half; m < n; m <<= 1, t >>= 1) {
      for (uint32_t b = threadIdx.x; b < half; b += blockDim.x) {
        const uint32_t grp = b / t, k = b % t;
        const uint32_t j = 2 * grp * t + k;
        const uint32_t s = w[m + grp], ss = ws[m + grp];
        const uint32_t u = a[j], v = mul_shoup(a[j + t], s, ss, q);
        a[j] = add_q(u, v, q);
        a[j + t] = sub_q(u, v, q);
      }
      __syncthreads();
    }
  } else {
    const uint32_t *w = T.ipsi + (uint64_t)i * n, *ws = T.ipsi_s + (uint64_t)i * n;
    for (uint32_t m = n, t = 1; m > 1; m >>= 1, t <<= 1) {
      const uint32_t h = m >> 1;
      for (uint32_t b = threadIdx.x; b < half; b += blockDim.x) {
        const uint32_t grp = b / t, k = b % t;
        const uint32_t j = 2 * grp * t + k;
        const uint32_t s = w[h + grp], ss = ws[h + grp];
        const uint32_t u = a[j], v = a[j + t];
        a[j] = add_q(u, v, q);
        a[j + t] = mul_shoup(sub_q(u, v, q), s, ss, q);
      }
      __syncthreads();
    }
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) a[j] = mul_shoup(a[j], T.p[i].ninv, T.p[i].ninv_s, q);
    __syncthreads();
  }
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) y[j] = a[j];
}

// ---- pointwise ----------------------------------------------------------------
// Key generation in the NTT domain: b = -a s + e, then a, b, s into
// Montgomery form.  All [L][N].
__global__ void k_keygen_finish(uint32_t n, Tables T, uint32_t *s, uint32_t *a, const uint32_t *e, uint32_t *b) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)kL * n) return;
  const Prime P = T.p[idx / n];
  const uint32_t sm = mont_q(s[idx], P.r2, P.q, P.qinv);  // s R
  const uint32_t am = mont_q(a[idx], P.r2, P.q, P.qinv);
  const uint32_t as = mont_q(am, s[idx], P.q, P.qinv);   // a s
  const uint32_t bv = sub_q(e[idx], as, P.q);
  b[idx] = mont_q(bv, P.r2, P.q, P.qinv);
  a[idx] = am;
  s[idx] = sm;
}

// out[p] = key (Montgomery, NTT domain) * x[p] (NTT domain), for `polys`
// polynomials [L][N] with strides sx and so (in words) between them.
__global__ void k_mul_key(uint32_t n, uint32_t polys, Tables T, const uint32_t *key, const uint32_t *x, uint64_t sx,
                          uint32_t *out, uint64_t so) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t per = (uint64_t)kL * n;
  if (idx >= (uint64_t)polys * per) return;
  const uint64_t p = idx / per, r = idx % per;
  const Prime P = T.p[r / n];
  out[p * so + r] = mont_q(key[r], x[p * sx + r], P.q, P.qinv);
}

// out = a + b + c (c optional), [polys][L][N] with independent strides.
__global__ void k_add3(uint32_t n, uint64_t polys, Tables T, const uint32_t *a, uint64_t sa, const uint32_t *b,
                       uint64_t sb, const uint32_t *c, uint64_t sc, uint32_t *out, uint64_t so) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t per = (uint64_t)kL * n;
  if (idx >= polys * per) return;
  const uint64_t p = idx / per, r = idx % per;
  const uint32_t q = T.p[r / n].q;
  uint32_t v = add_q(a[p * sa + r], b[p * sb + r], q);
  if (c) v = add_q(v, c[p * sc + r], q);
  out[p * so + r] = v;
}

// ---- encoding FFT ---------------------------------------------------------------
// One block per vector; n = N/2 complex values in LDS.  The evaluation points
// zeta^(5^k) (zeta = e^(i pi / N)) are zeta^(1 + 4 t) with t = (5^k mod 2N -
// 1) / 4, so with u_j = m_j + i m_(j + n):
//   z_k = sum_j u_j zeta^j omega^(t j),  omega = e^(2 pi i / n),
// a length-n DFT of the twisted u read at t_k.  Encoding inverts it.
struct Cx {
  double re, im;
};
__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// In-place radix-2 DIT FFT of length n (power of two) in LDS; sign +1 for
// sum x_j w^(t j), -1 for the conjugate.  tw[k] = e^(2 pi i k / n), k < n/2.
__device__ __forceinline__ void fft_lds(Cx *x, uint32_t n, uint32_t log_n, const Cx *tw, int sign) {
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const uint32_t r = __brev(j) >> (32 - log_n);
    if (r > j) {
      const Cx t = x[j];
      x[j] = x[r];
      x[r] = t;
    }
  }
  __syncthreads();
  for (uint32_t len = 2; len <= n; len <<= 1) {
    const uint32_t h = len >> 1, step = n / len;
    for (uint32_t b = threadIdx.x; b < n / 2; b += blockDim.x) {
      const uint32_t grp = b / h, k = b % h;
      const uint32_t j = grp * len + k;
      Cx w = tw[k * step];
      if (sign < 0) w.im = -w.im;
      const Cx v = cmul(x[j + h], w), u = x[j];
      x[j] = {u.re + v.re, u.im + v.im};
      x[j + h] = {u.re - v.re, u.im - v.im};
    }
    __syncthreads();
  }
}

// z: [count][n_values] doubles (n_values <= N/2) -> pt [count][L][N].
__global__ __launch_bounds__(kFftThreads) void k_encode(const double *z, uint32_t n_values, uint32_t N,
                                                        uint32_t log_n, double scale, const uint32_t *perm,
                                                        const Cx *tw, const Cx *zeta, Tables T, uint32_t *pt) {
  extern __shared__ Cx x[];
  const uint32_t n = N / 2;
  const double *zz = z + (uint64_t)blockIdx.x * n_values;
  for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) x[perm[k]] = {k < n_values ? zz[k] * scale : 0.0, 0.0};
  __syncthreads();
  fft_lds(x, n, log_n - 1, tw, -1);
  uint32_t *o = pt + (uint64_t)blockIdx.x * kL * N;
  const double inv_n = 1.0 / (double)n;
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    Cx c = x[j];
    c.re *= inv_n;
    c.im *= inv_n;
    const Cx zc = {zeta[j].re, -zeta[j].im};  // zeta^-j
    const Cx u = cmul(c, zc);
    const int64_t lo = (int64_t)rint(u.re), hi = (int64_t)rint(u.im);
    for (int i = 0; i < kL; ++i) {
      o[(uint64_t)i * N + j] = to_residue(lo, T.p[i].q);
      o[(uint64_t)i * N + j + n] = to_residue(hi, T.p[i].q);
    }
  }
}

// Centered value of the residues r_i of one coefficient, as a double:
// Garner's mixed-radix digits, the integer x = d0 + q0 (d1 + q1 d2) in 128
// bits, x - Q when x > Q/2.
struct Crt {
  uint32_t q0q1_inv_q2;  // (q0 q1)^-1 mod q2
  uint32_t q0_inv_q1, q0_inv_q2;
  uint64_t Q_lo, Q_hi;
};
__device__ __forceinline__ double crt_center(uint32_t r0, uint32_t r1, uint32_t r2, const Tables &T, const Crt &C) {
  const uint32_t q0 = T.p[0].q, q1 = T.p[1].q, q2 = T.p[2].q;
  const uint32_t d0 = r0;
  const uint32_t d1 = (uint32_t)((uint64_t)sub_q(r1, d0 % q1, q1) * C.q0_inv_q1 % q1);
  // d2 = ((r2 - d0) q0^-1 - d1) q1^-1 mod q2 = (r2 - d0 - q0 d1) (q0 q1)^-1
  const uint64_t t = ((uint64_t)q0 % q2) * d1 % q2;
  const uint32_t v = sub_q(sub_q(r2, d0 % q2, q2), (uint32_t)t, q2);
  const uint32_t d2 = (uint32_t)((uint64_t)v * C.q0q1_inv_q2 % q2);
  const unsigned __int128 x =
      (unsigned __int128)d0 + (unsigned __int128)q0 * ((unsigned __int128)d1 + (unsigned __int128)q1 * d2);
  const unsigned __int128 Q = ((unsigned __int128)C.Q_hi << 64) | C.Q_lo;
  const bool neg = x > (Q >> 1);
  const unsigned __int128 mag = neg ? Q - x : x;
  const double d = (double)(uint64_t)(mag >> 64) * 18446744073709551616.0 + (double)(uint64_t)mag;
  return neg ? -d : d;
}

// pt [count][L][N] -> z [count][n_values].
__global__ __launch_bounds__(kFftThreads) void k_decode(const uint32_t *pt, uint32_t n_values, uint32_t N,
                                                        uint32_t log_n, double inv_scale, const uint32_t *perm,
                                                        const Cx *tw, const Cx *zeta, Tables T, Crt C, double *z) {
  extern __shared__ Cx x[];
  const uint32_t n = N / 2;
  const uint32_t *p = pt + (uint64_t)blockIdx.x * kL * N;
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const double lo = crt_center(p[j], p[N + j], p[2 * N + j], T, C);
    const double hi = crt_center(p[j + n], p[N + j + n], p[2 * N + j + n], T, C);
    x[j] = cmul({lo * inv_scale, hi * inv_scale}, zeta[j]);
  }
  __syncthreads();
  fft_lds(x, n, log_n - 1, tw, +1);
  double *zz = z + (uint64_t)blockIdx.x * n_values;
  for (uint32_t k = threadIdx.x; k < n_values; k += blockDim.x) zz[k] = x[perm[k]].re;
}

// ---- host -----------------------------------------------------------------------
thread_local std::string g_err;
int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}
#define CK_TRY(expr)                                          \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) return fail(HE_ERR_DEVICE, hipGetErrorString(e_)); \
  } while (0)

uint64_t pow_mod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = (unsigned __int128)r * b % m;
    b = (unsigned __int128)b * b % m;
    e >>= 1;
  }
  return r;
}
bool is_prime32(uint64_t q) {
  if (q < 2 || q % 2 == 0) return q == 2;
  // deterministic Miller-Rabin for q < 2^32 with bases 2, 7, 61
  uint64_t d = q - 1;
  int s = 0;
  while (d % 2 == 0) {
    d /= 2;
    ++s;
  }
  for (uint64_t a : {2ull, 7ull, 61ull}) {
    if (a % q == 0) continue;
    uint64_t x = pow_mod(a, d, q);
    if (x == 1 || x == q - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = (unsigned __int128)x * x % q;
      if (x == q - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}
uint32_t bitrev(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t b = 0; b < bits; ++b) r |= ((x >> b) & 1u) << (bits - 1 - b);
  return r;
}

}  // namespace

struct he_ckks {
  uint32_t log_n = 0, n = 0, scale_bits = 0;
  uint64_t seed = 0;
  Tables T{};
  Crt C{};
  uint32_t *d_tab = nullptr;   // psi, psi_s, ipsi, ipsi_s: 4 [L][N]
  uint32_t *d_keys = nullptr;  // s, a, b: 3 [L][N] (NTT domain, Montgomery form)
  uint32_t *d_perm = nullptr;  // t_k for k < N/2
  Cx *d_tw = nullptr;          // e^(2 pi i k / (N/2)), k < N/4
  Cx *d_zeta = nullptr;        // zeta^j, j < N/2
  std::mutex mu;
  uint32_t *d_scratch = nullptr;  // encryption/decryption temporaries
  size_t scratch_words = 0;
};

namespace {

int scratch(he_ckks *c, size_t words, uint32_t **out) {
  if (c->scratch_words < words) {
    if (c->d_scratch) CK_TRY(hipFree(c->d_scratch));
    c->d_scratch = nullptr;
    c->scratch_words = 0;
    if (hipMalloc(&c->d_scratch, words * 4) != hipSuccess) return fail(HE_ERR_OOM, "out of device memory");
    c->scratch_words = words;
  }
  *out = c->d_scratch;
  return HE_OK;
}

inline uint32_t blocks(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

// polys polynomials [L][N], sin / sout words apart (0: packed), in -> out
// (may be the same buffer).
hipError_t ntt(const he_ckks *c, const uint32_t *in, uint32_t *out, uint64_t polys, bool inverse, hipStream_t s,
               uint64_t sin = 0, uint64_t sout = 0) {
  if (!polys) return hipSuccess;
  const uint64_t per = (uint64_t)kL * c->n;
  hipLaunchKernelGGL(k_ntt, dim3((uint32_t)(polys * kL)), dim3(kNttThreads), c->n * 4, s, in, sin ? sin : per, out,
                     sout ? sout : per, c->n, c->log_n, c->T, (int)inverse);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int he_ckks_create(uint32_t log_n, uint32_t scale_bits, uint64_t seed, he_ckks **out) {
  if (!out) return fail(HE_ERR_ARG, "null out");
  // Q is about 2^90: within the 128-bit classical security bounds of the
  // homomorphic encryption standard for a ternary secret (log Q at most 109
  // at N = 2^12, 218 at 2^13, 438 at 2^14), far outside them at N = 2^10 or
  // 2^11 (27 and 54), so smaller rings are refused.
  if (log_n < 12 || log_n > 14) return fail(HE_ERR_ARG, "log_n must be in [12, 14]");
  if (scale_bits < 10 || scale_bits > 60) return fail(HE_ERR_ARG, "scale_bits must be in [10, 60]");
  auto *c = new he_ckks();
  c->log_n = log_n;
  c->n = 1u << log_n;
  c->scale_bits = scale_bits;
  c->seed = seed;
  const uint32_t N = c->n;
  // primes: the largest below 2^30 that are 1 mod 2N
  std::vector<uint32_t> qs;
  for (uint64_t q = ((1ull << kPrimeBits) - 1) / (2 * N) * (2 * N) + 1; qs.size() < kL; q -= 2 * N)
    if (q < (1ull << kPrimeBits) && is_prime32(q)) qs.push_back((uint32_t)q);
  std::vector<uint32_t> tab(4ull * kL * N);
  for (int i = 0; i < kL; ++i) {
    const uint64_t q = qs[i];
    Prime &P = c->T.p[i];
    P.q = (uint32_t)q;
    uint32_t inv = 1;  // q^-1 mod 2^32 by Newton
    for (int k = 0; k < 5; ++k) inv *= 2u - (uint32_t)q * inv;
    P.qinv = 0u - inv;
    P.r2 = (uint32_t)(((unsigned __int128)1 << 64) % q);
    P.ninv = (uint32_t)pow_mod(N, q - 2, q);
    P.ninv_s = (uint32_t)(((uint64_t)P.ninv << 32) / q);
    uint64_t psi = 0;
    for (uint64_t g = 2; g < q; ++g) {
      const uint64_t cand = pow_mod(g, (q - 1) / (2 * N), q);
      if (pow_mod(cand, N, q) == q - 1) {
        psi = cand;
        break;
      }
    }
    const uint64_t ipsi = pow_mod(psi, q - 2, q);
    for (uint32_t k = 0; k < N; ++k) {
      const uint32_t e = bitrev(k, log_n);
      const uint64_t w = pow_mod(psi, e, q), iw = pow_mod(ipsi, e, q);
      tab[(0ull * kL + i) * N + k] = (uint32_t)w;
      tab[(1ull * kL + i) * N + k] = (uint32_t)((w << 32) / q);
      tab[(2ull * kL + i) * N + k] = (uint32_t)iw;
      tab[(3ull * kL + i) * N + k] = (uint32_t)((iw << 32) / q);
    }
  }
  {
    const uint64_t q0 = qs[0], q1 = qs[1], q2 = qs[2];
    c->C.q0_inv_q1 = (uint32_t)pow_mod(q0 % q1, q1 - 2, q1);
    c->C.q0_inv_q2 = (uint32_t)pow_mod(q0 % q2, q2 - 2, q2);
    c->C.q0q1_inv_q2 = (uint32_t)pow_mod((unsigned __int128)q0 * q1 % q2, q2 - 2, q2);
    const unsigned __int128 Q = (unsigned __int128)q0 * q1 * q2;
    c->C.Q_lo = (uint64_t)Q;
    c->C.Q_hi = (uint64_t)(Q >> 64);
  }
  // encoding tables
  const uint32_t n = N / 2;
  std::vector<uint32_t> perm(n);
  uint64_t e = 1;
  for (uint32_t k = 0; k < n; ++k) {
    perm[k] = (uint32_t)((e - 1) / 4);
    e = e * 5 % (2ull * N);
  }
  std::vector<Cx> tw(n / 2), zeta(n);
  for (uint32_t k = 0; k < n / 2; ++k) tw[k] = {std::cos(2.0 * M_PI * k / n), std::sin(2.0 * M_PI * k / n)};
  for (uint32_t j = 0; j < n; ++j) zeta[j] = {std::cos(M_PI * j / N), std::sin(M_PI * j / N)};

  auto cleanup = [&](int rc) {
    he_ckks_free(c);
    return rc;
  };
  // The N/2-point FFT holds up to 128 KiB of LDS, the NTT up to 64 KiB: ask
  // for that much dynamic LDS (best effort; a size the device refuses shows
  // up as a launch error of the kernel).
  (void)hipFuncSetAttribute((const void *)k_encode, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)((N / 2) * sizeof(Cx)));
  (void)hipFuncSetAttribute((const void *)k_decode, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)((N / 2) * sizeof(Cx)));
  (void)hipFuncSetAttribute((const void *)k_ntt, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(N * 4));
  (void)hipGetLastError();
  if (hipMalloc(&c->d_tab, tab.size() * 4) != hipSuccess || hipMalloc(&c->d_keys, 3ull * kL * N * 4) != hipSuccess ||
      hipMalloc(&c->d_perm, n * 4) != hipSuccess || hipMalloc(&c->d_tw, tw.size() * sizeof(Cx)) != hipSuccess ||
      hipMalloc(&c->d_zeta, n * sizeof(Cx)) != hipSuccess)
    return cleanup(fail(HE_ERR_OOM, "out of device memory"));
  if (hipMemcpy(c->d_tab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_perm, perm.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_tw, tw.data(), tw.size() * sizeof(Cx), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_zeta, zeta.data(), n * sizeof(Cx), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(HE_ERR_DEVICE, "copy of the tables failed"));
  c->T.psi = c->d_tab;
  c->T.psi_s = c->d_tab + 1ull * kL * N;
  c->T.ipsi = c->d_tab + 2ull * kL * N;
  c->T.ipsi_s = c->d_tab + 3ull * kL * N;
  // keys: s (ternary), e (centered binomial), a (uniform); b = -a s + e
  uint32_t *s = c->d_keys, *a = s + kL * N, *b = a + kL * N, *ek = nullptr;
  if (hipMalloc(&ek, (size_t)kL * N * 4) != hipSuccess) return cleanup(fail(HE_ERR_OOM, "out of device memory"));
  const uint32_t g = blocks(N, 256);
  hipLaunchKernelGGL(k_sample, dim3(g), dim3(256), 0, 0, 0, seed, 0ull, 0ull, N, 1u, c->T, s);
  hipLaunchKernelGGL(k_sample, dim3(g), dim3(256), 0, 0, 1, seed, kKeyEBase, 0ull, N, 1u, c->T, ek);
  hipLaunchKernelGGL(k_sample, dim3(g), dim3(256), 0, 0, 2, seed, kKeyABase, 0ull, N, 1u, c->T, a);
  hipError_t err = ntt(c, s, s, 1, false, 0);
  if (err == hipSuccess) err = ntt(c, a, a, 1, false, 0);
  if (err == hipSuccess) err = ntt(c, ek, ek, 1, false, 0);
  if (err == hipSuccess) {
    hipLaunchKernelGGL(k_keygen_finish, dim3(blocks((uint64_t)kL * N, 256)), dim3(256), 0, 0, N, c->T, s, a, ek, b);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipDeviceSynchronize();
  hipFree(ek);
  if (err != hipSuccess) return cleanup(fail(HE_ERR_DEVICE, hipGetErrorString(err)));
  *out = c;
  return HE_OK;
}

void he_ckks_free(he_ckks *c) {
  if (!c) return;
  hipFree(c->d_tab);
  hipFree(c->d_keys);
  hipFree(c->d_perm);
  hipFree(c->d_tw);
  hipFree(c->d_zeta);
  hipFree(c->d_scratch);
  delete c;
}

int he_ckks_params(const he_ckks *c, uint32_t *n, uint32_t *primes, uint32_t *scale_bits) {
  if (!c) return fail(HE_ERR_ARG, "null context");
  if (n) *n = c->n;
  if (primes)
    for (int i = 0; i < kL; ++i) primes[i] = c->T.p[i].q;
  if (scale_bits) *scale_bits = c->scale_bits;
  return HE_OK;
}

int he_ckks_encode(const he_ckks *c, const double *z, uint64_t count, uint32_t n_values, uint32_t *pt,
                   hipStream_t s) {
  if (!c) return fail(HE_ERR_ARG, "null context");
  if (n_values > c->n / 2) return fail(HE_ERR_ARG, "n_values exceeds N/2 slots");
  if (count == 0) return HE_OK;
  if (!pt || (n_values && !z)) return fail(HE_ERR_ARG, "null z or pt");
  if (count > 0x7FFFFFFFull) return fail(HE_ERR_ARG, "count too large");
  hipLaunchKernelGGL(k_encode, dim3((uint32_t)count), dim3(kFftThreads), (c->n / 2) * sizeof(Cx), s, z, n_values,
                     c->n, c->log_n, std::ldexp(1.0, (int)c->scale_bits), c->d_perm, c->d_tw, c->d_zeta, c->T, pt);
  CK_TRY(hipGetLastError());
  return HE_OK;
}

int he_ckks_decode(const he_ckks *c, const uint32_t *pt, uint64_t count, uint32_t n_values, double *z,
                   hipStream_t s) {
  if (!c) return fail(HE_ERR_ARG, "null context");
  if (n_values > c->n / 2) return fail(HE_ERR_ARG, "n_values exceeds N/2 slots");
  if (count == 0 || n_values == 0) return HE_OK;
  if (!pt || !z) return fail(HE_ERR_ARG, "null pt or z");
  if (count > 0x7FFFFFFFull) return fail(HE_ERR_ARG, "count too large");
  hipLaunchKernelGGL(k_decode, dim3((uint32_t)count), dim3(kFftThreads), (c->n / 2) * sizeof(Cx), s, pt, n_values,
                     c->n, c->log_n, std::ldexp(1.0, -(int)c->scale_bits), c->d_perm, c->d_tw, c->d_zeta, c->T,
                     c->C, z);
  CK_TRY(hipGetLastError());
  return HE_OK;
}

int he_ckks_encrypt(he_ckks *c, const uint32_t *pt, uint64_t count, uint64_t seed, uint64_t offset, uint32_t *ct,
                    hipStream_t s) {
  if (!c) return fail(HE_ERR_ARG, "null context");
  if (count == 0) return HE_OK;
  if (!pt || !ct) return fail(HE_ERR_ARG, "null pt or ct");
  const uint32_t N = c->n;
  const uint64_t per = (uint64_t)kL * N;
  if (count * 2 * kL > 0x7FFFFFFFull || count * N > 0xFFFFFFFFull) return fail(HE_ERR_ARG, "count too large");
  std::lock_guard<std::mutex> lk(c->mu);
  uint32_t *tmp = nullptr;
  int rc = scratch(c, 3 * count * per, &tmp);  // u, e0, e1 of every ciphertext
  if (rc) return rc;
  uint32_t *u = tmp, *e0 = tmp + count * per, *e1 = e0 + count * per;
  const uint32_t g = blocks(count * N, 256);
  // ciphertext t: u, e0, e1 at counters (offset + t) 3N + {0, N, 2N}
  hipLaunchKernelGGL(k_sample, dim3(g), dim3(256), 0, s, 0, seed, offset * 3 * N, 3ull * N, N, (uint32_t)count,
                     c->T, u);
  hipLaunchKernelGGL(k_sample, dim3(g), dim3(256), 0, s, 1, seed, offset * 3 * N + N, 3ull * N, N,
                     (uint32_t)count, c->T, e0);
  hipLaunchKernelGGL(k_sample, dim3(g), dim3(256), 0, s, 1, seed, offset * 3 * N + 2 * N, 3ull * N, N,
                     (uint32_t)count, c->T, e1);
  CK_TRY(hipGetLastError());
  CK_TRY(ntt(c, u, u, count, false, s));
  const uint32_t *a = c->d_keys + per, *b = a + per;
  // ct[t] = (INTT(b u) + e0 + m, INTT(a u) + e1); ct is [count][2][L][N]
  const uint32_t gp = blocks(count * per, 256);
  hipLaunchKernelGGL(k_mul_key, dim3(gp), dim3(256), 0, s, N, (uint32_t)count, c->T, b, u, per, ct, 2 * per);
  hipLaunchKernelGGL(k_mul_key, dim3(gp), dim3(256), 0, s, N, (uint32_t)count, c->T, a, u, per, ct + per, 2 * per);
  CK_TRY(hipGetLastError());
  CK_TRY(ntt(c, ct, ct, 2 * count, true, s));
  hipLaunchKernelGGL(k_add3, dim3(gp), dim3(256), 0, s, N, count, c->T, ct, 2 * per, e0, per, pt, per, ct, 2 * per);
  hipLaunchKernelGGL(k_add3, dim3(gp), dim3(256), 0, s, N, count, c->T, ct + per, 2 * per, e1, per,
                     (const uint32_t *)nullptr, 0ull, ct + per, 2 * per);
  CK_TRY(hipGetLastError());
  return HE_OK;
}

int he_ckks_add(const he_ckks *c, const uint32_t *x, const uint32_t *y, uint64_t count, uint32_t *out,
                hipStream_t s) {
  if (!c) return fail(HE_ERR_ARG, "null context");
  if (count == 0) return HE_OK;
  if (!x || !y || !out) return fail(HE_ERR_ARG, "null x, y or out");
  const uint64_t per = (uint64_t)kL * c->n;
  hipLaunchKernelGGL(k_add3, dim3(blocks(2 * count * per, 256)), dim3(256), 0, s, c->n, 2 * count, c->T, x, per, y,
                     per, (const uint32_t *)nullptr, 0ull, out, per);
  CK_TRY(hipGetLastError());
  return HE_OK;
}

int he_ckks_decrypt(const he_ckks *c, const uint32_t *ct, uint64_t count, uint32_t *pt, hipStream_t s) {
  if (!c) return fail(HE_ERR_ARG, "null context");
  if (count == 0) return HE_OK;
  if (!ct || !pt) return fail(HE_ERR_ARG, "null ct or pt");
  const uint64_t per = (uint64_t)kL * c->n;
  if (count * kL > 0x7FFFFFFFull) return fail(HE_ERR_ARG, "count too large");
  // pt = c0 + INTT(NTT(c1) s): NTT of every c1 into pt (strided input)
  CK_TRY(ntt(c, ct + per, pt, count, false, s, 2 * per, per));
  const uint32_t gp = blocks(count * per, 256);
  hipLaunchKernelGGL(k_mul_key, dim3(gp), dim3(256), 0, s, c->n, (uint32_t)count, c->T, c->d_keys, pt, per, pt, per);
  CK_TRY(hipGetLastError());
  CK_TRY(ntt(c, pt, pt, count, true, s));
  hipLaunchKernelGGL(k_add3, dim3(gp), dim3(256), 0, s, c->n, count, c->T, pt, per, ct, 2 * per,
                     (const uint32_t *)nullptr, 0ull, pt, per);
  CK_TRY(hipGetLastError());
  return HE_OK;
}

const char *he_ckks_last_error(void) { return g_err.c_str(); }

}  // extern "C"
