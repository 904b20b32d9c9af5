// Host runtime behind the C ABI in include/he.h: key objects with their
// device-resident constants, per-stream workspaces, argument checks and
// kernel dispatch.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <cmath>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/he.h"
#include "he_internal.hpp"
#include "hostbn.hpp"
#include "keysetup.hpp"

using hebn::Limbs;

struct he_key {
  uint32_t n_bits = 0;
  bool priv = false;
  Limbs n, p, q;
  int device = 0;
  void *blob = nullptr;   // device copy of every constant below
  he::DKey dk{};
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define HE_TRY_HIP(expr)                                                       \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess)                                                      \
      return fail(HE_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

he::DMod mk_mod(const uint32_t *base, const hekey::ModOff &o) {
  he::DMod m{base + o.N, base + o.R1, base + o.R2, base + o.R3, base + o.R4, o.ninv, {}, {}, {}};
  for (int v = 0; v < he29::kVariants; ++v) {
    m.N29[v] = base + o.N29[v];
    m.R1_29[v] = base + o.R1_29[v];
    m.R2_29[v] = base + o.R2_29[v];
  }
  return m;
}
he::DExp mk_exp(const uint32_t *base, const hekey::ExpOff &o) {
  return he::DExp{base + o.e, o.nwin, base + o.ops, o.nops};
}

// Builds every constant of the key and uploads them to the current device.
int build_key(he_key *k) {
  const hekey::KeyConsts kc = hekey::derive(k->n_bits, k->n, k->p, k->q, k->priv);
  const hekey::Blob &b = kc.blob;
  const hekey::ModOff &on = kc.n, &on2 = kc.n2;
  const hekey::ExpOff &oe = kc.e_n;
  const hekey::PrimeOff &op = kc.pr[0], &oq = kc.pr[1];
  const size_t o_nR = kc.nR_n2, o_half = kc.half, o_Cq = kc.Cq, o_q2R = kc.q2R_n2, o_qinv = kc.qinv_p,
               o_qR = kc.qR_n;
  HE_TRY_HIP(hipGetDevice(&k->device));
  HE_TRY_HIP(hipMalloc(&k->blob, b.words.size() * sizeof(uint32_t)));
  HE_TRY_HIP(hipMemcpy(k->blob, b.words.data(), b.words.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  const uint32_t *base = (const uint32_t *)k->blob;
  he::DKey &d = k->dk;
  d.n_bits = k->n_bits;
  d.has_priv = k->priv;
  d.n = mk_mod(base, on);
  d.n2 = mk_mod(base, on2);
  d.e_n = mk_exp(base, oe);
  d.nR_n2 = base + o_nR;
  d.half = base + o_half;
  if (k->priv) {
    const hekey::PrimeOff *po[2] = {&op, &oq};
    for (int w = 0; w < 2; ++w) {
      he::DPrime &P = d.pr[w];
      P.P = mk_mod(base, po[w]->P);
      P.P2 = mk_mod(base, po[w]->P2);
      P.e_enc = mk_exp(base, po[w]->e_enc);
      P.e_lift = mk_exp(base, po[w]->e_lift);
      P.e_dec = mk_exp(base, po[w]->e_dec);
      P.QR_P = base + po[w]->QR_P;
      P.PR_P2 = base + po[w]->PR_P2;
      P.Pinv = base + po[w]->Pinv;
      P.hR_P = base + po[w]->hR_P;
    }
    d.Cq = base + o_Cq;
    d.q2R_n2 = base + o_q2R;
    d.qinv_p = base + o_qinv;
    d.qR_n = base + o_qR;
  }
  return HE_OK;
}

int make_key(uint32_t n_bits, const Limbs &p, const Limbs &q, bool priv, he_key **out) {
  he_key *k = new (std::nothrow) he_key();
  if (!k) return fail(HE_ERR_OOM, "out of host memory");
  k->n_bits = n_bits;
  k->priv = priv;
  if (priv) {
    k->p = p;
    k->q = q;
    k->n = hebn::mul(p, q);
  } else {
    k->n = p;
  }
  int rc;
  try {
    rc = build_key(k);
  } catch (const std::exception &e) {
    rc = fail(HE_ERR_KEY, std::string("key setup: ") + e.what());
  }
  if (rc != HE_OK) {
    if (k->blob) hipFree(k->blob);
    delete k;
    return rc;
  }
  *out = k;
  return HE_OK;
}

bool valid_bits(uint32_t n_bits) { return n_bits == 1024 || n_bits == 2048; }
int kp_of(const he_key *k) { return k->n_bits == 2048 ? 2 : 1; }

// ---------------------------------------------------------------- workspace
// Grow-only device buffers, one set per stream.  Growing synchronises the
// stream first so that no queued kernel still uses the old buffer.
struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};
struct Workspace {
  Buf tab, tmp, hist, unpack, ctr;  // ctr: the exponentiation launches' work counters
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

Workspace *workspace(hipStream_t s) {
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto &w = g_ws[{dev, s}];
  if (!w) w = new Workspace();
  return w;
}

int ensure(Buf &b, size_t bytes, hipStream_t s) {
  if (b.bytes >= bytes) return HE_OK;
  if (b.p) {
    HE_TRY_HIP(hipStreamSynchronize(s));
    HE_TRY_HIP(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max(bytes, b.bytes * 3 / 2);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    hipGetLastError();
    b.p = nullptr;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      hipGetLastError();
      b.p = nullptr;
      return fail(HE_ERR_OOM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
    }
    want = bytes;
  }
  b.bytes = want;
  return HE_OK;
}

// ------------------------------------------------- exponentiation launch shapes
// Tuned shapes (lanes per integer, waves per SIMD) of the private-key
// exponentiations per (device, key size, kind, count class), filled by
// he_crt_autotune; count class = bit length of the count.
struct PowShape {
  int G = 0, waves = 0;  // waves 0: the kernel's own occupancy
  int tailG = 0;         // lanes per integer of the last partial round's launch (0: no separate launch)
};
std::mutex g_pow_mu;
std::map<std::tuple<int, int, int, int>, PowShape> g_pow_tuned;

int count_class(uint64_t count) {
  int b = 0;
  while (count) {
    ++b;
    count >>= 1;
  }
  return b;
}

// 32-bit limbs of the modulus of an exponentiation of `kind`: 4 mod P, 0
// and 2 mod P^2, 1 (public key) mod n^2.
int pow_s32(int KP, int kind) { return kind == 4 ? 16 * KP : (kind == 1 ? 64 * KP : 32 * KP); }

he::PowLaunch pow_launch_at(int KP, int kind, uint64_t count, PowShape sh) {
  const int S32 = pow_s32(KP, kind);
  if (sh.G == 0 || !he::pow_shape_valid(S32, sh.G)) sh = PowShape{he::pick_group(KP, kind, count), 0};
  const uint32_t dyn = he::pow_dyn_lds(S32, sh.G, sh.waves);
  const uint64_t per_wave = 64 / sh.G;
  const uint64_t work_blocks = (2 * ((count + per_wave - 1) / per_wave) + 3) / 4;
  const uint32_t grid =
      (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(he::pow_resident_blocks(S32, sh.G, dyn), work_blocks));
  return he::PowLaunch{sh.G, grid, dyn};
}

// The shape used when the autotuner has not run: pick_group's width, at the
// kernel's own occupancy unless two waves per SIMD take as many rounds of
// units (the resident waves each claiming one) to get through the batch.
// Fewer waves per SIMD each run faster, so in that case they finish sooner.
PowShape default_pow_shape(int KP, int kind, uint64_t count) {
  const int S32 = pow_s32(KP, kind);
  PowShape sh{he::pick_group(KP, kind, count), 0, 0};
  const uint32_t dyn2 = he::pow_dyn_lds(S32, sh.G, 2);
  if (dyn2 == 0) return sh;
  const uint64_t per_wave = 64 / sh.G;
  const uint64_t units = 2 * ((count + per_wave - 1) / per_wave);
  const uint64_t w_own = 4ull * he::pow_resident_blocks(S32, sh.G, 0);
  const uint64_t w_two = 4ull * he::pow_resident_blocks(S32, sh.G, dyn2);
  if (w_two < w_own && (units + w_two - 1) / w_two == (units + w_own - 1) / w_own) sh.waves = 2;
  return sh;
}

// The launches of shape `sh` over `count` ciphertexts.  With sh.tailG, the
// ciphertexts that fill whole rounds of the main launch's resident waves
// (as many units of 64 / G integers of one prime as a whole number of
// units per wave) go to the main launch and the rest, less than one round,
// to a launch at sh.tailG lanes per integer, whose fewer integers per wave
// spread that remainder over more waves.  No split when there is no whole
// round or no remainder.
he::PowPlan pow_plan_at(int KP, int kind, uint64_t count, PowShape sh) {
  he::PowPlan p{pow_launch_at(KP, kind, count, sh), count, he::PowLaunch{0, 0, 0}};
  const int S32 = pow_s32(KP, kind);
  if (sh.tailG == 0 || sh.tailG == p.main.G || !he::pow_shape_valid(S32, sh.tailG)) return p;
  const uint64_t per_wave = 64 / p.main.G;
  const uint64_t units = 2 * ((count + per_wave - 1) / per_wave);
  const uint64_t waves = 4ull * p.main.grid;
  const uint64_t rounds = units / waves;
  if (rounds == 0 || units % waves == 0) return p;
  p.main_count = rounds * waves / 2 * per_wave;  // < count: at least one unit pair is left
  p.tail = pow_launch_at(KP, kind, count - p.main_count, PowShape{sh.tailG, 0, 0});
  return p;
}

// Window-table bytes a plan's launches need (they run one after the other).
uint64_t plan_table_bytes(int KP, int kind, const he::PowPlan &p) {
  uint64_t b = (uint64_t)p.main.grid * he::table_bytes_per_block(KP, kind, p.main.G);
  if (p.tail.G) b = std::max<uint64_t>(b, (uint64_t)p.tail.grid * he::table_bytes_per_block(KP, kind, p.tail.G));
  return b;
}

// The launches of an exponentiation over `count` ciphertexts (units): the
// tuned shape for its class if the autotuner ran, else default_pow_shape's
// (one launch).
he::PowPlan pow_plan(int KP, int kind, uint64_t count) {
  PowShape sh = default_pow_shape(KP, kind, count);
  int dev = 0;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> lk(g_pow_mu);
    auto it = g_pow_tuned.find({dev, KP, kind, count_class(count)});
    if (it != g_pow_tuned.end()) sh = it->second;
  }
  return pow_plan_at(KP, kind, count, sh);
}

// m == nullptr encrypts zeros (the obfuscators r^n mod n^2).
int encrypt_impl(const he_key *key, const int64_t *m, uint64_t count, const uint32_t *r,
                 uint64_t r_seed, uint64_t r_offset, uint32_t *ct, hipStream_t stream, bool force_pub) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (count == 0) return HE_OK;
  if (!ct) return fail(HE_ERR_ARG, "null ct");
  Workspace *w = workspace(stream);
  const int KP = kp_of(key);
  const size_t L = key->n_bits / 32;
  if (key->priv && !force_pub) {
    he::PowPlan p1 = pow_plan(KP, 4, count), p2 = pow_plan(KP, 0, count);
    int rc = ensure(w->tab, std::max(plan_table_bytes(KP, 4, p1), plan_table_bytes(KP, 0, p2)), stream);
    if (rc) return rc;
    rc = ensure(w->ctr, 256, stream);
    if (rc) return rc;
    p1.ctr = (uint32_t *)w->ctr.p;
    p2.ctr = p1.ctr + 2;
    // omega / c_P per (ciphertext, prime) (2L limbs per ciphertext), then
    // r mod P / t per (ciphertext, prime) (L limbs)
    rc = ensure(w->tmp, count * 3 * L * sizeof(uint32_t), stream);
    if (rc) return rc;
    uint32_t *cpq = (uint32_t *)w->tmp.p, *tq = cpq + count * 2 * L;
    HE_TRY_HIP(he::launch_enc_crt(KP, key->dk, m, count, r, r_seed, r_offset, tq, cpq, ct, (uint32_t *)w->tab.p,
                                  p1, p2, stream));
  } else {
    // the exponentiation's units pair consecutive ciphertexts (both "primes"
    // of a public-key unit pair are n^2)
    he::PowPlan p = pow_plan(KP, 1, (count + 1) / 2);
    int rc = ensure(w->tab, plan_table_bytes(KP, 1, p), stream);
    if (rc) return rc;
    rc = ensure(w->ctr, 256, stream);
    if (rc) return rc;
    p.ctr = (uint32_t *)w->ctr.p;
    // r mod n^2, then r^n mod n^2 in place: count + (count & 1) rows of 2L limbs
    rc = ensure(w->tmp, (count + 1) * 2 * L * sizeof(uint32_t), stream);
    if (rc) return rc;
    HE_TRY_HIP(he::launch_enc_pub(KP, key->dk, m, count, r, r_seed, r_offset, (uint32_t *)w->tmp.p, ct,
                                  (uint32_t *)w->tab.p, p, stream));
  }
  return HE_OK;
}

}  // namespace

// ===================================================================== ABI
extern "C" {

const char *he_last_error(void) { return g_last_error.c_str(); }

int he_keygen(uint32_t n_bits, uint64_t seed, he_key **out) {
  if (!out) return fail(HE_ERR_ARG, "null out");
  if (!valid_bits(n_bits)) return fail(HE_ERR_ARG, "n_bits must be 1024 or 2048");
  try {
    const uint32_t half = n_bits / 2;
    Limbs p, q;
    for (uint64_t a = 0;; ++a) {
      p = hebn::prime_candidate(seed, 0, a, half);
      if (hebn::is_probable_prime(p)) break;
    }
    const Limbs one = hebn::from_u64(1);
    for (uint64_t a = 0;; ++a) {
      q = hebn::prime_candidate(seed, 1, a, half);
      if (hebn::cmp(q, p) == 0 || !hebn::is_probable_prime(q)) continue;
      Limbs g = hebn::gcd(hebn::mul(p, q), hebn::mul(hebn::sub(p, one), hebn::sub(q, one)));
      if (hebn::cmp(g, one) == 0) break;
    }
    return make_key(n_bits, p, q, true, out);
  } catch (const std::exception &e) {
    return fail(HE_ERR_KEY, std::string("keygen: ") + e.what());
  }
}

int he_key_import(uint32_t n_bits, const uint32_t *p, const uint32_t *q, he_key **out) {
  if (!out || !p) return fail(HE_ERR_ARG, "null argument");
  if (!valid_bits(n_bits)) return fail(HE_ERR_ARG, "n_bits must be 1024 or 2048");
  const size_t L = n_bits / 32;
  try {
    const Limbs one = hebn::from_u64(1);
    if (!q) {
      Limbs n = hebn::from_words(p, L);
      if (!hebn::is_odd(n) || hebn::bit_length(n) != n_bits)
        return fail(HE_ERR_KEY, "n must be odd with exactly n_bits bits");
      return make_key(n_bits, n, Limbs(), false, out);
    }
    Limbs P = hebn::from_words(p, L / 2), Q = hebn::from_words(q, L / 2);
    if (!hebn::is_odd(P) || !hebn::is_odd(Q) || hebn::cmp(P, one) <= 0 || hebn::cmp(Q, one) <= 0)
      return fail(HE_ERR_KEY, "p and q must be odd and > 1");
    if (hebn::cmp(P, Q) == 0) return fail(HE_ERR_KEY, "p == q");
    Limbs n = hebn::mul(P, Q);
    if (hebn::bit_length(n) != n_bits) return fail(HE_ERR_KEY, "p q must have exactly n_bits bits");
    Limbs g = hebn::gcd(n, hebn::mul(hebn::sub(P, one), hebn::sub(Q, one)));
    if (hebn::cmp(g, one) != 0) return fail(HE_ERR_KEY, "gcd(pq, (p-1)(q-1)) != 1");
    return make_key(n_bits, P, Q, true, out);
  } catch (const std::exception &e) {
    return fail(HE_ERR_KEY, std::string("import: ") + e.what());
  }
}

int he_key_export(const he_key *key, uint32_t *n, uint32_t *p, uint32_t *q) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  const size_t L = key->n_bits / 32;
  if ((p || q) && !key->priv) return fail(HE_ERR_NOPRIV, "public key has no p, q");
  if (n) hebn::to_words(key->n, n, L);
  if (p) hebn::to_words(key->p, p, L / 2);
  if (q) hebn::to_words(key->q, q, L / 2);
  return HE_OK;
}

int he_key_set_constant_time(he_key *key, int on) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  key->dk.ct = on ? 1 : 0;
  return HE_OK;
}

uint32_t he_key_bits(const he_key *key) { return key ? key->n_bits : 0; }
int he_key_has_private(const he_key *key) { return key && key->priv ? 1 : 0; }

void he_key_free(he_key *key) {
  if (!key) return;
  if (key->blob) hipFree(key->blob);
  delete key;
}

int he_encode(const double *x, uint64_t count, uint32_t frac_bits, int64_t *m, uint32_t *n_bad,
              hipStream_t stream) {
  if (count == 0) return HE_OK;
  if (!x || !m) return fail(HE_ERR_ARG, "null x or m");
  if (frac_bits > 62) return fail(HE_ERR_ARG, "frac_bits must be <= 62");
  HE_TRY_HIP(he::launch_encode(x, count, frac_bits, m, n_bad, stream));
  return HE_OK;
}

int he_encrypt(const he_key *key, const int64_t *m, uint64_t count, const uint32_t *r, uint64_t r_seed,
               uint64_t r_offset, uint32_t *ct, hipStream_t stream) {
  if (count && !m) return fail(HE_ERR_ARG, "null m");
  return encrypt_impl(key, m, count, r, r_seed, r_offset, ct, stream, false);
}

int he_obfuscators(const he_key *key, uint64_t count, const uint32_t *r, uint64_t r_seed, uint64_t r_offset,
                   uint32_t *rho, hipStream_t stream) {
  return encrypt_impl(key, nullptr, count, r, r_seed, r_offset, rho, stream, false);
}

int he_encrypt_obfuscated(const he_key *key, const int64_t *m, uint64_t count, const uint32_t *rho,
                          uint32_t *ct, hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (count == 0) return HE_OK;
  if (!m || !rho || !ct) return fail(HE_ERR_ARG, "null m, rho or ct");
  HE_TRY_HIP(he::launch_enc_obf(kp_of(key), key->dk, m, count, rho, ct, stream));
  return HE_OK;
}

int he_encrypt_public(const he_key *key, const int64_t *m, uint64_t count, const uint32_t *r,
                      uint64_t r_seed, uint64_t r_offset, uint32_t *ct, hipStream_t stream) {
  if (count && !m) return fail(HE_ERR_ARG, "null m");
  return encrypt_impl(key, m, count, r, r_seed, r_offset, ct, stream, true);
}

int he_hist_subtract(const he_key *key, const uint32_t *parent, const uint32_t *child, uint64_t count,
                     uint32_t batch, uint32_t *out, uint32_t *n_bad, hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (count == 0) return HE_OK;
  if (!parent || !child || !out) return fail(HE_ERR_ARG, "null parent, child or out");
  const uint64_t bytes = count * (key->n_bits / 16) * sizeof(uint32_t);
  auto overlap = [bytes](const void *x, const void *y) {
    const uintptr_t a = (uintptr_t)x, b = (uintptr_t)y;
    return a < b + bytes && b < a + bytes;
  };
  if (overlap(out, parent) || overlap(out, child)) return fail(HE_ERR_ARG, "out overlaps parent or child");
  if (batch == 0) batch = he::ct_div_batch(count);
  if ((count + batch - 1) / batch > (uint64_t)16 * 0x7FFFFFFF) return fail(HE_ERR_ARG, "batch too small");
  HE_TRY_HIP(he::launch_ct_div(kp_of(key), key->dk, parent, child, count, batch, out, n_bad, stream));
  return HE_OK;
}

static_assert(sizeof(he_split) == 32, "he_split layout");

int he_split_find(const int64_t *hist, const int64_t *minus, uint32_t nodes, uint32_t n_features, uint32_t n_bins,
                  uint32_t frac_bits, double lambda, double gamma, double min_child_weight, int64_t *derived,
                  he_split *out_feature, he_split *out_node, hipStream_t stream) {
  if (nodes == 0 || n_features == 0) return HE_OK;
  if (!hist || !out_node) return fail(HE_ERR_ARG, "null hist or out_node");
  if (n_bins < 1 || n_bins > 256) return fail(HE_ERR_ARG, "n_bins must be in [1, 256]");
  if (frac_bits > 62) return fail(HE_ERR_ARG, "frac_bits must be at most 62");
  if (!(lambda >= 0.0) || !(min_child_weight >= 0.0) || !(gamma == gamma))
    return fail(HE_ERR_ARG, "lambda and min_child_weight must be >= 0, gamma a number");
  HE_TRY_HIP(he::launch_split(hist, minus, nodes, n_features, n_bins, std::ldexp(1.0, -(int)frac_bits), lambda,
                              gamma, min_child_weight, derived, out_feature, out_node, stream));
  return HE_OK;
}

int he_ct_mul(const he_key *key, const uint32_t *a, const uint32_t *b, uint64_t count, uint32_t *out,
              hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (count == 0) return HE_OK;
  if (!a || !b || !out) return fail(HE_ERR_ARG, "null a, b or out");
  HE_TRY_HIP(he::launch_ct_mul(kp_of(key), key->dk, a, b, count, out, stream));
  return HE_OK;
}

int he_to_mont(const he_key *key, const uint32_t *in, uint64_t count, uint32_t *out, hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (count == 0) return HE_OK;
  if (!in || !out) return fail(HE_ERR_ARG, "null buffer");
  HE_TRY_HIP(he::launch_mont_convert(kp_of(key), key->dk, in, count, out, true, stream));
  return HE_OK;
}

int he_from_mont(const he_key *key, const uint32_t *in, uint64_t count, uint32_t *out, hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (count == 0) return HE_OK;
  if (!in || !out) return fail(HE_ERR_ARG, "null buffer");
  HE_TRY_HIP(he::launch_mont_convert(kp_of(key), key->dk, in, count, out, false, stream));
  return HE_OK;
}

int he_decrypt(const he_key *key, const uint32_t *ct, uint64_t count, int64_t *m, uint32_t *raw,
               uint32_t *n_overflow, hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (!key->priv) return fail(HE_ERR_NOPRIV, "decryption needs p and q");
  if (count == 0) return HE_OK;
  if (!ct || !m) return fail(HE_ERR_ARG, "null ct or m");
  Workspace *w = workspace(stream);
  const int KP = kp_of(key);
  const size_t L = key->n_bits / 32;
  he::PowPlan p = pow_plan(KP, 2, count);
  int rc = ensure(w->tab, plan_table_bytes(KP, 2, p), stream);
  if (rc) return rc;
  rc = ensure(w->ctr, 256, stream);
  if (rc) return rc;
  p.ctr = (uint32_t *)w->ctr.p;
  // c mod P^2, then c^(P-1) mod P^2, per (ciphertext, prime): 2L limbs per ciphertext
  rc = ensure(w->tmp, count * 2 * L * sizeof(uint32_t), stream);
  if (rc) return rc;
  HE_TRY_HIP(he::launch_dec(KP, key->dk, ct, count, (uint32_t *)w->tmp.p, m, raw, n_overflow,
                            (uint32_t *)w->tab.p, p, stream));
  return HE_OK;
}

}  // extern "C"

// ------------------------------------------------- allocation-free decryption
// Scratch of he_decrypt_noalloc: c mod p^2 and c mod q^2, then their powers
// (2L words per ciphertext, at most half of the array), followed by the
// exponentiation window tables of the persistent launch, whose grid is cut
// to what the rest of the array holds.  One copy per device, held until the
// process ends; in host code `scratch` only names the symbol, its device
// address comes from hipGetSymbolAddress.
namespace {
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kNoAllocDevices = 64;
}  // namespace
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];
namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device).
int scratch_address(void **out) {
  int dev = 0;
  HE_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices)
    return fail(HE_ERR_DEVICE, "device index " + std::to_string(dev) + " beyond the allocation-free path's table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HE_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(HE_ERR_DEVICE, "hipGetSymbolAddress returned a null address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HE_OK;
}
}  // namespace

extern "C" {

int he_decrypt_noalloc(const he_key *key, const uint32_t *ct, uint64_t count, int64_t *m, uint32_t *raw,
                       uint32_t *n_overflow, hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (!key->priv) return fail(HE_ERR_NOPRIV, "decryption needs p and q");
  if (count == 0) return HE_OK;
  if (!ct || !m) return fail(HE_ERR_ARG, "null ct or m");
  const int KP = kp_of(key);
  const size_t L = key->n_bits / 32;
  const uint64_t max_count = (kNoAllocBytes / 2) / (2 * L * sizeof(uint32_t));
  if (count > max_count)
    return fail(HE_ERR_ARG, "he_decrypt_noalloc: count " + std::to_string(count) + " exceeds the maximum of " +
                                std::to_string(max_count) + " ciphertexts at " + std::to_string(key->n_bits) +
                                "-bit keys (fixed scratch of " + std::to_string(kNoAllocBytes >> 20) + " MiB)");
  void *base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  const size_t xpq_bytes = (count * 2 * L * sizeof(uint32_t) + 255) / 256 * 256;
  // one launch whose grid is cut to the tables the scratch holds
  he::PowLaunch l = pow_plan(KP, 2, count).main;
  const uint64_t fit = (kNoAllocBytes - xpq_bytes) / he::table_bytes_per_block(KP, 2, l.G);
  if (fit == 0) return fail(HE_ERR_ARG, "he_decrypt_noalloc: no room for one block's window tables");
  l.grid = (uint32_t)std::min<uint64_t>(fit, l.grid);
  uint32_t *xpq = (uint32_t *)base;
  uint32_t *tab = (uint32_t *)((char *)base + xpq_bytes);
  // static units: no work counter in the scratch
  HE_TRY_HIP(he::launch_dec(KP, key->dk, ct, count, xpq, m, raw, n_overflow, tab,
                            he::PowPlan{l, count, he::PowLaunch{0, 0, 0}, nullptr}, stream));
  return HE_OK;
}

uint32_t he_pack_slots(const he_key *key, uint64_t count) {
  if (!key) return 0;
  return he::pack_slots((int)key->n_bits, count);
}

int he_pack(const he_key *key, const uint32_t *ct, uint64_t count, uint32_t slots, uint32_t *packed,
            hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (slots < 1 || slots > (key->n_bits - 1) / 64) return fail(HE_ERR_ARG, "slots must be in [1, (n_bits - 1) / 64]");
  if (count == 0) return HE_OK;
  if (!ct || !packed) return fail(HE_ERR_ARG, "null ct or packed");
  HE_TRY_HIP(he::launch_pack(kp_of(key), key->dk, ct, count, slots, packed, stream));
  return HE_OK;
}

int he_decrypt_packed(const he_key *key, const uint32_t *packed, uint64_t count, uint32_t slots, int64_t *m,
                      uint32_t *n_overflow, hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (!key->priv) return fail(HE_ERR_NOPRIV, "decryption needs p and q");
  if (slots < 1 || slots > (key->n_bits - 1) / 64) return fail(HE_ERR_ARG, "slots must be in [1, (n_bits - 1) / 64]");
  if (count == 0) return HE_OK;
  if (!packed || !m) return fail(HE_ERR_ARG, "null packed or m");
  const uint64_t n_packed = (count + slots - 1) / slots;
  const size_t L = key->n_bits / 32;
  Workspace *w = workspace(stream);
  const size_t raw_bytes = (n_packed * L * sizeof(uint32_t) + 255) & ~(size_t)255;
  int rc = ensure(w->unpack, raw_bytes + n_packed * sizeof(int64_t), stream);
  if (rc) return rc;
  uint32_t *raw = (uint32_t *)w->unpack.p;
  int64_t *whole = (int64_t *)((char *)w->unpack.p + raw_bytes);  // signed decode of the whole plaintext, unused
  rc = he_decrypt(key, packed, n_packed, whole, raw, nullptr, stream);
  if (rc) return rc;
  HE_TRY_HIP(he::launch_unpack(raw, count, slots, (uint32_t)L, m, n_overflow, stream));
  return HE_OK;
}

int he_hist_aggregate(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                      const he_hist_job *jobs, uint32_t n_jobs, hipStream_t stream) {
  return he_hist_aggregate_ex(key, ct, rows, ct_form, jobs, n_jobs, 0, stream);
}

}  // extern "C"

namespace {
size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Device layout of one histogram batch: job descriptors, flat per-(feature,
// bin) arrays, work items, the permutation and the partial products.
struct HistLayout {
  std::vector<he::DJob> dj;
  uint64_t total_fb = 0, total_f = 0, total_blocks = 0, total_perm = 0, items_cap = 0;
  uint64_t contributions = 0, rows = 0;
  size_t o_jobs = 0, o_counts = 0, o_offs = 0, o_cursor = 0, o_fch = 0, o_fitem = 0, o_border = 0, o_ftot = 0,
         o_fbase = 0, o_nitems = 0, o_items = 0, o_perm = 0, o_part = 0, o_ctm = 0, bytes = 0;
  uint32_t chunk = 64, split = 2;
  int G = he::kHistGroup, waves = 0;  // product kernel: lanes per ciphertext, waves per SIMD cap (0: none)
  bool convert = false;
};

int plan_layout(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form, const he_hist_job *jobs,
                uint32_t n_jobs, uint32_t chunk, uint32_t split, HistLayout &lay) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (!jobs) return fail(HE_ERR_ARG, "null jobs");
  if (ct_form != HE_FORM_CANONICAL && ct_form != HE_FORM_MONT) return fail(HE_ERR_ARG, "bad ct_form");
  if (chunk == 0) chunk = 64;
  if (chunk > (1u << 20)) return fail(HE_ERR_ARG, "chunk too large");
  if (split != 1 && split != 2) return fail(HE_ERR_ARG, "split must be 1 or 2");
  const size_t S = 2 * (key->n_bits / 32);
  lay.dj.assign(n_jobs, he::DJob{});
  lay.rows = rows;
  lay.chunk = chunk;
  lay.split = split;
  for (uint32_t j = 0; j < n_jobs; ++j) {
    const he_hist_job &J = jobs[j];
    const std::string tag = "job " + std::to_string(j) + ": ";
    if (J.n_features == 0 || J.n_bins == 0 || J.n_bins > 256)
      return fail(HE_ERR_ARG, tag + "need n_features >= 1 and 1 <= n_bins <= 256");
    if (!J.hist || !J.bins || (J.n_samples && !J.sample_idx)) return fail(HE_ERR_ARG, tag + "null pointer");
    if (J.n_samples > rows || J.n_samples >= (1ull << 32)) return fail(HE_ERR_ARG, tag + "n_samples exceeds rows");
    if (J.n_samples && !ct) return fail(HE_ERR_ARG, "null ct");
    if (J.bins_ld < rows) return fail(HE_ERR_ARG, tag + "bins_ld < rows");
    he::DJob &d = lay.dj[j];
    d.idx = J.sample_idx;
    d.bins = J.bins;
    d.hist = J.hist;
    d.n = J.n_samples;
    d.ld = J.bins_ld;
    d.F = J.n_features;
    d.B = J.n_bins;
    d.fb_off = lay.total_fb;
    d.perm_off = lay.total_perm;
    d.blk_off = lay.total_blocks;
    d.f_off = (uint32_t)lay.total_f;
    d.nblk = (uint32_t)((J.n_samples + he::kSampleBlock - 1) / he::kSampleBlock);
    d.n_bad = J.n_bad;
    lay.total_fb += (uint64_t)d.F * d.B;
    lay.total_f += d.F;
    lay.total_blocks += (uint64_t)d.F * d.nblk;
    lay.total_perm += (uint64_t)d.F * d.n;
    lay.items_cap += (uint64_t)d.F * ((d.n + chunk - 1) / chunk + std::min<uint64_t>(d.B, d.n));
    lay.contributions += 2ull * d.F * d.n;
  }
  if (lay.items_cap >= (1ull << 32)) return fail(HE_ERR_ARG, "too many work items; use a larger chunk");
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  lay.o_jobs = take(n_jobs * sizeof(he::DJob));
  lay.o_counts = take(lay.total_fb * 4);
  lay.o_offs = take(lay.total_fb * 4);
  lay.o_cursor = take(lay.total_fb * 4);
  lay.o_fch = take(lay.total_fb * 4);
  lay.o_fitem = take(lay.total_fb * 4);
  lay.o_border = take(lay.total_fb * 4);
  lay.o_ftot = take(lay.total_f * 4);
  lay.o_fbase = take(lay.total_f * 4);
  lay.o_nitems = take(8);  // item count, then the product kernel's work counter
  lay.o_items = take(std::max<uint64_t>(lay.items_cap, 1) * sizeof(he::HistItem));
  lay.o_perm = take(std::max<uint64_t>(lay.total_perm, 1) * 4);
  // partial products in the histogram kernels' 29-bit limbs
  const uint64_t S29 = (uint64_t)he29::limbs_for_group((int)S, he::kHistGroup);
  lay.o_part = take(std::max<uint64_t>(lay.items_cap, 1) * 2 * S29 * 4);
  lay.convert = ct_form == HE_FORM_CANONICAL && rows > 0;
  lay.o_ctm = lay.convert ? take(rows * 2 * S * 4) : 0;
  lay.bytes = off;
  return HE_OK;
}

he::HistWs bind_layout(const HistLayout &lay, char *base) {
  he::HistWs ws{};
  ws.jobs = (he::DJob *)(base + lay.o_jobs);
  ws.n_jobs = (uint32_t)lay.dj.size();
  ws.counts = (uint32_t *)(base + lay.o_counts);
  ws.offs = (uint32_t *)(base + lay.o_offs);
  ws.cursor = (uint32_t *)(base + lay.o_cursor);
  ws.fch = (uint32_t *)(base + lay.o_fch);
  ws.fitem = (uint32_t *)(base + lay.o_fitem);
  ws.border = (uint32_t *)(base + lay.o_border);
  ws.ftot = (uint32_t *)(base + lay.o_ftot);
  ws.fbase = (uint32_t *)(base + lay.o_fbase);
  ws.n_items = (uint32_t *)(base + lay.o_nitems);
  ws.next = ws.n_items + 1;
  ws.items = (he::HistItem *)(base + lay.o_items);
  ws.perm = (uint32_t *)(base + lay.o_perm);
  ws.partials = (uint32_t *)(base + lay.o_part);
  ws.total_fb = lay.total_fb;
  ws.total_f = lay.total_f;
  ws.total_blocks = lay.total_blocks;
  ws.items_cap = lay.items_cap;
  ws.rows = lay.rows;
  ws.chunk = lay.chunk;
  ws.split = lay.split;
  return ws;
}

// Enqueues every kernel of one batch on `stream` (no allocation, no
// memset: safe to capture into a graph).
int enqueue_hist(const he_key *key, const uint32_t *ct, uint64_t rows, const HistLayout &lay, char *base,
                 hipStream_t stream, uint64_t *mm_count = nullptr) {
  he::HistWs ws = bind_layout(lay, base);
  ws.mm_count = (unsigned long long *)mm_count;
  const int KP = kp_of(key);
  const uint32_t *ctm = ct;
  if (lay.convert) {
    uint32_t *dst = (uint32_t *)(base + lay.o_ctm);
    HE_TRY_HIP(he::launch_mont_convert(KP, key->dk, ct, rows * 2, dst, true, stream));
    ctm = dst;
  }
  he::HistLaunch hl{lay.G, 0, 0};
  if (!he::hist_shape_valid(KP, hl.G)) hl.G = he::kHistGroup;
  hl.dyn = he::hist_dyn_lds(KP, hl.G, lay.waves);
  hl.grid = he::hist_resident_blocks(KP, hl.G, hl.dyn);
  HE_TRY_HIP(he::launch_hist(KP, key->dk, ctm, lay.dj.data(), ws, hl, stream));
  return HE_OK;
}

int hist_run(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form, const he_hist_job *jobs,
             uint32_t n_jobs, uint32_t chunk, uint32_t split, hipStream_t stream, uint64_t *mm_count = nullptr,
             int G = he::kHistGroup, int waves = 0) {
  if (n_jobs == 0) return key ? HE_OK : fail(HE_ERR_ARG, "null key");
  HistLayout lay;
  int rc = plan_layout(key, ct, rows, ct_form, jobs, n_jobs, chunk, split, lay);
  if (rc) return rc;
  lay.G = G;
  lay.waves = waves;
  Workspace *w = workspace(stream);
  rc = ensure(w->hist, lay.bytes, stream);
  if (rc) return rc;
  return enqueue_hist(key, ct, rows, lay, (char *)w->hist.p, stream, mm_count);
}

// Autotuner cache: best (chunk, split) per shape class.
struct TuneKey {
  uint32_t bits, log2_contrib, log2_jobs, max_bins;
  bool operator<(const TuneKey &o) const {
    return std::tie(bits, log2_contrib, log2_jobs, max_bins) < std::tie(o.bits, o.log2_contrib, o.log2_jobs, o.max_bins);
  }
};
struct TuneVal {
  uint32_t chunk, split;
  float ms;
  int G = he::kHistGroup, waves = 0;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

uint32_t ilog2(uint64_t x) {
  uint32_t r = 0;
  while (x > 1) {
    x >>= 1;
    ++r;
  }
  return r;
}

TuneKey tune_key(const he_key *key, const he_hist_job *jobs, uint32_t n_jobs) {
  uint64_t contrib = 0;
  uint32_t mb = 0;
  for (uint32_t j = 0; j < n_jobs; ++j) {
    contrib += 2ull * jobs[j].n_features * jobs[j].n_samples;
    mb = std::max(mb, jobs[j].n_bins);
  }
  return TuneKey{key->n_bits, ilog2(contrib + 1), ilog2(n_jobs), mb};
}

// Work shape of an untuned batch (chunk 0, no autotuner entry for its
// class): at 2048-bit keys, a batch with enough items to fill the device
// several times over takes 8 lanes per ciphertext and items of up to 128
// samples (two items per wave, fewer instructions per product); a smaller
// one 16 lanes and items of up to 64 samples (one item per wave, so that
// its few items spread over more waves).
TuneVal default_hist_shape(const he_key *key, const he_hist_job *jobs, uint32_t n_jobs) {
  constexpr uint64_t kLargeBatchItems = 16384;
  uint64_t items = 0;
  for (uint32_t j = 0; j < n_jobs; ++j)
    items += (uint64_t)jobs[j].n_features *
             ((jobs[j].n_samples + 127) / 128 + std::min<uint64_t>(jobs[j].n_bins, jobs[j].n_samples));
  if (kp_of(key) == 2 && items >= kLargeBatchItems) return TuneVal{128, 2, 0.f, 8, 0};
  return TuneVal{64, 2, 0.f, he::kHistGroup, 0};
}

}  // namespace

extern "C" int he_hist_aggregate_ex(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                                    const he_hist_job *jobs, uint32_t n_jobs, uint32_t chunk,
                                    hipStream_t stream) {
  uint32_t split = 2;
  int G = he::kHistGroup, waves = 0;
  if (chunk == 0 && key && jobs && n_jobs) {
    TuneVal v = default_hist_shape(key, jobs, n_jobs);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(tune_key(key, jobs, n_jobs));
      if (it != g_tune.end()) v = it->second;
    }
    chunk = v.chunk;
    split = v.split;
    G = v.G;
    waves = v.waves;
  }
  return hist_run(key, ct, rows, ct_form, jobs, n_jobs, chunk, split, stream, nullptr, G, waves);
}

extern "C" int he_hist_aggregate_counted(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                                         const he_hist_job *jobs, uint32_t n_jobs, uint32_t chunk, uint32_t split,
                                         uint32_t lanes, uint32_t waves, uint64_t *mm_count, hipStream_t stream) {
  if (!mm_count) return fail(HE_ERR_ARG, "null mm_count");
  if (split != 1 && split != 2) return fail(HE_ERR_ARG, "split must be 1 or 2");
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (lanes == 0) lanes = he::kHistGroup;
  if (!he::hist_shape_valid(kp_of(key), (int)lanes))
    return fail(HE_ERR_ARG, "lanes must be 16, or 8 at 2048-bit keys");
  if (waves > 8) return fail(HE_ERR_ARG, "waves must be 0 (own occupancy) to 8");
  return hist_run(key, ct, rows, ct_form, jobs, n_jobs, chunk, split, stream, mm_count, (int)lanes, (int)waves);
}

extern "C" int he_hist_autotune(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                                const he_hist_job *jobs, uint32_t n_jobs, uint32_t *chunk_out,
                                uint32_t *split_out, uint32_t *lanes_out, uint32_t *waves_out, float *ms_out,
                                hipStream_t stream) {
  if (!key || !jobs || n_jobs == 0) return fail(HE_ERR_ARG, "need a key and at least one job");
  static const uint32_t chunks[] = {16, 32, 64, 128, 256, 512};
  hipEvent_t e0, e1;
  HE_TRY_HIP(hipEventCreate(&e0));
  HE_TRY_HIP(hipEventCreate(&e1));
  TuneVal best{64, 2, 1e30f};
  TuneVal best_g[2] = {{64, 2, 1e30f}, {64, 2, 1e30f}};  // per lanes per ciphertext: [0] 16, [1] 8
  int rc = HE_OK;
  auto trial = [&](uint32_t c, uint32_t split, int G, int waves) -> int {
    int r = hist_run(key, ct, rows, ct_form, jobs, n_jobs, c, split, stream, nullptr, G, waves);  // warm-up
    if (r) return r;
    HE_TRY_HIP(hipEventRecord(e0, stream));
    for (int k = 0; k < 2 && !r; ++k) r = hist_run(key, ct, rows, ct_form, jobs, n_jobs, c, split, stream, nullptr, G, waves);
    if (r) return r;
    HE_TRY_HIP(hipEventRecord(e1, stream));
    HE_TRY_HIP(hipEventSynchronize(e1));
    float ms = 0;
    HE_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms /= 2;
    const TuneVal v{c, split, ms, G, waves};
    if (ms < best.ms) best = v;
    TuneVal &bg = best_g[G == he::kHistGroup ? 0 : 1];
    if (ms < bg.ms) bg = v;
    return HE_OK;
  };
  // work items (chunk, groups per item) for each lane count at the kernel's
  // own occupancy (the 8-lane waves take two or four items at once, so their
  // best items differ), then waves per SIMD at the best items of each
  const int KP = kp_of(key);
  for (int G : {he::kHistGroup, 8}) {
    if (rc || !he::hist_shape_valid(KP, G)) continue;
    for (uint32_t split : {2u, 1u}) {
      for (uint32_t c : chunks) {
        if (G != he::kHistGroup && (c < 32 || c > 256)) continue;  // 8 lanes: the middle lengths only
        if ((rc = trial(c, split, G, 0))) break;
      }
      if (rc) break;
    }
  }
  for (int G : {he::kHistGroup, 8}) {
    if (rc || !he::hist_shape_valid(KP, G)) continue;
    const TuneVal bg = best_g[G == he::kHistGroup ? 0 : 1];
    for (int waves : {4, 3, 2}) {
      if (he::hist_dyn_lds(KP, G, waves) == 0) continue;  // no cap needed: same as its own occupancy
      if ((rc = trial(bg.chunk, bg.split, G, waves))) break;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(key, jobs, n_jobs)] = best;
  }
  if (chunk_out) *chunk_out = best.chunk;
  if (split_out) *split_out = best.split;
  if (lanes_out) *lanes_out = (uint32_t)best.G;
  if (waves_out) *waves_out = (uint32_t)best.waves;
  if (ms_out) *ms_out = best.ms;
  return HE_OK;
}

// ------------------------------------------- exponentiation shape autotuner
namespace {
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) hipFree(p);
  }
};

// Times `launch` (two runs after one warm-up) on `stream`; ms per run.
template <typename F>
int time_ms(F launch, hipStream_t stream, hipEvent_t e0, hipEvent_t e1, float *ms) {
  HE_TRY_HIP(launch());
  HE_TRY_HIP(hipEventRecord(e0, stream));
  for (int r = 0; r < 2; ++r) HE_TRY_HIP(launch());
  HE_TRY_HIP(hipEventRecord(e1, stream));
  HE_TRY_HIP(hipEventSynchronize(e1));
  HE_TRY_HIP(hipEventElapsedTime(ms, e0, e1));
  *ms /= 2;
  return HE_OK;
}
}  // namespace

extern "C" int he_crt_autotune(const he_key *key, uint64_t enc_count, uint64_t dec_count, uint32_t *choice,
                               float *ms_out, hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (!key->priv) return fail(HE_ERR_NOPRIV, "the CRT exponentiations need p and q");
  if (enc_count == 0 || dec_count == 0) return fail(HE_ERR_ARG, "need enc_count >= 1 and dec_count >= 1");
  const int KP = kp_of(key);
  const size_t L = key->n_bits / 32;
  const uint64_t n_ct = std::max(enc_count, dec_count);
  int dev = 0;
  HE_TRY_HIP(hipGetDevice(&dev));
  // trial buffers: r mod P / t, omega, ciphertexts, c mod P^2, window tables,
  // work counters
  DevBuf tq, cpq, ct, xpq, tab, ctr;
  size_t tab_bytes = 0;
  for (int kind : {4, 0, 2})
    for (int G : {2, 4, 8, 16})
      if (he::pow_shape_valid(pow_s32(KP, kind), G))
        tab_bytes = std::max<size_t>(tab_bytes, (size_t)he::pow_resident_blocks(pow_s32(KP, kind), G, 0) *
                                                   he::table_bytes_per_block(KP, kind, G));
  const size_t sizes[6] = {n_ct * L * 4, n_ct * 2 * L * 4, n_ct * 2 * L * 4, n_ct * 2 * L * 4, tab_bytes, 256};
  DevBuf *bufs[6] = {&tq, &cpq, &ct, &xpq, &tab, &ctr};
  for (int b = 0; b < 6; ++b)
    if (hipMalloc(&bufs[b]->p, sizes[b]) != hipSuccess) {
      hipGetLastError();
      return fail(HE_ERR_OOM, "autotuner trial buffers");
    }
  uint32_t *tq_p = (uint32_t *)tq.p, *cpq_p = (uint32_t *)cpq.p, *ct_p = (uint32_t *)ct.p,
           *xpq_p = (uint32_t *)xpq.p, *tab_p = (uint32_t *)tab.p;
  const uint32_t SP = 16 * KP, SP2 = 32 * KP;
  // real operands: r mod P, one encryption (default shapes), c mod P^2
  HE_TRY_HIP(he::launch_enc_r(KP, key->dk, enc_count, nullptr, 1, 0, tq_p, stream));
  int rc = encrypt_impl(key, nullptr, n_ct, nullptr, 1, 0, ct_p, stream, false);
  if (rc) return rc;
  HE_TRY_HIP(he::launch_dec_pre(KP, key->dk, ct_p, dec_count, xpq_p, stream));
  hipEvent_t e0, e1;
  HE_TRY_HIP(hipEventCreate(&e0));
  HE_TRY_HIP(hipEventCreate(&e1));
  PowShape best[3];
  float best_ms[3] = {1e30f, 1e30f, 1e30f};
  const int kinds[3] = {4, 0, 2};
  for (int t = 0; t < 3 && !rc; ++t) {
    const int kind = kinds[t];
    const uint64_t count = kind == 2 ? dec_count : enc_count;
    auto trial = [&](const PowShape &sh, he::PowPlan p) -> int {
      p.ctr = (uint32_t *)ctr.p;
      auto run = [&]() -> hipError_t {
        if (kind == 4) return he::launch_pow_kind(KP, key->dk, 4, tq_p, SP, SP, tq_p, SP, count, tab_p, p, stream);
        if (kind == 0) return he::launch_pow_kind(KP, key->dk, 0, tq_p, SP, SP, cpq_p, SP2, count, tab_p, p, stream);
        return he::launch_pow_kind(KP, key->dk, 2, xpq_p, SP2, SP2, xpq_p, SP2, count, tab_p, p, stream);
      };
      float ms = 0;
      const int r = time_ms(run, stream, e0, e1, &ms);
      if (r) return r;
      if (ms < best_ms[t]) {
        best_ms[t] = ms;
        best[t] = sh;
      }
      return HE_OK;
    };
    // lanes per integer and waves per SIMD in one launch, then, at the best
    // of those, a separate launch for the last partial round at each wider
    // group
    for (int G : {2, 4, 8, 16}) {
      if (!he::pow_shape_valid(pow_s32(KP, kind), G)) continue;
      for (int waves : {0, 3, 2}) {
        const PowShape sh{G, waves, 0};
        const he::PowPlan p = pow_plan_at(KP, kind, count, sh);
        if (waves && p.main.dyn == 0) continue;  // the kernel's own occupancy is already at most `waves`
        if ((rc = trial(sh, p))) break;
      }
      if (rc) break;
    }
    const PowShape one = best[t];
    for (int tg : {4, 8, 16}) {
      if (rc || tg <= one.G || !he::pow_shape_valid(pow_s32(KP, kind), tg)) continue;
      const PowShape sh{one.G, one.waves, tg};
      const he::PowPlan p = pow_plan_at(KP, kind, count, sh);
      if (p.tail.G == 0) break;  // whole rounds only, or less than one: nothing to split
      rc = trial(sh, p);
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HE_TRY_HIP(hipStreamSynchronize(stream));
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_pow_mu);
    for (int t = 0; t < 3; ++t)
      g_pow_tuned[{dev, KP, kinds[t], count_class(kinds[t] == 2 ? dec_count : enc_count)}] = best[t];
  }
  for (int t = 0; t < 3; ++t) {
    if (choice) {
      choice[3 * t] = (uint32_t)best[t].G;
      choice[3 * t + 1] = (uint32_t)best[t].waves;
      choice[3 * t + 2] = (uint32_t)best[t].tailG;
    }
    if (ms_out) ms_out[t] = best_ms[t];
  }
  return HE_OK;
}

extern "C" int he_crt_set_shape(const he_key *key, uint32_t kind, uint64_t count, uint32_t lanes, uint32_t waves,
                                uint32_t tail_lanes) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (kind > 3)
    return fail(HE_ERR_ARG, "kind must be 0 (mod p), 1 (lift), 2 (decryption) or 3 (public-key encryption)");
  if (count == 0) return fail(HE_ERR_ARG, "count must be at least 1");
  const int KP = kp_of(key), k = kind == 0 ? 4 : (kind == 1 ? 0 : (kind == 2 ? 2 : 1));
  // public-key encryption plans its exponentiation over unit pairs of two ciphertexts
  const uint64_t units = kind == 3 ? (count + 1) / 2 : count;
  const int S32 = pow_s32(KP, k);
  if (!he::pow_shape_valid(S32, (int)lanes))
    return fail(HE_ERR_ARG, "lanes " + std::to_string(lanes) + " not built for this kind and key size");
  if (waves != 0 && waves != 2 && waves != 3) return fail(HE_ERR_ARG, "waves must be 0 (own occupancy), 2 or 3");
  if (tail_lanes != 0 && (tail_lanes <= lanes || !he::pow_shape_valid(S32, (int)tail_lanes)))
    return fail(HE_ERR_ARG, "tail_lanes must be 0 or a built width above lanes");
  int dev = 0;
  HE_TRY_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_pow_mu);
  g_pow_tuned[{dev, KP, k, count_class(units)}] = PowShape{(int)lanes, (int)waves, (int)tail_lanes};
  return HE_OK;
}

// ------------------------------------------------------------ captured plans
struct he_hist_plan {
  const he_key *key = nullptr;
  HistLayout lay;
  void *ws = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" void he_hist_plan_free(he_hist_plan *plan) {
  if (!plan) return;
  if (plan->exec) hipGraphExecDestroy(plan->exec);
  if (plan->graph) hipGraphDestroy(plan->graph);
  if (plan->ws) hipFree(plan->ws);
  delete plan;
}

extern "C" int he_hist_plan_create(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                                   const he_hist_job *jobs, uint32_t n_jobs, uint32_t chunk, uint32_t split,
                                   he_hist_plan **out) {
  if (!out) return fail(HE_ERR_ARG, "null out");
  if (!key || !jobs || n_jobs == 0) return fail(HE_ERR_ARG, "need a key and at least one job");
  int G = he::kHistGroup, waves = 0;
  if (chunk == 0) {
    TuneVal v = default_hist_shape(key, jobs, n_jobs);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(tune_key(key, jobs, n_jobs));
      if (it != g_tune.end()) v = it->second;
    }
    chunk = v.chunk;
    if (split == 0) split = v.split;
    G = v.G;
    waves = v.waves;
  }
  if (split == 0) split = 2;
  he_hist_plan *p = new (std::nothrow) he_hist_plan();
  if (!p) return fail(HE_ERR_OOM, "out of host memory");
  p->key = key;
  int rc = plan_layout(key, ct, rows, ct_form, jobs, n_jobs, chunk, split, p->lay);
  if (rc) {
    delete p;
    return rc;
  }
  p->lay.G = G;
  p->lay.waves = waves;
  if (hipMalloc(&p->ws, std::max<size_t>(p->lay.bytes, 256)) != hipSuccess) {
    hipGetLastError();
    delete p;
    return fail(HE_ERR_OOM, "plan workspace allocation of " + std::to_string(p->lay.bytes) + " bytes failed");
  }
  // resident block counts and LDS caps are queried before capture
  // (occupancy calls are not stream work, but keep capture free of anything
  // but launches)
  (void)he::hist_resident_blocks(kp_of(key), G, he::hist_dyn_lds(kp_of(key), G, waves));
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    he_hist_plan_free(p);
    return fail(HE_ERR_DEVICE, "stream creation failed");
  }
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = enqueue_hist(key, ct, rows, p->lay, (char *)p->ws, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &p->graph);
    if (rc == HE_OK && e2 != hipSuccess) rc = fail(HE_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(e2));
  } else {
    rc = fail(HE_ERR_DEVICE, std::string("begin capture: ") + hipGetErrorString(e));
  }
  hipStreamDestroy(cs);
  if (rc == HE_OK) {
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = fail(HE_ERR_DEVICE, std::string("instantiate: ") + hipGetErrorString(e));
  }
  if (rc != HE_OK) {
    he_hist_plan_free(p);
    return rc;
  }
  *out = p;
  return HE_OK;
}

extern "C" int he_hist_plan_launch(he_hist_plan *plan, hipStream_t stream) {
  if (!plan || !plan->exec) return fail(HE_ERR_ARG, "null plan");
  HE_TRY_HIP(hipGraphLaunch(plan->exec, stream));
  return HE_OK;
}

extern "C" int he_probe_int_mul(uint64_t iters, uint32_t blocks, uint64_t *products, hipStream_t stream) {
  if (!blocks || !iters) return fail(HE_ERR_ARG, "iters and blocks must be > 0");
  Workspace *w = workspace(stream);
  int rc = ensure(w->tmp, 256, stream);
  if (rc) return rc;
  HE_TRY_HIP(he::launch_probe_mul(iters, blocks, (uint32_t *)w->tmp.p, stream));
  if (products) *products = (uint64_t)blocks * 256 * iters * 8;
  return HE_OK;
}
