// Host runtime behind the C ABI in include/he.h: key objects with their
// device-resident constants, per-stream workspaces, argument checks and
// kernel dispatch.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <map>
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
  return he::DMod{base + o.N, base + o.R1, base + o.R2, base + o.R3, base + o.R4, o.ninv};
}
he::DExp mk_exp(const uint32_t *base, const hekey::ExpOff &o) { return he::DExp{base + o.e, o.nwin}; }

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
  Buf tab, tmp, hist;
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

uint32_t persistent_grid(int KP, int kind, uint64_t work_blocks) {
  const uint32_t res = he::resident_blocks(KP, kind);
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(res, work_blocks));
}

int encrypt_impl(const he_key *key, const int64_t *m, uint64_t count, const uint32_t *r,
                 uint64_t r_seed, uint64_t r_offset, uint32_t *ct, hipStream_t stream, bool force_pub) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (count == 0) return HE_OK;
  if (!m || !ct) return fail(HE_ERR_ARG, "null m or ct");
  Workspace *w = workspace(stream);
  const int KP = kp_of(key);
  const size_t L = key->n_bits / 32;
  if (key->priv && !force_pub) {
    const uint32_t grid = persistent_grid(KP, 0, (2 * ((count + 3) / 4) + 3) / 4);
    int rc = ensure(w->tab, grid * he::table_bytes_per_block(KP, 0), stream);
    if (rc) return rc;
    rc = ensure(w->tmp, count * 2 * L * sizeof(uint32_t), stream);
    if (rc) return rc;
    HE_TRY_HIP(he::launch_enc_crt(KP, key->dk, m, count, r, r_seed, r_offset, (uint32_t *)w->tmp.p, ct,
                                  (uint32_t *)w->tab.p, grid, stream));
  } else {
    const uint32_t grid = persistent_grid(KP, 1, ((count + 3) / 4 + 3) / 4);
    int rc = ensure(w->tab, grid * he::table_bytes_per_block(KP, 1), stream);
    if (rc) return rc;
    HE_TRY_HIP(he::launch_enc_pub(KP, key->dk, m, count, r, r_seed, r_offset, ct, (uint32_t *)w->tab.p, grid,
                                  stream));
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
  return encrypt_impl(key, m, count, r, r_seed, r_offset, ct, stream, false);
}

int he_encrypt_public(const he_key *key, const int64_t *m, uint64_t count, const uint32_t *r,
                      uint64_t r_seed, uint64_t r_offset, uint32_t *ct, hipStream_t stream) {
  return encrypt_impl(key, m, count, r, r_seed, r_offset, ct, stream, true);
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
  const uint32_t grid = persistent_grid(KP, 2, (2 * ((count + 3) / 4) + 3) / 4);
  int rc = ensure(w->tab, grid * he::table_bytes_per_block(KP, 2), stream);
  if (rc) return rc;
  rc = ensure(w->tmp, count * L * sizeof(uint32_t), stream);
  if (rc) return rc;
  HE_TRY_HIP(he::launch_dec(KP, key->dk, ct, count, (uint32_t *)w->tmp.p, m, raw, n_overflow,
                            (uint32_t *)w->tab.p, grid, stream));
  return HE_OK;
}

int he_hist_aggregate(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                      const he_hist_job *jobs, uint32_t n_jobs, hipStream_t stream) {
  return he_hist_aggregate_ex(key, ct, rows, ct_form, jobs, n_jobs, 0, stream);
}

}  // extern "C"

namespace {
size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }
}  // namespace

extern "C" int he_hist_aggregate_ex(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                                    const he_hist_job *jobs, uint32_t n_jobs, uint32_t chunk,
                                    hipStream_t stream) {
  if (!key) return fail(HE_ERR_ARG, "null key");
  if (n_jobs == 0) return HE_OK;
  if (!jobs) return fail(HE_ERR_ARG, "null jobs");
  if (ct_form != HE_FORM_CANONICAL && ct_form != HE_FORM_MONT) return fail(HE_ERR_ARG, "bad ct_form");
  if (chunk == 0) chunk = 64;
  if (chunk > (1u << 20)) return fail(HE_ERR_ARG, "chunk too large");
  const size_t L = key->n_bits / 32, S = 2 * L;
  std::vector<he::DJob> dj(n_jobs);
  uint64_t total_fb = 0, total_f = 0, total_blocks = 0, total_perm = 0, items_cap = 0;
  for (uint32_t j = 0; j < n_jobs; ++j) {
    const he_hist_job &J = jobs[j];
    if (J.n_features == 0 || J.n_bins == 0 || J.n_bins > 256)
      return fail(HE_ERR_ARG, "job " + std::to_string(j) + ": need n_features >= 1 and 1 <= n_bins <= 256");
    if (!J.hist || !J.bins || (J.n_samples && !J.sample_idx))
      return fail(HE_ERR_ARG, "job " + std::to_string(j) + ": null pointer");
    if (J.n_samples > rows || J.n_samples >= (1ull << 32))
      return fail(HE_ERR_ARG, "job " + std::to_string(j) + ": n_samples exceeds rows");
    if (J.n_samples && !ct) return fail(HE_ERR_ARG, "null ct");
    if (J.bins_ld < rows) return fail(HE_ERR_ARG, "job " + std::to_string(j) + ": bins_ld < rows");
    he::DJob &d = dj[j];
    d.idx = J.sample_idx;
    d.bins = J.bins;
    d.hist = J.hist;
    d.n = J.n_samples;
    d.ld = J.bins_ld;
    d.F = J.n_features;
    d.B = J.n_bins;
    d.fb_off = total_fb;
    d.perm_off = total_perm;
    d.blk_off = total_blocks;
    d.f_off = (uint32_t)total_f;
    d.nblk = (uint32_t)((J.n_samples + he::kSampleBlock - 1) / he::kSampleBlock);
    total_fb += (uint64_t)d.F * d.B;
    total_f += d.F;
    total_blocks += (uint64_t)d.F * d.nblk;
    total_perm += (uint64_t)d.F * d.n;
    items_cap += (uint64_t)d.F * ((d.n + chunk - 1) / chunk + std::min<uint64_t>(d.B, d.n));
  }
  if (items_cap >= (1ull << 32)) return fail(HE_ERR_ARG, "too many work items; use a larger chunk");
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t o_jobs = take(n_jobs * sizeof(he::DJob));
  const size_t o_counts = take(total_fb * 4), o_offs = take(total_fb * 4), o_cursor = take(total_fb * 4);
  const size_t o_fch = take(total_fb * 4), o_fitem = take(total_fb * 4);
  const size_t o_ftot = take(total_f * 4), o_fbase = take(total_f * 4), o_nitems = take(4);
  const size_t o_items = take(std::max<uint64_t>(items_cap, 1) * sizeof(he::HistItem));
  const size_t o_perm = take(std::max<uint64_t>(total_perm, 1) * 4);
  const size_t o_part = take(std::max<uint64_t>(items_cap, 1) * 2 * S * 4);
  const size_t o_ctm = ct_form == HE_FORM_CANONICAL ? take(rows * 2 * S * 4) : 0;
  Workspace *w = workspace(stream);
  int rc = ensure(w->hist, off, stream);
  if (rc) return rc;
  char *base = (char *)w->hist.p;
  he::HistWs ws{};
  ws.jobs = (he::DJob *)(base + o_jobs);
  ws.n_jobs = n_jobs;
  ws.counts = (uint32_t *)(base + o_counts);
  ws.offs = (uint32_t *)(base + o_offs);
  ws.cursor = (uint32_t *)(base + o_cursor);
  ws.fch = (uint32_t *)(base + o_fch);
  ws.fitem = (uint32_t *)(base + o_fitem);
  ws.ftot = (uint32_t *)(base + o_ftot);
  ws.fbase = (uint32_t *)(base + o_fbase);
  ws.n_items = (uint32_t *)(base + o_nitems);
  ws.items = (he::HistItem *)(base + o_items);
  ws.perm = (uint32_t *)(base + o_perm);
  ws.partials = (uint32_t *)(base + o_part);
  ws.total_fb = total_fb;
  ws.total_f = total_f;
  ws.total_blocks = total_blocks;
  ws.items_cap = items_cap;
  ws.chunk = chunk;
  const uint32_t *ctm = ct;
  const int KP = kp_of(key);
  if (ct_form == HE_FORM_CANONICAL && rows) {
    uint32_t *dst = (uint32_t *)(base + o_ctm);
    HE_TRY_HIP(he::launch_mont_convert(KP, key->dk, ct, rows * 2, dst, true, stream));
    ctm = dst;
  }
  const uint32_t grid = he::resident_blocks(KP, 3);
  HE_TRY_HIP(he::launch_hist(KP, key->dk, ctm, dj.data(), ws, grid, stream));
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
