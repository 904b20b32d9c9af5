// Internal interfaces between the host runtime (he_api.cpp) and the kernels
// (he_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "radix29.hpp"

namespace he {

// One Montgomery modulus N of S limbs (R = 2^(32 S)); device pointers into
// the key's constant blob, each S limbs.  The radix-2^29 form (R' =
// 2^(29 S29), one set per limb-count variant) serves the exponentiations.
struct DMod {
  const uint32_t *N, *R1, *R2, *R3, *R4;  // N, R^k mod N
  uint32_t ninv;                          // -N^-1 mod 2^32
  const uint32_t *N29[he29::kVariants];   // N in S29 limbs of 29 bits
  const uint32_t *R1_29[he29::kVariants]; // R' mod N
  const uint32_t *R2_29[he29::kVariants]; // R'^2 mod N
};

// Exponent as limbs with one zero limb of padding and its fixed-window
// count, and its sliding-window schedule (keysetup.hpp, sliding_schedule).
struct DExp {
  const uint32_t *e;
  int nwin;
  const uint32_t *ops;
  int nops;
};

// Per-prime constants for the CRT paths; P is this prime, Q the other one.
// S_P = L/2 limbs for P, S_P2 = L limbs for P^2 (L = limbs of n).
struct DPrime {
  DMod P, P2;
  DExp e_enc;        // Q mod (P - 1): r^Q mod P = r^(Q mod (P-1)) mod P
  DExp e_lift;       // P: x -> x^P mod P^2 depends only on x mod P
  DExp e_dec;        // P - 1: decryption exponent
  const uint32_t *QR_P;   // Q R mod P          (S_P limbs)
  const uint32_t *PR_P2;  // P R' mod P^2       (S_P2 limbs)
  const uint32_t *Pinv;   // P^-1 mod 2^(32 S_P)
  const uint32_t *hR_P;   // h_P R mod P, h_P = L_P(g^(P-1) mod P^2)^-1 mod P
};

struct DKey {
  uint32_t n_bits;
  int has_priv;
  DMod n, n2;              // S_N = L, S_N2 = 2L limbs
  DExp e_n;                // n as an exponent (public encryption)
  const uint32_t *nR_n2;   // n R'' mod n^2
  const uint32_t *half;    // (n + 1) / 2 (L limbs) for the signed decode
  DPrime pr[2];            // [0]: P = p, Q = q; [1]: P = q, Q = p
  const uint32_t *Cq;      // (q^2)^-1 R' mod p^2
  const uint32_t *q2R_n2;  // q^2 R'' mod n^2
  const uint32_t *qinv_p;  // q^-1 mod p (canonical)
  const uint32_t *qR_n;    // q R_n mod n
  int ct;                  // private-key exponentiations read their window tables in full (secret digits)
};

// Histogram job as the kernels see it (host fills offsets).
struct DJob {
  const uint32_t *idx;
  const uint8_t *bins;
  uint32_t *hist;
  uint64_t n;          // samples in the node
  uint64_t ld;         // bins leading dimension
  uint32_t F, B;       // features, bins
  uint64_t fb_off;     // first (feature, bin) entry of this job in the flat lists
  uint64_t perm_off;   // first perm slot of this job (F * n slots)
  uint64_t blk_off;    // first sample block of this job (F * nblk blocks)
  uint32_t f_off;      // first (job, feature) entry
  uint32_t nblk;       // sample blocks per feature
  uint32_t *n_bad;     // optional: skipped (sample, feature) pairs, device counter
};

struct HistItem {      // one chunk of one (feature, bin): perm[start .. start+len)
  uint64_t start;
  uint32_t len;
  uint32_t pad;
};

// Flat device workspace of one histogram batch.
struct HistWs {
  DJob *jobs;
  uint32_t n_jobs;
  uint32_t *counts, *offs, *cursor, *fch, *fitem;  // [total_fb]
  uint32_t *border;                                // [total_fb]: per (job, feature), its bins by decreasing count
  uint32_t *ftot, *fbase;                          // [total_f]
  uint32_t *n_items;                               // device scalar
  uint32_t *next;                                  // device scalar: the product kernel's next wave unit
  HistItem *items;                                 // [items_cap]
  uint32_t *perm;                                  // [total_perm]
  uint32_t *partials;                              // [items_cap][2][S29], 29-bit limbs
  uint64_t total_fb, total_f, total_blocks, items_cap;
  uint64_t rows;                                   // resident ciphertext rows
  uint32_t chunk;                                  // most samples per item
  uint32_t split;                                  // groups per (item, slot): 1 or 2
  unsigned long long *mm_count;                    // optional debug counters [3], else null
};

constexpr int kWindowBits = 5;     // exponent window width (see mont.hpp)
constexpr int kSampleBlock = 4096;   // samples per bucketing block
constexpr int kBlockThreads = 256;   // 4 waves
constexpr int kHistGroup = 16;      // lanes per integer in the histogram kernels
constexpr int kHistWaves = 5;       // waves per SIMD asked of the histogram product kernel

// ---- launchers (he_kernels.hip) ------------------------------------------------
// KP = limbs per lane of a prime: 1 for 1024-bit keys, 2 for 2048-bit keys.
hipError_t launch_encode(const double *x, uint64_t count, uint32_t frac_bits, int64_t *m,
                         uint32_t *n_bad, hipStream_t s);
// Launch shape of a private-key exponentiation (k_pow): lanes per integer,
// grid, and dynamic LDS reserved only to cap the blocks per compute unit.
struct PowLaunch {
  int G;
  uint32_t grid;
  uint32_t dyn;
};
// A private-key exponentiation over `count` ciphertexts in up to two
// launches: the first main_count ciphertexts at `main`, whose resident waves
// then all take the same number of work units, and the rest (what would be
// a last, partly filled round) at `tail`, a narrower group per integer so
// that it spreads over more waves.  tail.G == 0: one launch of everything
// at `main` (main_count unused).  ctr: two device words for the launches'
// work counters (cleared by the launcher), or null for static units.
struct PowPlan {
  PowLaunch main;
  uint64_t main_count;
  PowLaunch tail;
  uint32_t *ctr;
};
// tq: [count][2][S_P] (r mod P, then t in place), cpq: [count][2][S_P2].
hipError_t launch_enc_crt(int KP, const DKey &k, const int64_t *m, uint64_t count, const uint32_t *r, uint64_t seed,
                          uint64_t roff, uint32_t *tq, uint32_t *cpq, uint32_t *ct, uint32_t *tab,
                          const PowPlan &p1, const PowPlan &p2, hipStream_t s);
// Public-key encryption: x holds count + (count & 1) rows of S_N2 limbs (r mod
// n^2, then x^n in place); p plans the exponentiation over (count + 1) / 2
// unit pairs (kind 1).
hipError_t launch_enc_pub(int KP, const DKey &k, const int64_t *m, uint64_t count, const uint32_t *r, uint64_t seed,
                          uint64_t roff, uint32_t *x, uint32_t *ct, uint32_t *tab, const PowPlan &p, hipStream_t s);
hipError_t launch_enc_obf(int KP, const DKey &k, const int64_t *m, uint64_t count, const uint32_t *rho,
                          uint32_t *ct, hipStream_t s);
uint32_t ct_div_batch(uint64_t count);
hipError_t launch_ct_div(int KP, const DKey &k, const uint32_t *num, const uint32_t *den, uint64_t count,
                         uint32_t batch, uint32_t *out, uint32_t *n_bad, hipStream_t s);
hipError_t launch_split(const int64_t *hist, const int64_t *minus, uint32_t nodes, uint32_t F, uint32_t B,
                        double scale, double lam, double gamma, double mcw, int64_t *derived, void *out_feat,
                        void *out_node, hipStream_t s);
hipError_t launch_ct_mul(int KP, const DKey &k, const uint32_t *a, const uint32_t *b, uint64_t count,
                         uint32_t *out, hipStream_t s);
hipError_t launch_pack(int KP, const DKey &k, const uint32_t *ct, uint64_t count, uint32_t slots,
                       uint32_t *packed, hipStream_t s);
hipError_t launch_unpack(const uint32_t *raw, uint64_t count, uint32_t slots, uint32_t L, int64_t *m,
                         uint32_t *n_overflow, hipStream_t s);
uint32_t pack_slots(int n_bits, uint64_t count);
hipError_t launch_mont_convert(int KP, const DKey &k, const uint32_t *in, uint64_t count,
                               uint32_t *out, bool to_mont, hipStream_t s);
// The pieces, for the autotuner: r mod P into tq; one private-key
// exponentiation of `kind` (4 mod P, 0 lift, 2 decryption; in/out strides
// and limbs per (ciphertext, prime) unit); c mod P^2 into xpq.
hipError_t launch_enc_r(int KP, const DKey &k, uint64_t count, const uint32_t *r, uint64_t seed, uint64_t roff,
                        uint32_t *tq, hipStream_t s);
hipError_t launch_pow_kind(int KP, const DKey &k, int kind, const uint32_t *in, uint32_t in_stride,
                           uint32_t in_limbs, uint32_t *out, uint32_t out_stride, uint64_t count, uint32_t *tab,
                           const PowPlan &p, hipStream_t s);
hipError_t launch_dec_pre(int KP, const DKey &k, const uint32_t *ct, uint64_t count, uint32_t *xpq, hipStream_t s);
// xpq: [count][2][S_P2] (c mod P^2, then c^(P-1) mod P^2 in place).
hipError_t launch_dec(int KP, const DKey &k, const uint32_t *ct, uint64_t count,
                      uint32_t *xpq, int64_t *m, uint32_t *raw, uint32_t *n_overflow,
                      uint32_t *tab, const PowPlan &p, hipStream_t s);
// Launch shape of the histogram product kernel: lanes per ciphertext (16,
// or 8 at 2048-bit keys), grid, and dynamic LDS reserved only to cap its
// blocks per compute unit.
struct HistLaunch {
  int G;
  uint32_t grid;
  uint32_t dyn;
};
bool hist_shape_valid(int KP, int G);
uint32_t hist_resident_blocks(int KP, int G, uint32_t dyn);
uint32_t hist_dyn_lds(int KP, int G, int waves);
hipError_t launch_hist(int KP, const DKey &k, const uint32_t *ctm, const DJob *host_jobs,
                       const HistWs &ws, const HistLaunch &l, hipStream_t s);
// Work items are equal parts (at most `chunk` samples) of one (feature, bin)'s
// sample run, laid out by decreasing bin count in each feature; with
// split 2 one wave takes one item (two groups per slot, halves combined),
// with split 1 one wave takes two items (one group per slot).
hipError_t launch_fill(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_probe_mul(uint64_t iters, uint32_t grid, uint32_t *sink, hipStream_t s);

// The private-key exponentiation k_pow over an S32-limb modulus (S_P or
// S_P2 32-bit limbs) at G lanes per integer: whether that shape is built,
// its resident blocks with `dyn` bytes of dynamic LDS, and the dynamic LDS
// that caps it at `waves` blocks per compute unit (0: no cap).
bool pow_shape_valid(int S32, int G);
uint32_t pow_resident_blocks(int S32, int G, uint32_t dyn);
uint32_t pow_dyn_lds(int S32, int G, int waves);
// Window-table scratch bytes per resident block of k_pow at G lanes: kinds 4
// (mod P), 0 (lift mod P^2), 2 (decryption mod P^2), 1 (public key, mod n^2).
uint64_t table_bytes_per_block(int KP, int kind, int G);
// Default lanes per integer for an exponentiation of `kind` over `count`
// unit pairs (ciphertexts for the private-key kinds).
int pick_group(int KP, int kind, uint64_t count);

}  // namespace he
