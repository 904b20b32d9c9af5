/*
 * he.h -- C ABI of the MI355X (gfx950) Paillier histogram library.
 *
 * The library implements the encrypted-gradient path of secure vertical
 * federated XGBoost (Xu et al., "Secure Federated XGBoost with CUDA-accelerated
 * Homomorphic Encryption via NVIDIA FLARE", Sec. III-B and Sec. III-C):
 *   1. the active party encrypts every per-sample gradient g and Hessian h
 *      as one Paillier plaintext (Sec. III-C: 2M encryptions for M samples);
 *   2. a passive party multiplies ciphertexts mod n^2 into per-(feature, bin)
 *      encrypted histograms (Sec. III-B; encrypted addition, Sec. III-C);
 *   3. the active party decrypts the returned histograms (Sec. III-B).
 * Paillier is the textbook scheme with g = n + 1:
 *   E(m; r) = (1 + m n) r^n mod n^2,   D(c) = L(c^lambda mod n^2) mu mod n,
 * computed here with Montgomery arithmetic on 32-bit limbs and, where the key
 * holds p and q, with the Chinese remainder theorem.  Results are bit-identical
 * to the textbook definitions.
 *
 * Conventions shared by every call:
 *  - Big integers are little-endian arrays of uint32_t limbs.  A key of
 *    n_bits bits has L = n_bits / 32 limbs for n and 2L limbs for n^2, so one
 *    ciphertext occupies 2L limbs (256 B at 1024 bits, 512 B at 2048 bits).
 *  - Ciphertexts crossing the ABI are canonical residues in [0, n^2) unless a
 *    parameter says HE_FORM_MONT: the Montgomery form x * R' mod n^2 of the
 *    histogram kernels, a canonical residue in the same 2L-limb layout, with
 *    R' = 2^(29 s) for their s limbs of 29 bits (s = 144 at 2048 bits, 80 at
 *    1024 bits).
 *  - Pointers documented as "device" are HIP device pointers owned by the
 *    caller; the library never frees or retains them after the call returns.
 *    Pointers documented as "host" are read or written before return.
 *  - Calls that take a hipStream_t enqueue work on that stream and return
 *    without waiting; argument checks are synchronous.  Work on one stream is
 *    ordered; calls on different streams may run concurrently (each stream
 *    gets its own library workspace).
 *  - Return value: 0 on success, a negative HE_ERR_* code otherwise; no C++
 *    exception crosses this boundary.  he_last_error() gives a message for the
 *    calling thread's last failure.
 *  - Only 1024- and 2048-bit keys are supported.
 */
#ifndef HE_MI355X_H
#define HE_MI355X_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HE_OK           0
#define HE_ERR_ARG     -1   /* null pointer, bad size or bad layout */
#define HE_ERR_KEY     -2   /* key material invalid (p, q not usable) */
#define HE_ERR_NOPRIV  -3   /* operation needs p and q but the key is public */
#define HE_ERR_RANGE   -4   /* value outside the representable range */
#define HE_ERR_OOM     -5   /* device workspace allocation failed */
#define HE_ERR_DEVICE  -6   /* a HIP runtime call failed */

#define HE_FORM_CANONICAL 0
#define HE_FORM_MONT      1

typedef struct he_key he_key;  /* opaque; immutable after creation */

/* Key generation (Paillier key setup; the paper fixes no key size, 1024 and
 * 2048 bits are supported).  Primes p, q of n_bits/2 bits each are the first
 * candidates of a SplitMix64 word stream keyed by `seed` (p from counter 0,
 * q from counter 2^48; n_bits/64 words per candidate, little-endian, top two
 * bits and bit 0 forced to 1) that pass trial division by the odd primes
 * below 2000 and 40 Miller-Rabin rounds with the first 40 prime bases; q must
 * differ from p and gcd(pq, (p-1)(q-1)) must be 1.  Deterministic in `seed`.
 * The key's device constants are uploaded to the current HIP device.
 * Returns HE_ERR_ARG for an unsupported n_bits or a null `out`. */
int he_keygen(uint32_t n_bits, uint64_t seed, he_key **out);

/* Builds a key from host limb arrays.  p and q hold n_bits/64 limbs each
 * (little-endian).  With q == NULL, p is taken as n (n_bits/32 limbs) and
 * the key is public-only: he_decrypt then fails with HE_ERR_NOPRIV and
 * he_encrypt uses the public-key path.  Checks: p, q odd, distinct, > 1,
 * gcd(pq, (p-1)(q-1)) = 1, and n = pq has exactly n_bits bits (HE_ERR_KEY). */
int he_key_import(uint32_t n_bits, const uint32_t *p, const uint32_t *q, he_key **out);

/* Copies n (n_bits/32 limbs) and, if non-NULL and the key is private, p and
 * q (n_bits/64 limbs each) into host buffers.  HE_ERR_NOPRIV if p or q is
 * requested from a public key. */
int he_key_export(const he_key *key, uint32_t *n, uint32_t *p, uint32_t *q);

/* Side-channel hardening of the private-key exponentiations (the CRT
 * encryption's r^(q mod (p-1)) mod p and x^p mod p^2, and decryption's
 * c^(p-1) mod p^2, whose exponents are secret; Sec. III-B: only the active
 * party holds p and q).  Off (the default), each exponentiation follows the
 * key's sliding-window schedule: the same sequence of operations for every
 * ciphertext and call, a function of p and q (not of the data), and each
 * window reads the one table entry it names.  With on != 0 they use fixed
 * 5-bit windows, one multiplication per window whatever its digit, and
 * every window reads all 32 table entries and keeps the one its digit names
 * by a mask, so neither the operations nor the device addresses touched
 * depend on the exponent (about 1.6x the default's encryption time on the
 * 2048-bit pass).  Results are identical bit for bit.  Applies to calls enqueued after it returns; must not run
 * concurrently with other calls on the same key.  HE_ERR_ARG for a null key. */
int he_key_set_constant_time(he_key *key, int on);

/* Number of bits of n, and whether the key holds p and q (1) or not (0). */
uint32_t he_key_bits(const he_key *key);
int he_key_has_private(const he_key *key);

/* Frees the key and its device constants.  The caller must make sure no
 * queued work still uses the key (synchronise its streams first). */
void he_key_free(he_key *key);

/* Fixed-point encoding of g or h (Sec. III-C encrypts each g and h as one
 * number but fixes no encoding): m[i] = rint(x[i] * 2^frac_bits),
 * ties to even, as int64.  x and m are device arrays of `count` elements.
 * Values whose scaled magnitude reaches 2^63 (or NaN) are stored as INT64_MIN
 * and counted into *n_bad (device, optional, atomically incremented). */
int he_encode(const double *x, uint64_t count, uint32_t frac_bits, int64_t *m,
              uint32_t *n_bad, hipStream_t stream);

/* Encryption (Sec. III-B: the active party encrypts every g and h;
 * Sec. III-C: one Paillier encryption per number):
 *   ct[i] = (1 + (m[i] mod n) n) * r_i^n mod n^2, canonical, 2L limbs.
 * m: device int64[count] (signed; taken mod n).
 * r: device uint32[count][L] explicit randomness (any value with
 *    gcd(r, n) = 1; only r mod n matters), or NULL for the seeded stream
 *    r_i = X_i mod n, X_i = sum_j w(r_seed, (r_offset + i) W + j) 2^(64 j),
 *    W = n_bits/64 + 1, w(s, k) the k-th SplitMix64 output from state s.
 * ct: device uint32[count][2L].
 * A private key uses the CRT path: r^n mod p^2 = (r^(q mod (p-1)) mod p)^p
 * mod p^2 (and likewise for q), then CRT to mod n^2; a public key
 * exponentiates mod n^2.  Both give bit-identical ciphertexts.
 * An r that is 0 mod p or mod q (for the seeded stream the chance is below
 * 2^-500) yields a ciphertext that is not a unit; this is not checked. */
int he_encrypt(const he_key *key, const int64_t *m, uint64_t count,
               const uint32_t *r, uint64_t r_seed, uint64_t r_offset,
               uint32_t *ct, hipStream_t stream);

/* Same as he_encrypt but forces the public-key path (r^n mod n^2 by one
 * exponentiation mod n^2) even for a private key. */
int he_encrypt_public(const he_key *key, const int64_t *m, uint64_t count,
                      const uint32_t *r, uint64_t r_seed, uint64_t r_offset,
                      uint32_t *ct, hipStream_t stream);

/* Obfuscators for encryption ahead of time: rho[i] = r_i^n mod n^2, i.e. the
 * encryption of 0 with the same r as he_encrypt (explicit r, or the seeded
 * stream with r_seed / r_offset).  rho: device uint32[count][2L], canonical.
 * This is the exponentiation part of encryption, which does not depend on
 * the plaintext, so the encrypting party can run it before the gradients
 * exist. */
int he_obfuscators(const he_key *key, uint64_t count, const uint32_t *r, uint64_t r_seed,
                   uint64_t r_offset, uint32_t *rho, hipStream_t stream);

/* Encryption with precomputed obfuscators: ct[i] = (1 + (m[i] mod n) n)
 * rho[i] mod n^2 -- the same ciphertext as he_encrypt with the r that
 * produced rho[i], for three Montgomery products per value.  Each obfuscator
 * must be used for one plaintext only.  m: device int64[count]; rho, ct:
 * device uint32[count][2L] (ct may alias rho). */
int he_encrypt_obfuscated(const he_key *key, const int64_t *m, uint64_t count, const uint32_t *rho,
                          uint32_t *ct, hipStream_t stream);

/* Montgomery conversion of ciphertexts: out = in * R' mod n^2 (to_mont) or
 * in * R'^-1 mod n^2 (from_mont), R' as for HE_FORM_MONT above (the radix-2^29
 * Montgomery factor of the histogram kernels).  Device uint32[count][2L]; in-place
 * (in == out) is allowed.  Keeps gradients resident in the form the
 * histogram kernels consume, so the conversion is paid once per round. */
int he_to_mont(const he_key *key, const uint32_t *in, uint64_t count, uint32_t *out,
               hipStream_t stream);
int he_from_mont(const he_key *key, const uint32_t *in, uint64_t count, uint32_t *out,
                 hipStream_t stream);

/* One tree-node histogram job (Sec. III-B: each passive party sums the
 * encrypted gradients into the bins of its own features).
 *  sample_idx: device uint32[n_samples], rows of `ct` in this node (any order;
 *              a row listed twice is multiplied in twice);
 *  bins:       device uint8[n_features][bins_ld]; bins[f][row] is the bin of
 *              sample `row` for feature f (bins_ld >= rows);
 *  n_bins:     1..256;
 *  hist:       device uint32[n_features][n_bins][2][2L] output, canonical;
 *              slot 0 accumulates g, slot 1 accumulates h;
 *  n_bad:      device uint32, optional (NULL): receives (atomically, not
 *              cleared) the number of skipped (sample, feature) pairs.
 * Device data is checked, not trusted: a sample whose row is not below the
 * call's `rows` is skipped for every feature, and a sample whose bin for a
 * feature is not below n_bins is skipped for that feature; skipped pairs
 * join no bin and are only counted.  (Reading a device value out of range
 * never indexes memory.)  The call cannot detect ciphertexts made under a
 * different key of the same size: they are multiplied like any others. */
typedef struct he_hist_job {
  const uint32_t *sample_idx;
  uint64_t n_samples;
  const uint8_t *bins;
  uint64_t bins_ld;
  uint32_t n_features;
  uint32_t n_bins;
  uint32_t *hist;
  uint32_t *n_bad;
} he_hist_job;

/* Encrypted histogram aggregation for n_jobs nodes in one batch:
 *   hist[f][b][t] = prod over i in sample_idx with bins[f][i] = b of
 *                   ct[i][t] mod n^2,   empty bins hold 1.
 * ct: device uint32[rows][2][2L] (g and h ciphertext of each row), in the
 *     form given by ct_form (HE_FORM_MONT avoids a conversion per call).
 * jobs: host array of n_jobs descriptors.  All jobs' (feature, bin, chunk)
 * work items run in one persistent launch; the result is independent of
 * batching, chunking and order (exact modular products).  Work shape: the
 * one he_hist_autotune found for the batch's shape class, else, at 2048-bit
 * keys for batches of at least 16384 items (estimated at 128 samples per
 * item), 8 lanes per ciphertext and items of up to 128 samples, and 16
 * lanes with items of up to 64 samples otherwise. */
int he_hist_aggregate(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                      const he_hist_job *jobs, uint32_t n_jobs, hipStream_t stream);

/* he_hist_aggregate with an explicit work-item length: at most `chunk`
 * samples of one (feature, bin) per item, each bin's samples split into
 * equal parts (0 picks the library default).  The result does not depend
 * on `chunk`; only the load balance does. */
int he_hist_aggregate_ex(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                         const he_hist_job *jobs, uint32_t n_jobs, uint32_t chunk,
                         hipStream_t stream);

/* Autotuner for the batched aggregation: times he_hist_aggregate on these
 * jobs (synchronising `stream`), first for work-item lengths of 16..512
 * samples (32..256 at 8 lanes) and one or two groups per (item, slot) at
 * each of the product kernel's lanes per ciphertext (16, and 8 at 2048-bit
 * keys), then, at the best items of each, for waves per SIMD (4, 3 or 2 by
 * reserving LDS, where that is below the kernel's own occupancy), and
 * remembers the fastest choice for the shape class (key
 * size, total contributions and job count rounded to powers of two, largest
 * bin count).  Later he_hist_aggregate calls and plans with chunk 0 in the
 * same class use it.  The histograms are written (correctly) several times.
 * Outputs are host pointers, each optional; waves 0 = own occupancy. */
int he_hist_autotune(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                     const he_hist_job *jobs, uint32_t n_jobs, uint32_t *chunk, uint32_t *split,
                     uint32_t *lanes, uint32_t *waves, float *ms, hipStream_t stream);

/* Autotuner for the private-key exponentiations: the CRT encryption's
 * exponentiation mod p and p-th-power lift mod p^2 (Sec. III-C: 2M
 * encryptions for M samples) and decryption's exponentiation mod p^2.  Times
 * every built launch shape of each -- lanes per integer (2, 4, 8 or 16) and
 * waves per SIMD (the kernel's own occupancy, or 3 or 2 by reserving LDS) --
 * and then, at the best of those, the same work in two launches: the
 * ciphertexts that fill whole rounds of the resident waves at that shape,
 * and the remainder (less than one round) at a wider group per integer, so
 * that the last partial round spreads over more waves.  Trials run on
 * enc_count encryptions and dec_count decryptions of trial operands (the
 * sliding-window schedule is fixed per key, so the running time does not
 * depend on the data), and the fastest per kind is remembered for the
 * count's size class (bit length) on this device and key size; later
 * he_encrypt, he_obfuscators and he_decrypt calls of that class use it.
 * Results never depend on the shape.  Without a tuned (or pinned) shape a
 * kind runs at the narrowest built width that gives every SIMD two waves,
 * at the kernel's own occupancy, or at two waves per SIMD where those take
 * as many rounds of units (units / resident waves, rounded up).  Allocates
 * trial buffers and synchronises `stream`.
 * choice: optional host uint32[9]: per kind (the mod-p exponentiation, the
 *         lift, decryption) lanes, waves (0 = own occupancy) and lanes of
 *         the remainder's launch (0 = one launch).
 * ms: optional host float[3]: their launch times.
 * HE_ERR_NOPRIV for a public key, HE_ERR_ARG for a zero count. */
int he_crt_autotune(const he_key *key, uint64_t enc_count, uint64_t dec_count, uint32_t *choice, float *ms,
                    hipStream_t stream);

/* Sets the launch shape he_crt_autotune would remember, without timing (a
 * shape measured once, pinned in a deployment): for kind 0 (the mod-p
 * exponentiation of encryption), 1 (the lift), 2 (decryption) or 3 (the
 * exponentiation by n mod n^2 of public-key encryption, also the path of a
 * key holding n only) at this key's size, on the current device, for counts
 * of count's size class (bit length; for kind 3 of (count + 1) / 2): lanes
 * per integer (2, 4, 8 or 16 where built for the kind; 8 or 16 for kind 3 at
 * 2048-bit keys),
 * waves per SIMD (0 = own occupancy, 2 or 3) and lanes of the last partial
 * round's launch (0 = one launch, else a built width above lanes).  Results
 * never depend on the shape.  HE_ERR_ARG for anything else. */
int he_crt_set_shape(const he_key *key, uint32_t kind, uint64_t count, uint32_t lanes, uint32_t waves,
                     uint32_t tail_lanes);

/* Work-count check of the aggregation: he_hist_aggregate_ex at an explicit
 * work shape -- work-item length (chunk, 0 = default), groups per item
 * (split, 1 or 2), lanes per ciphertext of the product kernel (lanes, 0 =
 * 16; 8 only at 2048-bit keys, else HE_ERR_ARG) and its waves per SIMD
 * (waves, 0 = own occupancy, at most 8) -- that also adds, into the device
 * counters mm_count[3] (not cleared):
 *   [0] the Montgomery products that join two partial products of real
 *       samples -- for every (job, feature, slot) the node's sample count
 *       minus its number of non-empty bins, the algorithm's count;
 *   [1] the products the kernels executed, padding of uneven work items and
 *       the conversions out of Montgomery form included;
 *   [2] the conversions out of Montgomery form (one per histogram entry).
 * The conversion of canonical input rows into Montgomery form is not counted. */
int he_hist_aggregate_counted(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                              const he_hist_job *jobs, uint32_t n_jobs, uint32_t chunk, uint32_t split,
                              uint32_t lanes, uint32_t waves, uint64_t *mm_count, hipStream_t stream);

/* A batched aggregation captured once into a HIP graph (all of its kernels,
 * with a workspace the plan owns), to be replayed with one launch, e.g. once
 * per tree level per boosting round.  Each replay reads the buffers that the
 * job descriptors and `ct` point to at replay time, so the caller refreshes
 * their contents in place; the sizes are fixed at creation.  chunk/split 0
 * take the autotuned or default values.  Replays of one plan must not
 * overlap (one plan per concurrent stream). */
typedef struct he_hist_plan he_hist_plan;
int he_hist_plan_create(const he_key *key, const uint32_t *ct, uint64_t rows, int ct_form,
                        const he_hist_job *jobs, uint32_t n_jobs, uint32_t chunk, uint32_t split,
                        he_hist_plan **out);
int he_hist_plan_launch(he_hist_plan *plan, hipStream_t stream);
void he_hist_plan_free(he_hist_plan *plan);

/* Encrypted addition of two ciphertext arrays (Sec. III-C: addition of
 * plaintexts is the product of ciphertexts mod n^2): out[i] = a[i] b[i] mod
 * n^2.  Uses: re-randomising returned histograms (multiply by obfuscators
 * from he_obfuscators, i.e. encryptions of 0 under fresh r, which needs only
 * the public key), and combining partial histograms of sample shards.
 * a, b, out: device uint32[count][2L] canonical; out may alias a or b. */
int he_ct_mul(const he_key *key, const uint32_t *a, const uint32_t *b, uint64_t count, uint32_t *out,
              hipStream_t stream);

/* Encrypted histogram subtraction (the sibling trick of tree building: the
 * samples of a node split into its two children, so the larger child's
 * histogram is the parent's "minus" the smaller child's).  By the additive
 * homomorphism (Sec. III-C), out[i] = parent[i] child[i]^-1 mod n^2 is an
 * encryption of m_parent - m_child; when the child's samples are a subset of
 * the parent's, it equals bit for bit the product over the remaining samples.
 * Needs only the public key.  Inverses come from Kaliski's binary
 * almost-inverse with Montgomery's batch trick (one inversion per `batch`
 * consecutive elements, 0 = chosen from the count and the device).
 * parent, child, out: device uint32[count][2L] canonical, any layout of
 * histograms flattened to ciphertexts (e.g. [F][B][2]); out must not
 * overlap parent or child (it holds intermediate products).  Elements whose
 * child is not a unit mod n^2 (never the case for ciphertexts) get 0 and are
 * counted into *n_bad (device uint32, optional, not cleared). */
int he_hist_subtract(const he_key *key, const uint32_t *parent, const uint32_t *child, uint64_t count,
                     uint32_t batch, uint32_t *out, uint32_t *n_bad, hipStream_t stream);

/* Split finding, the active party's step after decryption (Sec. III-B: the
 * decrypted histograms go to tree building).  The criterion is XGBoost's
 * split gain (Chen & Guestrin 2016): splitting a feature's bins after bin b
 * sends bins 0..b left, and
 *   gain = 1/2 [G_L^2/(H_L+lambda) + G_R^2/(H_R+lambda) - G^2/(H+lambda)] - gamma,
 * admissible when H_L, H_R >= min_child_weight and H_L+lambda, H_R+lambda > 0.
 * Sums are exact int64 (prefix sums), converted to double and scaled by
 * 2^-frac_bits; the gain is evaluated in IEEE double exactly as written (no
 * fused multiply-add).  Ties: the lowest bin, then the lowest feature; no
 * admissible split gives gain -inf, feature and bin -1.
 * hist: device int64 [nodes][F][B][2] (G, H sums, e.g. he_decrypt's output).
 * minus: optional, same shape: the node's histogram is hist - minus (a
 *   larger sibling from its parent and the smaller child, in plaintext).
 * derived: optional, same shape, receives the histogram used (may alias hist).
 * out_feature: optional device he_split [nodes][F]; out_node: device he_split [nodes].
 * B must be in [1, 256]. */
typedef struct he_split {
  double gain;
  int32_t feature; /* -1: no admissible split */
  int32_t bin;     /* left = bins 0..bin */
  int64_t g_left;  /* fixed-point sums of the left side */
  int64_t h_left;
} he_split;
int he_split_find(const int64_t *hist, const int64_t *minus, uint32_t nodes, uint32_t n_features, uint32_t n_bins,
                  uint32_t frac_bits, double lambda, double gamma, double min_child_weight, int64_t *derived,
                  he_split *out_feature, he_split *out_node, hipStream_t stream);

/* Decryption (Sec. III-B: the active party decrypts the returned
 * histograms), by the CRT: m_p = L_p(c^(p-1) mod p^2) h_p mod p with
 * h_p = (-q mod p)^-1 mod p, likewise m_q, then m = m_q + q ((m_p - m_q)
 * q^-1 mod p), which equals L(c^lambda mod n^2) mu mod n.
 * ct: device uint32[count][2L] canonical.
 * m: device int64[count] signed decode (m >= (n+1)/2 means m - n); values
 *    outside [-2^63, 2^63) are saturated and counted into *n_overflow
 *    (device uint32, optional).
 * raw: device uint32[count][L] plaintext in [0, n), optional (NULL).
 * HE_ERR_NOPRIV for a public key. */
int he_decrypt(const he_key *key, const uint32_t *ct, uint64_t count, int64_t *m,
               uint32_t *raw, uint32_t *n_overflow, hipStream_t stream);

/* Decryption that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, results and errors as he_decrypt,
 * bit for bit; the kernels are he_decrypt's.  Its working memory is one
 * 64 MiB array in the library's device image, one copy per device, held
 * until the process ends: count must not exceed 2^22 / L ciphertexts
 * (65,536 at 2048-bit keys, 131,072 at 1024-bit), else HE_ERR_ARG before
 * any device work; the exponentiation launch is cut to the blocks whose
 * window tables fit beside the count's residues mod p^2 and q^2, so large
 * calls run on part of the device.  Nothing in the array needs to start at zero.  Every
 * call on a device shares that device's array: calls that overlap on one
 * device (other streams, other threads) race and must be serialised by the
 * caller. */
int he_decrypt_noalloc(const he_key *key, const uint32_t *ct, uint64_t count, int64_t *m,
                       uint32_t *raw, uint32_t *n_overflow, hipStream_t stream);

/* Ciphertext packing for cheaper decryption.  The holder of encrypted
 * histograms (public key only) folds `slots` consecutive ciphertexts into
 * one: packed = prod_j c_j^(2^(64 j)) (1 + K n) mod n^2 with
 * K = sum_j 2^(64 j + 63), an encryption of sum_j 2^(64 j) (m_j + 2^63)
 * (additive homomorphism, Sec. III-C; multiplying by 1 + K n adds K).  The
 * key holder decrypts count / slots ciphertexts instead of count; each slot
 * value must lie in [-2^63, 2^63).  Costs 64 squarings mod n^2 per slot.
 * slots in [1, (n_bits - 1) / 64] (31 for 2048-bit keys, 15 for 1024-bit);
 * he_pack_slots gives the count the library would pick for `count`
 * ciphertexts on this device (enough packed ciphertexts to occupy it).
 * ct: device uint32[count][2L] canonical; packed: device
 * uint32[ceil(count / slots)][2L] (the last may hold fewer slots). */
uint32_t he_pack_slots(const he_key *key, uint64_t count);
int he_pack(const he_key *key, const uint32_t *ct, uint64_t count, uint32_t slots, uint32_t *packed,
            hipStream_t stream);
/* Decrypts he_pack's output: m: device int64[count] (the original order).
 * Plaintexts with bits above their last slot (which a slot value outside the
 * signed 64-bit range at the top slot, or a negative total, produces) are
 * counted into *n_overflow (device uint32, optional, not cleared).
 * HE_ERR_NOPRIV for a public key. */
int he_decrypt_packed(const he_key *key, const uint32_t *packed, uint64_t count, uint32_t slots, int64_t *m,
                      uint32_t *n_overflow, hipStream_t stream);

/* Measurement probe for the roofline denominator: launches `blocks` blocks
 * of 256 threads that each run `iters` iterations of 8 independent 32x32->64
 * integer multiply-adds; *products receives the number of products issued
 * (host).  Time it with events on `stream`. */
int he_probe_int_mul(uint64_t iters, uint32_t blocks, uint64_t *products, hipStream_t stream);

/* Message describing the calling thread's last non-zero return. */
const char *he_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HE_MI355X_H */
