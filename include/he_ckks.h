/* CKKS for the secure horizontal path (Sec. III-A, III-C: each client
 * encrypts its local G/H histogram vectors, the federated server adds the
 * ciphertexts, the clients decrypt the global histograms; CKKS because one
 * ciphertext carries a whole histogram vector).  Public-key encryption,
 * addition and decryption only.
 *
 * Ring Z_Q[X]/(X^N + 1), N = 2^log_n (log_n in [12, 14]), Q = q0 q1 q2 with
 * the three largest primes below 2^30 that are 1 mod 2N, kept in RNS form.
 * Q is about 2^90, inside the 128-bit classical security bounds of the
 * homomorphic encryption standard for a ternary secret at these N (log Q up
 * to 109, 218, 438 for N = 2^12, 2^13, 2^14); smaller N would not be, and
 * he_ckks_create refuses them (HE_ERR_ARG).
 * Encoding of n <= N/2 reals z: the integer polynomial m with
 * m(zeta^(5^k)) ~ 2^scale_bits z_k (zeta = e^(i pi / N)); |2^scale_bits z| summed
 * over the ciphertexts that are added must stay below Q/2 (about 2^89).
 * Keys (ternary secret s, uniform a, centered-binomial error e, b = -a s + e)
 * come from a seed and stay on the device; encryption randomness (ternary u,
 * centered-binomial e0, e1) comes from (seed, offset + index) counters of the
 * SplitMix64 stream, so results are reproducible.
 *
 * Layouts: a plaintext polynomial is uint32 [L = 3][N] residues; a
 * ciphertext is uint32 [2][3][N] (c0, c1), coefficient domain.  All data
 * pointers are device pointers owned by the caller; calls enqueue on the
 * given stream.  Errors are negative HE_ERR_* codes (he.h) with a message
 * from he_ckks_last_error(). */
#ifndef HE_CKKS_H
#define HE_CKKS_H
#include <hip/hip_runtime.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct he_ckks he_ckks;

/* Context with keys from `seed` (synchronous; allocates device memory). */
int he_ckks_create(uint32_t log_n, uint32_t scale_bits, uint64_t seed, he_ckks **out);
void he_ckks_free(he_ckks *ctx);
/* N, the three primes (host array of 3, optional), scale bits. */
int he_ckks_params(const he_ckks *ctx, uint32_t *n, uint32_t *primes, uint32_t *scale_bits);

/* z: device double [count][n_values] -> pt: [count][3][N]. */
int he_ckks_encode(const he_ckks *ctx, const double *z, uint64_t count, uint32_t n_values, uint32_t *pt,
                   hipStream_t stream);
/* Encrypts count plaintexts; ciphertext t uses the randomness of index
 * offset + t under `seed`.  ct: [count][2][3][N].  Not reentrant per context
 * (a context-owned scratch buffer holds the randomness). */
int he_ckks_encrypt(he_ckks *ctx, const uint32_t *pt, uint64_t count, uint64_t seed, uint64_t offset, uint32_t *ct,
                    hipStream_t stream);
/* out = x + y for count ciphertexts (out may alias x or y). */
int he_ckks_add(const he_ckks *ctx, const uint32_t *x, const uint32_t *y, uint64_t count, uint32_t *out,
                hipStream_t stream);
/* pt = c0 + c1 s for count ciphertexts: [count][3][N]. */
int he_ckks_decrypt(const he_ckks *ctx, const uint32_t *ct, uint64_t count, uint32_t *pt, hipStream_t stream);
/* Centered plaintext coefficients (by the CRT) -> z: double [count][n_values]. */
int he_ckks_decode(const he_ckks *ctx, const uint32_t *pt, uint64_t count, uint32_t n_values, double *z,
                   hipStream_t stream);
const char *he_ckks_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HE_CKKS_H */
