// Index logic of the histogram bucketing kernels (counting sort of a node's
// samples by bin, per feature), shared by the gfx950 kernels and the CPU
// harness that checks it under AddressSanitizer.
//
// A node lists row indices of the resident ciphertext array; bins[f][row] is
// the bin of that row for feature f.  Both come from device memory the caller
// fills, so a row at or past the number of resident rows, or a bin at or past
// the job's bin count, must not index anything: such a sample is skipped by
// every kernel (the count, the scatter and therefore the products) and
// counted as bad.  The count and the scatter take the same decision for a
// sample, so every per-bin run of the permutation holds exactly the samples
// counted for it.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define HE_HD __host__ __device__
#else
#define HE_HD
#endif

namespace he {

// Row and bin of sample s of a node for one feature; false when the sample
// is skipped (row >= rows or bin >= n_bins).  `bins_f` is the feature's row
// of the bin table (at least `rows` entries); it is read only for a row
// below `rows`.
HE_HD inline bool bucket_sample(const uint32_t *idx, const uint8_t *bins_f, uint64_t rows, uint32_t n_bins,
                                uint64_t s, uint32_t &row, uint32_t &bin) {
  row = idx[s];
  if ((uint64_t)row >= rows) return false;
  bin = bins_f[row];
  return bin < n_bins;
}

// Feature and sample range [s0, s1) of bucketing block `local` of a job with
// n samples and nblk blocks of `block` samples per feature.
HE_HD inline void bucket_block(uint64_t local, uint32_t nblk, uint64_t n, uint32_t block, uint32_t &f,
                               uint64_t &s0, uint64_t &s1) {
  f = (uint32_t)(local / nblk);
  s0 = (local % nblk) * block;
  s1 = s0 + block < n ? s0 + block : n;
}

// Slot of a sample in the feature's permutation row: the start of its bin's
// run reserved by its block (`block_base`, taken from the bin's cursor, which
// starts at the bin's offset) plus its rank among the block's samples of
// that bin.  Below offset + count of the bin when the count and the scatter
// skip the same samples.
HE_HD inline uint64_t bucket_slot(uint32_t block_base, uint32_t rank) { return (uint64_t)block_base + rank; }

}  // namespace he
