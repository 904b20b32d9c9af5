// Size of the radix-2^29 Montgomery representation used by the modular
// exponentiation loops (shared by the host key set-up and the kernels).
//
// A modulus N below 2^(32 S) is written in S29 limbs of 29 bits with
// R = 2^(29 S29).  S29 is the fewest limbs with R > 4N, so that Montgomery
// products of operands below 2N stay below 2N without a final subtraction,
// rounded up so that every lane of a G-lane group holds the same number of
// limbs.  Three roundings cover the group widths: variant 0 (multiple of 4:
// groups of 2 or 4 lanes), 1 (multiple of 8: 8 lanes), 2 (multiple of 16:
// 16 lanes); the key stores constants for each.
#pragma once

namespace he29 {

constexpr int kBits = 29;
constexpr int kVariants = 3;

constexpr int variant(int G) { return G <= 4 ? 0 : (G == 8 ? 1 : 2); }
constexpr int multiple(int v) { return v == 0 ? 4 : (v == 1 ? 8 : 16); }
constexpr int limbs(int S, int v) {
  const int m = (32 * S + 2 + kBits - 1) / kBits;
  const int u = multiple(v);
  return (m + u - 1) / u * u;
}
constexpr int limbs_for_group(int S, int G) { return limbs(S, variant(G)); }

}  // namespace he29
