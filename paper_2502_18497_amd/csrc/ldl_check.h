// Launchers of the device-side invariant recount (definitions in kernels_check.hip).
#pragma once

#include "ldl_kernels.h"

namespace ldl {

// Sums of one check pass (see kernels_check.hip), cleared by launch_inv_clear.  Row words:
// entries, weight sum, fingerprints of the keys (h1, h2), of the transposed keys (h1, h2), of the
// parent-mapped keys (h1, h2), intra-community weight.  Node words: sum h1(parent) over alive
// nodes, sum rsize h1(node), sum kout h1(label), sum kin h2(label), sum Kout(c) h1(c),
// sum Kin(c) h2(c), sum Kout, sum Kin; then sum Kout Kin as (lo, hi).
constexpr int kInvRowWords = 9;
constexpr int kInvNodeWords = 8;
constexpr uint32_t kInvDegrees = 1u, kInvTranspose = 2u, kInvAggregate = 4u, kInvLabels = 8u, kInvRoots = 16u,
                   kInvTotals = 32u, kInvRange = 64u;
struct InvScratch {
  u64a out[kInvRowWords];
  u64a in[kInvRowWords];
  u64a node[kInvNodeWords + 1];   // the last word is the low word of sum Kout Kin
  u64a skk_hi;
  uint32_t flags;
  uint32_t pad;
};
void launch_inv_clear(InvScratch* sc, hipStream_t s);
// row pass over one orientation (transposed = the CSR holds in-rows); par / lab optional
void launch_inv_rows(CsrRef c, uint32_t n, const uint8_t* alive, const int64_t* deg, const uint32_t* par,
                     const uint32_t* lab, int transposed, InvScratch* sc, hipStream_t s);
// node pass over level r (up_* null at the top level; Kout / Kin only at level 0)
void launch_inv_nodes(uint32_t n, const uint8_t* alive, const uint32_t* lab, const uint32_t* par,
                      const uint32_t* rsize, const int64_t* kout, const int64_t* kin, const uint8_t* up_alive,
                      const uint32_t* up_lab, const int64_t* Kout, const int64_t* Kin, InvScratch* sc, hipStream_t s);

}  // namespace ldl
