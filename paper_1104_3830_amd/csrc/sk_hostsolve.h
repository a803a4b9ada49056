// Host exact solvers of the reduced instance (no device code), shared by the
// scaling paths and the C entry points.
#pragma once
#include <cstdint>

#include "../../include/sk.h"

namespace sk {

// sk_solve_reduced with a column per row to try first in the greedy start
// of the matching (nullptr: none).
sk_status solve_reduced_seeded(const sk_csr *csr, const int32_t *hint, int32_t *perm,
                               int64_t *weight);

// Maximum-weight perfect matching of the CSR (rp, col, w) with float weights
// by shortest augmenting paths; hint as above. SK_EINVAL for a malformed
// CSR or a non-finite weight, SK_EINFEASIBLE when no perfect matching exists.
sk_status solve_real_impl(int n, const int64_t *rp, const int32_t *col, const float *w,
                          const int32_t *hint, int32_t *perm, double *weight);

}  // namespace sk
