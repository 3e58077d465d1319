// Instances of the persistent CG solve for stencil half-width n = 2.
#include "solve_impl.h"

namespace exx {

hipError_t solve_dispatch_n2(const SolveKArgs& a, bool mixed, int max_cols, int threads, int depth, int groups,
                             size_t lds, hipStream_t s, int* occ) {
  return solve_ns_dispatch<2>(a, mixed, max_cols, threads, depth, groups, lds, s, occ);
}

}  // namespace exx
