// Choice of the variables fixed before the degree of the elements is raised
// (Sec. 6.1).
#pragma once

#include "../../include/mgcg.h"
#include "common.h"

namespace mgcg {

void fix_variables(const mgcg_fix_desc& d, const double* rho, const double* grad,
                   unsigned char* kind_out, unsigned char* design_out, unsigned char* mask,
                   mgcg_fix_counts* counts, int mem);
// The same on device arrays, with the scratch in a static per-GPU array
// (allocates nothing); counts_dev: int64[4] on the device; stream-ordered.
void fix_variables_noalloc(const mgcg_fix_desc& d, const double* rho, const double* grad,
                           unsigned char* kind_out, unsigned char* design_out, unsigned char* mask,
                           int64_t* counts_dev, hipStream_t st);

}  // namespace mgcg
