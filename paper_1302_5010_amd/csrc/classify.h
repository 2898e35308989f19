// Launcher of the class-residual classification kernel (classify.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmpl {

struct ClassifyArgs {
    const float* At; int64_t lda; int n; int m;   // padded float32 atoms
    const float* B; int64_t ldb; int p;           // signals, one per row
    const int32_t* x_idx; const float* x_val; const int32_t* supp_len; int ld_x;   // the codes
    const int32_t* class_of_atom;                 // [m]
    int32_t* labels; double* resid;               // [p]; resid may be null
};
hipError_t launch_classify(const ClassifyArgs& a, hipStream_t stream);

}  // namespace bmpl
