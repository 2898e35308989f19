// Launchers of the Q-route correlation (qroute.hip): g = beta - Q_{:,S} x_S.
#pragma once

#include "bmpl_internal.h"

namespace bmpl {

// beta[i][j] = a_j^T b_i (float64 sums of float32 products), i < p, j < m.
hipError_t launch_atb_f64(const float* At, int64_t lda, int m, const float* Bw, int64_t ldb, int p, int n,
                          double* beta, int64_t ldbeta, hipStream_t s);

struct QCorrArgs {
    Workspace w;
    const double* Q; int64_t ldq;         // Gram table
    const double* beta; int64_t ldbeta;   // [p][ldbeta]
    const int* act; const int* n_act_dev; int p_grid;
    float* G; int64_t ldg;                // output rows by running index, as the MFMA product
};
hipError_t launch_q_corr(const QCorrArgs& a, hipStream_t s);

}  // namespace bmpl
