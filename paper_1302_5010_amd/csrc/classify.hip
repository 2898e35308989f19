// Sparse-representation classification: the face-recognition use of the batch
// solver (Section V follows the class-residual rule of sparse-representation-based
// classification).  For signal i with code x_i, every class with an atom in the
// support is scored by ||b_i - A delta_c(x_i)||_2 (delta_c keeps that class's
// coefficients); the label is the class with the smallest residual, ties to the
// lower class index, -1 for an empty support.  Float64 sums from float32 data.
//
// One 256-thread workgroup per signal; the support is staged in LDS in chunks, the
// classes are visited in increasing order, and for each class the threads stream the
// signal once over n with that class's atoms.
#include <float.h>
#include <limits.h>

#include "bmpl_internal.h"
#include "classify.h"

namespace bmpl {
namespace {

constexpr int NTC = 256;

__device__ inline double block_sum_c(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

__device__ inline int block_min_int(int v, int* redi)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    __syncthreads();
    if (lane == 0) redi[wave] = v;
    __syncthreads();
    return min(min(redi[0], redi[1]), min(redi[2], redi[3]));
}

__global__ __launch_bounds__(NTC) void classify_kernel(ClassifyArgs a)
{
    __shared__ double red[4];
    __shared__ int redi[4];
    const int sig = blockIdx.x;
    const int tid = threadIdx.x;
    const int len = min(a.supp_len[sig], a.ld_x);
    const int* idx = a.x_idx + (int64_t)sig * a.ld_x;
    const float* val = a.x_val + (int64_t)sig * a.ld_x;
    const float* b = a.B + (int64_t)sig * a.ldb;
    int best = -1;
    double best_r = DBL_MAX;
    int prev = INT_MIN;
    for (;;) {
        // next class: the smallest class index above `prev` among the support's atoms
        int c = INT_MAX;
        for (int k = tid; k < len; k += NTC) {
            const int j = idx[k];
            if (j < 0 || j >= a.m) continue;
            const int cj = a.class_of_atom[j];
            if (cj > prev && cj < c) c = cj;
        }
        c = block_min_int(c, redi);
        if (c == INT_MAX) break;
        // residual of that class
        double part = 0.0;
        for (int r = tid; r < a.n; r += NTC) {
            double v = (double)b[r];
            for (int k = 0; k < len; ++k) {
                const int j = idx[k];
                if (j < 0 || j >= a.m || a.class_of_atom[j] != c) continue;
                v -= (double)val[k] * (double)a.At[(int64_t)j * a.lda + r];
            }
            part += v * v;
        }
        const double rr = sqrt(block_sum_c(part, red));
        if (rr < best_r) { best_r = rr; best = c; }   // classes in increasing order: ties keep the lower
        prev = c;
    }
    if (tid == 0) {
        a.labels[sig] = best;
        if (a.resid) a.resid[sig] = best >= 0 ? best_r : 0.0;
    }
}

}  // namespace

hipError_t launch_classify(const ClassifyArgs& a, hipStream_t stream)
{
    if (a.p <= 0) return hipSuccess;
    hipLaunchKernelGGL(classify_kernel, dim3(a.p), dim3(NTC), 0, stream, a);
    return hipGetLastError();
}

}  // namespace bmpl
