// Log-domain Gibbs contraction along one axis (see logpass.hip).
#pragma once

#include "jko_internal.h"

namespace jko {

// One axis pass of the log-domain product: the field is [outer][n][inner]
// (the axis has stride inner), Y[o][i][j] = log sum_k exp(X[o][k][j] -
// alpha (i - k)^2) with alpha = 1 / (n^2 gamma), written in the same layout
// or handed (as logs) to the pointwise epilogue.
struct LogPass {
    int64_t outer, inner;
    int n;
    int W;                 // float32 band half-width of the factor (where the max search starts)
    double alpha;
    const float* X;
    int F;                 // fibres staged per block
    int TI;                // outputs per block along the axis
    int chunks;            // blocks per fibre group
    int64_t fibre_blocks;  // fibre groups
};

LogPass make_log_pass(int64_t outer, int n, int64_t inner, int W, double gamma, const float* X);
int64_t log_pass_blocks(const LogPass& L);
// Every epilogue but the adjoint's; partial sums go to slot blockIdx (at most epi.part.cap blocks).
hipError_t launch_log_pass(const LogPass& L, const EpiArgs& epi, int* nblocks, hipStream_t st);

}  // namespace jko
