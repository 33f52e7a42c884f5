// Gibbs contractions in the log domain (the absorbed iteration), exact up to
// float rounding.
//
// After the absorption switch the scalings are carried as logs, and one axis
// of a product xi x becomes, per output i of a fibre X of length n,
//     Y[i] = log sum_k exp(X[k] - alpha (i - k)^2),   alpha = 1 / (n^2 gamma)
// (the log of the separable factor K1[i][k] = exp(-(x_i - x_k)^2 / gamma)).
// Each output takes its own shift, the largest term M[i] = max_k (X[k] -
// alpha (i - k)^2), so the largest term is exp(0) = 1 and no term that
// matters to float precision is lost.  No band is assumed: a log input may
// exceed its neighbours by more than the factor's float range, so the max and
// the sum run over windows derived from the fibre's largest value Xmax:
//   - the max starts on the float band |i - k| <= W and widens to
//     alpha (i - k)^2 <= Xmax - M (no term beyond can be larger);
//   - the sum runs over alpha (i - k)^2 <= Xmax - M + 104 (every term beyond
//     is below e^-104 of the largest, under float resolution).
// This is plain ALU work (a max-plus pass and exponentials), not a dense
// contraction, so it does not use MFMA; it runs only in the log domain.
//
// Layout: the field is [outer][n][inner] (the contracted axis has stride
// inner); outputs keep that layout, so d passes (contiguous axis first) apply
// xi, the last one handing its values (logs) to the pointwise epilogue.  A
// block stages F whole fibres in LDS and computes a chunk of TI outputs of
// each.
#include <math.h>

#include <algorithm>

#include "epilogue.h"
#include "logpass.h"

namespace jko {

namespace {

constexpr int kLThr = 256;
constexpr int kLds = 16640;   // floats of staged fibres (F (n + 1) <= kLds)

__device__ __forceinline__ float sq_term(double alpha, int d) { return (float)(alpha * (double)d * (double)d); }

template <int EK>
__global__ void __launch_bounds__(kLThr) log_pass_kernel(LogPass L, EpiArgs E) {
    __shared__ float xs[kLds];
    __shared__ float xmax[64];
    __shared__ double shd[8];
    if (E.ctl && E.ctl->done) return;   // the step has stopped (uniform)

    const int tid = threadIdx.x;
    const int n = L.n, F = L.F, ld = n + 1;
    const bool contig = L.inner == 1;
    const int64_t fb = blockIdx.x / L.chunks;          // fibre block
    const int i0 = (int)(blockIdx.x % L.chunks) * L.TI;
    const int TI = min(L.TI, n - i0);
    // fibre f of this block: contiguous axis: row r0 + f; strided: (o, j0 + f)
    int64_t r0 = 0, o = 0, j0 = 0;
    int nf;
    if (contig) {
        r0 = fb * F;
        nf = (int)(L.outer - r0 < F ? L.outer - r0 : F);
    } else {
        const int64_t jb = (L.inner + F - 1) / F;
        o = fb / jb;
        j0 = (fb % jb) * F;
        nf = (int)(L.inner - j0 < F ? L.inner - j0 : F);
    }
    auto gidx = [&](int f, int c) -> int64_t {
        return contig ? (r0 + f) * n + c : (o * n + c) * L.inner + j0 + f;
    };

    // stage the fibres (coalesced along the memory-contiguous index)
    for (int u = tid; u < F * n; u += kLThr) {
        const int f = contig ? u / n : u % F;
        const int c = contig ? u % n : u / F;
        xs[f * ld + c] = (f < nf) ? L.X[gidx(f, c)] : -INFINITY;
    }
    __syncthreads();
    // largest value of each fibre: four lanes per fibre
    for (int f0 = 0; f0 < F; f0 += kLThr / 4) {
        const int f = f0 + tid / 4;
        float m = -INFINITY;
        if (f < F)
            for (int c = tid % 4; c < n; c += 4) m = fmaxf(m, xs[f * ld + c]);
        m = fmaxf(m, __shfl_xor(m, 1, 64));
        m = fmaxf(m, __shfl_xor(m, 2, 64));
        if (f < F && tid % 4 == 0) xmax[f] = m;
    }
    __syncthreads();

    const double alpha = L.alpha;
    EpiAcc acc;
    for (int u = tid; u < F * TI; u += kLThr) {
        const int f = contig ? u / TI : u % F;
        const int i = i0 + (contig ? u % TI : u / F);
        const float* x = xs + f * ld;
        const float xm = xmax[f];
        float y = -INFINITY;
        if (f < nf && xm > -INFINITY) {
            // largest term: the float band first, then as far as a term could beat it
            const int lo = max(0, i - L.W), hi = min(n - 1, i + L.W);
            float best = -INFINITY;
            for (int c = lo; c <= hi; ++c) best = fmaxf(best, x[c] - sq_term(alpha, i - c));
            const double reach = (best == -INFINITY) ? (double)n : sqrt((double)(xm - best) / alpha) + 1.0;
            const int R = (int)fmin(reach, (double)n);
            for (int c = max(0, i - R); c < lo; ++c) best = fmaxf(best, x[c] - sq_term(alpha, i - c));
            for (int c = hi + 1; c <= min(n - 1, i + R); ++c) best = fmaxf(best, x[c] - sq_term(alpha, i - c));
            // the sum over every term within e^-104 of the largest
            const double M = best;
            const int R2 = (int)fmin(sqrt(((double)xm - M + 104.0) / alpha) + 1.0, (double)n);
            float s = 0.f;
            for (int c = max(0, i - R2); c <= min(n - 1, i + R2); ++c) {
                const int d = i - c;
                s += expf((float)(((double)x[c] - M) - alpha * (double)d * (double)d));
            }
            y = (float)(M + (double)logf(s));
        }
        const int64_t idx = gidx(f, i);
        const int cnt = (f < nf) ? 1 : 0;
        if (EK == EK_STORE) {
            if (cnt) E.y[idx] = y;
        } else {
            const EpiIn in = epi_prefetch<EK>(E, (int)idx, cnt);
            epi_apply<EK, false, 1>(E, (int)idx, cnt, f4{y, 0.f, 0.f, 0.f}, true, in, acc);
        }
    }
    epi_finish<false>(E, acc, (int)blockIdx.x, shd);
}

int fibres_of(int n, int64_t inner) {
    int F = 64;
    while (F > 1 && F * (n + 1) > kLds) F /= 2;
    if (inner > 1) F = (int)std::min<int64_t>(F, inner);
    return F;
}

}  // namespace

LogPass make_log_pass(int64_t outer, int n, int64_t inner, int W, double gamma, const float* X) {
    LogPass L{};
    L.outer = outer;
    L.n = n;
    L.inner = inner;
    L.W = W;
    L.alpha = 1.0 / ((double)n * (double)n * gamma);
    L.X = X;
    L.F = fibres_of(n, inner);
    const int64_t fibres = (inner == 1) ? (outer + L.F - 1) / L.F : outer * ((inner + L.F - 1) / L.F);
    // enough blocks to fill the chip: split the outputs of each fibre into chunks
    int chunks = 1;
    while (fibres * chunks < 1024 && n / (2 * chunks) >= 16) chunks *= 2;
    L.TI = (n + chunks - 1) / chunks;
    L.chunks = (n + L.TI - 1) / L.TI;
    L.fibre_blocks = fibres;
    return L;
}

int64_t log_pass_blocks(const LogPass& L) { return L.fibre_blocks * L.chunks; }

hipError_t launch_log_pass(const LogPass& L, const EpiArgs& epi, int* nblocks, hipStream_t st) {
    const int64_t nb = log_pass_blocks(L);
    if (nb > epi.part.cap && epi.kind != EpiKind::STORE) return hipErrorInvalidValue;
    if (nblocks) *nblocks = (int)nb;
    const dim3 grid((unsigned)nb), block(kLThr);
    switch (ek_of(epi)) {
        case EK_STORE: log_pass_kernel<EK_STORE><<<grid, block, 0, st>>>(L, epi); break;
        case EK_BUPDATE: log_pass_kernel<EK_BUPDATE><<<grid, block, 0, st>>>(L, epi); break;
        case EK_MONITOR: log_pass_kernel<EK_MONITOR><<<grid, block, 0, st>>>(L, epi); break;
        case EK_PROX + JKO_F_ZERO: log_pass_kernel<EK_PROX + JKO_F_ZERO><<<grid, block, 0, st>>>(L, epi); break;
        case EK_PROX + JKO_F_CONGESTION:
            log_pass_kernel<EK_PROX + JKO_F_CONGESTION><<<grid, block, 0, st>>>(L, epi);
            break;
        case EK_PROX + JKO_F_POROUS: log_pass_kernel<EK_PROX + JKO_F_POROUS><<<grid, block, 0, st>>>(L, epi); break;
        case EK_PROX + JKO_F_ENTROPY: log_pass_kernel<EK_PROX + JKO_F_ENTROPY><<<grid, block, 0, st>>>(L, epi); break;
        case EK_PROX + JKO_F_CONGESTION_BINARY:
            log_pass_kernel<EK_PROX + JKO_F_CONGESTION_BINARY><<<grid, block, 0, st>>>(L, epi);
            break;
        case EK_PROX + JKO_F_GEN_ENTROPY:
            log_pass_kernel<EK_PROX + JKO_F_GEN_ENTROPY><<<grid, block, 0, st>>>(L, epi);
            break;
        default: return hipErrorInvalidValue;   // the adjoint has no log domain
    }
    return hipGetLastError();
}

}  // namespace jko
