// Set-up, control and pointwise kernels of libjko (gfx950).
//
//  * the one-axis Gibbs factor K1[i][j] = exp(-(x_i - x_j)^2 / gamma) on the
//    cell-centred grid x_i = (i + 1/2)/n (Section 3.1 of the paper, cost
//    |x - y|^2), evaluated in FP64 and rounded to float32, plus its
//    bfloat16 hi/lo split for the split-precision contractions;
//  * per-call energy fields: exp(-sigma w) for the congestion prox
//    (Proposition 4.1), 1/(1 + sigma c) for the entropy prox (Proposition 4.2,
//    m = 1), log((m-1) k) = log(sigma c m D^{m-1}) for the porous prox;
//  * the single-block control kernel that turns the per-block FP64 partial sums
//    of the fused epilogues into the marginal violation of Listing 1 and the
//    stop decision (fixed summation order: bitwise reproducible);
//  * the FP64 input check (mass, capacity, finiteness);
//  * the pointwise parts of the adjoint sweep.
#include <math.h>

#include "adjoint.h"
#include "control.h"
#include "jko_internal.h"

namespace jko {

namespace {

__device__ __forceinline__ uint16_t f2bf_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

unsigned blocks_for(int64_t n, int per = 256) {
    int64_t b = (n + per - 1) / per;
    if (b > 65535 * 16) b = 65535 * 16;
    if (b < 1) b = 1;
    return (unsigned)b;
}

__global__ void k_build_factor(float* K1, uint16_t* hi, uint16_t* lo, int n, double gamma) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    const double d = (double)(i - j) / (double)n;
    const double kd = exp(-(d * d) / gamma);
    K1[idx] = (float)kd;
    if (hi) {
        const uint16_t h = f2bf_rne((float)kd);
        hi[idx] = h;
        lo[idx] = f2bf_rne((float)(kd - (double)bf2f(h)));
    }
}

__global__ void k_fill(float* x, float v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_copy_scaled(float* __restrict__ d, const float* __restrict__ s, double f, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (float)((double)s[i] * f);
}

__global__ void k_copy(float* __restrict__ d, const float* __restrict__ s, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

__global__ void k_prepare(int kind, const float* w, const float* coef, float coef_s, float m, const float* mf,
                          float D, double sigma, int64_t N, float* g, float* kf) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (kind == JKO_F_CONGESTION) {
            if (g) g[i] = (float)exp(-sigma * (double)w[i]);
        } else if (kind == JKO_F_ENTROPY) {
            const double c = coef ? (double)coef[i] : (double)coef_s;
            kf[i] = (float)(1.0 / (1.0 + sigma * c));
        } else if (kind == JKO_F_GEN_ENTROPY) {
            // c = sigma b m and eps = m - 1 (exponents below 1 are taken as 1)
            const double b = coef ? (double)coef[i] : (double)coef_s;
            const double mi = fmax(mf ? (double)mf[i] : (double)m, 1.0);
            kf[i] = (float)(sigma * b * mi);
            g[i] = (float)(mi - 1.0);
        } else if (kind == JKO_F_POROUS) {
            const double c = coef ? (double)coef[i] : (double)coef_s;
            const double mm = (double)m;
            kf[i] = (float)log(sigma * c * mm * pow((double)D, mm - 1.0));
        }
    }
}

// Proximal half-step of the Wasserstein attraction (eq. prox-psi-attraction,
// h = iota_[0,kappa]) on the two stacked couplings: s = (s_1, s_2),
// p = min(s_1^alpha s_2^{1-alpha}, kappa) with alpha = 1/(1+tau), a_m = p / s_m
// (0/0 = 0).  Log domain (ctl->logmode): s and a hold logs,
// log p = min(alpha log s_1 + (1-alpha) log s_2, log kappa), log a_m = log p - log s_m.
// Nothing is written once the step has stopped.
__global__ void k_attraction_prox(const float* __restrict__ s, float* __restrict__ a, float* __restrict__ p,
                                  const float* __restrict__ kappa, float kappa_s, float alpha, int64_t N,
                                  const Ctl* ctl) {
    // the first cell's inputs are loaded before the control block is looked
    // at, so that the two memory latencies overlap
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float s1 = 0.f, s2 = 0.f, k = kappa_s;
    if (i < N) {
        s1 = s[i];
        s2 = s[N + i];
        if (kappa) k = kappa[i];
    }
    if (ctl && ctl->done) return;
    const bool logx = ctl && ctl->logmode;
    for (; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        if (i != (int64_t)blockIdx.x * blockDim.x + threadIdx.x) {
            s1 = s[i];
            s2 = s[N + i];
            k = kappa ? kappa[i] : kappa_s;
        }
        if (logx) {
            const float lp = fminf(alpha * s1 + (1.f - alpha) * s2, logf(k));
            p[i] = expf(lp);
            a[i] = lp == -INFINITY ? -INFINITY : lp - s1;
            a[N + i] = lp == -INFINITY ? -INFINITY : lp - s2;
            continue;
        }
        const float g = (s1 > 0.f && s2 > 0.f) ? expf(alpha * logf(s1) + (1.f - alpha) * logf(s2)) : 0.f;
        const float pv = fminf(g, k);
        p[i] = pv;
        a[i] = pv == 0.f ? 0.f : pv / s1;
        a[N + i] = pv == 0.f ? 0.f : pv / s2;
    }
}

__global__ void k_ctl_reset(Ctl* c, int logmode) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->done = 0;
        c->stop_iter = 0;
        c->nonfinite = 0;
        c->absorptions = logmode ? 1 : 0;
        c->absorb_pending = 0;
        c->logmode = logmode;
        c->exit_iter = 0;
        c->err = 0.0;
        c->mass = 0.0;
        c->maxloga = 0.0;
        c->maxlogb = 0.0;
        for (int i = 0; i < 4; ++i) c->aux[i] = 0.0;
    }
}

// Deterministic single-block sum of `n` partials.
__device__ double fixed_sum(const double* v, int n, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += v[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// plain: queued as part of plain-domain iterations, which are void once a
// switch to the log domain has been committed (their kernels returned early).
__global__ void __launch_bounds__(64) k_ctl_check(Ctl* c, Partials part, int nparts, int iter,
                                                  double tol, int check_mass, double absorb, int a_only,
                                                  int plain) {
    if (c->done || (plain && c->logmode)) return;
    ctl_update(c, part, nparts, iter, tol, check_mass, absorb, a_only);
}

__global__ void k_absorb(const Ctl* c, float* __restrict__ a, float* __restrict__ b, int64_t N) {
    if (!c->absorb_pending || c->done) return;
    const float ninf = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float av = a[i], bv = b[i];
        a[i] = av > 0.f ? logf(av) : ninf;
        b[i] = bv > 0.f ? logf(bv) : ninf;
    }
}

__global__ void k_ctl_commit(Ctl* c, int iter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (c->absorb_pending && !c->done) {
            c->logmode = 1;
            c->exit_iter = iter;
        }
        c->absorb_pending = 0;
    }
}

__global__ void __launch_bounds__(256) k_input_partial(const float* p, const float* kappa, float kappa_s,
                                                       int64_t N, int congestion, double* part) {
    __shared__ double sh[256];
    double sp = 0.0, sk = 0.0, bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = p[i];
        if (!isfinite(v) || v < 0.f) bad += 1.0;
        else sp += (double)v;
        if (congestion) {
            const float k = kappa ? kappa[i] : kappa_s;
            if (isnan(k) || k < 0.f) bad += 1.0;
            else sk += (double)k;   // +inf propagates: no cap
        }
    }
    const double vals[3] = {sp, sk, bad};
    for (int q = 0; q < 3; ++q) {
        sh[threadIdx.x] = vals[q];
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[q * gridDim.x + blockIdx.x] = sh[0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_input_final(const double* part, int nb, double* out) {
    __shared__ double sh[256];
    for (int q = 0; q < 3; ++q) {
        const double s = fixed_sum(part + q * nb, nb, sh);
        if (threadIdx.x == 0) out[q] = s;
    }
}

// ---------------------------------------------------------------- adjoint

// Reverse of p = prox(s), a = p / s over the field (adj_prox_cell per cell).
template <int KIND>
__global__ void k_adj_prox(const float* __restrict__ s, const float* __restrict__ pbar_ext,
                           const float* __restrict__ abar, float* __restrict__ sbar,
                           float* __restrict__ wbar, ProxArgs px, float sigma, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        float fu = 0.f, fv = 0.f;
        if (KIND == JKO_F_CONGESTION) {
            fu = px.g ? px.g[i] : 1.f;
            fv = px.kappa ? px.kappa[i] : px.kappa_s;
        } else if (KIND == JKO_F_ENTROPY || KIND == JKO_F_POROUS) {
            fu = px.kf ? px.kf[i] : px.kf_s;
        } else if (KIND == JKO_F_GEN_ENTROPY) {
            fu = px.kf ? px.kf[i] : px.kf_s;
            fv = px.g ? px.g[i] : px.eps_s;
        }
        float dw;
        sbar[i] = adj_prox_cell<KIND>(px, sigma, s[i], pbar_ext ? pbar_ext[i] : 0.f, abar ? abar[i] : 0.f, fu,
                                      fv, &dw);
        if (wbar && dw != 0.f) wbar[i] += dw;
    }
}

// Reverse of b = q / t over the field (adj_b_cell per cell).
__global__ void k_adj_b(const float* __restrict__ t, const float* __restrict__ q,
                        const float* __restrict__ bbar, float* __restrict__ tbar,
                        float* __restrict__ qbar, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        float dq;
        tbar[i] = adj_b_cell(t[i], q[i], bbar[i], &dq);
        if (dq != 0.f) qbar[i] += dq;
    }
}

__global__ void k_axpy(float* __restrict__ y, const float* __restrict__ x, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] += x[i];
}

}  // namespace

hipError_t launch_build_factor(float* K1, uint16_t* hi, uint16_t* lo, int n, double gamma,
                               hipStream_t s) {
    const int64_t nn = (int64_t)n * n;
    hipLaunchKernelGGL(k_build_factor, dim3(blocks_for(nn)), dim3(256), 0, s, K1, hi, lo, n, gamma);
    return hipGetLastError();
}

hipError_t launch_fill(float* x, float v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 1024)), dim3(256), 0, s, x, v, n);
    return hipGetLastError();
}

hipError_t launch_copy_scaled(float* dst, const float* src, double f, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_scaled, dim3(blocks_for(n, 1024)), dim3(256), 0, s, dst, src, f, n);
    return hipGetLastError();
}

hipError_t launch_copy(float* dst, const float* src, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(blocks_for(n, 1024)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_prepare_energy(const jko_energy* en, double sigma, int64_t N, float* g, float* kf,
                                 hipStream_t s) {
    // both congestion kinds prepare g = exp(-sigma w)
    const int kind = en->kind == JKO_F_CONGESTION_BINARY ? JKO_F_CONGESTION : en->kind;
    hipLaunchKernelGGL(k_prepare, dim3(blocks_for(N, 1024)), dim3(256), 0, s, kind, en->w, en->coef,
                       en->coef_scalar, en->m, en->m_field, en->density_scale, sigma, N, g, kf);
    return hipGetLastError();
}

hipError_t launch_attraction_prox(const float* s, float* a, float* p, const float* kappa, float kappa_s,
                                  double alpha, int64_t N, const Ctl* ctl, hipStream_t st) {
    hipLaunchKernelGGL(k_attraction_prox, dim3(blocks_for(N, 1024)), dim3(256), 0, st, s, a, p, kappa, kappa_s,
                       (float)alpha, N, ctl);
    return hipGetLastError();
}

hipError_t launch_ctl_reset(Ctl* ctl, int logmode, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, s, ctl, logmode);
    return hipGetLastError();
}

hipError_t launch_ctl_check(Ctl* ctl, Partials part, int nparts, int iter, double tol, int check_mass,
                            double absorb, int a_only, int plain, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_check, dim3(1), dim3(64), 0, s, ctl, part, nparts, iter, tol, check_mass, absorb,
                       a_only, plain);
    return hipGetLastError();
}

hipError_t launch_absorb(Ctl* ctl, float* a, float* b, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_absorb, dim3(blocks_for(N, 1024)), dim3(256), 0, s, ctl, a, b, N);
    return hipGetLastError();
}

hipError_t launch_ctl_commit(Ctl* ctl, int iter, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_commit, dim3(1), dim3(64), 0, s, ctl, iter);
    return hipGetLastError();
}

hipError_t launch_input_check(const float* p_in, const float* kappa, float kappa_s, int64_t N,
                              int congestion, double* part, int part_cap, double* out, hipStream_t s) {
    int nb = part_cap / 3;
    if (nb > 256) nb = 256;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_input_partial, dim3(nb), dim3(256), 0, s, p_in, kappa, kappa_s, N, congestion, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_input_final, dim3(1), dim3(256), 0, s, part, nb, out);
    return hipGetLastError();
}

hipError_t launch_adj_prox(const float* s, const float* pbar_ext, const float* abar, float* sbar,
                           float* wbar, const ProxArgs& px, double sigma, int64_t N, hipStream_t st) {
    const dim3 grid(blocks_for(N, 1024)), block(256);
    switch (px.kind) {
        case JKO_F_CONGESTION:
            hipLaunchKernelGGL(k_adj_prox<JKO_F_CONGESTION>, grid, block, 0, st, s, pbar_ext, abar, sbar, wbar, px,
                               (float)sigma, N);
            break;
        case JKO_F_ENTROPY:
            hipLaunchKernelGGL(k_adj_prox<JKO_F_ENTROPY>, grid, block, 0, st, s, pbar_ext, abar, sbar, wbar, px,
                               (float)sigma, N);
            break;
        case JKO_F_POROUS:
            hipLaunchKernelGGL(k_adj_prox<JKO_F_POROUS>, grid, block, 0, st, s, pbar_ext, abar, sbar, wbar, px,
                               (float)sigma, N);
            break;
        case JKO_F_GEN_ENTROPY:
            hipLaunchKernelGGL(k_adj_prox<JKO_F_GEN_ENTROPY>, grid, block, 0, st, s, pbar_ext, abar, sbar, wbar, px,
                               (float)sigma, N);
            break;
        default:
            hipLaunchKernelGGL(k_adj_prox<JKO_F_ZERO>, grid, block, 0, st, s, pbar_ext, abar, sbar, wbar, px,
                               (float)sigma, N);
    }
    return hipGetLastError();
}

hipError_t launch_adj_b(const float* t, const float* q, const float* bbar, float* tbar, float* qbar,
                        int64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_b, dim3(blocks_for(N, 1024)), dim3(256), 0, st, t, q, bbar, tbar, qbar, N);
    return hipGetLastError();
}

hipError_t launch_axpy_inplace(float* y, const float* x, int64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy, dim3(blocks_for(N, 1024)), dim3(256), 0, st, y, x, N);
    return hipGetLastError();
}

}  // namespace jko
