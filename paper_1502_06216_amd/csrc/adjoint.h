// Per-cell reverse steps of the iteration (3.2), shared by the pointwise
// adjoint kernels and the contraction epilogues that fuse them.
#pragma once

#include <math.h>

#include "jko_internal.h"

namespace jko {

// Generalised entropy (Proposition 4.2 with weight b, exponent m = 1 + eps and
// density scale D): Y = log(D psi) is the root of
//   F(Y) = Y + c (e^{eps Y} - 1) / eps - L = 0,   c = sigma b m,  L = log(D s),
// continuous down to eps = 0 (where Y = L / (1 + c)).  F is increasing and
// convex, and both L / (1 + c) and, for L > 0, log(1 + eps L / c) / eps lie at
// or right of the root (e^x >= 1 + x), so Newton from their minimum descends
// monotonically onto it.  (e^x - 1) / x is taken as 1 + x/2 for |x| < 1e-4.
//
// Stopping rule of the Newton proxes (this one and the porous one): both
// converge quadratically with a constant of at most 1/2 (here in Y, F''/(2F')
// <= eps/2; the porous form in the log of its variable), so once a step's
// update is within 2^-20 of the iterate's scale the error left is about 2^-41
// of it, far below float32 rounding, and further steps would only move the
// iterate by rounding.  `steps` caps the count.  The update's divisor F' only
// sets the speed, not the root, so it takes the hardware reciprocal, and here
// e^x comes from the residual's (e^x - 1) / x.
constexpr float kNewtonTol = 0x1p-20f;

__device__ __forceinline__ float gen_newton_step(float y, float L, float c, float eps) {
    const float x = eps * y;
    const float phi = fabsf(x) < 1e-4f ? 1.f + 0.5f * x : expm1f(x) / x;
    const float f = y + c * y * phi - L;
    return y - f * __builtin_amdgcn_rcpf(1.f + c * (1.f + x * phi));
}

__device__ __forceinline__ bool gen_newton_settled(float y, float yn) {
    return fabsf(yn - y) <= kNewtonTol * fmaxf(fabsf(yn), 1.f);
}

__device__ __forceinline__ float log_prox_gen(float L, float c, float eps, int steps) {
    float y = L / (1.f + c);
    if (eps > 0.f && c > 0.f) {
        if (L > 0.f) y = fminf(y, log1pf(eps * L / c) / eps);
        for (int it = 0; it < steps; ++it) {
            const float yn = gen_newton_step(y, L, c, eps);
            const bool done = gen_newton_settled(y, yn);
            y = yn;
            if (done) break;
        }
    }
    return y;
}

// Porous prox in the variable v = (m-1) k psi^{m-1}: the root equation
// log psi + k psi^{m-1} = log s becomes v + log v = lz with
// lz = log((m-1) k) + (m-1) log s (Lambert W of e^lz).  Newton steps on it in
// residual form, v <- v - (log v + v - lz) v / (1 + v); the start
// v0 = log(1 + e^lz) (lz < 1) or lz - log lz is within 2% of the root
// everywhere, so a few steps settle it under the stopping rule of the Newton
// proxes.
__device__ __forceinline__ float porous_newton_step(float v, float lz) {
    const float r = logf(v) + v - lz;
    return v - r * v * __builtin_amdgcn_rcpf(1.f + v);
}

// The residual carries rounding noise of a few ulps of |lz|, so the relative
// update is compared with 2^-20 max(1, |lz|) (at |lz| <= 60 the error left is
// still below 2^-29 of v).
__device__ __forceinline__ bool porous_newton_settled(float v, float vn, float lz) {
    return fabsf(vn - v) <= kNewtonTol * fmaxf(fabsf(lz), 1.f) * fabsf(vn);
}

__device__ __forceinline__ float porous_start(float lz) { return (lz < 1.f) ? log1pf(expf(lz)) : lz - logf(lz); }

// The root v of v + log v = lz.
__device__ __forceinline__ float porous_root(float lz, int steps) {
    float v = porous_start(lz);
    for (int it = 0; it < steps; ++it) {
        const float vn = porous_newton_step(v, lz);
        const bool done = porous_newton_settled(v, vn, lz);
        v = vn;
        if (done) break;
    }
    return v;
}

// Reverse of p = prox(s), a = p / s at one cell:
//   pbar = pbar_ext + abar / s
//   sbar = -abar a / s + pbar dp/ds          (abar p / s^2 written with a = p / s)
//   wbar += pbar dp/dw          (congestion: dp/dw = -sigma s g on the free branch;
//                                generalised entropy: the weight b in place of w)
// Ties s g = kappa take the capped branch (derivative 0).  Terms whose factor
// is structurally zero (a = 0, dp/ds = 0) are skipped, so cells with s, p at
// the float32 underflow limit contribute 0 rather than 0 * inf.
// fu, fv: the cell's energy fields (congestion: g, kappa; entropy: 1/(1 + sigma c);
// porous: log((m-1) k); generalised entropy: c = sigma b m, eps = m - 1).
// Returns sbar; *dw receives the wbar increment.
template <int KIND>
__device__ __forceinline__ float adj_prox_cell(const ProxArgs& px, float sigma, float sv, float pb, float ab,
                                               float fu, float fv, float* dw) {
    float p = 0.f, dpds = 0.f, dpdw = 0.f, sb = 0.f;
    *dw = 0.f;
    if (!(sv > 0.f)) return 0.f;
    if (KIND == JKO_F_CONGESTION) {
        const float sg = sv * fu;
        if (sg < fv) {
            p = sg;
            dpds = fu;
            dpdw = -sigma * sg;
        } else {
            p = fv;
        }
    } else if (KIND == JKO_F_ENTROPY) {
        p = expf(fu * logf(sv));
        dpds = fu * p / sv;
    } else if (KIND == JKO_F_POROUS) {
        const float m = px.m;
        const float ls = logf(sv);
        const float lz = fu + (m - 1.f) * ls;
        if (lz < -60.f) {   // k psi^{m-1} negligible: psi = s
            p = sv;
            dpds = 1.f;
        } else {
            const float v = porous_root(lz, px.newton);
            p = expf(ls - v / (m - 1.f));
            // implicit derivative of log psi + k psi^{m-1} = log s
            dpds = (p / sv) / (1.f + v);
        }
    } else if (KIND == JKO_F_GEN_ENTROPY) {
        // implicit derivatives of Y + c (e^{eps Y} - 1) / eps = log(D s),
        // c = sigma b m: dY / dlog s = 1 / (1 + c e^{eps Y}) and
        // dY / db = -sigma m (e^{eps Y} - 1) / eps / (1 + c e^{eps Y})
        const float y = log_prox_gen(logf(sv) + px.lD, fu, fv, px.newton);
        const float x = fv * y;
        const float inv = 1.f / (1.f + fu * expf(x));
        const float phi = fabsf(x) < 1e-4f ? y * (1.f + 0.5f * x) : expm1f(x) / fv;
        p = expf(y - px.lD);
        dpds = (p / sv) * inv;
        dpdw = -p * sigma * (1.f + fv) * phi * inv;
    } else {
        p = sv;
        dpds = 1.f;
    }
    const float a = (p == 0.f) ? 0.f : p / sv;
    const float abs_ = (ab != 0.f) ? ab / sv : 0.f;
    pb += abs_;
    if (a != 0.f) sb -= abs_ * a;
    if (dpds != 0.f) sb += pb * dpds;
    if (dpdw != 0.f) *dw = pb * dpdw;
    return sb;
}

// Reverse of b = q / t at one cell: tbar = -bbar q / t^2 = -bbar b / t and the
// qbar increment bbar / t (zero where t = 0).
__device__ __forceinline__ float adj_b_cell(float tv, float qv, float bb, float* dq) {
    if (!(tv > 0.f)) {
        *dq = 0.f;
        return 0.f;
    }
    const float bv = (qv == 0.f) ? 0.f : qv / tv;
    *dq = bb / tv;
    return (bv == 0.f || bb == 0.f) ? 0.f : -bb * (bv / tv);
}

}  // namespace jko
