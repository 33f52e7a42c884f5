// Device-side helpers shared by the contraction kernels: bfloat16 split,
// block reductions, the proximal maps of the energies and the pointwise
// epilogues that finish an iteration's half-step (plain and log domain).
#pragma once

#include <math.h>

#include "adjoint.h"
#include "jko_internal.h"

namespace jko {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ uint16_t f2bf_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Block-wide FP64 reductions; every thread of the block must call them.
__device__ inline double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
    return r;  // valid in thread 0
}
__device__ inline double block_max(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, sh[w]);
    return r;
}

// --------------------------------------------------------- proximal maps

// log Prox(e^ls) of the porous energy: log psi = ls - v / (m - 1) with v the
// root of v + log v = lz (porous_root).
__device__ __forceinline__ float log_prox_porous(float ls, float lk, float m, int steps) {
    if (ls == -INFINITY) return -INFINITY;
    const float lz = lk + (m - 1.f) * ls;
    if (lz < -60.f) return ls;   // v < 1e-26: psi = s to float32 rounding (also k = 0)
    return ls - porous_root(lz, steps) / (m - 1.f);
}

// The porous and generalised-entropy proxes of a thread's NE cells at once,
// in the log domain (ls = log s, -inf for s = 0): log_prox_porous and
// log_prox_gen cell by cell (a cell stops stepping once settled, as there),
// with the loop running until every cell has settled or the cap is reached.
// Cells that take no Newton step (s = 0, lz < -60, a zero coefficient or
// exponent) keep their closed form.
template <int KIND, int NE>
__device__ __forceinline__ f4 log_prox_cells(const ProxArgs& px, f4 ls, f4 pu, f4 pv) {
    static_assert(KIND == JKO_F_POROUS || KIND == JKO_F_GEN_ENTROPY, "Newton proxes only");
    f4 out;
    if constexpr (KIND == JKO_F_POROUS) {
        const float m = px.m;
        float lz[NE], v[NE];
        bool go[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const float z = pu[e] + (m - 1.f) * ls[e];
            go[e] = !(ls[e] == -INFINITY) && !(z < -60.f);
            lz[e] = go[e] ? z : 1.f;
            v[e] = go[e] ? porous_start(z) : 1.f;
        }
        for (int it = 0; it < px.newton; ++it) {
            bool any = false;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const float vn = porous_newton_step(v[e], lz[e]);
                const bool done = porous_newton_settled(v[e], vn, lz[e]);
                v[e] = go[e] ? vn : v[e];
                go[e] = go[e] && !done;
                any |= go[e];
            }
            if (!any) break;
        }
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const float z = pu[e] + (m - 1.f) * ls[e];
            out[e] = (ls[e] == -INFINITY) ? -INFINITY : (z < -60.f) ? ls[e] : ls[e] - v[e] / (m - 1.f);
        }
    } else {
        float y0[NE], y[NE], L[NE];
        bool nw[NE], go[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const float Le = ls[e] + px.lD, ce = pu[e], ee = pv[e];
            y0[e] = Le / (1.f + ce);
            nw[e] = !(ls[e] == -INFINITY) && ee > 0.f && ce > 0.f;
            if (nw[e] && Le > 0.f) y0[e] = fminf(y0[e], log1pf(ee * Le / ce) / ee);
            go[e] = nw[e];
            y[e] = nw[e] ? y0[e] : 0.f;
            L[e] = nw[e] ? Le : 0.f;
        }
        for (int it = 0; it < px.newton; ++it) {
            bool any = false;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const float yn = gen_newton_step(y[e], L[e], go[e] ? pu[e] : 0.f, go[e] ? pv[e] : 0.f);
                const bool done = gen_newton_settled(y[e], yn);
                y[e] = go[e] ? yn : y[e];
                go[e] = go[e] && !done;
                any |= go[e];
            }
            if (!any) break;
        }
#pragma unroll
        for (int e = 0; e < NE; ++e)
            out[e] = (ls[e] == -INFINITY) ? -INFINITY : (nw[e] ? y[e] : y0[e]) - px.lD;
    }
    return out;
}


// Epilogue codes: the epilogue kind and, for the proximal epilogue, the
// energy, fixed at compile time so that each kernel carries only its own code.
// EK_PROX + energy kind, EK_ADJ_B, EK_ADJ_PROX + energy kind
// (the binary congestion prox, kind 4, has no adjoint epilogue)
// EK_ATTR: the attraction's proximal step over two stacked couplings (only
// the rotating pass has it).
enum : int { EK_STORE = 0, EK_BUPDATE = 1, EK_MONITOR = 2, EK_PROX = 3, EK_ADJ_B = 9, EK_ADJ_PROX = 10,
             EK_ATTR = 32 };

__host__ __device__ constexpr EpiKind ek_kind(int ek) {
    return ek == EK_STORE ? EpiKind::STORE : ek == EK_BUPDATE ? EpiKind::BUPDATE
         : ek == EK_MONITOR ? EpiKind::MONITOR : ek == EK_ADJ_B ? EpiKind::ADJ_B
         : ek == EK_ATTR ? EpiKind::ATTR_PROX
         : ek >= EK_ADJ_PROX ? EpiKind::ADJ_PROX : EpiKind::PROX;
}

inline int ek_of(const EpiArgs& e) {
    switch (e.kind) {
        case EpiKind::STORE: return EK_STORE;
        case EpiKind::BUPDATE: return EK_BUPDATE;
        case EpiKind::MONITOR: return EK_MONITOR;
        case EpiKind::ADJ_B: return EK_ADJ_B;
        case EpiKind::ADJ_PROX: return EK_ADJ_PROX + e.prox.kind;
        case EpiKind::ATTR_PROX: return EK_ATTR;
        default: return EK_PROX + e.prox.kind;
    }
}

// Prox of one cell; pu, pv are the cell's prefetched energy parameters
// (congestion: exp(-sigma w), kappa; entropy: 1/(1 + sigma c); porous:
// log((m-1) k)).
// Binary congestion: kappa where z = s e^{-sigma w} reaches kappa/e, else 0
// (the tie takes kappa).
constexpr float kInvE = 0.36787944117144233f;   // 1 / e

template <int KIND>
__device__ __forceinline__ float prox_val(const ProxArgs& px, float s, float pu, float pv) {
    if (KIND == JKO_F_CONGESTION) return fminf(s * pu, pv);
    if (KIND == JKO_F_CONGESTION_BINARY) return s * pu >= pv * kInvE ? pv : 0.f;
    if (KIND == JKO_F_ENTROPY) return s > 0.f ? expf(pu * logf(s)) : 0.f;
    if (KIND == JKO_F_POROUS) return s > 0.f ? expf(log_prox_porous(logf(s), pu, px.m, px.newton)) : 0.f;
    if (KIND == JKO_F_GEN_ENTROPY)
        return s > 0.f ? expf(log_prox_gen(logf(s) + px.lD, pu, pv, px.newton) - px.lD) : 0.f;
    return s;
}

// log Prox(exp(ls)) of one cell.
template <int KIND>
__device__ __forceinline__ float log_prox_val(const ProxArgs& px, float ls, float pu, float pv) {
    if (KIND == JKO_F_CONGESTION) return fminf(ls + logf(pu), logf(pv));
    if (KIND == JKO_F_CONGESTION_BINARY) {
        const float lk = logf(pv);
        return (pv > 0.f && ls + logf(pu) >= lk - 1.f) ? lk : -INFINITY;
    }
    if (KIND == JKO_F_ENTROPY) return pu * ls;
    if (KIND == JKO_F_POROUS) return log_prox_porous(ls, pu, px.m, px.newton);
    if (KIND == JKO_F_GEN_ENTROPY)
        return ls == -INFINITY ? -INFINITY : log_prox_gen(ls + px.lD, pu, pv, px.newton) - px.lD;
    return ls;
}

// ------------------------------------------------------------- epilogues

// Per-thread accumulators of the epilogue reductions.
struct EpiAcc {
    double err = 0.0, mass = 0.0, maxla = 0.0, maxlb = 0.0;
};

// Inputs of the pointwise epilogue for a run of up to 4 consecutive outputs,
// loaded before they are needed so that their latency overlaps the
// contraction.  BUPDATE/MONITOR: u = q, v = old b;  PROX: u, v = the energy
// parameters of prox_val.
struct EpiIn {
    f4 u, v, w;
};

__device__ __forceinline__ f4 ld4(const float* __restrict__ p, int idx, int cnt, bool vec, float fill) {
    if (vec && cnt == 4) return *reinterpret_cast<const f4*>(p + idx);
    f4 r = f4{fill, fill, fill, fill};
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (e < cnt) r[e] = p[idx + e];
    return r;
}

// Four consecutive values at any float index: the hardware needs only dword
// alignment for a 16-byte load, so this is one load with no branch.
typedef float f4_dw __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ f4 ld4_full(const float* __restrict__ p, int idx) {
    return *reinterpret_cast<const f4_dw*>(p + idx);
}

// Epilogue results are written with the non-temporal (streaming) hint: each
// is read once, by the next kernel or pass, usually from another XCD.
__device__ __forceinline__ void st4(float* __restrict__ p, int idx, int cnt, bool vec, f4 v) {
    if (vec && cnt == 4) {
        __builtin_nontemporal_store(v, reinterpret_cast<f4*>(p + idx));
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (e < cnt) __builtin_nontemporal_store(v[e], p + idx + e);
}


// Split 8 consecutive floats into bfloat16 hi + lo, x = hi + lo + O(2^-16 x),
// with the hardware's round-to-nearest-even conversion.
__device__ __forceinline__ void split_bf16(f4 v0, f4 v1, bf8& hi, bf8& lo) {
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    typedef float fl2 __attribute__((ext_vector_type(2)));
    const fl2 x[4] = {fl2{v0[0], v0[1]}, fl2{v0[2], v0[3]}, fl2{v1[0], v1[1]}, fl2{v1[2], v1[3]}};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const b2 h = __builtin_convertvector(x[q], b2);
        const b2 l = __builtin_convertvector(x[q] - __builtin_convertvector(h, fl2), b2);
        hi[2 * q] = h[0];
        hi[2 * q + 1] = h[1];
        lo[2 * q] = l[0];
        lo[2 * q + 1] = l[1];
    }
}

// Device-scope (coherent across XCDs) element stores and loads, for data one
// block of the resident kernel writes and another reads within the launch.
// A whole aligned run goes out as one 16-byte buffer store with the device
// scope bit (SC1); the descriptor spans the 2^31 bytes a 32-bit offset reaches.
__device__ __forceinline__ void st4_coh(float* p, int idx, int cnt, bool vec, f4 v) {
    if (vec && cnt == 4) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(p, (short)0, 0x7fffffff, 0x00020000);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rs, 4 * idx, 0, 16);
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (e < cnt) __hip_atomic_store(p + idx + e, v[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ f4 ld4_coh(const float* p, int idx, int cnt, float fill) {
    f4 r;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        r[e] = (e < cnt) ? __hip_atomic_load(p + idx + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : fill;
    return r;
}

// COH: accumulators of the adjoint epilogues are read with device-scope loads
// (the resident reverse sweep writes them with device-scope stores).
template <int EK, bool COH = false, bool FULL = false>
__device__ __forceinline__ EpiIn epi_prefetch(const EpiArgs& E, int idx, int cnt) {
    EpiIn in;
    in.u = f4{0.f, 0.f, 0.f, 0.f};
    in.v = f4{0.f, 0.f, 0.f, 0.f};
    in.w = f4{0.f, 0.f, 0.f, 0.f};
    if (!FULL && cnt <= 0) return in;
    const bool vec = E.vec_ok && ((idx & 3) == 0);
    // FULL: every group of four is whole (cnt == 4): branch-free loads, so no
    // register copy at a join waits for the load to land
    auto ld4 = [&](const float* p, int i, int c, bool v, float fill) {
        if constexpr (FULL) return ld4_full(p, i);
        else return jko::ld4(p, i, c, v, fill);
    };
    if (EK == EK_BUPDATE || EK == EK_MONITOR) {
        in.u = ld4(E.q, idx, cnt, vec, 0.f);
        if (EK == EK_MONITOR || E.check) in.v = ld4(E.b, idx, cnt, vec, 0.f);
    } else if (EK == EK_ADJ_B) {
        in.u = ld4(E.hin, idx, cnt, vec, 0.f);
        in.v = ld4(E.q, idx, cnt, vec, 0.f);
        in.w = COH ? ld4_coh(E.acc, idx, cnt, 0.f) : ld4(E.acc, idx, cnt, vec, 0.f);
    } else if (EK >= EK_ADJ_PROX) {
        const ProxArgs& px = E.prox;
        in.u = ld4(E.hin, idx, cnt, vec, 0.f);
        if (EK - EK_ADJ_PROX == JKO_F_CONGESTION) {
            in.v = px.g ? ld4(px.g, idx, cnt, vec, 1.f) : f4{1.f, 1.f, 1.f, 1.f};
            in.w = px.kappa ? ld4(px.kappa, idx, cnt, vec, 0.f)
                            : f4{px.kappa_s, px.kappa_s, px.kappa_s, px.kappa_s};
        } else if (EK - EK_ADJ_PROX == JKO_F_ENTROPY || EK - EK_ADJ_PROX == JKO_F_POROUS) {
            in.v = px.kf ? ld4(px.kf, idx, cnt, vec, 0.f) : f4{px.kf_s, px.kf_s, px.kf_s, px.kf_s};
        } else if (EK - EK_ADJ_PROX == JKO_F_GEN_ENTROPY) {
            in.v = px.kf ? ld4(px.kf, idx, cnt, vec, 0.f) : f4{px.kf_s, px.kf_s, px.kf_s, px.kf_s};
            in.w = px.g ? ld4(px.g, idx, cnt, vec, 0.f) : f4{px.eps_s, px.eps_s, px.eps_s, px.eps_s};
        }
    } else if (EK >= EK_PROX) {
        const ProxArgs& px = E.prox;
        if (EK - EK_PROX == JKO_F_CONGESTION || EK - EK_PROX == JKO_F_CONGESTION_BINARY) {
            in.u = px.g ? ld4(px.g, idx, cnt, vec, 1.f) : f4{1.f, 1.f, 1.f, 1.f};
            in.v = px.kappa ? ld4(px.kappa, idx, cnt, vec, 0.f)
                            : f4{px.kappa_s, px.kappa_s, px.kappa_s, px.kappa_s};
        } else if (EK - EK_PROX == JKO_F_ENTROPY || EK - EK_PROX == JKO_F_POROUS) {
            in.u = px.kf ? ld4(px.kf, idx, cnt, vec, 0.f) : f4{px.kf_s, px.kf_s, px.kf_s, px.kf_s};
        } else if (EK - EK_PROX == JKO_F_GEN_ENTROPY) {
            in.u = px.kf ? ld4(px.kf, idx, cnt, vec, 0.f) : f4{px.kf_s, px.kf_s, px.kf_s, px.kf_s};
            in.v = px.g ? ld4(px.g, idx, cnt, vec, 0.f) : f4{px.eps_s, px.eps_s, px.eps_s, px.eps_s};
        }
    }
    return in;
}

// Finish `cnt` consecutive outputs idx .. idx+cnt-1 of a contraction whose
// values are `val` (logs of the values when logx).  Plain domain:
//   STORE    y = v
//   BUPDATE  t = v; [err += |b_old t - q|]; b = q / t          (0/0 = 0)
//   MONITOR  err += |b t - q|
//   PROX     s = v; p = prox(s); a = p / s; [p_out = p]       (0/0 = 0)
// Log domain: the same with b, a held as log b, log a.
// COH: b (b-update) and a (prox) are stored with device-scope stores.
// NE: elements of `val` computed (cnt <= NE); 1 for one output per lane.
template <int EK, bool COH = false, int NE = 4>
__device__ __forceinline__ void epi_apply(const EpiArgs& E, int idx, int cnt, f4 val, bool logx,
                                          const EpiIn& in, EpiAcc& acc) {
    if (cnt <= 0) return;
    const bool vec = E.vec_ok && ((idx & 3) == 0);
    if (EK == EK_STORE) {
        st4(E.y, idx, cnt, vec, val);
    } else if (EK == EK_BUPDATE) {
        f4 bn;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const float q = in.u[e], t = val[e];
            if (logx) {
                bn[e] = (q == 0.f) ? -INFINITY : logf(q) - t;
                if (E.check && e < cnt) {
                    acc.err += fabs((double)expf(in.v[e] + t) - (double)q);
                    if (bn[e] > -INFINITY) acc.maxlb = fmax(acc.maxlb, fabs((double)bn[e]));
                }
            } else {
                bn[e] = (q == 0.f) ? 0.f : q / t;
                if (E.check && e < cnt) {
                    acc.err += fabs((double)in.v[e] * (double)t - (double)q);
                    if (bn[e] > 0.f) acc.maxlb = fmax(acc.maxlb, fabs((double)logf(bn[e])));
                }
            }
        }
        if (COH) st4_coh(E.b, idx, cnt, vec, bn);
        else st4(E.b, idx, cnt, vec, bn);
        if (E.t_out) st4(E.t_out, idx, cnt, vec, val);
    } else if (EK == EK_ADJ_B) {
        f4 tb, qb;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            float dq;
            tb[e] = adj_b_cell(in.u[e], in.v[e], val[e], &dq);
            qb[e] = (dq != 0.f) ? in.w[e] + dq : in.w[e];
        }
        if (COH) {
            st4_coh(E.y, idx, cnt, vec, tb);
            st4_coh(E.acc, idx, cnt, vec, qb);
        } else {
            st4(E.y, idx, cnt, vec, tb);
            st4(E.acc, idx, cnt, vec, qb);
        }
    } else if (EK >= EK_ADJ_PROX) {
        constexpr int KIND = EK - EK_ADJ_PROX;
        f4 sb, dw;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            float d;
            sb[e] = adj_prox_cell<KIND>(E.prox, E.sigma, in.u[e], 0.f, val[e], in.v[e], in.w[e], &d);
            dw[e] = d;
        }
        if (COH) st4_coh(E.y, idx, cnt, vec, sb);
        else st4(E.y, idx, cnt, vec, sb);
        if ((KIND == JKO_F_CONGESTION || KIND == JKO_F_GEN_ENTROPY) && E.acc) {
            f4 wb = COH ? ld4_coh(E.acc, idx, cnt, 0.f) : ld4(E.acc, idx, cnt, vec, 0.f);
#pragma unroll
            for (int e = 0; e < NE; ++e)
                if (dw[e] != 0.f) wb[e] += dw[e];
            if (COH) st4_coh(E.acc, idx, cnt, vec, wb);
            else st4(E.acc, idx, cnt, vec, wb);
        }
    } else if (EK == EK_MONITOR) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            if (e >= cnt) continue;
            const double bt = logx ? (double)expf(in.v[e] + val[e]) : (double)in.v[e] * (double)val[e];
            acc.err += fabs(bt - (double)in.u[e]);
        }
    } else {
        constexpr int KIND = EK - EK_PROX;
        constexpr bool kNewton = KIND == JKO_F_POROUS || KIND == JKO_F_GEN_ENTROPY;
        f4 an, pn, lpn;
        if constexpr (kNewton) {
            f4 ls;
#pragma unroll
            for (int e = 0; e < NE; ++e) ls[e] = logx ? val[e] : (val[e] > 0.f ? logf(val[e]) : -INFINITY);
            lpn = log_prox_cells<KIND, NE>(E.prox, ls, in.u, in.v);
        }
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            if (logx) {
                const float lp = kNewton ? lpn[e] : log_prox_val<KIND>(E.prox, val[e], in.u[e], in.v[e]);
                an[e] = (lp == -INFINITY) ? -INFINITY : lp - val[e];
                pn[e] = expf(lp);
                if (E.check && e < cnt && an[e] > -INFINITY) acc.maxla = fmax(acc.maxla, fabs((double)an[e]));
            } else {
                const float p = kNewton ? (val[e] > 0.f ? expf(lpn[e]) : 0.f)
                                        : prox_val<KIND>(E.prox, val[e], in.u[e], in.v[e]);
                pn[e] = p;
                an[e] = (p == 0.f) ? 0.f : p / val[e];
                if (E.check && e < cnt && an[e] > 0.f) acc.maxla = fmax(acc.maxla, fabs((double)logf(an[e])));
            }
            if (E.check && e < cnt) acc.mass += (double)pn[e];
        }
        if (COH) st4_coh(E.a, idx, cnt, vec, an);
        else st4(E.a, idx, cnt, vec, an);
        if (E.write_p) st4(E.p_out, idx, cnt, vec, pn);
        if (E.s_out) st4(E.s_out, idx, cnt, vec, val);
    }
}

// COH: the partials are stored with device-scope stores.
template <bool COH = false>
__device__ __forceinline__ void epi_finish(const EpiArgs& E, const EpiAcc& acc, int slot, double* sh) {
    if (E.kind == EpiKind::STORE) return;
    const bool want_err = (E.kind == EpiKind::MONITOR) || (E.kind == EpiKind::BUPDATE && E.check);
    const bool want_pm = (E.kind == EpiKind::PROX && E.check);
    if (want_err) {
        const double e = block_sum(acc.err, sh);
        const double mb = block_max(acc.maxlb, sh);
        if (threadIdx.x == 0) {
            if (COH) {
                __hip_atomic_store(E.part.err + slot, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(E.part.maxlogb + slot, mb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                E.part.err[slot] = e;
                E.part.maxlogb[slot] = mb;
            }
        }
    }
    if (want_pm) {
        const double ms = block_sum(acc.mass, sh);
        const double ma = block_max(acc.maxla, sh);
        if (threadIdx.x == 0) {
            if (COH) {
                __hip_atomic_store(E.part.mass + slot, ms, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(E.part.maxloga + slot, ma, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                E.part.mass[slot] = ms;
                E.part.maxloga[slot] = ma;
            }
        }
    }
}

}  // namespace jko
