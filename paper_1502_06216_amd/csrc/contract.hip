// Per-axis Gibbs contractions on MFMA for gfx950, with fused pointwise epilogues.
//
// The Gibbs kernel of a uniform grid with squared Euclidean cost is the
// Kronecker product of one-axis factors K1[i][k] = exp(-(x_i - x_k)^2/gamma)
// (the separable Gaussian of Section 4.1 of the paper), so xi x is d dense
// contractions of one axis each.  A pass contracts the contiguous axis of its
// input and writes the result with that axis moved to the front:
//     Y[i][r] = sum_k K1[i][k] X[r][k],     X: R x n (rows contiguous in k)
// After d passes the axes are back in their original order, and every pass
// reads rows with k contiguous, so both MFMA operands are plain row copies
// staged through LDS (no transposes).  The MFMA row dimension is r, so each
// lane ends with 4 consecutive r of one output row i: contiguous runs for the
// epilogue.
//
// In float32, K1[i][k] is exactly zero for |i - k| > W (exp underflows), so
// the K loop of an output tile covers only its band [i0 - W, i0 + TI + W):
// exact, and a large saving for small gamma.
//
// FP32 path: v_mfma_f32_16x16x4_f32.  Split path: each operand x = hi + lo in
// bfloat16 (round to nearest even); acc += lo*hi + hi*lo + hi*hi with
// v_mfma_f32_16x16x32_bf16, float32 accumulation.  LDS is double-buffered:
// the global loads of chunk c+1 are in flight while chunk c is multiplied,
// with one barrier per chunk.
//
// These passes run the plain domain only: after an absorption switch every
// product runs on the exact log-sum-exp passes of logpass.hip.
//
// 3D grids whose axes are multiples of 32 use two other kernels defined here,
// which keep the layout: a plane pass (axes 2 and 1 of each plane, the
// intermediate in LDS) and a slow-axis pass (axis 0, X staged transposed),
// with the same arithmetic in the same order as the three axis passes.
#include <math.h>

#include <algorithm>

#include "epilogue.h"
#include "panel.h"

namespace jko {

namespace {

// BK: k per chunk.  STAGES = 2: double-buffered chunks; STAGES = 1: the whole
// band of a tile fits in one chunk (loaded once, then multiplied).
template <int TR, int TI, int WR, int WI, bool SPLIT, int BK, int STAGES, int EK>
__global__ void __launch_bounds__(kThreads)
contract_rot(Pass P, EpiArgs E) {
    static_assert(WR * WI == 4, "four waves per block");
    constexpr int FM = TR / WR / 16;           // 16-row fragments per wave along r
    constexpr int FN = TI / WI / 16;           // 16-col fragments per wave along i
    static_assert(FM >= 1 && FN >= 1, "tile too small for the wave grid");
    static_assert(BK % (SPLIT ? 32 : 16) == 0, "chunk must hold whole MFMA k-steps");
    constexpr int SF = BK + 4;                 // FP32 LDS row (floats)
    constexpr int SB = BK + 8;                 // split LDS row (bf16)
    constexpr int NF = SPLIT ? 1 : STAGES * (TR + TI) * SF;
    constexpr int NB = SPLIT ? STAGES * (TR + TI) * SB : 1;
    __shared__ __attribute__((aligned(16))) float ldsf[NF];        // [stage][TR+TI][SF]
    __shared__ __attribute__((aligned(16))) uint16_t ldsh[NB];     // [stage][TR+TI][SB] hi
    __shared__ __attribute__((aligned(16))) uint16_t ldsl[NB];     //                    lo
    __shared__ double shd[8];

    // The control flags are read here but acted on only after the first chunk's
    // loads are in flight, so their latencies overlap.
    int done = 0;
    if (E.ctl) done = E.ctl->done | E.ctl->logmode;

    // EK_ATTR: paired tiles (pair_row)
    constexpr bool PAIR = EK == EK_ATTR;
    constexpr int TH = TR / 2;

    // Every field has at most 2^30 cells, so 32-bit element offsets suffice.
    const int n = P.n;
    const int R = (int)P.R;
    const int Rb = P.B > 1 ? R / P.B : R;
    const int IT = (n + TI - 1) / TI;
    const int logical = xcd_logical_block();
    const int r0 = (logical / IT) * (PAIR ? TH : TR);
    const int i0 = (logical % IT) * TI;
    // band of the output tile, start aligned down to 4 (the extra columns meet exact zeros)
    const int kb0 = max(0, i0 - P.W) & ~3;
    const int kb1 = min(n, i0 + TI + P.W);
    const int nch = (kb1 - kb0 + BK - 1) / BK;
    const bool vec = (n & 3) == 0;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave % WR, wi = wave / WR;

    // Staging: one unit = 4 consecutive k of one row.
    constexpr int UX = (TR * BK / 4 + kThreads - 1) / kThreads;
    constexpr int UK = (TI * BK / 4 + kThreads - 1) / kThreads;
    struct Regs {   // one chunk of X and K1 on its way from HBM to LDS
        f4 x[UX];
        f4 k[SPLIT ? 1 : UK];
        u16x4 kh[SPLIT ? UK : 1], kl[SPLIT ? UK : 1];
    };

    auto load = [&](int c, Regs& g) {
        const int kc = kb0 + c * BK;
#pragma unroll
        for (int u = 0; u < UX; ++u) {
            const int unit = tid + u * kThreads;
            f4 v = f4{0.f, 0.f, 0.f, 0.f};
            if (unit < TR * BK / 4) {
                const int d = unit / (BK / 4), k = kc + 4 * (unit % (BK / 4));
                const int row = PAIR ? pair_row(d, r0, Rb, TH) : r0 + d;
                if (PAIR ? r0 + (d < TH ? d : d - TH) < Rb : row < R) {
                    const float* src = P.X + (row * n + k);
                    if (vec && k + 3 < kb1) v = *reinterpret_cast<const f4*>(src);
                    else
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = (k + e < kb1) ? src[e] : 0.f;
                }
            }
            g.x[u] = v;
        }
#pragma unroll
        for (int u = 0; u < UK; ++u) {
            const int unit = tid + u * kThreads;
            const int d = unit / (BK / 4), k = kc + 4 * (unit % (BK / 4));
            const bool ok = unit < TI * BK / 4 && i0 + d < n;
            const int off = (i0 + d) * n + k;
            if (SPLIT) {
                u16x4 h = u16x4{0, 0, 0, 0}, l = u16x4{0, 0, 0, 0};
                if (ok) {
                    if (vec && k + 3 < kb1) {
                        h = *reinterpret_cast<const u16x4*>(P.K1hi + off);
                        l = *reinterpret_cast<const u16x4*>(P.K1lo + off);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            h[e] = (k + e < kb1) ? P.K1hi[off + e] : (uint16_t)0;
                            l[e] = (k + e < kb1) ? P.K1lo[off + e] : (uint16_t)0;
                        }
                    }
                }
                g.kh[u] = h;
                g.kl[u] = l;
            } else {
                f4 v = f4{0.f, 0.f, 0.f, 0.f};
                if (ok) {
                    if (vec && k + 3 < kb1) v = *reinterpret_cast<const f4*>(P.K1 + off);
                    else
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = (k + e < kb1) ? P.K1[off + e] : 0.f;
                }
                g.k[u] = v;
            }
        }
    };

    auto store = [&](int buf, const Regs& g) {
#pragma unroll
        for (int u = 0; u < UX; ++u) {
            const int unit = tid + u * kThreads;
            if (unit >= TR * BK / 4) continue;
            const int d = unit / (BK / 4), kq = unit % (BK / 4);
            const f4 v = g.x[u];
            if (SPLIT) {
                u16x4 h, l;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    h[e] = f2bf_rne(v[e]);
                    l[e] = f2bf_rne(v[e] - bf2f(h[e]));
                }
                const int o = (buf * (TR + TI) + d) * SB + 4 * kq;
                *reinterpret_cast<u16x4*>(&ldsh[o]) = h;
                *reinterpret_cast<u16x4*>(&ldsl[o]) = l;
            } else {
                *reinterpret_cast<f4*>(&ldsf[(buf * (TR + TI) + d) * SF + 4 * kq]) = v;
            }
        }
#pragma unroll
        for (int u = 0; u < UK; ++u) {
            const int unit = tid + u * kThreads;
            if (unit >= TI * BK / 4) continue;
            const int d = unit / (BK / 4), kq = unit % (BK / 4);
            if (SPLIT) {
                const int o = (buf * (TR + TI) + TR + d) * SB + 4 * kq;
                *reinterpret_cast<u16x4*>(&ldsh[o]) = g.kh[u];
                *reinterpret_cast<u16x4*>(&ldsl[o]) = g.kl[u];
            } else {
                *reinterpret_cast<f4*>(&ldsf[(buf * (TR + TI) + TR + d) * SF + 4 * kq]) = g.k[u];
            }
        }
    };

    f4 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

    auto compute = [&](int buf) {
        if (SPLIT) {
#pragma unroll
            for (int kk = 0; kk < BK / 32; ++kk) {
                const int koff = 32 * kk + 8 * (lane >> 4);
                bf8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
                for (int a = 0; a < FM; ++a) {
                    const int o = (buf * (TR + TI) + wr * 16 * FM + a * 16 + (lane & 15)) * SB + koff;
                    ah[a] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&ldsh[o]));
                    al[a] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&ldsl[o]));
                }
#pragma unroll
                for (int b = 0; b < FN; ++b) {
                    const int o = (buf * (TR + TI) + TR + wi * 16 * FN + b * 16 + (lane & 15)) * SB + koff;
                    bh[b] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&ldsh[o]));
                    bl[b] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&ldsl[o]));
                }
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b) {
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                    }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK / 16; ++kk) {
                const int koff = 16 * kk + 4 * (lane >> 4);
                f4 av[FM], bv[FN];
#pragma unroll
                for (int a = 0; a < FM; ++a)
                    av[a] = *reinterpret_cast<const f4*>(
                        &ldsf[(buf * (TR + TI) + wr * 16 * FM + a * 16 + (lane & 15)) * SF + koff]);
#pragma unroll
                for (int b = 0; b < FN; ++b)
                    bv[b] = *reinterpret_cast<const f4*>(
                        &ldsf[(buf * (TR + TI) + TR + wi * 16 * FN + b * 16 + (lane & 15)) * SF + koff]);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int a = 0; a < FM; ++a)
#pragma unroll
                        for (int b = 0; b < FN; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][s], bv[b][s], acc[a][b], 0, 0, 0);
            }
        }
    };

    // Epilogue: the accumulator tile goes through LDS as [i][r] rows, and each
    // thread finishes UE runs of 4 consecutive r of one output row i (row i of
    // the output tile is TR contiguous floats: coalesced loads and stores).
    // Their inputs are fetched now, before the K loop.
    constexpr int UE = (TI * TR / 4 + kThreads - 1) / kThreads;
    constexpr int TS = TR + 4;   // LDS row of the staged tile
    static_assert(TI * TS * 4 <= (SPLIT ? NB * 2 : NF * 4), "staged tile must fit in the staging LDS");
    EpiIn ein[UE];
    int eidx[UE], ecnt[UE];
    f4 kap[UE];   // EK_ATTR: the capacity of the unit's cells
    tile_units<TR, TI, UE, PAIR>(tid, i0, r0, n, R, Rb, eidx, ecnt);
    if (PAIR) {
        attr_capacity<UE>(E, eidx, ecnt, kap);
    } else {
#pragma unroll
        for (int u = 0; u < UE; ++u) ein[u] = epi_prefetch<EK>(E, eidx[u], ecnt[u]);
    }

    // The first chunks are in flight before the control flags are looked at.
    // Pipelined form: two register sets keep the loads of chunk c+2 in flight
    // while chunk c is multiplied and chunk c+1 is written to LDS.
    Regs ra, rb;
    load(0, ra);
    if (STAGES == 2 && nch > 1) load(1, rb);
    store(0, ra);
    if (done) return;   // the step has stopped: nothing to compute (uniform)
    __syncthreads();
    if (STAGES == 2) {
        for (int c = 0; c < nch; c += 2) {
            // chunk c in stage 0, rb holds chunk c+1, ra is free
            if (c + 2 < nch) load(c + 2, ra);
            compute(0);
            if (c + 1 < nch) store(1, rb);
            __syncthreads();
            if (c + 1 >= nch) break;
            // chunk c+1 in stage 1, ra holds chunk c+2, rb is free
            if (c + 3 < nch) load(c + 3, rb);
            compute(1);
            if (c + 2 < nch) store(0, ra);
            __syncthreads();
        }
    } else {
        for (int c = 0; c < nch; ++c) {
            if (c > 0) {
                load(c, ra);
                __syncthreads();
                store(0, ra);
                __syncthreads();
            }
            compute(0);
        }
    }

    // (the K loop ended on a barrier: the staging LDS is free)
    float* tile = SPLIT ? reinterpret_cast<float*>(ldsh) : ldsf;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int rl = wr * 16 * FM + a * 16 + 4 * (lane >> 4);
            const int il = wi * 16 * FN + b * 16 + (lane & 15);
            *reinterpret_cast<f4*>(&tile[il * TS + rl]) = acc[a][b];
        }
    __syncthreads();
    if (PAIR) {
        attr_finish<TR, TS, UE>(E, tile, tid, n, Rb, eidx, ecnt, kap);
        return;
    }
    EpiAcc ea;
#pragma unroll
    for (int u = 0; u < UE; ++u) {
        const int unit = tid + u * kThreads;
        const int il = unit / (TR / 4), rl = 4 * (unit % (TR / 4));
        if (ecnt[u] == 0) continue;
        const f4 v = *reinterpret_cast<const f4*>(&tile[il * TS + rl]);
        epi_apply<EK>(E, eidx[u], ecnt[u], v, false, ein[u], ea);
    }
    epi_finish(E, ea, (int)blockIdx.x, shd);
}

// Panel form (panel.h), for axes whose length is a multiple of 32.
template <int TR, int TI, int WR, int WI, bool SPLIT, int EK>
__global__ void __launch_bounds__(kThreads)
contract_panel(Pass P, EpiArgs E) {
    static_assert(WR * WI == 4, "four waves per block");
    constexpr int FM = TR / WR / 16;
    constexpr int FN = TI / WI / 16;
    static_assert(FM >= 1 && FN >= 1 && TR % 16 == 0 && TI % 16 == 0, "tile shape");
    extern __shared__ __attribute__((aligned(16))) float dyn[];
    __shared__ double shd[8];

    int done = 0;
    if (E.ctl) done = E.ctl->done | E.ctl->logmode;
    // EK_ATTR: paired tiles (pair_row)
    constexpr bool PAIR = EK == EK_ATTR;
    constexpr int TH = TR / 2;
    const int n = P.n;
    const int R = (int)P.R;
    const int Rb = P.B > 1 ? R / P.B : R;
    const int IT = n / TI;
    const int logical = xcd_logical_block();
    const int r0 = (logical / IT) * (PAIR ? TH : TR);
    const int i0 = (logical % IT) * TI;
    const int kb0 = panel_k0(i0, P.W);
    const int kb1 = panel_k1(i0, TI, P.W, n);
    const int NP = (kb1 - kb0) >> 5;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave % WR, wi = wave / WR;
    float* Xs = dyn;                                               // NP * TR * 32 floats
    float* Kf = dyn + NP * TR * 32;                                // NP * TI * 32 floats
    uint16_t* Kh = reinterpret_cast<uint16_t*>(dyn + NP * TR * 32);   // NP * TI * 32 bf16
    uint16_t* Kl = Kh + NP * TI * 32;

    // epilogue inputs first, then the staging copies; one wait covers both
    constexpr int UE = (TI * TR / 4 + kThreads - 1) / kThreads;
    EpiIn ein[UE];
    int eidx[UE], ecnt[UE];
    f4 kap[UE];   // EK_ATTR: the capacity of the unit's cells
    tile_units<TR, TI, UE, PAIR>(tid, i0, r0, n, R, Rb, eidx, ecnt);
    if (PAIR) {
        attr_capacity<UE>(E, eidx, ecnt, kap);
    } else {
#pragma unroll
        for (int u = 0; u < UE; ++u) ein[u] = epi_prefetch<EK>(E, eidx[u], ecnt[u]);
    }
    // Staging copies panel by panel (this wave's X rows of the panel, then its
    // K rows), CPP copies per wave and panel, so that panel p has landed once
    // at most (NP - 1 - p) * CPP of this wave's copies are outstanding.
    constexpr int XPP = TR / 8;                     // 8-row X copies per panel
    constexpr int KQ = SPLIT ? 2 * (TI / 16) : TI / 8;   // K copies per panel (hi and lo rows)
    static_assert(XPP % 4 == 0 && KQ % 4 == 0, "copies spread evenly over the four waves");
    constexpr int CPP = XPP / 4 + KQ / 4;
    static_assert((kPanelMaxRot - 1) * CPP <= 31, "per-panel wait counts fit wait_vm");
    {
        const __amdgpu_buffer_rsrc_t rx =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(P.X), (short)0, R * n * 4, kBufRsrcWord3);
        const __amdgpu_buffer_rsrc_t rk = __builtin_amdgcn_make_buffer_rsrc(
            SPLIT ? (void*)const_cast<uint16_t*>(P.K1hi) : (void*)const_cast<float*>(P.K1), (short)0,
            SPLIT ? n * n * 2 : n * n * 4, kBufRsrcWord3);
        const __amdgpu_buffer_rsrc_t rkl = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(SPLIT ? P.K1lo : P.K1hi), (short)0, n * n * 2, kBufRsrcWord3);
        // rows past R read as zeros; a paired tile's field-0 rows past Rb read
        // field-1 rows, which only reach outputs never written
        auto row_of = [&](int d) { return PAIR ? pair_row(d, r0, Rb, TH) : r0 + d; };
        for (int pnl = 0; pnl < NP; ++pnl) {
            const int kc = kb0 + 32 * pnl;
            panel_copy_x<TR, 0>(rx, Xs + pnl * TR * 32, n, kc, wave, lane, row_of);
            panel_copy_k<TI, SPLIT>(rk, rkl, Kf + pnl * TI * 32, Kh + pnl * TI * 32, Kl + pnl * TI * 32, n, i0, kc,
                                    wave, lane);
        }
    }
    if (done) {   // the step has stopped: nothing to compute (uniform)
        __builtin_amdgcn_s_waitcnt(0);
        return;
    }

    f4 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    for (int pnl = 0; pnl < NP; ++pnl) {
        // this panel's copies of every wave have landed (a bare barrier:
        // __syncthreads would first wait for every copy)
        wait_vm((NP - 1 - pnl) * CPP);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        panel_mma<TR, TI, WR, WI, SPLIT>(acc, Xs + pnl * TR * 32, Kf + pnl * TI * 32, Kh + pnl * TI * 32,
                                         Kl + pnl * TI * 32, lane, wr, wi);
    }
    __syncthreads();

    // epilogue through LDS as in contract_rot
    constexpr int TS = TR + 4;
    float* tile = dyn;
    panel_stage_acc<TR, TI, WR, WI>(tile, acc, lane, wr, wi);
    __syncthreads();
    if (PAIR) {
        attr_finish<TR, TS, UE>(E, tile, tid, n, Rb, eidx, ecnt, kap);
        return;
    }
    EpiAcc ea;
#pragma unroll
    for (int u = 0; u < UE; ++u) {
        const int unit = tid + u * kThreads;
        const int il = unit / (TR / 4), rl = 4 * (unit % (TR / 4));
        if (ecnt[u] == 0) continue;
        const f4 v = *reinterpret_cast<const f4*>(&tile[il * TS + rl]);
        epi_apply<EK>(E, eidx[u], ecnt[u], v, false, ein[u], ea);
    }
    epi_finish(E, ea, (int)blockIdx.x, shd);
}

// Tile configurations (TR, TI, WR, WI):
//  0: 32 x 32, 2 x 2 waves of one fragment, chunked K loop
//  1: 16 x 64, 1 x 4 waves (few rows: 1D grids)
//  2: 64 x 16, 4 x 1 waves (short axes)
//  3: 32 x 32 panel form (axes of a multiple of 32, band of at most 224 k)
//  4: 64 x 32 panel form, when it still leaves 4 blocks per CU (band of at
//     most 160 k)
// The chunked forms run K in 32-wide chunks through two LDS stages.
constexpr int kCfgTR[5] = {32, 16, 64, 32, 64};
constexpr int kCfgTI[5] = {32, 64, 16, 32, 32};
constexpr int64_t kPanelWideBlocks = 1024;

int64_t tiles_of(const Pass& p, int c) {
    return ((p.R + kCfgTR[c] - 1) / kCfgTR[c]) * (int64_t)((p.n + kCfgTI[c] - 1) / kCfgTI[c]);
}

// Panels of the widest tile band of the pass (0 if the panel form does not apply).
int panel_count(const Pass& p) {
    if (p.n % 32 != 0 || p.R * (int64_t)p.n * 4 >= ((int64_t)1 << 31)) return 0;
    int np = 0;
    for (int i0 = 0; i0 < p.n; i0 += 32) {
        const int kb0 = std::max(0, i0 - p.W) & ~31;
        const int kb1 = std::min(p.n, (i0 + 32 + p.W + 31) & ~31);
        np = std::max(np, (kb1 - kb0) >> 5);
    }
    return np <= kPanelMaxRot ? np : 0;
}

int pick_cfg(const Pass& p) {
    if (p.n <= 16) return 2;
    if (p.R <= 16) return 1;
    const int np = panel_count(p);
    if (np > 0) return (np <= kPanelMax && tiles_of(p, 4) >= kPanelWideBlocks) ? 4 : 3;
    return 0;
}

template <bool SPLIT, int EK>
hipError_t launch_cfg(int cfg, int64_t nb, const Pass& p, const EpiArgs& e, hipStream_t st) {
    const dim3 grid((unsigned)nb), block(kThreads);
    switch (cfg) {
        case 0: hipLaunchKernelGGL((contract_rot<32, 32, 2, 2, SPLIT, 32, 2, EK>), grid, block, 0, st, p, e); break;
        case 1: hipLaunchKernelGGL((contract_rot<16, 64, 1, 4, SPLIT, 32, 2, EK>), grid, block, 0, st, p, e); break;
        case 2: hipLaunchKernelGGL((contract_rot<64, 16, 4, 1, SPLIT, 32, 2, EK>), grid, block, 0, st, p, e); break;
        case 3:
            hipLaunchKernelGGL((contract_panel<32, 32, 2, 2, SPLIT, EK>), grid, block,
                               panel_lds_bytes(32, 32, panel_count(p)), st, p, e);
            break;
        default:
            hipLaunchKernelGGL((contract_panel<64, 32, 2, 2, SPLIT, EK>), grid, block,
                               panel_lds_bytes(64, 32, panel_count(p)), st, p, e);
            break;
    }
    return hipGetLastError();
}

template <bool SPLIT>
hipError_t launch_ek(int ek, int cfg, int64_t nb, const Pass& p, const EpiArgs& e, hipStream_t st) {
    switch (ek) {
        case EK_STORE: return launch_cfg<SPLIT, EK_STORE>(cfg, nb, p, e, st);
        case EK_BUPDATE: return launch_cfg<SPLIT, EK_BUPDATE>(cfg, nb, p, e, st);
        case EK_MONITOR: return launch_cfg<SPLIT, EK_MONITOR>(cfg, nb, p, e, st);
        case EK_PROX + JKO_F_ZERO: return launch_cfg<SPLIT, EK_PROX + JKO_F_ZERO>(cfg, nb, p, e, st);
        case EK_PROX + JKO_F_CONGESTION: return launch_cfg<SPLIT, EK_PROX + JKO_F_CONGESTION>(cfg, nb, p, e, st);
        case EK_PROX + JKO_F_CONGESTION_BINARY:
            return launch_cfg<SPLIT, EK_PROX + JKO_F_CONGESTION_BINARY>(cfg, nb, p, e, st);
        case EK_PROX + JKO_F_GEN_ENTROPY: return launch_cfg<SPLIT, EK_PROX + JKO_F_GEN_ENTROPY>(cfg, nb, p, e, st);
        case EK_PROX + JKO_F_POROUS: return launch_cfg<SPLIT, EK_PROX + JKO_F_POROUS>(cfg, nb, p, e, st);
        case EK_PROX + JKO_F_ENTROPY: return launch_cfg<SPLIT, EK_PROX + JKO_F_ENTROPY>(cfg, nb, p, e, st);
        case EK_ADJ_B: return launch_cfg<SPLIT, EK_ADJ_B>(cfg, nb, p, e, st);
        case EK_ADJ_PROX + JKO_F_ZERO: return launch_cfg<SPLIT, EK_ADJ_PROX + JKO_F_ZERO>(cfg, nb, p, e, st);
        case EK_ADJ_PROX + JKO_F_CONGESTION:
            return launch_cfg<SPLIT, EK_ADJ_PROX + JKO_F_CONGESTION>(cfg, nb, p, e, st);
        case EK_ADJ_PROX + JKO_F_POROUS: return launch_cfg<SPLIT, EK_ADJ_PROX + JKO_F_POROUS>(cfg, nb, p, e, st);
        case EK_ADJ_PROX + JKO_F_GEN_ENTROPY:
            return launch_cfg<SPLIT, EK_ADJ_PROX + JKO_F_GEN_ENTROPY>(cfg, nb, p, e, st);
        default: return launch_cfg<SPLIT, EK_ADJ_PROX + JKO_F_ENTROPY>(cfg, nb, p, e, st);
    }
}

// ---------------------------------------------------------------- 3D planes
//
// A 3D application of xi as a plane pass (axes 2 and 1 of each plane a, the
// intermediate kept in LDS) and a slow-axis pass (axis 0, with the epilogue),
// both keeping the layout [a][b][c].  The arithmetic is that of the three
// axis passes, in the same order: the plane pass's first stage is the axis-2
// pass (rows b, outputs c' in 32-wide chunks over their 32-aligned bands), its
// second stage the axis-1 pass on the staged intermediate (outputs b' in
// 32-wide chunks, one per wave, each over its own band), and the slow-axis
// pass is the axis-0 pass with X staged transposed.  Two launches per application instead of three, and one trip
// of the field through memory fewer.

constexpr int kPlaneMaxN1 = 128;             // one 16-row fragment of b per wave in the first stage
constexpr int kPlaneQ = kPlaneMaxN1 / 32;    // band panels of a b' chunk

__host__ __device__ inline int band_lo32(int i0, int W) { return (i0 - W > 0 ? i0 - W : 0) & ~31; }
__host__ __device__ inline int band_hi32(int i0, int W, int n) {
    const int h = (i0 + 32 + W + 31) & ~31;
    return h < n ? h : n;
}

// Dynamic LDS of the plane pass: the X and K2 panels of the block's band (the
// split K2 hi + lo take the bytes of the FP32 panels), later the intermediate.
int plane_lds_bytes(int n1, int NP) { return std::max(NP * (n1 + 32) * 128, 32 * (n1 + 4) * 4); }

constexpr int kPlaneWaves = 8;                 // 512 threads: two waves per SIMD per block
constexpr int kPlaneThr = 64 * kPlaneWaves;

template <bool SPLIT>
__global__ void __launch_bounds__(kPlaneThr)
plane_pass(Plane3D P) {
    extern __shared__ __attribute__((aligned(16))) float dyn[];

    int done = 0;
    if (P.ctl) done = P.ctl->done | P.ctl->logmode;
    const int n1 = P.n1, n2 = P.n2;
    const int chunks = n2 >> 5;
    const int logical = xcd_logical_block();
    const int a = logical / chunks, c0 = (logical % chunks) * 32;
    const int kb0 = band_lo32(c0, P.W2), kb1 = band_hi32(c0, P.W2, n2);
    const int NP = (kb1 - kb0) >> 5;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4;
    float* Xs = dyn;                                                   // [NP][n1][32]
    float* K2f = dyn + NP * n1 * 32;                                   // [NP][32][32]
    uint16_t* K2h = reinterpret_cast<uint16_t*>(dyn + NP * n1 * 32);   // [NP][32][32] bf16
    uint16_t* K2l = K2h + NP * 32 * 32;
    const int ZS = n1 + 4;
    float* Zt = dyn;                                                   // [32][ZS] after the first stage

    // Second stage: waves 2q and 2q + 1 share the 32-row chunk q of b', one
    // 16-row fragment each.  Their factor rows over the chunk's band are
    // fetched from global memory ahead of everything else.
    const int bq0 = 32 * (wave >> 1);
    const int bt = bq0 + 16 * (wave & 1);   // first b' of this wave's fragment
    const bool s2 = bq0 < n1;
    const int qb0 = s2 ? band_lo32(bq0, P.W1) : 0;
    const int NQ = s2 ? (band_hi32(bq0, P.W1, n1) - qb0) >> 5 : 0;
    f4 kq[kPlaneQ][2];
    bf8 kqh[kPlaneQ], kql[kPlaneQ];
#pragma unroll
    for (int q = 0; q < kPlaneQ; ++q) {
        if (q >= NQ) continue;
        const int row = bt + (lane & 15);
        const int kb = qb0 + 32 * q;
        if (SPLIT) {
            kqh[q] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(P.K1hi + row * n1 + kb + 8 * g));
            kql[q] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(P.K1lo + row * n1 + kb + 8 * g));
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h)
                kq[q][h] = *reinterpret_cast<const f4*>(P.K1 + row * n1 + kb + 4 * (4 * h + g));
        }
    }

    // First-stage staging: the plane's rows over the band, and the K2 rows of
    // the chunk (layout and swizzle of the panel form).
    {
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(P.X), (short)0, P.n0 * n1 * n2 * 4, kBufRsrcWord3);
        const __amdgpu_buffer_rsrc_t rk = __builtin_amdgcn_make_buffer_rsrc(
            SPLIT ? (void*)const_cast<uint16_t*>(P.K2hi) : (void*)const_cast<float*>(P.K2), (short)0,
            SPLIT ? n2 * n2 * 2 : n2 * n2 * 4, kBufRsrcWord3);
        const __amdgpu_buffer_rsrc_t rkl = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(SPLIT ? P.K2lo : P.K2hi), (short)0, n2 * n2 * 2, kBufRsrcWord3);
        const int xrow = lane >> 3, xch = lane & 7;
        const int krow = lane >> 2, kch = lane & 3;
        const int XC = n1 / 8;   // 8-row X copies per panel
        for (int j = wave; j < NP * XC; j += kPlaneWaves) {
            const int pnl = j / XC, row = (j % XC) * 8 + xrow;
            const int col = kb0 + 32 * pnl + 4 * (xch ^ ((row >> 1) & 7));
            lds_copy16(rx, Xs + j * 256, 4 * ((a * n1 + row) * n2 + col));
        }
        // K2: four copies per panel (FP32: 8 rows each; split: 16 rows of hi, then lo)
        for (int j = wave; j < NP * 4; j += kPlaneWaves) {
            const int pnl = j >> 2, q = j & 3;
            if (SPLIT) {
                const int qq = q & 1, row = qq * 16 + krow;
                const int col = kb0 + 32 * pnl + 8 * (kch ^ ((row >> 2) & 3));
                const int voff = 2 * ((c0 + row) * n2 + col);
                if (q < 2) lds_copy16(rk, K2h + (pnl * 2 + qq) * 512, voff);
                else lds_copy16(rkl, K2l + (pnl * 2 + qq) * 512, voff);
            } else {
                const int row = q * 8 + xrow;
                const int col = kb0 + 32 * pnl + 4 * (xch ^ ((row >> 1) & 7));
                lds_copy16(rk, K2f + j * 256, 4 * ((c0 + row) * n2 + col));
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    if (done) return;   // the step has stopped: nothing to compute (uniform)
    __syncthreads();

    // ---- first stage: Z[b][c'] = sum_c X[b][c] K2[c'][c]; wave w owns the
    // 16-row fragment w of b and both 16-column fragments of c'
    const int fb = wave;
    const bool s1 = fb < (n1 >> 4);
    const int s8 = (lane >> 1) & 7;
    f4 acc[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
    if (s1) {
        for (int pnl = 0; pnl < NP; ++pnl) {
            const float* xr = Xs + (pnl * n1 + fb * 16 + (lane & 15)) * 32;
            if (SPLIT) {
                const int s4 = (lane >> 2) & 3;
                bf8 ah, al, bh[2], bl[2];
                const f4 v0 = *reinterpret_cast<const f4*>(xr + 4 * ((2 * g) ^ s8));
                const f4 v1 = *reinterpret_cast<const f4*>(xr + 4 * ((2 * g + 1) ^ s8));
                split_bf16(v0, v1, ah, al);
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    const int o = (pnl * 32 + f * 16 + (lane & 15)) * 32 + 8 * (g ^ s4);
                    bh[f] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(K2h + o));
                    bl[f] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(K2l + o));
                }
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    acc[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[f], acc[f], 0, 0, 0);
                    acc[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[f], acc[f], 0, 0, 0);
                    acc[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[f], acc[f], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int ch = 4 * ((4 * h + g) ^ s8);
                    const f4 av = *reinterpret_cast<const f4*>(xr + ch);
                    f4 bv[2];
#pragma unroll
                    for (int f = 0; f < 2; ++f)
                        bv[f] = *reinterpret_cast<const f4*>(K2f + (pnl * 32 + f * 16 + (lane & 15)) * 32 + ch);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
#pragma unroll
                        for (int f = 0; f < 2; ++f)
                            acc[f] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[f][s], acc[f], 0, 0, 0);
                }
            }
        }
    }
    __syncthreads();   // every wave is done with the staged panels: the intermediate replaces them
    if (s1) {
        const int b = fb * 16 + 4 * g;
#pragma unroll
        for (int f = 0; f < 2; ++f) *reinterpret_cast<f4*>(&Zt[(f * 16 + (lane & 15)) * ZS + b]) = acc[f];
    }
    __syncthreads();

    // ---- second stage: Y[b'][c'] = sum_b K1[b'][b] Z[b][c'] over the band of
    // this wave's chunk of b' (rows of the MFMA: c'; columns: b')
    if (!s2) return;
    f4 acc2[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int q = 0; q < kPlaneQ; ++q) {
        if (q >= NQ) continue;
        const int kb = qb0 + 32 * q;
        if (SPLIT) {
            bf8 ah[2], al[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const float* zr = Zt + (f * 16 + (lane & 15)) * ZS + kb + 8 * g;
                const f4 v0 = *reinterpret_cast<const f4*>(zr);
                const f4 v1 = *reinterpret_cast<const f4*>(zr + 4);
                split_bf16(v0, v1, ah[f], al[f]);
            }
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                acc2[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[f], kqh[q], acc2[f], 0, 0, 0);
                acc2[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[f], kql[q], acc2[f], 0, 0, 0);
                acc2[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[f], kqh[q], acc2[f], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                f4 av[2];
#pragma unroll
                for (int f = 0; f < 2; ++f)
                    av[f] = *reinterpret_cast<const f4*>(Zt + (f * 16 + (lane & 15)) * ZS + kb + 4 * (4 * h + g));
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int f = 0; f < 2; ++f)
                        acc2[f] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[f][s], kq[q][h][s], acc2[f], 0, 0, 0);
            }
        }
    }
    // lane: c' = 16 f + 4 g + e, b' = bt + (lane & 15)
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const int cl = f * 16 + 4 * g;
        const int bp = bt + (lane & 15);
        __builtin_nontemporal_store(acc2[f], reinterpret_cast<f4*>(P.Y + ((int64_t)a * n1 + bp) * n2 + c0 + cl));
    }
}

// Slow-axis pass: Y[i][r] = sum_k K1[i][k] X[k][r] (X: n x R, rows contiguous
// in r), tiles of TR = 64 r x TI = 32 i, the MFMA rows r as in the panel form.
// The band's X rows are staged as [panel][32 k][64 r]; within a row the
// 16-byte chunk c of r is stored at c ^ (4 ((k >> 2) & 3)), so the operand
// reads of four k at once fall in distinct banks.
__device__ __forceinline__ int slow_pos(int k, int r) { return (((r >> 2) ^ (4 * ((k >> 2) & 3))) << 2) | (r & 3); }

template <bool SPLIT, int EK>
__global__ void __launch_bounds__(kThreads)
contract_slow(Pass P, EpiArgs E) {
    constexpr int TR = 64, TI = 32, WR = 2, WI = 2;
    constexpr int FM = TR / WR / 16;
    constexpr int FN = TI / WI / 16;
    extern __shared__ __attribute__((aligned(16))) float dyn[];
    __shared__ double shd[8];

    int done = 0;
    if (E.ctl) done = E.ctl->done | E.ctl->logmode;
    const int n = P.n;
    const int R = (int)P.R;
    const int IT = n / TI;
    const int logical = xcd_logical_block();
    const int r0 = (logical / IT) * TR;
    const int i0 = (logical % IT) * TI;
    const int kb0 = band_lo32(i0, P.W), kb1 = band_hi32(i0, P.W, n);
    const int NP = (kb1 - kb0) >> 5;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave % WR, wi = wave / WR;
    float* Xs = dyn;                                                   // NP * 32 * TR floats
    float* Kf = dyn + NP * TR * 32;                                    // NP * TI * 32 floats
    uint16_t* Kh = reinterpret_cast<uint16_t*>(dyn + NP * TR * 32);    // NP * TI * 32 bf16
    uint16_t* Kl = Kh + NP * TI * 32;

    constexpr int UE = (TI * TR / 4 + kThreads - 1) / kThreads;
    EpiIn ein[UE];
    int eidx[UE], ecnt[UE];
#pragma unroll
    for (int u = 0; u < UE; ++u) {
        const int unit = tid + u * kThreads;
        const int il = unit / (TR / 4), rl = 4 * (unit % (TR / 4));
        const int i = i0 + il, r = r0 + rl;
        ecnt[u] = (unit < TI * TR / 4 && i < n) ? max(0, min(4, R - r)) : 0;
        eidx[u] = i * R + r;
        ein[u] = epi_prefetch<EK, false, true>(E, eidx[u], ecnt[u]);   // whole tiles
    }
    {
        // copies issued untracked, K first, then X panel by panel: each
        // wave issues two X copies per panel, so panel p has landed for this
        // wave once at most 2 (NP - 1 - p) copies are outstanding
        const int xrow = lane >> 3, xch = lane & 7;
        if (SPLIT) {
            const i4v rh = buffer_desc(P.K1hi, n * n * 2), rl = buffer_desc(P.K1lo, n * n * 2);
            constexpr int KPP = TI / 16;
            const int nK = NP * KPP;
            const int kr = lane >> 2, kch = lane & 3;
            for (int j = wave; j < 2 * nK; j += kThreads / 64) {
                const int jj = j < nK ? j : j - nK;
                const int pnl = jj / KPP, row = (jj % KPP) * 16 + kr;
                const int col = kb0 + 32 * pnl + 8 * (kch ^ ((row >> 2) & 3));
                const int voff = 2 * ((i0 + row) * n + col);
                if (j < nK) lds_copy16_untracked(rh, Kh + jj * 512, voff);
                else lds_copy16_untracked(rl, Kl + jj * 512, voff);
            }
        } else {
            const i4v rk = buffer_desc(P.K1, n * n * 4);
            constexpr int KPP = TI / 8;
            for (int j = wave; j < NP * KPP; j += kThreads / 64) {
                const int pnl = j / KPP, row = (j % KPP) * 8 + xrow;
                const int col = kb0 + 32 * pnl + 4 * (xch ^ ((row >> 1) & 7));
                lds_copy16_untracked(rk, Kf + j * 256, 4 * ((i0 + row) * n + col));
            }
        }
        // X: 4 rows of 64 r per wave-wide copy; lane L fills position L & 15 of
        // row 4 j + (L >> 4) with the chunk that the swizzle puts there
        const i4v rx = buffer_desc(P.X, R * n * 4);
        const int krow = lane >> 4, pos = lane & 15;
        for (int j = wave; j < NP * 8; j += kThreads / 64) {
            const int pnl = j / 8, k = (j % 8) * 4 + krow;
            const int c = pos ^ (4 * ((k >> 2) & 3));
            lds_copy16_untracked(rx, Xs + j * 256, 4 * ((kb0 + 32 * pnl + k) * R + r0 + 4 * c));
        }
    }
    if (done) {   // the step has stopped: nothing to compute (uniform)
        __builtin_amdgcn_s_waitcnt(0);
        return;
    }

    f4 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    const int s8 = (lane >> 1) & 7;
    const int g = lane >> 4;
    for (int pnl = 0; pnl < NP; ++pnl) {
        // this panel's copies of every wave have landed
        wait_vm(2 * (NP - 1 - pnl));
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const float* xp = Xs + pnl * 32 * TR;
        if (SPLIT) {
            const int s4 = (lane >> 2) & 3;
            bf8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
            for (int a = 0; a < FM; ++a) {
                const int r = wr * 16 * FM + a * 16 + (lane & 15);
                f4 v0, v1;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v0[e] = xp[(8 * g + e) * TR + slow_pos(8 * g + e, r)];
                    v1[e] = xp[(8 * g + 4 + e) * TR + slow_pos(8 * g + 4 + e, r)];
                }
                split_bf16(v0, v1, ah[a], al[a]);
            }
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                const int o = (pnl * TI + wi * 16 * FN + b * 16 + (lane & 15)) * 32 + 8 * (g ^ s4);
                bh[b] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(Kh + o));
                bl[b] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(Kl + o));
            }
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int kk = 4 * (4 * h + g);
                const int ch = 4 * ((4 * h + g) ^ s8);
                f4 av[FM], bv[FN];
#pragma unroll
                for (int a = 0; a < FM; ++a) {
                    const int r = wr * 16 * FM + a * 16 + (lane & 15);
                    const int pr = slow_pos(kk, r);   // the same position in the four rows kk .. kk + 3
#pragma unroll
                    for (int s = 0; s < 4; ++s) av[a][s] = xp[(kk + s) * TR + pr];
                }
#pragma unroll
                for (int b = 0; b < FN; ++b)
                    bv[b] = *reinterpret_cast<const f4*>(
                        Kf + (pnl * TI + wi * 16 * FN + b * 16 + (lane & 15)) * 32 + ch);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int a = 0; a < FM; ++a)
#pragma unroll
                        for (int b = 0; b < FN; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][s], bv[b][s], acc[a][b], 0, 0, 0);
            }
        }
    }
    __syncthreads();

    // epilogue through LDS as in the panel form
    constexpr int TS = TR + 4;
    float* tile = dyn;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int rl = wr * 16 * FM + a * 16 + 4 * (lane >> 4);
            const int il = wi * 16 * FN + b * 16 + (lane & 15);
            *reinterpret_cast<f4*>(&tile[il * TS + rl]) = acc[a][b];
        }
    __syncthreads();
    // the prefetched inputs landed long ago; waiting for them here, before
    // any store, keeps the compiler from placing that wait after a store
    wait_vm_n<0>();
    EpiAcc ea;
#pragma unroll
    for (int u = 0; u < UE; ++u) {
        const int unit = tid + u * kThreads;
        const int il = unit / (TR / 4), rl = 4 * (unit % (TR / 4));
        if (ecnt[u] == 0) continue;
        const f4 v = *reinterpret_cast<const f4*>(&tile[il * TS + rl]);
        epi_apply<EK>(E, eidx[u], ecnt[u], v, false, ein[u], ea);
    }
    epi_finish(E, ea, (int)blockIdx.x, shd);
}

template <bool SPLIT>
hipError_t launch_slow_ek(int ek, int64_t nb, const Pass& p, const EpiArgs& e, int lds, hipStream_t st) {
    const dim3 grid((unsigned)nb), block(kThreads);
#define JKO_SLOW(EKV) hipLaunchKernelGGL((contract_slow<SPLIT, EKV>), grid, block, lds, st, p, e); break
    switch (ek) {
        case EK_STORE: JKO_SLOW(EK_STORE);
        case EK_BUPDATE: JKO_SLOW(EK_BUPDATE);
        case EK_MONITOR: JKO_SLOW(EK_MONITOR);
        case EK_PROX + JKO_F_ZERO: JKO_SLOW(EK_PROX + JKO_F_ZERO);
        case EK_PROX + JKO_F_CONGESTION: JKO_SLOW(EK_PROX + JKO_F_CONGESTION);
        case EK_PROX + JKO_F_CONGESTION_BINARY: JKO_SLOW(EK_PROX + JKO_F_CONGESTION_BINARY);
        case EK_PROX + JKO_F_GEN_ENTROPY: JKO_SLOW(EK_PROX + JKO_F_GEN_ENTROPY);
        case EK_PROX + JKO_F_POROUS: JKO_SLOW(EK_PROX + JKO_F_POROUS);
        case EK_PROX + JKO_F_ENTROPY: JKO_SLOW(EK_PROX + JKO_F_ENTROPY);
        case EK_ADJ_B: JKO_SLOW(EK_ADJ_B);
        case EK_ADJ_PROX + JKO_F_ZERO: JKO_SLOW(EK_ADJ_PROX + JKO_F_ZERO);
        case EK_ADJ_PROX + JKO_F_CONGESTION: JKO_SLOW(EK_ADJ_PROX + JKO_F_CONGESTION);
        case EK_ADJ_PROX + JKO_F_POROUS: JKO_SLOW(EK_ADJ_PROX + JKO_F_POROUS);
        case EK_ADJ_PROX + JKO_F_GEN_ENTROPY: JKO_SLOW(EK_ADJ_PROX + JKO_F_GEN_ENTROPY);
        default: JKO_SLOW(EK_ADJ_PROX + JKO_F_ENTROPY);
    }
#undef JKO_SLOW
    return hipGetLastError();
}

// Widest band (in 32-panels) of the 32-chunks of an axis of length n.
int band_panels(int n, int W) {
    int np = 0;
    for (int i0 = 0; i0 < n; i0 += 32) np = std::max(np, (band_hi32(i0, W, n) - band_lo32(i0, W)) >> 5);
    return np;
}

}  // namespace

int64_t contract_max_blocks(const Pass& pass, int32_t /*precision*/) { return tiles_of(pass, pick_cfg(pass)); }

bool plane3d_fits(int n0, int n1, int n2, int W0, int W1, int W2) {
    if (n0 % 32 != 0 || n1 % 32 != 0 || n2 % 32 != 0 || n1 > kPlaneMaxN1) return false;
    if ((int64_t)n0 * n1 * n2 * 4 >= ((int64_t)1 << 31)) return false;
    const int np2 = band_panels(n2, W2), np0 = band_panels(n0, W0);
    if (np2 > kPanelMax || np0 > kPanelMax || band_panels(n1, W1) > kPlaneQ) return false;
    // dynamic LDS within 64 KiB with the static arrays beside it
    return plane_lds_bytes(n1, np2) <= 65536 - 2048 && panel_lds_bytes(64, 32, np0) <= 65536 - 2048;
}

hipError_t launch_plane3d(const Plane3D& p, int32_t precision, int* nblocks, hipStream_t stream) {
    const int64_t nb = (int64_t)p.n0 * (p.n2 / 32);
    if (nblocks) *nblocks = (int)nb;
    const int lds = plane_lds_bytes(p.n1, band_panels(p.n2, p.W2));
    if (precision == JKO_SPLIT_BF16)
        hipLaunchKernelGGL(plane_pass<true>, dim3((unsigned)nb), dim3(kPlaneThr), lds, stream, p);
    else
        hipLaunchKernelGGL(plane_pass<false>, dim3((unsigned)nb), dim3(kPlaneThr), lds, stream, p);
    return hipGetLastError();
}

int64_t contract_slow_blocks(const Pass& pass) { return (pass.R / 64) * (int64_t)(pass.n / 32); }

hipError_t launch_contract_slow(const Pass& pass, int32_t precision, const EpiArgs& epi, int* nblocks,
                                hipStream_t stream) {
    // whole tiles only: every output group of four is complete
    if (pass.R % 64 != 0 || pass.n % 32 != 0) return hipErrorInvalidValue;
    const int64_t nb = contract_slow_blocks(pass);
    if (nblocks) *nblocks = (int)nb;
    if (nb <= 0) return hipSuccess;
    const int lds = panel_lds_bytes(64, 32, band_panels(pass.n, pass.W));
    if (precision == JKO_SPLIT_BF16) return launch_slow_ek<true>(ek_of(epi), nb, pass, epi, lds, stream);
    return launch_slow_ek<false>(ek_of(epi), nb, pass, epi, lds, stream);
}

hipError_t launch_contract(const Pass& pass, int32_t precision, const EpiArgs& epi, int* nblocks,
                           hipStream_t stream) {
    if (pass.B > 1 && (pass.R % pass.B != 0 || (pass.R / pass.B) % 4 != 0)) return hipErrorInvalidValue;
    if (epi.kind == EpiKind::ATTR_PROX) {
        // paired 32 x 32 tiles: the panel form where the band fits it, else
        // the chunked form
        if (pass.B != 2) return hipErrorInvalidValue;
        const int64_t nb = tiles_of(pass, 0);
        if (nblocks) *nblocks = (int)nb;
        const dim3 grid((unsigned)nb), block(kThreads);
        const int np = panel_count(pass);
        if (np > 0) {
            const int lds = panel_lds_bytes(32, 32, np);
            if (precision == JKO_SPLIT_BF16)
                hipLaunchKernelGGL((contract_panel<32, 32, 2, 2, true, EK_ATTR>), grid, block, lds, stream, pass, epi);
            else
                hipLaunchKernelGGL((contract_panel<32, 32, 2, 2, false, EK_ATTR>), grid, block, lds, stream, pass, epi);
        } else if (precision == JKO_SPLIT_BF16) {
            hipLaunchKernelGGL((contract_rot<32, 32, 2, 2, true, 32, 2, EK_ATTR>), grid, block, 0, stream, pass, epi);
        } else {
            hipLaunchKernelGGL((contract_rot<32, 32, 2, 2, false, 32, 2, EK_ATTR>), grid, block, 0, stream, pass, epi);
        }
        return hipGetLastError();
    }
    const int c = pick_cfg(pass);
    const int64_t nb = tiles_of(pass, c);
    if (nblocks) *nblocks = (int)nb;
    if (nb <= 0) return hipSuccess;
    const int ek = ek_of(epi);
    if (precision == JKO_SPLIT_BF16) return launch_ek<true>(ek, c, nb, pass, epi, stream);
    return launch_ek<false>(ek, c, nb, pass, epi, stream);
}

}  // namespace jko
