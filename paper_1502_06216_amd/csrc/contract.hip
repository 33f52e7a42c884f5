// Per-axis Gibbs contractions on MFMA for gfx950, with fused pointwise epilogues.
//
// The Gibbs kernel of a uniform grid with squared Euclidean cost is the
// Kronecker product of one-axis factors K1[i][j] = exp(-(x_i - x_j)^2/gamma)
// (the separable Gaussian of Section 4.1 of the paper), so xi x is d dense
// contractions of one axis each.  Every contraction is a short-K GEMM
// (K = n <= 1024):
//   LAST  axis:  Y[r][i]    = sum_k X[r][k] K1[k][i]
//   OUTER axis:  Y[b][i][m] = sum_k K1[i][k] X[b][k][m]
// Both operands are staged through LDS as [dim][k] tiles (k contiguous, padded
// rows) so that every lane fetches its MFMA operands with one 16-byte LDS read.
// The MFMA "row" dimension is always mapped to the contiguous dimension of the
// output, so each lane ends with 4 (FP32 path) consecutive output elements and
// the epilogue works on contiguous runs.
//
// FP32 path: v_mfma_f32_16x16x4_f32.  Split path: each operand x = hi + lo in
// bfloat16 (round to nearest even); acc += hi*hi + hi*lo + lo*hi with
// v_mfma_f32_16x16x32_bf16, float32 accumulation.
//
// The last pass of a Gibbs application carries the pointwise work of the
// iteration (b = q / t with the marginal-violation partial sums, or the
// proximal map and a = p / s), so t and s never round-trip through HBM.
#include <float.h>
#include <math.h>

#include "epilogue.h"

namespace jko {

// ----------------------------------------------------------- tile mapping

template <int FM, int FN, int WM, int WN, int WK>
struct Cfg {
    static_assert(WM * WN * WK == 4, "four waves per block");
    static constexpr int TM = 16 * FM * WM;   // tile extent along the MFMA row (contiguous output) dim
    static constexpr int TN = 16 * FN * WN;   // tile extent along the MFMA column dim
};

struct TileCoord {
    int64_t batch, row0, col0;
};

// The hardware hands consecutive blocks to the 8 XCDs in turn; give each XCD
// a contiguous range of tiles so that tiles sharing an X strip share an L2.
__device__ __forceinline__ int64_t xcd_logical_block() {
    const int64_t nb = gridDim.x, bid = blockIdx.x;
    if (nb % 8 != 0) return bid;
    return (bid % 8) * (nb / 8) + bid / 8;
}

// OUTER: rows = m (tiles RT over M), cols = i (CT over n), batches B; col tile fastest.
// LAST : rows = i (RT over n), cols = r (CT over R); row tile fastest.
template <bool OUTER>
__device__ __forceinline__ TileCoord tile_of(int64_t logical, int64_t RT, int64_t CT) {
    TileCoord t;
    if (OUTER) {
        const int64_t ct = logical % CT;
        const int64_t rest = logical / CT;
        t.row0 = rest % RT;
        t.batch = rest / RT;
        t.col0 = ct;
    } else {
        t.row0 = logical % RT;
        t.col0 = logical / RT;
        t.batch = 0;
    }
    return t;
}

// Log domain: per-fibre shift M_f = max over the contracted axis of the log
// input, so that the contraction of exp(L - M_f) stays in float range and the
// output is M_f + log(sum).  Fibres of a block: OUTER the TM columns m of its
// row tile, LAST the TN rows r of its column tile.  Empty fibres get M_f = 0.
template <bool OUTER, int FIB>
__device__ void fibre_max(const float* __restrict__ X, int n, int64_t M, int64_t R, int64_t first,
                          float* fshift, float* scratch) {
    constexpr int G = kThreads / FIB;
    const int tid = threadIdx.x;
    float mx = -INFINITY;
    if (OUTER) {
        const int f = tid % FIB, g = tid / FIB;
        const int64_t m = first + f;
        if (m < M)
            for (int k = g; k < n; k += G) mx = fmaxf(mx, X[(int64_t)k * M + m]);
        scratch[g * FIB + f] = mx;
    } else {
        const int f = tid / G, g = tid % G;
        const int64_t r = first + f;
        if (r < R)
            for (int k = g; k < n; k += G) mx = fmaxf(mx, X[r * (int64_t)n + k]);
        scratch[g * FIB + f] = mx;
    }
    __syncthreads();
    if (tid < FIB) {
        float v = -INFINITY;
        for (int g = 0; g < G; ++g) v = fmaxf(v, scratch[g * FIB + tid]);
        fshift[tid] = (v == -INFINITY) ? NAN : v;   // NaN marks an all-zero fibre
    }
    __syncthreads();
}

// exp(L - shift) for a staged log input (an all-zero fibre stages zeros).
__device__ __forceinline__ float shifted_exp(float L, float shift) {
    return (shift == shift) ? expf(L - shift) : 0.f;
}

// log of a log-domain contraction output.  A non-empty fibre whose sum
// underflowed (every contribution below e^-87 of the fibre maximum) is held at
// the floor shift - 104 instead of -inf, so that b = q / t stays finite.
__device__ __forceinline__ float shifted_log(float acc, float shift) {
    if (shift != shift) return -INFINITY;
    return acc > 0.f ? shift + logf(acc) : shift - 104.f;
}

// ======================================================= FP32 MFMA kernel

template <int FM, int FN, int WM, int WN, int WK, bool OUTER>
__global__ void __launch_bounds__(kThreads)
contract_f32(Pass P, EpiArgs E) {
    using C = Cfg<FM, FN, WM, WN, WK>;
    constexpr int TM = C::TM, TN = C::TN;
    constexpr int BK = 16 * WK;        // k per chunk (each wave takes a 16-wide slice)
    constexpr int S = BK + 4;          // padded LDS row (floats): conflict-free 16-B reads
    __shared__ __attribute__((aligned(16))) float Ps[TM * S];   // MFMA A: [row][k]
    __shared__ __attribute__((aligned(16))) float Qs[TN * S];   // MFMA B: [col][k]
    __shared__ float red[(WK > 1) ? (WK - 1) * WM * WN * 64 * FM * FN * 4 : 1];
    __shared__ double sh[8];

    if (E.ctl && E.ctl->done) return;

    const int n = P.n;
    const int64_t rowsLim = OUTER ? P.M : (int64_t)n;
    const int64_t colsLim = OUTER ? (int64_t)n : P.R;
    const int64_t RT = (rowsLim + TM - 1) / TM;
    const int64_t CT = (colsLim + TN - 1) / TN;
    TileCoord tc = tile_of<OUTER>(xcd_logical_block(), RT, CT);
    const int64_t row0 = tc.row0 * TM, col0 = tc.col0 * TN;
    const float* __restrict__ K1 = P.K1;
    const float* __restrict__ X = P.X + (OUTER ? tc.batch * (int64_t)n * P.M : 0);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wk = wave / (WM * WN), wmn = wave % (WM * WN), wm = wmn % WM, wn = wmn / WM;

    // Log domain (after the absorption switch): inputs are logs, shifted per fibre.
    const bool logx = (E.ctl != nullptr) && (E.ctl->logmode != 0);
    constexpr int FIB = OUTER ? TM : TN;
    __shared__ float fshift[FIB];
    __shared__ float fscr[kThreads];
    if (logx) fibre_max<OUTER, FIB>(X, n, P.M, P.R, OUTER ? row0 : col0, fshift, fscr);
    const float xfill = logx ? -INFINITY : 0.f;

    f4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // Staging registers: one float4 unit = 4 consecutive k (direct) or 4 consecutive m (transposed).
    constexpr int UP = (TM * BK / 4 + kThreads - 1) / kThreads;
    constexpr int UQ = (TN * BK / 4 + kThreads - 1) / kThreads;
    f4 rp[UP], rq[UQ];

    // Direct tile loader: rows [base, base+D) of a row-major matrix G (ld = n
    // for K1 and for LAST-axis X), k in [k0, k0+BK).
    auto load_direct = [&](f4* r, const float* __restrict__ G, int64_t base, int64_t lim, int D,
                           int k0, int U, float fill) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int unit = tid + u * kThreads;
            f4 v = f4{fill, fill, fill, fill};
            if (unit < D * BK / 4) {
                const int d = unit / (BK / 4), kq = unit % (BK / 4);
                const int64_t row = base + d;
                const int k = k0 + 4 * kq;
                if (row < lim) {
                    const float* src = G + row * (int64_t)n + k;
                    if (k + 3 < n && ((n & 3) == 0)) {
                        v = *reinterpret_cast<const f4*>(src);
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) v[j] = (k + j < n) ? src[j] : fill;
                    }
                }
            }
            r[u] = v;
        }
    };
    auto store_direct = [&](const f4* r, float* L, int D, int U, bool xform) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int unit = tid + u * kThreads;
            if (unit < D * BK / 4) {
                const int d = unit / (BK / 4), kq = unit % (BK / 4);
                f4 v = r[u];
                if (xform) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) v[j] = shifted_exp(v[j], fshift[d]);
                }
                *reinterpret_cast<f4*>(&L[d * S + 4 * kq]) = v;
            }
        }
    };
    // Transposed loader (OUTER X): element (m, k) = X[k][m], units of 4 consecutive m.
    auto load_trans = [&](f4* r, int k0) {
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            const int unit = tid + u * kThreads;
            f4 v = f4{xfill, xfill, xfill, xfill};
            if (unit < TM * BK / 4) {
                const int mq = unit % (TM / 4), kk = unit / (TM / 4);
                const int k = k0 + kk;
                const int64_t m = row0 + 4 * mq;
                if (k < n) {
                    const float* src = X + (int64_t)k * P.M + m;
                    if (m + 3 < P.M && ((P.M & 3) == 0)) {
                        v = *reinterpret_cast<const f4*>(src);
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) v[j] = (m + j < P.M) ? src[j] : xfill;
                    }
                }
            }
            r[u] = v;
        }
    };
    auto store_trans = [&](const f4* r) {
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            const int unit = tid + u * kThreads;
            if (unit < TM * BK / 4) {
                const int mq = unit % (TM / 4), kk = unit / (TM / 4);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    Ps[(4 * mq + j) * S + kk] = logx ? shifted_exp(r[u][j], fshift[4 * mq + j]) : r[u][j];
            }
        }
    };
    auto load_chunk = [&](int k0) {
        if (OUTER) {
            load_trans(rp, k0);
            load_direct(rq, K1, col0, n, TN, k0, UQ, 0.f);
        } else {
            load_direct(rp, K1, row0, n, TM, k0, UP, 0.f);
            load_direct(rq, X, col0, P.R, TN, k0, UQ, xfill);
        }
    };
    auto store_chunk = [&]() {
        if (OUTER) store_trans(rp);
        else store_direct(rp, Ps, TM, UP, false);
        store_direct(rq, Qs, TN, UQ, !OUTER && logx);
    };

    const int nchunks = (n + BK - 1) / BK;
    load_chunk(0);
    for (int c = 0; c < nchunks; ++c) {
        __syncthreads();
        store_chunk();
        __syncthreads();
        if (c + 1 < nchunks) load_chunk((c + 1) * BK);
        f4 af[FM], bfr[FN];
        const int koff = 16 * wk + 4 * (lane >> 4);
#pragma unroll
        for (int i = 0; i < FM; ++i)
            af[i] = *reinterpret_cast<const f4*>(&Ps[(wm * 16 * FM + i * 16 + (lane & 15)) * S + koff]);
#pragma unroll
        for (int j = 0; j < FN; ++j)
            bfr[j] = *reinterpret_cast<const f4*>(&Qs[(wn * 16 * FN + j * 16 + (lane & 15)) * S + koff]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s], bfr[j][s], acc[i][j], 0, 0, 0);
    }

    // Split-K: waves wk > 0 hand their partial tiles to wave group 0.
    if (WK > 1) {
        __syncthreads();
        if (wk > 0) {
            float* dst = &red[(((wk - 1) * WM * WN + wmn) * 64 + lane) * FM * FN * 4];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) dst[(i * FN + j) * 4 + e] = acc[i][j][e];
        }
        __syncthreads();
        if (wk == 0) {
            for (int w = 1; w < WK; ++w) {
                const float* src = &red[(((w - 1) * WM * WN + wmn) * 64 + lane) * FM * FN * 4];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[i][j][e] += src[(i * FN + j) * 4 + e];
            }
        }
    }

    EpiAcc ea;
    if (wk == 0) {
        EpiIn ein[FM][FN];
        int64_t ebase[FM][FN];
        int ecnt[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int64_t row = row0 + wm * 16 * FM + i * 16 + 4 * (lane >> 4);
                const int64_t col = col0 + wn * 16 * FN + j * 16 + (lane & 15);
                int64_t left = rowsLim - row;
                ecnt[i][j] = (col < colsLim) ? (int)(left < 0 ? 0 : (left > 4 ? 4 : left)) : 0;
                // OUTER: element (b, i = col, m = row);  LAST: element (r = col, i = row)
                ebase[i][j] = OUTER ? tc.batch * (int64_t)n * P.M + col * P.M + row : col * (int64_t)n + row;
                ein[i][j] = epi_prefetch(E, ebase[i][j], ecnt[i][j]);
            }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                f4 v = acc[i][j];
                if (logx && ecnt[i][j] > 0) {
                    const int64_t row = row0 + wm * 16 * FM + i * 16 + 4 * (lane >> 4);
                    const int64_t col = col0 + wn * 16 * FN + j * 16 + (lane & 15);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int64_t fr = OUTER ? (row + e - row0) : (col - col0);
                        const float sh_ = fshift[(fr < FIB && fr >= 0) ? fr : 0];
                        v[e] = shifted_log(acc[i][j][e], sh_);
                    }
                }
                epi_apply(E, ebase[i][j], ecnt[i][j], v, logx, ein[i][j], ea);
            }
    }
    epi_finish(E, ea, (int)blockIdx.x, sh);
}

// ================================================= split-BF16 MFMA kernel

template <int FM, int FN, int WM, int WN, int WK, bool OUTER>
__global__ void __launch_bounds__(kThreads)
contract_split(Pass P, EpiArgs E) {
    using C = Cfg<FM, FN, WM, WN, WK>;
    constexpr int TM = C::TM, TN = C::TN;
    constexpr int BK = 32 * WK;          // k per chunk (a 32-wide slice per wave)
    constexpr int S = BK + 8;            // padded LDS row in bf16 elements
    __shared__ __attribute__((aligned(16))) uint16_t Ph[TM * S];
    __shared__ __attribute__((aligned(16))) uint16_t Pl[TM * S];
    __shared__ __attribute__((aligned(16))) uint16_t Qh[TN * S];
    __shared__ __attribute__((aligned(16))) uint16_t Ql[TN * S];
    __shared__ float red[(WK > 1) ? (WK - 1) * WM * WN * 64 * FM * FN * 4 : 1];
    __shared__ double sh[8];

    if (E.ctl && E.ctl->done) return;

    const int n = P.n;
    const int64_t rowsLim = OUTER ? P.M : (int64_t)n;
    const int64_t colsLim = OUTER ? (int64_t)n : P.R;
    const int64_t RT = (rowsLim + TM - 1) / TM;
    const int64_t CT = (colsLim + TN - 1) / TN;
    TileCoord tc = tile_of<OUTER>(xcd_logical_block(), RT, CT);
    const int64_t row0 = tc.row0 * TM, col0 = tc.col0 * TN;
    const float* __restrict__ X = P.X + (OUTER ? tc.batch * (int64_t)n * P.M : 0);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wk = wave / (WM * WN), wmn = wave % (WM * WN), wm = wmn % WM, wn = wmn / WM;

    const bool logx = (E.ctl != nullptr) && (E.ctl->logmode != 0);
    constexpr int FIB = OUTER ? TM : TN;
    __shared__ float fshift[FIB];
    __shared__ float fscr[kThreads];
    if (logx) fibre_max<OUTER, FIB>(X, n, P.M, P.R, OUTER ? row0 : col0, fshift, fscr);
    const float xfill = logx ? -INFINITY : 0.f;

    f4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // X staging: float4 units (split on store); K1 staging: 4 bf16 (hi and lo) units.
    constexpr int UX = ((OUTER ? TM : TN) * BK / 4 + kThreads - 1) / kThreads;
    constexpr int UK = ((OUTER ? TN : TM) * BK / 4 + kThreads - 1) / kThreads;
    f4 rx[UX];
    u16x4 rkh[UK], rkl[UK];
    uint16_t* Xh = OUTER ? Ph : Qh;
    uint16_t* Xl = OUTER ? Pl : Ql;
    uint16_t* Kh = OUTER ? Qh : Ph;
    uint16_t* Kl = OUTER ? Ql : Pl;
    const int DX = OUTER ? TM : TN;
    const int DK = OUTER ? TN : TM;
    const int64_t kbase = OUTER ? col0 : row0;

    auto load_k1 = [&](int k0) {
#pragma unroll
        for (int u = 0; u < UK; ++u) {
            const int unit = tid + u * kThreads;
            u16x4 h = u16x4{0, 0, 0, 0}, l = u16x4{0, 0, 0, 0};
            if (unit < DK * BK / 4) {
                const int d = unit / (BK / 4), kq = unit % (BK / 4);
                const int64_t row = kbase + d;
                const int k = k0 + 4 * kq;
                if (row < n) {
                    const uint16_t* sh_ = P.K1hi + row * (int64_t)n + k;
                    const uint16_t* sl_ = P.K1lo + row * (int64_t)n + k;
                    if (k + 3 < n && ((n & 3) == 0)) {
                        h = *reinterpret_cast<const u16x4*>(sh_);
                        l = *reinterpret_cast<const u16x4*>(sl_);
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            h[j] = (k + j < n) ? sh_[j] : (uint16_t)0;
                            l[j] = (k + j < n) ? sl_[j] : (uint16_t)0;
                        }
                    }
                }
            }
            rkh[u] = h;
            rkl[u] = l;
        }
    };
    auto store_k1 = [&]() {
#pragma unroll
        for (int u = 0; u < UK; ++u) {
            const int unit = tid + u * kThreads;
            if (unit < DK * BK / 4) {
                const int d = unit / (BK / 4), kq = unit % (BK / 4);
                *reinterpret_cast<u16x4*>(&Kh[d * S + 4 * kq]) = rkh[u];
                *reinterpret_cast<u16x4*>(&Kl[d * S + 4 * kq]) = rkl[u];
            }
        }
    };
    auto load_x = [&](int k0) {
#pragma unroll
        for (int u = 0; u < UX; ++u) {
            const int unit = tid + u * kThreads;
            f4 v = f4{xfill, xfill, xfill, xfill};
            if (unit < DX * BK / 4) {
                if (OUTER) {
                    const int mq = unit % (TM / 4), kk = unit / (TM / 4);
                    const int k = k0 + kk;
                    const int64_t m = row0 + 4 * mq;
                    if (k < n) {
                        const float* src = X + (int64_t)k * P.M + m;
                        if (m + 3 < P.M && ((P.M & 3) == 0)) v = *reinterpret_cast<const f4*>(src);
                        else
#pragma unroll
                            for (int j = 0; j < 4; ++j) v[j] = (m + j < P.M) ? src[j] : xfill;
                    }
                } else {
                    const int d = unit / (BK / 4), kq = unit % (BK / 4);
                    const int64_t row = col0 + d;
                    const int k = k0 + 4 * kq;
                    if (row < P.R) {
                        const float* src = X + row * (int64_t)n + k;
                        if (k + 3 < n && ((n & 3) == 0)) v = *reinterpret_cast<const f4*>(src);
                        else
#pragma unroll
                            for (int j = 0; j < 4; ++j) v[j] = (k + j < n) ? src[j] : xfill;
                    }
                }
            }
            rx[u] = v;
        }
    };
    auto store_x = [&]() {
#pragma unroll
        for (int u = 0; u < UX; ++u) {
            const int unit = tid + u * kThreads;
            if (unit < DX * BK / 4) {
                f4 x = rx[u];
                if (logx) {
                    if (OUTER) {
                        const int mq = unit % (TM / 4);
#pragma unroll
                        for (int j = 0; j < 4; ++j) x[j] = shifted_exp(x[j], fshift[4 * mq + j]);
                    } else {
                        const int d = unit / (BK / 4);
#pragma unroll
                        for (int j = 0; j < 4; ++j) x[j] = shifted_exp(x[j], fshift[d]);
                    }
                }
                u16x4 h, l;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    h[j] = f2bf_rne(x[j]);
                    l[j] = f2bf_rne(x[j] - bf2f(h[j]));
                }
                if (OUTER) {
                    const int mq = unit % (TM / 4), kk = unit / (TM / 4);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        Xh[(4 * mq + j) * S + kk] = h[j];
                        Xl[(4 * mq + j) * S + kk] = l[j];
                    }
                } else {
                    const int d = unit / (BK / 4), kq = unit % (BK / 4);
                    *reinterpret_cast<u16x4*>(&Xh[d * S + 4 * kq]) = h;
                    *reinterpret_cast<u16x4*>(&Xl[d * S + 4 * kq]) = l;
                }
            }
        }
    };

    const int nchunks = (n + BK - 1) / BK;
    load_k1(0);
    load_x(0);
    for (int c = 0; c < nchunks; ++c) {
        __syncthreads();
        store_k1();
        store_x();
        __syncthreads();
        if (c + 1 < nchunks) {
            load_k1((c + 1) * BK);
            load_x((c + 1) * BK);
        }
        const int koff = 32 * wk + 8 * (lane >> 4);
        bf8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const int r = (wm * 16 * FM + i * 16 + (lane & 15)) * S + koff;
            ah[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Ph[r]));
            al[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Pl[r]));
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int r = (wn * 16 * FN + j * 16 + (lane & 15)) * S + koff;
            bh[j] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Qh[r]));
            bl[j] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Ql[r]));
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
    }

    if (WK > 1) {
        __syncthreads();
        if (wk > 0) {
            float* dst = &red[(((wk - 1) * WM * WN + wmn) * 64 + lane) * FM * FN * 4];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) dst[(i * FN + j) * 4 + e] = acc[i][j][e];
        }
        __syncthreads();
        if (wk == 0) {
            for (int w = 1; w < WK; ++w) {
                const float* src = &red[(((w - 1) * WM * WN + wmn) * 64 + lane) * FM * FN * 4];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[i][j][e] += src[(i * FN + j) * 4 + e];
            }
        }
    }

    EpiAcc ea;
    if (wk == 0) {
        EpiIn ein[FM][FN];
        int64_t ebase[FM][FN];
        int ecnt[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int64_t row = row0 + wm * 16 * FM + i * 16 + 4 * (lane >> 4);
                const int64_t col = col0 + wn * 16 * FN + j * 16 + (lane & 15);
                int64_t left = rowsLim - row;
                ecnt[i][j] = (col < colsLim) ? (int)(left < 0 ? 0 : (left > 4 ? 4 : left)) : 0;
                // OUTER: element (b, i = col, m = row);  LAST: element (r = col, i = row)
                ebase[i][j] = OUTER ? tc.batch * (int64_t)n * P.M + col * P.M + row : col * (int64_t)n + row;
                ein[i][j] = epi_prefetch(E, ebase[i][j], ecnt[i][j]);
            }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                f4 v = acc[i][j];
                if (logx && ecnt[i][j] > 0) {
                    const int64_t row = row0 + wm * 16 * FM + i * 16 + 4 * (lane >> 4);
                    const int64_t col = col0 + wn * 16 * FN + j * 16 + (lane & 15);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int64_t fr = OUTER ? (row + e - row0) : (col - col0);
                        const float sh_ = fshift[(fr < FIB && fr >= 0) ? fr : 0];
                        v[e] = shifted_log(acc[i][j][e], sh_);
                    }
                }
                epi_apply(E, ebase[i][j], ecnt[i][j], v, logx, ein[i][j], ea);
            }
    }
    epi_finish(E, ea, (int)blockIdx.x, sh);
}

// ================================================================ launcher

namespace {

struct Shape {
    int64_t rows, cols, batch;
};

Shape shape_of(const Pass& p) {
    if (p.form == Form::OUTER) return Shape{p.M, (int64_t)p.n, p.B};
    return Shape{(int64_t)p.n, p.R, 1};
}

int64_t tiles(const Shape& s, int TM, int TN) {
    return ((s.rows + TM - 1) / TM) * ((s.cols + TN - 1) / TN) * s.batch;
}

// Tile configurations, largest first: (FM, FN, WM, WN, WK).
//  0: 64 x 64 tile, 2x2 waves of 2x2 fragments
//  1: 32 x 32 tile, 2x2 waves of 1 fragment
//  2: 32 x 32 tile, 1 wave-plane of 2x2 fragments, 4-way split K
//  3: 16 x 16 tile, 4-way split K
constexpr int kCfgTM[4] = {64, 32, 32, 16};
constexpr int kCfgTN[4] = {64, 32, 32, 16};

// Pick the largest tile that still gives every CU (256) a couple of blocks.
int pick_cfg(const Shape& s) {
    const int64_t want = 512;
    for (int c = 0; c < 4; ++c)
        if (tiles(s, kCfgTM[c], kCfgTN[c]) >= want) return c;
    return (tiles(s, 32, 32) >= 256) ? 2 : 3;
}

template <bool OUTER>
hipError_t launch_f32(int cfg, int64_t nb, const Pass& p, const EpiArgs& e, hipStream_t st) {
    dim3 grid((unsigned)nb), block(kThreads);
    switch (cfg) {
        case 0: hipLaunchKernelGGL((contract_f32<2, 2, 2, 2, 1, OUTER>), grid, block, 0, st, p, e); break;
        case 1: hipLaunchKernelGGL((contract_f32<1, 1, 2, 2, 1, OUTER>), grid, block, 0, st, p, e); break;
        case 2: hipLaunchKernelGGL((contract_f32<2, 2, 1, 1, 4, OUTER>), grid, block, 0, st, p, e); break;
        default: hipLaunchKernelGGL((contract_f32<1, 1, 1, 1, 4, OUTER>), grid, block, 0, st, p, e); break;
    }
    return hipGetLastError();
}

template <bool OUTER>
hipError_t launch_split(int cfg, int64_t nb, const Pass& p, const EpiArgs& e, hipStream_t st) {
    dim3 grid((unsigned)nb), block(kThreads);
    switch (cfg) {
        case 0: hipLaunchKernelGGL((contract_split<2, 2, 2, 2, 1, OUTER>), grid, block, 0, st, p, e); break;
        case 1: hipLaunchKernelGGL((contract_split<1, 1, 2, 2, 1, OUTER>), grid, block, 0, st, p, e); break;
        case 2: hipLaunchKernelGGL((contract_split<2, 2, 1, 1, 4, OUTER>), grid, block, 0, st, p, e); break;
        default: hipLaunchKernelGGL((contract_split<1, 1, 1, 1, 4, OUTER>), grid, block, 0, st, p, e); break;
    }
    return hipGetLastError();
}

}  // namespace

int64_t contract_max_blocks(const Pass& pass, int32_t /*precision*/) {
    const Shape s = shape_of(pass);
    const int c = pick_cfg(s);
    return tiles(s, kCfgTM[c], kCfgTN[c]);
}

hipError_t launch_contract(const Pass& pass, int32_t precision, const EpiArgs& epi, int* nblocks,
                           hipStream_t stream) {
    const Shape s = shape_of(pass);
    const int c = pick_cfg(s);
    const int64_t nb = tiles(s, kCfgTM[c], kCfgTN[c]);
    if (nblocks) *nblocks = (int)nb;
    if (nb <= 0) return hipSuccess;
    const bool outer = pass.form == Form::OUTER;
    if (precision == JKO_SPLIT_BF16)
        return outer ? launch_split<true>(c, nb, pass, epi, stream) : launch_split<false>(c, nb, pass, epi, stream);
    return outer ? launch_f32<true>(c, nb, pass, epi, stream) : launch_f32<false>(c, nb, pass, epi, stream);
}

}  // namespace jko
