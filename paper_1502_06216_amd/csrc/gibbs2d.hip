// Fused 2D Gibbs application  Y = K1_0 X K1_1  on MFMA (gfx950), one launch.
//
// On a uniform 2D grid xi = K1_0 (x) K1_1 (separable Gaussian, Section 4.1 of
// the paper).  In float32 the factor K1[i][j] = exp(-(x_i - x_j)^2/gamma) is
// exactly zero beyond a band |i - j| > W (exp underflows), so the output tile
// Y[I][J] (16 x 16) only needs the input halo X[I +- W][J +- W]:
//     Z[ib][j] = sum_jb X[ib][jb] K1_1[j][jb]        (ib in I +- W, j in J)
//     Y[i][j]  = sum_ib K1_0[i][ib] Z[ib][j]
// Skipping the zero band is exact, and the intermediate Z never leaves LDS, so
// one application costs one launch instead of one per axis.  Each block owns
// one output tile; the tile order is XCD-aware so that neighbouring tiles,
// which share most of their halo, share an L2.
//
// Log domain (after the absorption switch): X holds log values; the halo rows
// are shifted by their maximum over the halo before the first contraction, Z
// is carried to the second in log form and re-shifted per output column, so
// each shift is local to the band around the outputs it serves.
#include <algorithm>

#include "epilogue.h"

namespace jko {

namespace {

constexpr int kT = 16;          // output tile edge
constexpr int kHalo = 128;      // largest halo edge held in LDS
constexpr int kS = kHalo + 4;   // padded LDS row (floats)

__device__ __forceinline__ int64_t xcd_block() {
    const int64_t nb = gridDim.x, bid = blockIdx.x;
    if (nb % 8 != 0) return bid;
    return (bid % 8) * (nb / 8) + bid / 8;
}

constexpr int kThr = 512;   // 8 waves per block

template <int EK>
__global__ void __launch_bounds__(kThr)
gibbs2d_f32(Band2D B, EpiArgs E) {
    __shared__ __attribute__((aligned(16))) float Xs[kHalo * kS];   // [ib][jb]
    __shared__ __attribute__((aligned(16))) float Kj[kT * kS];      // [j][jb]  = K1_1[j0+j][jb0+jb]
    __shared__ __attribute__((aligned(16))) float Ki[kT * kS];      // [i][ib]  = K1_0[i0+i][ib0+ib]
    __shared__ __attribute__((aligned(16))) float Zs[kT * kS];      // [j][ib]
    __shared__ float red[7 * 64 * 4];
    __shared__ float sh1[kHalo];     // log domain: row shifts of the halo
    __shared__ float sh2[kT];        // log domain: column shifts of Z
    __shared__ double shd[8];

    // The control flags are read here but acted on only after the halo loads
    // are in flight, so their latencies overlap.
    int done = 0, lmode = 0;
    if (E.ctl) {
        done = E.ctl->done;
        lmode = E.ctl->logmode;
    }

    const int n0 = B.n0, n1 = B.n1;
    const int tiles_j = (n1 + kT - 1) / kT;
    const int64_t logical = xcd_block();
    const int i0 = (int)(logical / tiles_j) * kT;
    const int j0 = (int)(logical % tiles_j) * kT;
    // halo, start aligned down to a multiple of 4 (the extra entries meet
    // exact zeros of the band)
    const int ib0 = max(0, i0 - B.W0) & ~3;
    const int ib1 = min(n0, i0 + kT + B.W0);
    const int jb0 = max(0, j0 - B.W1) & ~3;
    const int jb1 = min(n1, j0 + kT + B.W1);
    const int LI = ib1 - ib0, LJ = jb1 - jb0;
    const int LIp = (LI + 15) & ~15, LJp = (LJ + 15) & ~15;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool vec1 = (n1 & 3) == 0, vec0 = (n0 & 3) == 0;

    // Wave 0 finishes the tile: lane (i = lane & 15, j = 4 (lane >> 4) + e).
    // Its epilogue inputs are fetched now, ahead of the contraction.
    const int koff = 4 * (lane >> 4);
    const int oi = i0 + (lane & 15);
    const int obase = oi * n1 + j0 + koff;
    const int ocnt = (oi < n0) ? max(0, min(4, n1 - (j0 + koff))) : 0;
    EpiIn ein;
    if (wave == 0) ein = epi_prefetch<EK>(E, obase, ocnt);

    // ---- stage the halo of X and the two factor bands: every load is issued
    // before the first LDS store
    constexpr int UXM = kHalo * (kHalo / 4) / kThr;     // max halo units per thread
    constexpr int UKM = kT * (kHalo / 4) / kThr;        // max factor units per thread
    const int nux = LIp * (LJp / 4), nkj = kT * (LJp / 4), nki = kT * (LIp / 4);
    f4 bx[UXM], bj[UKM], bi[UKM];
#pragma unroll
    for (int u = 0; u < UXM; ++u) {
        const int unit = tid + u * kThr;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (unit < nux) {
            const int r = unit / (LJp / 4), c = 4 * (unit % (LJp / 4));
            if (r < LI) {
                const float* src = B.X + (int64_t)(ib0 + r) * n1 + jb0 + c;
                if (vec1 && c + 3 < LJ) v = *reinterpret_cast<const f4*>(src);
                else
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = (c + e < LJ) ? src[e] : 0.f;
            }
        }
        bx[u] = v;
    }
#pragma unroll
    for (int u = 0; u < UKM; ++u) {
        const int unit = tid + u * kThr;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (unit < nkj) {
            const int j = unit / (LJp / 4), c = 4 * (unit % (LJp / 4));
            if (j0 + j < n1) {
                const float* src = B.K1 + (int64_t)(j0 + j) * n1 + jb0 + c;
                if (vec1 && c + 3 < LJ) v = *reinterpret_cast<const f4*>(src);
                else
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = (c + e < LJ) ? src[e] : 0.f;
            }
        }
        bj[u] = v;
        f4 w = f4{0.f, 0.f, 0.f, 0.f};
        if (unit < nki) {
            const int i = unit / (LIp / 4), c = 4 * (unit % (LIp / 4));
            if (i0 + i < n0) {
                const float* src = B.K0 + (int64_t)(i0 + i) * n0 + ib0 + c;
                if (vec0 && c + 3 < LI) w = *reinterpret_cast<const f4*>(src);
                else
#pragma unroll
                    for (int e = 0; e < 4; ++e) w[e] = (c + e < LI) ? src[e] : 0.f;
            }
        }
        bi[u] = w;
    }
    const bool logx = lmode != 0;
#pragma unroll
    for (int u = 0; u < UXM; ++u) {
        const int unit = tid + u * kThr;
        if (unit < nux) {
            const int r = unit / (LJp / 4), c = 4 * (unit % (LJp / 4));
            f4 v = bx[u];
            if (logx)   // staged logs: cells outside the halo are exact zeros
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (r >= LI || c + e >= LJ) v[e] = -INFINITY;
            *reinterpret_cast<f4*>(&Xs[r * kS + c]) = v;
        }
    }
#pragma unroll
    for (int u = 0; u < UKM; ++u) {
        const int unit = tid + u * kThr;
        if (unit < nkj) {
            const int j = unit / (LJp / 4), c = 4 * (unit % (LJp / 4));
            *reinterpret_cast<f4*>(&Kj[j * kS + c]) = bj[u];
        }
        if (unit < nki) {
            const int i = unit / (LIp / 4), c = 4 * (unit % (LIp / 4));
            *reinterpret_cast<f4*>(&Ki[i * kS + c]) = bi[u];
        }
    }
    if (done) return;   // the step has stopped: nothing to compute (uniform)
    __syncthreads();

    if (logx) {
        // row shifts over the halo, then exponentiate the staged logs
        for (int r = tid; r < LIp; r += kThr) {
            float m = -INFINITY;
            for (int c = 0; c < LJ; ++c) m = fmaxf(m, Xs[r * kS + c]);
            sh1[r] = (m == -INFINITY) ? NAN : m;
        }
        __syncthreads();
        for (int u = tid; u < LIp * LJp; u += kThr) {
            const int r = u / LJp, c = u % LJp;
            const float m = sh1[r];
            Xs[r * kS + c] = (m == m) ? expf(Xs[r * kS + c] - m) : 0.f;
        }
        __syncthreads();
    }

    // ---- Z = X K1_1^T over the halo rows: wave f owns the 16-row fragment f;
    // even and odd k-chunks go to two accumulators (independent MFMA chains)
    const int F = LIp / 16;
    if (wave < F) {
        const int f = wave;
        f4 acc0 = f4{0.f, 0.f, 0.f, 0.f}, acc1 = f4{0.f, 0.f, 0.f, 0.f};
        const float* xr = &Xs[(16 * f + (lane & 15)) * kS + koff];
        const float* kr = &Kj[(lane & 15) * kS + koff];
        int c0 = 0;
        for (; c0 + 16 < LJp; c0 += 32) {
            const f4 a0 = *reinterpret_cast<const f4*>(xr + c0);
            const f4 b0 = *reinterpret_cast<const f4*>(kr + c0);
            const f4 a1 = *reinterpret_cast<const f4*>(xr + c0 + 16);
            const f4 b1 = *reinterpret_cast<const f4*>(kr + c0 + 16);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[s], b0[s], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[s], b1[s], acc1, 0, 0, 0);
            }
        }
        if (c0 < LJp) {
            const f4 a0 = *reinterpret_cast<const f4*>(xr + c0);
            const f4 b0 = *reinterpret_cast<const f4*>(kr + c0);
#pragma unroll
            for (int s = 0; s < 4; ++s) acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[s], b0[s], acc0, 0, 0, 0);
        }
        f4 acc = acc0 + acc1;
        // acc holds Z[ib = 16f + koff + e][j = lane & 15]
        if (logx) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float m = sh1[16 * f + koff + e];
                acc[e] = (m != m) ? -INFINITY : (acc[e] > 0.f ? m + logf(acc[e]) : m - 104.f);
            }
        }
        *reinterpret_cast<f4*>(&Zs[(lane & 15) * kS + 16 * f + koff]) = acc;
    }
    __syncthreads();

    if (logx) {
        // column shifts of Z over the valid halo rows, then exponentiate
        if (tid < kT) {
            float m = -INFINITY;
            for (int r = 0; r < LI; ++r) m = fmaxf(m, Zs[tid * kS + r]);
            sh2[tid] = (m == -INFINITY) ? NAN : m;
        }
        __syncthreads();
        for (int u = tid; u < kT * LIp; u += kThr) {
            const int j = u / LIp, r = u % LIp;
            const float m = sh2[j];
            Zs[j * kS + r] = (m == m && r < LI) ? expf(Zs[j * kS + r] - m) : 0.f;
        }
        __syncthreads();
    }

    // ---- Y^T = Z^T K1_0^T: one 16 x 16 fragment, its 16-wide k-chunks spread
    // over the waves (at most 8 chunks), partial sums combined in a fixed order
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    if (16 * wave < LIp) {
        const int c0 = 16 * wave;
        const f4 a = *reinterpret_cast<const f4*>(&Zs[(lane & 15) * kS + c0 + koff]);
        const f4 b = *reinterpret_cast<const f4*>(&Ki[(lane & 15) * kS + c0 + koff]);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], acc, 0, 0, 0);
    }
    if (wave > 0) *reinterpret_cast<f4*>(&red[((wave - 1) * 64 + lane) * 4]) = acc;
    __syncthreads();
    EpiAcc ea;
    if (wave == 0) {
#pragma unroll
        for (int w = 0; w < 7; ++w) acc += *reinterpret_cast<const f4*>(&red[(w * 64 + lane) * 4]);
        // acc holds Y[i = i0 + (lane & 15)][j = j0 + koff + e]
        if (logx) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float m = sh2[koff + e];
                acc[e] = (m != m) ? -INFINITY : (acc[e] > 0.f ? m + logf(acc[e]) : m - 104.f);
            }
        }
        epi_apply<EK>(E, obase, ocnt, acc, logx, ein, ea);
    }
    epi_finish(E, ea, (int)blockIdx.x, shd);
}

}  // namespace

int band_halfwidth(int n, double gamma) {
    // distances d with (d/n)^2/gamma > 152 ln 2 give exp(.) < 2^-152: zero in float32
    const double dmax = sqrt(152.0 * log(2.0) * gamma) * (double)n;
    const int W = (int)floor(dmax) + 1;
    return std::min(W, n - 1);
}

int64_t gibbs2d_blocks(int n0, int n1) {
    return (int64_t)((n0 + kT - 1) / kT) * ((n1 + kT - 1) / kT);
}

bool gibbs2d_fits(int n0, int n1, int W0, int W1) {
    // halo = tile + 2 W + 3 (alignment), rounded up to 16
    const int h0 = ((std::min(n0, kT + 2 * W0 + 3)) + 15) & ~15;
    const int h1 = ((std::min(n1, kT + 2 * W1 + 3)) + 15) & ~15;
    return h0 <= kHalo && h1 <= kHalo;
}

hipError_t launch_gibbs2d(const Band2D& b, int32_t precision, const EpiArgs& epi, int* nblocks,
                          hipStream_t stream) {
    (void)precision;
    const int64_t nb = gibbs2d_blocks(b.n0, b.n1);
    if (nblocks) *nblocks = (int)nb;
    const dim3 grid((unsigned)nb), block(kThr);
    switch (ek_of(epi)) {
        case EK_STORE: hipLaunchKernelGGL(gibbs2d_f32<EK_STORE>, grid, block, 0, stream, b, epi); break;
        case EK_BUPDATE: hipLaunchKernelGGL(gibbs2d_f32<EK_BUPDATE>, grid, block, 0, stream, b, epi); break;
        case EK_MONITOR: hipLaunchKernelGGL(gibbs2d_f32<EK_MONITOR>, grid, block, 0, stream, b, epi); break;
        case EK_PROX + JKO_F_ZERO:
            hipLaunchKernelGGL(gibbs2d_f32<EK_PROX + JKO_F_ZERO>, grid, block, 0, stream, b, epi); break;
        case EK_PROX + JKO_F_CONGESTION:
            hipLaunchKernelGGL(gibbs2d_f32<EK_PROX + JKO_F_CONGESTION>, grid, block, 0, stream, b, epi); break;
        case EK_PROX + JKO_F_POROUS:
            hipLaunchKernelGGL(gibbs2d_f32<EK_PROX + JKO_F_POROUS>, grid, block, 0, stream, b, epi); break;
        default: hipLaunchKernelGGL(gibbs2d_f32<EK_PROX + JKO_F_ENTROPY>, grid, block, 0, stream, b, epi); break;
    }
    return hipGetLastError();
}

}  // namespace jko
