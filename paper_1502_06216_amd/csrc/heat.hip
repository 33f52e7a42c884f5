// Heat-kernel Gibbs operator (Section 4.1, eq. heat-kernel) on a masked 2D
// grid: construction of the dense operator and its application with the
// scaling iteration's pointwise epilogues.
//
// The paper applies xi~ = (Id - (gamma/L) Delta_M)^{-L} by L sparse
// back-substitutions per product, a sequential sweep.  On this device the
// operator of a grid of up to 2^16 cells fits HBM as a dense float32 matrix,
// so it is built once per (domain, gamma, L), and every product of the
// iteration becomes one memory-bound pass over it whose tiles run in
// parallel.  The operator acts on the free cells only, and only its upper
// triangle is stored (xi~ is symmetric): the 9556 free cells of a 100 x 100
// room take 187 MB, which fits the device's 256 MB last-level cache.
//
// Grids of more than 2^16 cells (or on request) take the paper's own form
// instead: each product is L successive solves of (Id - (gamma/L) Delta_M) y
// = rhs on the grid, by the same Chebyshev iteration in FP64 with one vector
// (a stencil sweep per iteration, linear in the grid's size), and its result
// goes through the same epilogues.  No operator is stored.
//
// Construction: the columns of xi~ are L successive solves of
// M x = rhs, M = Id + nu_0 G_0 + nu_1 G_1, from unit vectors, all columns of
// a chunk at once (C columns, element (cell i, column c) at i*C + c, so the
// five-point stencil reads whole rows of C consecutive doubles).  M is
// symmetric with spectrum in [1, 1 + 4 nu_0 + 4 nu_1] (Gershgorin; G_k is
// positive semi-definite), so each solve is a Chebyshev iteration
// (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 12.1)
// with no inner products: one stencil sweep per iteration, in FP64.
#include <algorithm>

#include "heat.h"
#include "epilogue.h"

namespace jko {

static_assert(HEAT_EK_STORE == EK_STORE && HEAT_EK_BUPDATE == EK_BUPDATE && HEAT_EK_MONITOR == EK_MONITOR &&
                  HEAT_EK_PROX == EK_PROX,
              "heat epilogue codes follow the band contractions' codes");

namespace {

__device__ __forceinline__ bool is_free(const uint8_t* mask, int64_t i) { return !mask || mask[i]; }

// (M x)_(i, c) over a chunk: x_i + sum over free neighbours j of nu_k (x_i - x_j)
// for a free cell; x_i (zero) for an obstacle.
__device__ __forceinline__ double heat_mx(const double* __restrict__ x, const uint8_t* __restrict__ mask,
                                          int64_t i, int64_t e, int C, int n0, int n1, double nu0, double nu1) {
    const double xi = x[e];
    if (!is_free(mask, i)) return xi;
    const int r = (int)(i / n1), col = (int)(i - (int64_t)r * n1);
    double acc = xi;
    if (r > 0 && is_free(mask, i - n1)) acc += nu0 * (xi - x[e - (int64_t)n1 * C]);
    if (r + 1 < n0 && is_free(mask, i + n1)) acc += nu0 * (xi - x[e + (int64_t)n1 * C]);
    if (col > 0 && is_free(mask, i - 1)) acc += nu1 * (xi - x[e - C]);
    if (col + 1 < n1 && is_free(mask, i + 1)) acc += nu1 * (xi - x[e + C]);
    return acc;
}

// X = the unit columns of free cells j0 .. j0+C-1 (grid cell gidx[j]; none
// at or beyond nf).
__global__ void k_heat_unit(double* __restrict__ X, const int32_t* __restrict__ gidx, int64_t nf, int64_t N,
                            int logC, int64_t j0) {
    const int64_t n = N << logC;
    const int C = 1 << logC;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e >> logC;
        const int64_t j = j0 + (e & (C - 1));
        X[e] = (j < nf && i == gidx[j]) ? 1.0 : 0.0;
    }
}

// Start of one solve with right-hand side and first guess X:
// R = X - M X, D = R / theta.
__global__ void k_heat_cheb_init(const double* __restrict__ X, double* __restrict__ R, double* __restrict__ D,
                                 const uint8_t* __restrict__ mask, int64_t N, int logC, int n0, int n1,
                                 double nu0, double nu1, double inv_theta) {
    const int64_t n = N << logC;
    const int C = 1 << logC;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e >> logC;
        const double r = X[e] - heat_mx(X, mask, i, e, C, n0, n1, nu0, nu1);
        R[e] = r;
        D[e] = r * inv_theta;
    }
}

// One Chebyshev iteration: X += D, R -= M D, Dn = c1 D + c2 R (new R).
// D is only read (at the cell and its neighbours); X, R, Dn only at the cell.
__global__ void k_heat_cheb_step(double* __restrict__ X, double* __restrict__ R, const double* __restrict__ D,
                                 double* __restrict__ Dn, const uint8_t* __restrict__ mask, int64_t N, int logC,
                                 int n0, int n1, double nu0, double nu1, double c1, double c2) {
    const int64_t n = N << logC;
    const int C = 1 << logC;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e >> logC;
        const double d = D[e];
        const double md = heat_mx(D, mask, i, e, C, n0, n1, nu0, nu1);
        X[e] += d;
        const double r = R[e] - md;
        R[e] = r;
        Dn[e] = c1 * d + c2 * r;
    }
}

// Several Chebyshev iterations per launch for one grid vector (the
// per-product solves), blocked in time: a block owns a kHB x kHB tile,
// stages R and D over the tile and a halo of kHS cells in LDS, and runs up
// to kHS iterations there; each iteration reads D at the neighbours, so the
// cells it can update shrink by one per iteration, and after kHS of them the
// tile is still exact.  It then writes X, R and the new D of its tile (R and
// D to the other buffers of a pair: other blocks still read the old ones as
// their halos).  Per cell the arithmetic is k_heat_cheb_step's, in the same
// order (absent neighbour terms add exact zeros).
constexpr int kHB = 16;                  // tile edge
constexpr int kHS = 8;                   // iterations per launch (halo width)
constexpr int kHR = kHB + 2 * kHS;       // staged region edge
constexpr int kHBThr = 256;
static_assert(kHR * kHR % kHBThr == 0, "whole cells per thread");

__global__ void __launch_bounds__(kHBThr)
k_heat_cheb_block(double* __restrict__ X, const double* __restrict__ Rin, const double* __restrict__ Din,
                  double* __restrict__ Rout, double* __restrict__ Dout, const uint8_t* __restrict__ mask, int n0,
                  int n1, double nu0, double nu1, HeatChebSteps cf) {
    constexpr int PER = kHR * kHR / kHBThr;
    __shared__ double sR[kHR * kHR];
    __shared__ double sD[2][kHR * kHR];
    __shared__ uint8_t sM[kHR * kHR];   // 1 free cell, 0 obstacle or outside the grid
    const int tiles_j = (n1 + kHB - 1) / kHB;
    const int gi0 = (int)(blockIdx.x / tiles_j) * kHB - kHS;
    const int gj0 = (int)(blockIdx.x % tiles_j) * kHB - kHS;
    const int tid = threadIdx.x;
    double xr[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int c = tid + q * kHBThr;
        const int li = c / kHR, lj = c % kHR, gi = gi0 + li, gj = gj0 + lj;
        const bool in = gi >= 0 && gi < n0 && gj >= 0 && gj < n1;
        const int64_t g = (int64_t)gi * n1 + gj;
        sR[c] = in ? Rin[g] : 0.0;
        sD[0][c] = in ? Din[g] : 0.0;
        sM[c] = (in && is_free(mask, g)) ? 1 : 0;
        const bool own = li >= kHS && li < kHS + kHB && lj >= kHS && lj < kHS + kHB;
        xr[q] = (in && own) ? X[g] : 0.0;
    }
    __syncthreads();
    // Each cell's stencil once for the launch, branch-free: the weight of a
    // neighbour is nu_k when both cells are free and 0 otherwise (an absent
    // term adds an exact zero, so the sum is the same as skipping it; an
    // obstacle's row is the identity).  Cells of the region's outer ring use
    // themselves as neighbours: their values are never read by a cell that
    // is still exact (the exact region shrinks by one cell per iteration).
    int nb[PER][4];
    double wt[PER][4];
    double ownf[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int c = tid + q * kHBThr;
        const int li = c / kHR, lj = c % kHR;
        const bool ring = li == 0 || li == kHR - 1 || lj == 0 || lj == kHR - 1;
        const bool f = sM[c] == 1 && !ring;
        nb[q][0] = ring ? c : c - kHR;
        nb[q][1] = ring ? c : c + kHR;
        nb[q][2] = ring ? c : c - 1;
        nb[q][3] = ring ? c : c + 1;
        wt[q][0] = (f && sM[c - kHR] == 1) ? nu0 : 0.0;
        wt[q][1] = (f && sM[c + kHR] == 1) ? nu0 : 0.0;
        wt[q][2] = (f && sM[c - 1] == 1) ? nu1 : 0.0;
        wt[q][3] = (f && sM[c + 1] == 1) ? nu1 : 0.0;
        ownf[q] = (li >= kHS && li < kHS + kHB && lj >= kHS && lj < kHS + kHB) ? 1.0 : 0.0;
    }
    for (int st = 0; st < cf.steps; ++st) {
        const double* D = sD[st & 1];
        double* Dn = sD[(st + 1) & 1];
        const double c1 = cf.c1[st], c2 = cf.c2[st];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int c = tid + q * kHBThr;
            const double d = D[c];
            const double du = D[nb[q][0]], dd = D[nb[q][1]], dl = D[nb[q][2]], dr = D[nb[q][3]];
            double md = d;
            md += wt[q][0] * (d - du);
            md += wt[q][1] * (d - dd);
            md += wt[q][2] * (d - dl);
            md += wt[q][3] * (d - dr);
            xr[q] += ownf[q] * d;
            const double r = sR[c] - md;
            sR[c] = r;
            Dn[c] = c1 * d + c2 * r;
        }
        __syncthreads();
    }
    const double* Df = sD[cf.steps & 1];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int c = tid + q * kHBThr;
        const int li = c / kHR, lj = c % kHR, gi = gi0 + li, gj = gj0 + lj;
        const bool own = li >= kHS && li < kHS + kHB && lj >= kHS && lj < kHS + kHB;
        if (!own || gi >= n0 || gj >= n1) continue;
        const int64_t g = (int64_t)gi * n1 + gj;
        X[g] = xr[q];
        Rout[g] = sR[c];
        Dout[g] = Df[c];
    }
}

__global__ void k_heat_zero(float* __restrict__ A, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        A[e] = 0.f;
}

// Packed index of the upper-triangular tile (I, J), I <= J, of nT x nT.
__host__ __device__ __forceinline__ int64_t tile_index(int64_t I, int64_t J, int64_t nT) {
    return I * nT - I * (I - 1) / 2 + (J - I);
}

// Element (free row cidx[i], free column j0 + c) of xi~ = X[i, c] rounded to
// float32, stored where its tile lies in the upper triangle (xi~ is
// symmetric: the solves give every column, the lower half is the
// transpose).  Columns at or beyond nf are zero in X; padding rows are never
// written and stay zero.
__global__ void k_heat_store(const double* __restrict__ X, float* __restrict__ A, const int32_t* __restrict__ cidx,
                             int64_t N, int logC, int64_t ld, int64_t j0) {
    const int64_t n = N << logC;
    const int C = 1 << logC;
    const int64_t nT = ld / kHeatTile;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e >> logC;
        const int64_t r = cidx[i];
        const int64_t j = j0 + (e & (C - 1));
        const int64_t I = r / kHeatTile, J = j / kHeatTile;
        if (r >= 0 && j < ld && I <= J)
            A[tile_index(I, J, nT) * kHeatTile * kHeatTile + (r - I * kHeatTile) * kHeatTile + (j - J * kHeatTile)] =
                (float)X[e];
    }
}

// Free cells in row-major order: each of the 256 threads counts a contiguous
// run of cells, an exclusive scan of the counts gives each run's first free
// index, and the runs are numbered in order.
__global__ void __launch_bounds__(256) k_heat_compact(const uint8_t* __restrict__ mask, int64_t N,
                                                      int32_t* __restrict__ cidx, int32_t* __restrict__ gidx,
                                                      int64_t* __restrict__ count) {
    __shared__ int64_t base[257];
    const int t = threadIdx.x;
    const int64_t per = (N + 255) / 256;
    const int64_t lo = t * per < N ? t * per : N, hi = lo + per < N ? lo + per : N;
    int64_t c = 0;
    for (int64_t i = lo; i < hi; ++i) c += is_free(mask, i) ? 1 : 0;
    base[t + 1] = c;
    __syncthreads();
    if (t == 0) {
        base[0] = 0;
        for (int k = 1; k <= 256; ++k) base[k] += base[k - 1];
        *count = base[256];
    }
    __syncthreads();
    int64_t r = base[t];
    for (int64_t i = lo; i < hi; ++i) {
        if (is_free(mask, i)) {
            cidx[i] = (int32_t)r;
            gidx[r] = (int32_t)i;
            ++r;
        } else {
            cidx[i] = -1;
        }
    }
}

__global__ void k_heat_gather(float* __restrict__ x, const float* __restrict__ src, const int32_t* __restrict__ gidx,
                              int64_t nf, int64_t ld) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ld; r += (int64_t)gridDim.x * blockDim.x)
        x[r] = r < nf ? src[gidx[r]] : 0.f;
}

// ------------------------------------------------------------------ products

// X (grid, FP64) = the free-cell vector x scattered to its cells, 0 on obstacles.
__global__ void k_heat_scatter(double* __restrict__ X, const float* __restrict__ x, const int32_t* __restrict__ cidx,
                               int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = cidx[i];
        X[i] = r >= 0 ? (double)x[r] : 0.0;
    }
}

// Finish row r (free cell i = gidx[r]) of y = A x (value v): the epilogue of
// the iteration's half-step.
template <int EK>
__device__ __forceinline__ void heat_epilogue(const HeatGemv& g, int64_t r, float v) {
    const int64_t i = g.gidx[r];
    if constexpr (EK == EK_STORE) {
        g.y[i] = v;
    } else if constexpr (EK == EK_BUPDATE || EK == EK_MONITOR) {
        const float q = g.q[i];
        if (EK == EK_MONITOR || g.check) g.errrow[r] = fabs((double)g.b[r] * (double)v - (double)q);
        if (EK == EK_BUPDATE) g.b[r] = q == 0.f ? 0.f : q / v;
    } else {
        constexpr int KIND = EK - EK_PROX;
        const ProxArgs& px = g.px;
        float pu = 1.f, pv = 0.f;
        if (KIND == JKO_F_CONGESTION || KIND == JKO_F_CONGESTION_BINARY) {
            pu = px.g ? px.g[i] : 1.f;
            pv = px.kappa ? px.kappa[i] : px.kappa_s;
        } else if (KIND == JKO_F_ENTROPY || KIND == JKO_F_POROUS) {
            pu = px.kf ? px.kf[i] : px.kf_s;
        } else if (KIND == JKO_F_GEN_ENTROPY) {
            pu = px.kf ? px.kf[i] : px.kf_s;
            pv = px.g ? px.g[i] : px.eps_s;
        }
        const float p = prox_val<KIND>(px, v, pu, pv);
        g.a[r] = p == 0.f ? 0.f : p / v;
        g.p[i] = p;
    }
}

// Plain loads: the packed operator of a 100 x 100 room stays largely
// resident in the last-level cache between passes; with the non-temporal
// hint the room's flow ran 12 % slower (measured on the full-grid operator:
// 11.8 K against 13.4 K iterations/s).
#ifndef JKO_HEAT_NT
#define JKO_HEAT_NT 0
#endif
// One float4 of an operator tile, with the non-temporal hint when JKO_HEAT_NT.
__device__ __forceinline__ f4 ld_nt(const f4* p) {
#if JKO_HEAT_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// Tile pass: block b takes the packed tile (I, J), I <= J, and writes
//   part[I][J] = A_IJ x_J             (its row sums, the tile's share of y_I)
//   part[J][I] = A_IJ^T x_I  (I < J)  (its column sums, the share of y_J
//                                      from the transposed lower tile)
// so that every (row block, tile) slot of part is written exactly once.  A
// tile row is 32 float4s: thread (group g, lane c) takes float4 c of rows
// g, g + 8, ..., g + 120 (plain loads, see ld_nt), keeps one partial row sum per
// row and four column sums in registers; the row partials are then summed
// through LDS (one row per thread), the column sums over the 8 groups.
__global__ void __launch_bounds__(256) k_heat_tiles(const float* __restrict__ A, const float* __restrict__ x,
                                                    float* __restrict__ part, int nT) {
    constexpr int T = kHeatTile, R = T / 8;
    const int b = blockIdx.x;
    int I = 0, start = 0;
    while (start + (nT - I) <= b) {    // uniform over the block; at most nT steps
        start += nT - I;
        ++I;
    }
    const int J = I + (b - start);
    const f4* __restrict__ tile = reinterpret_cast<const f4*>(A + (int64_t)b * T * T);
    const int t = threadIdx.x, cl = t & 31, rg = t >> 5;
    const f4 xj = reinterpret_cast<const f4*>(x + (int64_t)J * T)[cl];
    const float* __restrict__ xi = x + (int64_t)I * T;
    const bool off = I != J;
    __shared__ float red[T][33];      // row partials, padded against bank conflicts
    __shared__ f4 cols[8][32];
    float rp[R];
    f4 cacc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = rg + 8 * k;
        const f4 a = ld_nt(tile + r * 32 + cl);
        rp[k] = (a.x * xj.x + a.y * xj.y) + (a.z * xj.z + a.w * xj.w);
        if (off) cacc += a * xi[r];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) red[rg + 8 * k][cl] = rp[k];
    if (off) cols[rg][cl] = cacc;
    __syncthreads();
    if (t < T) {
        float y = 0.f;
#pragma unroll
        for (int c = 0; c < 32; ++c) y += red[t][c];
        part[((int64_t)I * nT + J) * T + t] = y;
    } else if (off && t < T + 32) {
        const int c = t - T;
        f4 v = cols[0][c];
#pragma unroll
        for (int g = 1; g < 8; ++g) v += cols[g][c];
        reinterpret_cast<f4*>(part + ((int64_t)J * nT + I) * T)[c] = v;
    }
}

// Finish pass: y_i = the sum of the nT slots of i's row block, split over 8
// slices (slice s takes slots s, s + 8, ...) whose results are added in slice
// order, then the pointwise epilogue of row i.  A block takes 32 consecutive
// cells x 8 slices.
template <int EK>
__global__ void __launch_bounds__(256) k_heat_finish(HeatGemv g) {
    __shared__ float red[8][33];
    const int t = threadIdx.x, c = t & 31, sl = t >> 5;
    const int64_t i = (int64_t)blockIdx.x * 32 + c;
    float y = 0.f;
    if (i < g.N) {
        const int64_t I = i / kHeatTile, il = i - I * kHeatTile;
        const float* __restrict__ p = g.part + I * g.nT * kHeatTile + il;
#pragma unroll 4
        for (int K = sl; K < g.nT; K += 8) y += p[(int64_t)K * kHeatTile];
    }
    red[sl][c] = y;
    __syncthreads();
    if (sl == 0 && i < g.N) {
        float v = red[0][c];
#pragma unroll
        for (int q = 1; q < 8; ++q) v += red[q][c];
        heat_epilogue<EK>(g, i, v);
    }
}

// Finish of a product computed by the solves: row r takes its cell's value of
// X (rounded to float32) through the epilogue.
template <int EK>
__global__ void __launch_bounds__(256) k_heat_solve_finish(HeatGemv g, const double* __restrict__ X) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < g.N; r += (int64_t)gridDim.x * blockDim.x)
        heat_epilogue<EK>(g, r, (float)X[g.gidx[r]]);
}

__global__ void k_heat_fill(float* __restrict__ x, float v, int64_t n, int64_t ld) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ld; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = i < n ? v : 0.f;
}

__global__ void __launch_bounds__(256) k_heat_sums(const double* __restrict__ errrow, int64_t ne,
                                                   const float* __restrict__ p, int64_t np, double* __restrict__ out) {
    __shared__ double sh[4];
    double e = 0.0, m = 0.0, bad = 0.0;
    if (errrow)
        for (int64_t i = threadIdx.x; i < ne; i += blockDim.x) {
            const double v = errrow[i];
            if (isfinite(v)) e += v;
            else bad += 1.0;
        }
    if (p)
        for (int64_t i = threadIdx.x; i < np; i += blockDim.x) m += (double)p[i];
    e = block_sum(e, sh);
    if (threadIdx.x == 0) out[0] = e;
    m = block_sum(m, sh);
    if (threadIdx.x == 0) out[1] = m;
    bad = block_sum(bad, sh);
    if (threadIdx.x == 0) out[2] = bad;
}

__global__ void __launch_bounds__(256) k_heat_input(const float* __restrict__ p, const uint8_t* __restrict__ mask,
                                                    const float* __restrict__ kappa, float kappa_s, int64_t N,
                                                    double* __restrict__ out) {
    __shared__ double sh[4];
    double m = 0.0, cap = 0.0, bad = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
        const float v = p[i];
        const bool fr = is_free(mask, i);
        if (!(v >= 0.f) || !isfinite(v) || (!fr && v != 0.f)) bad += 1.0;
        else m += (double)v;
        const float k = kappa ? kappa[i] : kappa_s;
        if (!(k >= 0.f)) bad += 1.0;
        else if (fr) cap += (double)k;
    }
    m = block_sum(m, sh);
    if (threadIdx.x == 0) out[0] = m;
    cap = block_sum(cap, sh);
    if (threadIdx.x == 0) out[1] = cap;
    bad = block_sum(bad, sh);
    if (threadIdx.x == 0) out[2] = bad;
}

int grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

int chunk_log2(int64_t N) {
    int lg = 2;                                   // at least 4 columns
    while (lg < 10 && ((int64_t)1 << lg) < N) ++lg;
    return lg;                                    // at most 1024 columns per chunk
}

// L solves of M y = X in place on the grid vector X (obstacles stay zero),
// each a Chebyshev iteration of K steps from the first guess X, kHS steps per
// launch (k_heat_cheb_block; R and D alternate between their two buffers).
void heat_solves(const HeatSolve& h, int K, hipStream_t st) {
    const int64_t N = (int64_t)h.n0 * h.n1;
    const double nu0 = h.n0 > 1 ? h.gamma * (double)h.n0 * h.n0 / h.L : 0.0;
    const double nu1 = h.n1 > 1 ? h.gamma * (double)h.n1 * h.n1 / h.L : 0.0;
    const double beta = 1.0 + 4.0 * (nu0 + nu1);
    const double theta = 0.5 * (beta + 1.0), delta = 0.5 * (beta - 1.0);
    const int gb = grid_for(N);
    const unsigned tiles = (unsigned)(((h.n0 + kHB - 1) / kHB) * ((h.n1 + kHB - 1) / kHB));
    double* R[2] = {h.R, h.R1};
    double* D[2] = {h.D0, h.D1};
    for (int l = 0; l < h.L && K > 0; ++l) {
        hipLaunchKernelGGL(k_heat_cheb_init, dim3(gb), dim3(256), 0, st, h.X, R[0], D[0], h.mask, N, 0, h.n0, h.n1,
                           nu0, nu1, 1.0 / theta);
        const double sigma1 = theta / delta;
        double rho = 1.0 / sigma1;
        int cur = 0;
        for (int k = 0; k < K; k += kHS) {
            HeatChebSteps cf{};
            cf.steps = std::min(kHS, K - k);
            for (int j = 0; j < cf.steps; ++j) {
                const double rho_n = 1.0 / (2.0 * sigma1 - rho);
                cf.c1[j] = rho_n * rho;
                cf.c2[j] = 2.0 * rho_n / delta;
                rho = rho_n;
            }
            hipLaunchKernelGGL(k_heat_cheb_block, dim3(tiles), dim3(kHBThr), 0, st, h.X, R[cur], D[cur], R[1 - cur],
                               D[1 - cur], h.mask, h.n0, h.n1, nu0, nu1, cf);
            cur = 1 - cur;
        }
    }
}

template <int EK>
hipError_t solve_as(const HeatGemv& g, const HeatSolve& h, hipStream_t st) {
    const int64_t N = (int64_t)h.n0 * h.n1;
    hipLaunchKernelGGL(k_heat_scatter, dim3(grid_for(N)), dim3(256), 0, st, h.X, g.x, h.cidx, N);
    const double nu0 = h.n0 > 1 ? h.gamma * (double)h.n0 * h.n0 / h.L : 0.0;
    const double nu1 = h.n1 > 1 ? h.gamma * (double)h.n1 * h.n1 / h.L : 0.0;
    heat_solves(h, heat_cheb_iters(1.0 + 4.0 * (nu0 + nu1), kHeatSolveTol), st);
    if (g.N > 0) hipLaunchKernelGGL(k_heat_solve_finish<EK>, dim3(grid_for(g.N)), dim3(256), 0, st, g, h.X);
    return hipGetLastError();
}

template <int EK>
hipError_t gemv_as(const HeatGemv& g, hipStream_t st) {
    if (g.nT == 0) return hipSuccess;   // no free cell
    const int64_t tiles = (int64_t)g.nT * (g.nT + 1) / 2;
    hipLaunchKernelGGL(k_heat_tiles, dim3((unsigned)tiles), dim3(256), 0, st, g.A, g.x, g.part, g.nT);
    hipLaunchKernelGGL(k_heat_finish<EK>, dim3((unsigned)((g.N + 31) / 32)), dim3(256), 0, st, g);
    return hipGetLastError();
}

}  // namespace

int heat_cheb_iters(double beta, double tol) {
    if (!(beta > 1.0)) return 0;
    const double sk = sqrt(beta);
    const double c = (sk - 1.0) / (sk + 1.0);
    return (int)ceil(log(0.5 * tol) / log(c));
}

int64_t heat_build_scratch(int64_t N) { return 4 * N * ((int64_t)1 << chunk_log2(N)); }

hipError_t heat_build_operator(const uint8_t* mask, int n0, int n1, double gamma, int L, const int32_t* cidx,
                               const int32_t* gidx, int64_t nf, float* A, double* scratch, hipStream_t st) {
    const int64_t N = (int64_t)n0 * n1;
    const int64_t ld = heat_ld(nf);
    const int logC = chunk_log2(N);
    const int64_t C = (int64_t)1 << logC;
    const double nu0 = n0 > 1 ? gamma * (double)n0 * n0 / L : 0.0;
    const double nu1 = n1 > 1 ? gamma * (double)n1 * n1 / L : 0.0;
    const double beta = 1.0 + 4.0 * (nu0 + nu1);
    const int K = heat_cheb_iters(beta, 1e-14);
    const double theta = 0.5 * (beta + 1.0), delta = 0.5 * (beta - 1.0);
    hipLaunchKernelGGL(k_heat_zero, dim3(grid_for(heat_operator_floats(nf))), dim3(256), 0, st, A,
                       heat_operator_floats(nf));
    double* X = scratch;
    double* R = X + N * C;
    double* D[2] = {R + N * C, R + 2 * N * C};
    const int gb = grid_for(N * C);
    for (int64_t j0 = 0; j0 < ld; j0 += C) {
        hipLaunchKernelGGL(k_heat_unit, dim3(gb), dim3(256), 0, st, X, gidx, nf, N, logC, j0);
        for (int l = 0; l < L && K > 0; ++l) {
            // solve M x = X from the first guess X
            hipLaunchKernelGGL(k_heat_cheb_init, dim3(gb), dim3(256), 0, st, X, R, D[0], mask, N, logC, n0, n1,
                               nu0, nu1, 1.0 / theta);
            const double sigma1 = theta / delta;
            double rho = 1.0 / sigma1;
            for (int k = 0; k < K; ++k) {
                const double rho_n = 1.0 / (2.0 * sigma1 - rho);
                hipLaunchKernelGGL(k_heat_cheb_step, dim3(gb), dim3(256), 0, st, X, R, D[k & 1], D[(k + 1) & 1],
                                   mask, N, logC, n0, n1, nu0, nu1, rho_n * rho, 2.0 * rho_n / delta);
                rho = rho_n;
            }
        }
        hipLaunchKernelGGL(k_heat_store, dim3(gb), dim3(256), 0, st, X, A, cidx, N, logC, ld, j0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_heat_gemv(int ek, const HeatGemv& g, hipStream_t st) {
    switch (ek) {
        case EK_STORE: return gemv_as<EK_STORE>(g, st);
        case EK_BUPDATE: return gemv_as<EK_BUPDATE>(g, st);
        case EK_MONITOR: return gemv_as<EK_MONITOR>(g, st);
        case EK_PROX + JKO_F_ZERO: return gemv_as<EK_PROX + JKO_F_ZERO>(g, st);
        case EK_PROX + JKO_F_CONGESTION: return gemv_as<EK_PROX + JKO_F_CONGESTION>(g, st);
        case EK_PROX + JKO_F_POROUS: return gemv_as<EK_PROX + JKO_F_POROUS>(g, st);
        case EK_PROX + JKO_F_ENTROPY: return gemv_as<EK_PROX + JKO_F_ENTROPY>(g, st);
        case EK_PROX + JKO_F_CONGESTION_BINARY: return gemv_as<EK_PROX + JKO_F_CONGESTION_BINARY>(g, st);
        case EK_PROX + JKO_F_GEN_ENTROPY: return gemv_as<EK_PROX + JKO_F_GEN_ENTROPY>(g, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_heat_solve(int ek, const HeatGemv& g, const HeatSolve& h, hipStream_t st) {
    switch (ek) {
        case EK_STORE: return solve_as<EK_STORE>(g, h, st);
        case EK_BUPDATE: return solve_as<EK_BUPDATE>(g, h, st);
        case EK_MONITOR: return solve_as<EK_MONITOR>(g, h, st);
        case EK_PROX + JKO_F_ZERO: return solve_as<EK_PROX + JKO_F_ZERO>(g, h, st);
        case EK_PROX + JKO_F_CONGESTION: return solve_as<EK_PROX + JKO_F_CONGESTION>(g, h, st);
        case EK_PROX + JKO_F_POROUS: return solve_as<EK_PROX + JKO_F_POROUS>(g, h, st);
        case EK_PROX + JKO_F_ENTROPY: return solve_as<EK_PROX + JKO_F_ENTROPY>(g, h, st);
        case EK_PROX + JKO_F_CONGESTION_BINARY: return solve_as<EK_PROX + JKO_F_CONGESTION_BINARY>(g, h, st);
        case EK_PROX + JKO_F_GEN_ENTROPY: return solve_as<EK_PROX + JKO_F_GEN_ENTROPY>(g, h, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_heat_fill(float* x, float v, int64_t n, int64_t ld, hipStream_t st) {
    hipLaunchKernelGGL(k_heat_fill, dim3(grid_for(ld)), dim3(256), 0, st, x, v, n, ld);
    return hipGetLastError();
}

hipError_t launch_heat_sums(const double* errrow, int64_t ne, const float* p, int64_t np, double* out,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_heat_sums, dim3(1), dim3(256), 0, st, errrow, ne, p, np, out);
    return hipGetLastError();
}

hipError_t launch_heat_input(const float* p, const uint8_t* mask, const float* kappa, float kappa_s, int64_t N,
                             double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_heat_input, dim3(1), dim3(256), 0, st, p, mask, kappa, kappa_s, N, out);
    return hipGetLastError();
}

hipError_t launch_heat_compact(const uint8_t* mask, int64_t N, int32_t* cidx, int32_t* gidx, int64_t* count,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_heat_compact, dim3(1), dim3(256), 0, st, mask, N, cidx, gidx, count);
    return hipGetLastError();
}

hipError_t launch_heat_gather(float* x, const float* src, const int32_t* gidx, int64_t nf, int64_t ld,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_heat_gather, dim3(grid_for(ld)), dim3(256), 0, st, x, src, gidx, nf, ld);
    return hipGetLastError();
}

}  // namespace jko
