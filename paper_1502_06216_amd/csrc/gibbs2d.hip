// Fused 2D Gibbs application  Y = K1_0 X K1_1  on MFMA (gfx950), and the
// resident 2D kernel that runs a whole step's iteration in one launch.
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
// These kernels run the plain domain only: after an absorption switch every
// product runs on the exact log-sum-exp passes of logpass.hip.
//
// Resident kernel: when every tile's block fits on the chip at once, the
// iteration of a step (3.2: t = xi^T a, b = q / t, s = xi b, a = prox(s) / s,
// the stop test and the absorption switch) runs in one cooperative launch.
// Each block keeps its factor bands and its tile's epilogue inputs on chip
// and, between applications, waits only for the blocks whose tiles its halo
// reaches; the stop test is evaluated by every block from the same partials
// in the same order, so all blocks take the same decision.  Results are
// bit-identical to the launch-per-application path.
#include <algorithm>
#include <type_traits>

#include "control.h"
#include "epilogue.h"

namespace jko {

namespace {

constexpr int kT = 16;          // output tile edge
constexpr int kHalo = 128;      // largest halo edge held in LDS
constexpr int kS = kHalo + 4;   // padded LDS row (floats)
constexpr int kThr = 512;       // 8 waves per block
constexpr int kMaxNeighbours = 9 * 9;   // halo reach of at most 4 tiles per side

constexpr int kS2 = kHalo + 8;   // padded LDS row of a bfloat16 band (16-byte aligned)
constexpr int kRS = 68;          // padded row of the partial sums (64 lanes)

struct Smem {
    float Xs[kHalo * kS];   // [ib][jb]
    float Kj[kT * kS];      // [j][jb]  = K1_1[j0+j][jb0+jb]
    float Ki[kT * kS];      // [i][ib]  = K1_0[i0+i][ib0+ib]
    uint16_t Kjh[kT * kS2], Kjl[kT * kS2];   // split path: bfloat16 hi / lo of the bands
    uint16_t Kih[kT * kS2], Kil[kT * kS2];
    float Zs[kT * kS];      // [j][ib]
    float red[8 * 4 * kRS];  // [wave][element][lane] partial sums of the second contraction
    double shd[8];
};

__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, bid = blockIdx.x;
    if (nb % 8 != 0) return bid;
    return (bid % 8) * (nb / 8) + bid / 8;
}

// Geometry of one block's tile.  The halo start is aligned down to a
// multiple of 4 (the extra entries meet exact zeros of the band).
struct Tile {
    int i0, j0, ib0, jb0, LI, LJ, LIp, LJp;
    int eidx, ecnt;    // the output this thread finishes (waves 0-3; ecnt = 0 elsewhere or outside the grid)
};

// Halo extents are padded to whole MFMA k-steps: 16 (FP32) or 32 (split).
template <bool SPLIT = false>
__device__ __forceinline__ Tile tile_of(const Band2D& B, int logical, int lane) {
    constexpr int RND = SPLIT ? 32 : 16;
    Tile T;
    const int tiles_j = (B.n1 + kT - 1) / kT;
    T.i0 = (logical / tiles_j) * kT;
    T.j0 = (logical % tiles_j) * kT;
    T.ib0 = max(0, T.i0 - B.W0) & ~3;
    T.jb0 = max(0, T.j0 - B.W1) & ~3;
    T.LI = min(B.n0, T.i0 + kT + B.W0) - T.ib0;
    T.LJ = min(B.n1, T.j0 + kT + B.W1) - T.jb0;
    T.LIp = (T.LI + RND - 1) & ~(RND - 1);
    T.LJp = (T.LJ + RND - 1) & ~(RND - 1);
    // wave v < 4, lane l finish row i0 + 4 v + (l >> 4), column j0 + (l & 15):
    // each store instruction writes whole row segments
    const int wave = threadIdx.x >> 6;
    const int ei = T.i0 + 4 * wave + (lane >> 4), ej = T.j0 + (lane & 15);
    T.eidx = ei * B.n1 + ej;
    T.ecnt = (wave < 4 && ei < B.n0 && ej < B.n1) ? 1 : 0;
    return T;
}

constexpr int UXM = kHalo * (kHalo / 4) / kThr;   // max halo units per thread
constexpr int UKM = kT * (kHalo / 4) / kThr;      // max factor units per thread

// Issue the loads of the X halo (zero outside the grid).  COH: device-scope
// loads (buffer loads with scope bit SC1, range-checked by the descriptor) of
// a field other blocks of the same launch wrote.
constexpr int kCpolDevice = 16;   // SC1: device scope

template <bool COH = false>
__device__ __forceinline__ void load_halo(const Band2D& B, const Tile& T, f4 (&bx)[UXM]) {
    const int tid = threadIdx.x;
    const int nux = T.LIp * (T.LJp / 4);
    const bool vec1 = (B.n1 & 3) == 0;
    __amdgpu_buffer_rsrc_t rs;
    if (COH)
        rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(B.X), (short)0, B.n0 * B.n1 * 4, 0x00020000);
#pragma unroll
    for (int u = 0; u < UXM; ++u) {
        const int unit = tid + u * kThr;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (unit < nux) {
            const int r = unit / (T.LJp / 4), c = 4 * (unit % (T.LJp / 4));
            if (r < T.LI) {
                const int off = (T.ib0 + r) * B.n1 + T.jb0 + c;
                if (COH) {
                    if (vec1 && c + 3 < T.LJ)
                        v = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, 4 * off, 0, kCpolDevice));
                    else
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            v[e] = (c + e < T.LJ) ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                                                  rs, 4 * (off + e), 0, kCpolDevice))
                                                  : 0.f;
                } else {
                    const float* src = B.X + off;
                    if (vec1 && c + 3 < T.LJ) v = *reinterpret_cast<const f4*>(src);
                    else
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = (c + e < T.LJ) ? src[e] : 0.f;
                }
            }
        }
        bx[u] = v;
    }
}

__device__ __forceinline__ void store_halo(Smem& S, const Tile& T, const f4 (&bx)[UXM]) {
    const int tid = threadIdx.x;
    const int nux = T.LIp * (T.LJp / 4);
#pragma unroll
    for (int u = 0; u < UXM; ++u) {
        const int unit = tid + u * kThr;
        if (unit < nux) {
            const int r = unit / (T.LJp / 4), c = 4 * (unit % (T.LJp / 4));
            *reinterpret_cast<f4*>(&S.Xs[r * kS + c]) = bx[u];
        }
    }
}

// Issue the loads of the two factor bands of the tile.
__device__ __forceinline__ void load_bands(const Band2D& B, const Tile& T, f4 (&bj)[UKM], f4 (&bi)[UKM]) {
    const int tid = threadIdx.x;
    const int nkj = kT * (T.LJp / 4), nki = kT * (T.LIp / 4);
    const bool vec1 = (B.n1 & 3) == 0, vec0 = (B.n0 & 3) == 0;
#pragma unroll
    for (int u = 0; u < UKM; ++u) {
        const int unit = tid + u * kThr;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (unit < nkj) {
            const int j = unit / (T.LJp / 4), c = 4 * (unit % (T.LJp / 4));
            if (T.j0 + j < B.n1) {
                const float* src = B.K1 + (int64_t)(T.j0 + j) * B.n1 + T.jb0 + c;
                if (vec1 && c + 3 < T.LJ) v = *reinterpret_cast<const f4*>(src);
                else
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = (c + e < T.LJ) ? src[e] : 0.f;
            }
        }
        bj[u] = v;
        f4 w = f4{0.f, 0.f, 0.f, 0.f};
        if (unit < nki) {
            const int i = unit / (T.LIp / 4), c = 4 * (unit % (T.LIp / 4));
            if (T.i0 + i < B.n0) {
                const float* src = B.K0 + (int64_t)(T.i0 + i) * B.n0 + T.ib0 + c;
                if (vec0 && c + 3 < T.LI) w = *reinterpret_cast<const f4*>(src);
                else
#pragma unroll
                    for (int e = 0; e < 4; ++e) w[e] = (c + e < T.LI) ? src[e] : 0.f;
            }
        }
        bi[u] = w;
    }
}

__device__ __forceinline__ void store_bands(Smem& S, const Tile& T, const f4 (&bj)[UKM], const f4 (&bi)[UKM]) {
    const int tid = threadIdx.x;
    const int nkj = kT * (T.LJp / 4), nki = kT * (T.LIp / 4);
#pragma unroll
    for (int u = 0; u < UKM; ++u) {
        const int unit = tid + u * kThr;
        if (unit < nkj) {
            const int j = unit / (T.LJp / 4), c = 4 * (unit % (T.LJp / 4));
            *reinterpret_cast<f4*>(&S.Kj[j * kS + c]) = bj[u];
        }
        if (unit < nki) {
            const int i = unit / (T.LIp / 4), c = 4 * (unit % (T.LIp / 4));
            *reinterpret_cast<f4*>(&S.Ki[i * kS + c]) = bi[u];
        }
    }
}

// Split path: stage the bfloat16 hi / lo factor bands (built from the exact
// factor in double precision), zero outside the band.
constexpr int UKS = kT * (kHalo / 4) / kThr;   // 4-element units per thread, per array

__device__ __forceinline__ void stage_bands_split(const Band2D& B, const Tile& T, Smem& S) {
    const int tid = threadIdx.x;
    const int nkj = kT * (T.LJp / 4), nki = kT * (T.LIp / 4);
    u16x4 jh[UKS], jl[UKS], ih[UKS], il[UKS];
#pragma unroll
    for (int u = 0; u < UKS; ++u) {
        const int unit = tid + u * kThr;
        jh[u] = jl[u] = ih[u] = il[u] = u16x4{0, 0, 0, 0};
        if (unit < nkj) {
            const int j = unit / (T.LJp / 4), c = 4 * (unit % (T.LJp / 4));
            if (T.j0 + j < B.n1) {
                const int64_t off = (int64_t)(T.j0 + j) * B.n1 + T.jb0 + c;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    jh[u][e] = (c + e < T.LJ) ? B.K1hi[off + e] : (uint16_t)0;
                    jl[u][e] = (c + e < T.LJ) ? B.K1lo[off + e] : (uint16_t)0;
                }
            }
        }
        if (unit < nki) {
            const int i = unit / (T.LIp / 4), c = 4 * (unit % (T.LIp / 4));
            if (T.i0 + i < B.n0) {
                const int64_t off = (int64_t)(T.i0 + i) * B.n0 + T.ib0 + c;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ih[u][e] = (c + e < T.LI) ? B.K0hi[off + e] : (uint16_t)0;
                    il[u][e] = (c + e < T.LI) ? B.K0lo[off + e] : (uint16_t)0;
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < UKS; ++u) {
        const int unit = tid + u * kThr;
        if (unit < nkj) {
            const int j = unit / (T.LJp / 4), c = 4 * (unit % (T.LJp / 4));
            *reinterpret_cast<u16x4*>(&S.Kjh[j * kS2 + c]) = jh[u];
            *reinterpret_cast<u16x4*>(&S.Kjl[j * kS2 + c]) = jl[u];
        }
        if (unit < nki) {
            const int i = unit / (T.LIp / 4), c = 4 * (unit % (T.LIp / 4));
            *reinterpret_cast<u16x4*>(&S.Kih[i * kS2 + c]) = ih[u];
            *reinterpret_cast<u16x4*>(&S.Kil[i * kS2 + c]) = il[u];
        }
    }
}

// Both contractions of the staged tile and its epilogue (waves 0-3), then the
// block's partials into slot `slot`.  Xs, Kj, Ki are staged, not yet synced.
// COH: the scalings and partials the epilogue writes use device-scope stores.
// SPLIT: each FP32 operand (X, then Z) is split into bfloat16 hi + lo as it is
// read and multiplied with the factor bands' hi / lo, three products
// (hi*hi + hi*lo + lo*hi) on v_mfma_f32_16x16x32_bf16, FP32 accumulation.
template <int EK, bool COH = false, bool SPLIT = false>
__device__ __forceinline__ void contract_tile(const EpiArgs& E, const Tile& T, const EpiIn& ein, Smem& S,
                                              int slot) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int koff = 4 * (lane >> 4);
    const int LIp = T.LIp, LJp = T.LJp;
    __syncthreads();

    // ---- Z = X K1_1^T over the halo rows: wave f owns the 16-row fragment f;
    // even and odd k-chunks go to two accumulators (independent MFMA chains)
    const int F = LIp / 16;
    if (SPLIT && wave < F) {
        const int f = wave;
        const int k8 = 8 * (lane >> 4);
        f4 acc = f4{0.f, 0.f, 0.f, 0.f};
        const float* xr = &S.Xs[(16 * f + (lane & 15)) * kS + k8];
        const uint16_t* khr = &S.Kjh[(lane & 15) * kS2 + k8];
        const uint16_t* klr = &S.Kjl[(lane & 15) * kS2 + k8];
        for (int c0 = 0; c0 < LJp; c0 += 32) {
            bf8 ah, al;
            split_bf16(*reinterpret_cast<const f4*>(xr + c0), *reinterpret_cast<const f4*>(xr + c0 + 4), ah, al);
            const bf8 bh = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(khr + c0));
            const bf8 bl = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(klr + c0));
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
        }
        *reinterpret_cast<f4*>(&S.Zs[(lane & 15) * kS + 16 * f + koff]) = acc;
    } else if (!SPLIT && wave < F) {
        const int f = wave;
        f4 acc0 = f4{0.f, 0.f, 0.f, 0.f}, acc1 = f4{0.f, 0.f, 0.f, 0.f};
        const float* xr = &S.Xs[(16 * f + (lane & 15)) * kS + koff];
        const float* kr = &S.Kj[(lane & 15) * kS + koff];
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
        const f4 acc = acc0 + acc1;
        // acc holds Z[ib = 16f + koff + e][j = lane & 15]
        *reinterpret_cast<f4*>(&S.Zs[(lane & 15) * kS + 16 * f + koff]) = acc;
    }
    __syncthreads();

    // ---- Y^T = Z^T K1_0^T: one 16 x 16 fragment, its 16-wide k-chunks spread
    // over the waves (at most 8 chunks), partial sums combined in a fixed order
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    if (SPLIT) {
        if (32 * wave < LIp) {   // 32-wide k-chunks over the waves
            const int c0 = 32 * wave + 8 * (lane >> 4);
            bf8 ah, al;
            const float* zr = &S.Zs[(lane & 15) * kS + c0];
            split_bf16(*reinterpret_cast<const f4*>(zr), *reinterpret_cast<const f4*>(zr + 4), ah, al);
            const bf8 bh = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&S.Kih[(lane & 15) * kS2 + c0]));
            const bf8 bl = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&S.Kil[(lane & 15) * kS2 + c0]));
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
        }
    } else if (16 * wave < LIp) {
        const int c0 = 16 * wave;
        const f4 a = *reinterpret_cast<const f4*>(&S.Zs[(lane & 15) * kS + c0 + koff]);
        const f4 b = *reinterpret_cast<const f4*>(&S.Ki[(lane & 15) * kS + c0 + koff]);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) S.red[(wave * 4 + e) * kRS + lane] = acc[e];
    __syncthreads();
    EpiAcc ea;
    if (wave < 4) {
        // One output per lane (Tile::eidx): Y[i][j] sits in element j & 3 of
        // MFMA lane (i - i0) + 16 ((j - j0) >> 2); its partial sums are added
        // in wave order.
        const int il = 4 * wave + (lane >> 4), jl = lane & 15;
        const int src = il + 16 * (jl >> 2), e = jl & 3;
        float y = S.red[e * kRS + src];
#pragma unroll
        for (int w = 1; w < 8; ++w) y += S.red[(w * 4 + e) * kRS + src];
        epi_apply<EK, COH, 1>(E, T.eidx, T.ecnt, f4{y, 0.f, 0.f, 0.f}, false, ein, ea);
    }
    epi_finish<COH>(E, ea, slot, S.shd);
}

template <int EK, bool SPLIT>
__global__ void __launch_bounds__(kThr)
gibbs2d_kernel(Band2D B, EpiArgs E) {
    __shared__ __attribute__((aligned(16))) Smem S;

    // The control flags are read here but acted on only after the halo loads
    // are in flight, so their latencies overlap.
    int done = 0;
    if (E.ctl) done = E.ctl->done;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Tile T = tile_of<SPLIT>(B, xcd_block(), lane);

    // Waves 0-3 finish the tile (one output per lane each); their epilogue
    // inputs are fetched now, ahead of the contraction.
    EpiIn ein;
    if (wave < 4) ein = epi_prefetch<EK>(E, T.eidx, T.ecnt);

    // the staging loads are issued before the LDS stores
    f4 bx[UXM];
    load_halo(B, T, bx);
    if (SPLIT) {
        stage_bands_split(B, T, S);
    } else {
        f4 bj[UKM], bi[UKM];
        load_bands(B, T, bj, bi);
        store_bands(S, T, bj, bi);
    }
    store_halo(S, T, bx);
    if (done) return;   // the step has stopped: nothing to compute (uniform)
    contract_tile<EK, false, SPLIT>(E, T, ein, S, (int)blockIdx.x);
}

// ------------------------------------------------------------ resident kernel
//
// Synchronisation without atomics read-modify-write and without cache-wide
// fences: every value one block writes for another (a, b, the partials) is
// stored and loaded at device scope, which is coherent across the XCDs'
// separate L2s.  After a phase's stores have completed (s_waitcnt), block t
// publishes its phase count in flags[t]; before a phase that reads other
// blocks' values, a block waits until each block it reads from has published
// at least its own count.  Tiles only read the tiles within their halo, so
// most phases wait on those neighbours only (the relation is symmetric, which
// also keeps a block from overwriting values a neighbour is still reading);
// at a stop-test check, block 0 waits on every block, evaluates the test
// from all partials and publishes the decision, which the others wait for.
// Each wait polls a bounded number of times; one that runs out raises the
// abort word, which every waiting block also polls, so every wave ends.

// Sync region layout (uint32 words): [0] abort, [16] decision bits of the
// last check (1 done, 2 absorb), [32] the phase count that decision belongs
// to, flags[t] at kFlag0 + kFlagStride * t.
constexpr int kDecision = 16;
constexpr int kDecisionSeq = 32;
constexpr int kFlag0 = 64;
constexpr int kFlagStride = 16;   // one 64-byte line per block

__device__ __forceinline__ uint32_t* flag_of(uint32_t* sync, int t) { return sync + kFlag0 + kFlagStride * t; }

// All stores of this block completed, then publish `count` for it.
__device__ __forceinline__ void publish(uint32_t* sync, int slot, uint32_t count) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag_of(sync, slot), count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until blocks list[0 .. n) (one per thread) have published >= count.
// Returns false (in every thread) if the wait ran out or another block aborted.
__device__ __forceinline__ bool wait_for(uint32_t* sync, int n, const int* list, uint32_t count, int spin_limit) {
    int ok = 1;
    const int t = threadIdx.x;
    if (t < n) {
        const uint32_t* f = flag_of(sync, list[t]);
        for (int spins = 0; __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < count; ++spins) {
            if ((spins & 31) == 31 &&
                __hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            if (spins >= spin_limit) {
                __hip_atomic_store(sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return __syncthreads_and(ok) != 0;
}

// All stores of this block completed, then store `value` to `word`.
__device__ __forceinline__ void publish_word(uint32_t* word, uint32_t value) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(word, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until `word` >= value (bounded, watching the abort word);
// false in every thread if the wait ran out or another block aborted.
__device__ __forceinline__ bool wait_word(const uint32_t* word, uint32_t value, uint32_t* sync, int spin_limit,
                                          uint32_t* shared_ok) {
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        for (int spins = 0; __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < value; ++spins) {
            if ((spins & 31) == 31 && __hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            if (spins >= spin_limit) {
                __hip_atomic_store(sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        *shared_ok = ok;
    }
    __syncthreads();
    return *shared_ok != 0;
}

// The blocks whose tiles lie within a tile's halo reach (and itself); returns
// their number (at most kMaxNeighbours).
__device__ __forceinline__ int neighbours_of(const Band2D& B, int logical, int nb, int* nbr) {
    const int tiles_i = (B.n0 + kT - 1) / kT, tiles_j = (B.n1 + kT - 1) / kT;
    const int ri = (B.W0 + 3 + kT - 1) / kT, rj = (B.W1 + 3 + kT - 1) / kT;
    const int ti = logical / tiles_j, tj = logical % tiles_j;
    int m = 0;
    for (int a = max(0, ti - ri); a <= min(tiles_i - 1, ti + ri); ++a)
        for (int b = max(0, tj - rj); b <= min(tiles_j - 1, tj + rj); ++b) {
            const int lg = a * tiles_j + b;   // logical tile -> block index (inverse of xcd_block)
            nbr[m++] = (nb % 8 != 0) ? lg : (lg % (nb / 8)) * 8 + lg / (nb / 8);
        }
    return m;
}

template <int PK, bool SPLIT>
__global__ void __launch_bounds__(kThr)
resident2d(Resident2D R) {
    __shared__ __attribute__((aligned(16))) Smem S;
    __shared__ Ctl C;                // this block's copy of the control state
    __shared__ int nbr[kMaxNeighbours];
    __shared__ int all[kFusedMaxBlocks];
    __shared__ int n_nbr;
    __shared__ uint32_t okw, word;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = (int)gridDim.x;
    const int slot = (int)blockIdx.x;
    Band2D B = R.B;
    const int logical = xcd_block();
    const Tile T = tile_of<SPLIT>(B, logical, lane);

    if (tid == 0) {
        n_nbr = neighbours_of(B, logical, nb, nbr);
        C = *R.ctl;
    }
    for (int t = tid; t < nb; t += kThr) all[t] = t;

    EpiArgs eb{};
    eb.kind = EpiKind::BUPDATE;
    eb.q = R.q;
    eb.b = R.b;
    eb.vec_ok = R.vec_ok;
    eb.part = R.part;
    EpiArgs ep{};
    ep.kind = EpiKind::PROX;
    ep.a = R.a;
    ep.p_out = R.p_out;
    ep.prox = R.prox;
    ep.vec_ok = R.vec_ok;
    ep.part = R.part;

    // factor bands: staged once for the whole launch
    if (SPLIT) {
        stage_bands_split(B, T, S);
    } else {
        f4 bj[UKM], bi[UKM];
        load_bands(B, T, bj, bi);
        store_bands(S, T, bj, bi);
    }
    // epilogue inputs that do not change over the iteration (q; the energy's fields)
    EpiIn inq, inp;
    if (wave < 4) {
        inq = epi_prefetch<EK_BUPDATE>(eb, T.eidx, T.ecnt);
        inp = epi_prefetch<PK>(ep, T.eidx, T.ecnt);
    }
    __syncthreads();
    const int nn = n_nbr;
    uint32_t count = 0;   // phases this block has published

    // One phase: stage the halo of X, contract, epilogue.  Specialised at
    // compile time on whether the epilogue accumulates the stop-test
    // partials, so the common iteration runs straight-line code.
    using yes = std::true_type;
    using no = std::false_type;
    auto phase = [&](auto ek, auto chkc, EpiArgs& E, const EpiIn& in, const float* X) {
        constexpr int EKv = decltype(ek)::value;
        constexpr bool CHK = decltype(chkc)::value;
        E.check = CHK ? 1 : 0;
        if (EKv >= EK_PROX) E.write_p = CHK ? 1 : 0;
        B.X = X;
        f4 bx[UXM];
        load_halo<true>(B, T, bx);
        store_halo(S, T, bx);
        contract_tile<EKv, true, SPLIT>(E, T, in, S, slot);
    };
    const std::integral_constant<int, EK_BUPDATE> ekb;
    const std::integral_constant<int, PK> ekp;

    for (int k = 1; k <= R.K; ++k) {
        // ---- t = xi^T a, b = q / t (and the violation of the previous iterate at checks)
        const bool chk = R.checks && k > 1 && (k - 1) % R.ce == 0;
        eb.t_out = R.hist ? R.hist + (2 * (int64_t)(k - 1)) * R.hist_stride : nullptr;
        EpiIn ia = inq;
        if (chk && wave < 4) ia.v = ld4_coh(R.b, T.eidx, T.ecnt, 0.f);
        if (!wait_for(R.sync, nn, nbr, count, R.spin_limit)) return;
        if (chk) phase(ekb, yes(), eb, ia, R.a);
        else phase(ekb, no(), eb, ia, R.a);
        publish(R.sync, slot, ++count);

        // Stop test: block 0 waits for every block's partials, takes the
        // decision and publishes it.  No block writes partials again before
        // it has seen the decision, so block 0 has read them all by then.
        // With check_every >= 2 and k < K the proximal half-step of this
        // iteration writes no partials and no p, so the other blocks run it
        // while block 0 decides and read the decision afterwards; a stop
        // then discards only scalings.  Otherwise they wait for it first.
        const bool spec = chk && R.ce >= 2 && k < R.K;
        const uint32_t chk_count = count;
        uint32_t decision = 0;
        if (chk) {
            if (slot == 0) {
                if (!wait_for(R.sync, nb, all, count, R.spin_limit)) return;
                if (wave == 0) ctl_update<true>(&C, R.part, nb, k, R.tol, 1, R.absorb, R.a_only);
                __syncthreads();
                if (tid == 0) {
                    Ctl* g = R.ctl;
                    g->done = C.done;
                    g->stop_iter = C.stop_iter;
                    g->nonfinite = C.nonfinite;
                    g->absorptions = C.absorptions;
                    g->absorb_pending = C.absorb_pending;
                    g->logmode = C.logmode;
                    g->exit_iter = C.absorb_pending ? k : 0;
                    g->err = C.err;
                    g->mass = C.mass;
                    g->maxloga = C.maxloga;
                    g->maxlogb = C.maxlogb;
                    __hip_atomic_store(R.sync + kDecision, (uint32_t)(C.done | (C.absorb_pending << 1)),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                publish_word(R.sync + kDecisionSeq, chk_count);
            }
            if (!spec) {
                if (!wait_word(R.sync + kDecisionSeq, chk_count, R.sync, R.spin_limit, &okw)) return;
                if (tid == 0)
                    word = __hip_atomic_load(R.sync + kDecision, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
                decision = word;
                if (decision & 1u) return;   // same decision in every block
            }
        }

        // ---- s = xi b, p = prox(s), a = p / s (p kept at candidate iterations)
        const bool cand = (R.checks && k % R.ce == 0) || k == R.K;
        ep.s_out = R.hist ? R.hist + (2 * (int64_t)(k - 1) + 1) * R.hist_stride : nullptr;
        if (!wait_for(R.sync, nn, nbr, count, R.spin_limit)) return;
        if (cand) phase(ekp, yes(), ep, inp, R.b);
        else phase(ekp, no(), ep, inp, R.b);
        publish(R.sync, slot, ++count);

        if (chk) {
            if (spec) {
                if (!wait_word(R.sync + kDecisionSeq, chk_count, R.sync, R.spin_limit, &okw)) return;
                if (tid == 0)
                    word = __hip_atomic_load(R.sync + kDecision, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
                decision = word;
                if (decision & 1u) return;   // same decision in every block
            }
            // An absorption switch takes effect after this proximal half-step:
            // the launch returns here (every block), and the host converts
            // the scalings to logs and runs the rest of the step on the
            // log-domain passes (recorded in ctl->exit_iter).
            if (decision & 2u) return;
        }
    }
}

// Reverse sweep of one step in one cooperative launch (same tiles, halo
// waits and device-scope exchange as resident2d): for k = K .. 1,
//   bbar = xi sbar_k  -> tbar_k = -bbar b / t,  qbar += bbar / t        (ADJ_B)
//   abar = xi tbar_k  -> sbar_{k-1}, wbar += ...                         (ADJ_PROX, k > 1)
// with t_k, s_k read from the recomputation's history.  Same tile code and
// order as the launch path: bit-identical results.
template <int AK, bool SPLIT>
__global__ void __launch_bounds__(kThr)
resident_adj(ResidentAdj R) {
    __shared__ __attribute__((aligned(16))) Smem S;
    __shared__ int nbr[kMaxNeighbours];
    __shared__ int n_nbr;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = (int)gridDim.x;
    const int slot = (int)blockIdx.x;
    Band2D B = R.B;
    const int logical = xcd_block();
    const Tile T = tile_of<SPLIT>(B, logical, lane);
    if (tid == 0) n_nbr = neighbours_of(B, logical, nb, nbr);
    if (SPLIT) {
        stage_bands_split(B, T, S);
    } else {
        f4 bj[UKM], bi[UKM];
        load_bands(B, T, bj, bi);
        store_bands(S, T, bj, bi);
    }
    EpiArgs eb{};
    eb.kind = EpiKind::ADJ_B;
    eb.q = R.q;
    eb.y = R.tbar;
    eb.acc = R.qbar;
    eb.vec_ok = R.vec_ok;
    EpiArgs ep{};
    ep.kind = EpiKind::ADJ_PROX;
    ep.y = R.sbar;
    ep.acc = R.wbar;
    ep.prox = R.prox;
    ep.sigma = R.sigma;
    ep.vec_ok = R.vec_ok;
    __syncthreads();
    const int nn = n_nbr;
    uint32_t count = 0;
    for (int k = R.K; k >= 1; --k) {
        eb.hin = R.hist + (2 * (int64_t)(k - 1)) * R.hist_stride;
        EpiIn ia;
        if (wave < 4) ia = epi_prefetch<EK_ADJ_B, true>(eb, T.eidx, T.ecnt);
        if (!wait_for(R.sync, nn, nbr, count, R.spin_limit)) return;
        {
            B.X = R.sbar;
            f4 bx[UXM];
            load_halo<true>(B, T, bx);
            store_halo(S, T, bx);
        }
        contract_tile<EK_ADJ_B, true, SPLIT>(eb, T, ia, S, slot);
        publish(R.sync, slot, ++count);
        if (k == 1) break;
        ep.hin = R.hist + (2 * (int64_t)(k - 2) + 1) * R.hist_stride;
        EpiIn ip;
        if (wave < 4) ip = epi_prefetch<AK, true>(ep, T.eidx, T.ecnt);
        if (!wait_for(R.sync, nn, nbr, count, R.spin_limit)) return;
        {
            B.X = R.tbar;
            f4 bx[UXM];
            load_halo<true>(B, T, bx);
            store_halo(S, T, bx);
        }
        contract_tile<AK, true, SPLIT>(ep, T, ip, S, slot);
        publish(R.sync, slot, ++count);
    }
}

template <bool SPLIT>
const void* adjoint_kernel_of(int prox_kind) {
    switch (prox_kind) {
        case JKO_F_ZERO: return reinterpret_cast<const void*>(&resident_adj<EK_ADJ_PROX + JKO_F_ZERO, SPLIT>);
        case JKO_F_CONGESTION:
            return reinterpret_cast<const void*>(&resident_adj<EK_ADJ_PROX + JKO_F_CONGESTION, SPLIT>);
        case JKO_F_POROUS: return reinterpret_cast<const void*>(&resident_adj<EK_ADJ_PROX + JKO_F_POROUS, SPLIT>);
        case JKO_F_GEN_ENTROPY:
            return reinterpret_cast<const void*>(&resident_adj<EK_ADJ_PROX + JKO_F_GEN_ENTROPY, SPLIT>);
        default: return reinterpret_cast<const void*>(&resident_adj<EK_ADJ_PROX + JKO_F_ENTROPY, SPLIT>);
    }
}

template <bool SPLIT>
const void* resident_kernel_of(int prox_kind) {
    switch (prox_kind) {
        case JKO_F_ZERO: return reinterpret_cast<const void*>(&resident2d<EK_PROX + JKO_F_ZERO, SPLIT>);
        case JKO_F_CONGESTION: return reinterpret_cast<const void*>(&resident2d<EK_PROX + JKO_F_CONGESTION, SPLIT>);
        case JKO_F_CONGESTION_BINARY:
            return reinterpret_cast<const void*>(&resident2d<EK_PROX + JKO_F_CONGESTION_BINARY, SPLIT>);
        case JKO_F_GEN_ENTROPY: return reinterpret_cast<const void*>(&resident2d<EK_PROX + JKO_F_GEN_ENTROPY, SPLIT>);
        case JKO_F_POROUS: return reinterpret_cast<const void*>(&resident2d<EK_PROX + JKO_F_POROUS, SPLIT>);
        default: return reinterpret_cast<const void*>(&resident2d<EK_PROX + JKO_F_ENTROPY, SPLIT>);
    }
}

const void* resident_kernel(int prox_kind, bool split) {
    return split ? resident_kernel_of<true>(prox_kind) : resident_kernel_of<false>(prox_kind);
}

template <bool SPLIT>
void launch_g2(int ek, dim3 grid, dim3 block, const Band2D& b, const EpiArgs& epi, hipStream_t stream) {
    switch (ek) {
        case EK_STORE: hipLaunchKernelGGL((gibbs2d_kernel<EK_STORE, SPLIT>), grid, block, 0, stream, b, epi); break;
        case EK_BUPDATE: hipLaunchKernelGGL((gibbs2d_kernel<EK_BUPDATE, SPLIT>), grid, block, 0, stream, b, epi); break;
        case EK_MONITOR: hipLaunchKernelGGL((gibbs2d_kernel<EK_MONITOR, SPLIT>), grid, block, 0, stream, b, epi); break;
        case EK_PROX + JKO_F_ZERO:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_PROX + JKO_F_ZERO, SPLIT>), grid, block, 0, stream, b, epi); break;
        case EK_PROX + JKO_F_CONGESTION:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_PROX + JKO_F_CONGESTION, SPLIT>), grid, block, 0, stream, b, epi);
            break;
        case EK_PROX + JKO_F_CONGESTION_BINARY:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_PROX + JKO_F_CONGESTION_BINARY, SPLIT>), grid, block, 0, stream, b,
                               epi);
            break;
        case EK_PROX + JKO_F_GEN_ENTROPY:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_PROX + JKO_F_GEN_ENTROPY, SPLIT>), grid, block, 0, stream, b, epi);
            break;
        case EK_PROX + JKO_F_POROUS:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_PROX + JKO_F_POROUS, SPLIT>), grid, block, 0, stream, b, epi); break;
        case EK_PROX + JKO_F_ENTROPY:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_PROX + JKO_F_ENTROPY, SPLIT>), grid, block, 0, stream, b, epi); break;
        case EK_ADJ_B: hipLaunchKernelGGL((gibbs2d_kernel<EK_ADJ_B, SPLIT>), grid, block, 0, stream, b, epi); break;
        case EK_ADJ_PROX + JKO_F_ZERO:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_ADJ_PROX + JKO_F_ZERO, SPLIT>), grid, block, 0, stream, b, epi);
            break;
        case EK_ADJ_PROX + JKO_F_CONGESTION:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_ADJ_PROX + JKO_F_CONGESTION, SPLIT>), grid, block, 0, stream, b,
                               epi);
            break;
        case EK_ADJ_PROX + JKO_F_GEN_ENTROPY:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_ADJ_PROX + JKO_F_GEN_ENTROPY, SPLIT>), grid, block, 0, stream, b,
                               epi);
            break;
        case EK_ADJ_PROX + JKO_F_POROUS:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_ADJ_PROX + JKO_F_POROUS, SPLIT>), grid, block, 0, stream, b, epi);
            break;
        default:
            hipLaunchKernelGGL((gibbs2d_kernel<EK_ADJ_PROX + JKO_F_ENTROPY, SPLIT>), grid, block, 0, stream, b, epi);
            break;
    }
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

bool gibbs2d_fits(int n0, int n1, int W0, int W1, int32_t precision) {
    // halo = tile + 2 W + 3 (alignment), rounded up to 16 (32 for split)
    const int rnd = precision == JKO_SPLIT_BF16 ? 31 : 15;
    const int h0 = ((std::min(n0, kT + 2 * W0 + 3)) + rnd) & ~rnd;
    const int h1 = ((std::min(n1, kT + 2 * W1 + 3)) + rnd) & ~rnd;
    return h0 <= kHalo && h1 <= kHalo;
}

hipError_t launch_gibbs2d(const Band2D& b, int32_t precision, const EpiArgs& epi, int* nblocks,
                          hipStream_t stream) {
    const int64_t nb = gibbs2d_blocks(b.n0, b.n1);
    if (nblocks) *nblocks = (int)nb;
    const dim3 grid((unsigned)nb), block(kThr);
    if (precision == JKO_SPLIT_BF16) launch_g2<true>(ek_of(epi), grid, block, b, epi, stream);
    else launch_g2<false>(ek_of(epi), grid, block, b, epi, stream);
    return hipGetLastError();
}

// Every block of `fn` co-resident on the device (cooperative launch possible).
bool grid_fits(const void* fn, int64_t blocks) {
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThr, 0) != hipSuccess) return false;
    return (int64_t)per_cu * cus >= blocks;
}

bool resident_adj_fits(int n0, int n1, int W0, int W1, int prox_kind, int32_t precision) {
    const int ti = (n0 + kT - 1) / kT, tj = (n1 + kT - 1) / kT;
    const int ri = (W0 + 3 + kT - 1) / kT, rj = (W1 + 3 + kT - 1) / kT;
    if ((int64_t)std::min(ti, 2 * ri + 1) * std::min(tj, 2 * rj + 1) > kMaxNeighbours) return false;
    if (gibbs2d_blocks(n0, n1) > kFusedMaxBlocks) return false;
    const void* fn = precision == JKO_SPLIT_BF16 ? adjoint_kernel_of<true>(prox_kind) : adjoint_kernel_of<false>(prox_kind);
    return grid_fits(fn, gibbs2d_blocks(n0, n1));
}

hipError_t launch_resident_adj(const ResidentAdj& r, hipStream_t stream) {
    const int64_t nb = gibbs2d_blocks(r.B.n0, r.B.n1);
    ResidentAdj arg = r;
    void* args[] = {&arg};
    const void* fn = r.split ? adjoint_kernel_of<true>(r.prox.kind) : adjoint_kernel_of<false>(r.prox.kind);
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)nb), dim3(kThr), args, 0, stream);
}

bool resident2d_fits(int n0, int n1, int W0, int W1, int prox_kind, int32_t precision) {
    const int ti = (n0 + kT - 1) / kT, tj = (n1 + kT - 1) / kT;
    const int ri = (W0 + 3 + kT - 1) / kT, rj = (W1 + 3 + kT - 1) / kT;
    if ((int64_t)std::min(ti, 2 * ri + 1) * std::min(tj, 2 * rj + 1) > kMaxNeighbours) return false;
    if (gibbs2d_blocks(n0, n1) > kFusedMaxBlocks) return false;
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, resident_kernel(prox_kind, precision == JKO_SPLIT_BF16),
                                                     kThr, 0) != hipSuccess)
        return false;
    return (int64_t)per_cu * cus >= gibbs2d_blocks(n0, n1);
}

hipError_t launch_resident2d(const Resident2D& r, hipStream_t stream) {
    const int64_t nb = gibbs2d_blocks(r.B.n0, r.B.n1);
    Resident2D arg = r;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(resident_kernel(r.prox.kind, r.split != 0), dim3((unsigned)nb), dim3(kThr), args, 0,
                                      stream);
}

}  // namespace jko
