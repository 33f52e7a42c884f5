// Fused 2D Gibbs application  Y = K1_0 X K1_1  on MFMA (gfx950), and the
// resident 2D kernels that run a whole step's iteration (and its reverse
// sweep) in one launch.
//
// On a uniform 2D grid xi = K1_0 (x) K1_1 (separable Gaussian, Section 4.1 of
// the paper).  In float32 the factor K1[i][j] = exp(-(x_i - x_j)^2/gamma) is
// exactly zero beyond a band |i - j| > W (exp underflows), so an output tile
// Y[I][J] (TT x TT) only needs the input halo X[I +- W][J +- W]:
//     Z[ib][j] = sum_jb X[ib][jb] K1_1[j][jb]        (ib in I +- W, j in J)
//     Y[i][j]  = sum_ib K1_0[i][ib] Z[ib][j]
// Skipping the zero band is exact, and the intermediate Z never leaves LDS, so
// one application costs one launch instead of one per axis.  Each block owns
// one output tile; the tile order is XCD-aware so that neighbouring tiles,
// which share most of their halo, share an L2.
//
// Two tile edges: TT = 16 while the grid has at most 256 such tiles (one
// block per CU), TT = 32 for grids of up to 256 tiles of 32 x 32 (512 x 512
// at most).  The larger tile spends fewer redundant halo rows per output
// (the first contraction runs over all (TT + 2W) halo rows) and keeps the
// whole grid resident where 16 x 16 tiles would need four blocks per CU.  Its
// halo takes most of the LDS, so its intermediate Z reuses the halo's space
// once the first contraction has read it.
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
// bit-identical to the launch-per-application path with the same tile edge.
#include <algorithm>
#include <type_traits>

#include "control.h"
#include "epilogue.h"
#include "resident_sync.h"

namespace jko {

namespace {

constexpr int kThr = 512;       // 8 waves per block
constexpr int kMaxNeighbours = 9 * 9;   // halo reach of at most 4 tiles per side
constexpr int kRS = 68;          // padded row of the partial sums (64 lanes)

// Per tile edge TT: the largest halo edge held in LDS, the outputs each
// thread finishes and the waves that finish them.
template <int TT> struct Geom;
template <> struct Geom<16> {
    static constexpr int kHalo = 128;
    static constexpr bool kAliasZ = false;   // Z has its own LDS
    static constexpr int kOut = 1;           // waves 0-3, one output per lane
};
template <> struct Geom<32> {
    static constexpr int kHalo = 160;
    static constexpr bool kAliasZ = true;    // Z reuses the halo's LDS
    static constexpr int kOut = 2;           // all 8 waves, two outputs per lane
};

template <int TT, bool SPLIT>
struct Smem {
    static constexpr int H = Geom<TT>::kHalo;
    static constexpr int S = H + 4;    // padded LDS row (floats)
    static constexpr int S2 = H + 8;   // padded LDS row of a bfloat16 band (16-byte aligned)
    // every array starts on a 16-byte boundary (the unused one-element arrays
    // of the other precision would otherwise shift the rest by 8 bytes and
    // split the 16-byte LDS accesses)
    alignas(16) float Xs[H * S];                   // [ib][jb]
    alignas(16) float Kj[SPLIT ? 1 : TT * S];      // [j][jb]  = K1_1[j0+j][jb0+jb]
    alignas(16) float Ki[SPLIT ? 1 : TT * S];      // [i][ib]  = K1_0[i0+i][ib0+ib]
    alignas(16) uint16_t Kjh[SPLIT ? TT * S2 : 1];   // split: bfloat16 hi / lo of the bands
    alignas(16) uint16_t Kjl[SPLIT ? TT * S2 : 1];
    alignas(16) uint16_t Kih[SPLIT ? TT * S2 : 1];
    alignas(16) uint16_t Kil[SPLIT ? TT * S2 : 1];
    alignas(16) float Zown[Geom<TT>::kAliasZ ? 1 : TT * S];   // [j][ib]
    alignas(16) float red[8 * 4 * kRS];            // [wave][element][lane] partial sums of the second contraction
    double shd[8];
    __device__ float* Z() { return Geom<TT>::kAliasZ ? Xs : Zown; }
};

__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, bid = blockIdx.x;
    if (nb % 8 != 0) return bid;
    return (bid % 8) * (nb / 8) + bid / 8;
}

// Geometry of one block's tile.  The halo start is aligned down to a
// multiple of 4 (the extra entries meet exact zeros of the band).
template <int TT>
struct Tile {
    int fld;                                          // field of a batch (0 without one)
    int i0, j0, ib0, jb0, LI, LJ, LIp, LJp;
    int eidx[Geom<TT>::kOut], ecnt[Geom<TT>::kOut];   // outputs this thread finishes (ecnt = 0: none)
};

// Halo extents are padded to whole MFMA k-steps: 16 (FP32) or 32 (split).
template <int TT, bool SPLIT = false>
__device__ __forceinline__ Tile<TT> tile_of(const Band2D& B, int logical, int lane) {
    constexpr int RND = SPLIT ? 32 : 16;
    Tile<TT> T;
    const int tiles_j = (B.n1 + TT - 1) / TT;
    const int per = ((B.n0 + TT - 1) / TT) * tiles_j;   // tiles of one field
    T.fld = logical / per;
    const int t = logical - T.fld * per;
    T.i0 = (t / tiles_j) * TT;
    T.j0 = (t % tiles_j) * TT;
    T.ib0 = max(0, T.i0 - B.W0) & ~3;
    T.jb0 = max(0, T.j0 - B.W1) & ~3;
    T.LI = min(B.n0, T.i0 + TT + B.W0) - T.ib0;
    T.LJ = min(B.n1, T.j0 + TT + B.W1) - T.jb0;
    T.LIp = (T.LI + RND - 1) & ~(RND - 1);
    T.LJp = (T.LJ + RND - 1) & ~(RND - 1);
    // each store instruction writes whole row segments: TT = 16, wave v < 4,
    // lane l finish row i0 + 4 v + (l >> 4), column j0 + (l & 15); TT = 32,
    // thread t finishes outputs t and t + 512 of the tile in row-major order
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < Geom<TT>::kOut; ++u) {
        int il, jl;
        bool mine;
        if (TT == 16) {
            il = 4 * wave + (lane >> 4);
            jl = lane & 15;
            mine = wave < 4;
        } else {
            const int o = threadIdx.x + kThr * u;
            il = o / TT;
            jl = o % TT;
            mine = true;
        }
        const int ei = T.i0 + il, ej = T.j0 + jl;
        T.eidx[u] = (T.fld * B.n0 + ei) * B.n1 + ej;
        T.ecnt[u] = (mine && ei < B.n0 && ej < B.n1) ? 1 : 0;
    }
    return T;
}

template <int TT> constexpr int halo_units() {   // max halo units (4 floats) per thread
    return (Geom<TT>::kHalo * (Geom<TT>::kHalo / 4) + kThr - 1) / kThr;
}
template <int TT> constexpr int band_units() {   // max factor-band units per thread
    return (TT * (Geom<TT>::kHalo / 4) + kThr - 1) / kThr;
}

// Issue the loads of the X halo (zero outside the grid).  COH: device-scope
// loads (buffer loads with scope bit SC1, range-checked by the descriptor) of
// a field other blocks of the same launch wrote.
constexpr int kCpolDevice = 16;   // SC1: device scope

template <int TT, bool COH = false>
__device__ __forceinline__ void load_halo(const Band2D& B, const Tile<TT>& T, f4 (&bx)[halo_units<TT>()]) {
    const int tid = threadIdx.x;
    const int nux = T.LIp * (T.LJp / 4);
    const bool vec1 = (B.n1 & 3) == 0;
    __amdgpu_buffer_rsrc_t rs;
    if (COH)
        rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(B.X), (short)0, B.n0 * B.n1 * 4, 0x00020000);
#pragma unroll
    for (int u = 0; u < halo_units<TT>(); ++u) {
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

template <int TT, bool SPLIT>
__device__ __forceinline__ void store_halo(Smem<TT, SPLIT>& S, const Tile<TT>& T,
                                           const f4 (&bx)[halo_units<TT>()]) {
    constexpr int kS = Smem<TT, SPLIT>::S;
    const int tid = threadIdx.x;
    const int nux = T.LIp * (T.LJp / 4);
#pragma unroll
    for (int u = 0; u < halo_units<TT>(); ++u) {
        const int unit = tid + u * kThr;
        if (unit < nux) {
            const int r = unit / (T.LJp / 4), c = 4 * (unit % (T.LJp / 4));
            *reinterpret_cast<f4*>(&S.Xs[r * kS + c]) = bx[u];
        }
    }
}

// Stage the two FP32 factor bands of the tile (zero outside the band).
template <int TT>
__device__ __forceinline__ void stage_bands(const Band2D& B, const Tile<TT>& T, Smem<TT, false>& S) {
    constexpr int kS = Smem<TT, false>::S;
    constexpr int UK = band_units<TT>();
    const int tid = threadIdx.x;
    const int nkj = TT * (T.LJp / 4), nki = TT * (T.LIp / 4);
    const bool vec1 = (B.n1 & 3) == 0, vec0 = (B.n0 & 3) == 0;
    f4 bj[UK], bi[UK];
#pragma unroll
    for (int u = 0; u < UK; ++u) {
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
#pragma unroll
    for (int u = 0; u < UK; ++u) {
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
template <int TT>
__device__ __forceinline__ void stage_bands(const Band2D& B, const Tile<TT>& T, Smem<TT, true>& S) {
    constexpr int kS2 = Smem<TT, true>::S2;
    constexpr int UK = band_units<TT>();
    const int tid = threadIdx.x;
    const int nkj = TT * (T.LJp / 4), nki = TT * (T.LIp / 4);
    u16x4 jh[UK], jl[UK], ih[UK], il[UK];
#pragma unroll
    for (int u = 0; u < UK; ++u) {
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
    for (int u = 0; u < UK; ++u) {
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

// Both contractions of the staged tile and its epilogue, then the block's
// partials into slot `slot`.  Xs and the factor bands are staged, not yet
// synced.  COH: the scalings and partials the epilogue writes use
// device-scope stores.  SPLIT: each FP32 operand (X, then Z) is split into
// bfloat16 hi + lo as it is read and multiplied with the factor bands' hi /
// lo, three products (hi*hi + hi*lo + lo*hi) on v_mfma_f32_16x16x32_bf16,
// FP32 accumulation.
//
// The first contraction computes Z in 16 x 16 fragments (16 halo rows x 16
// output columns).  TT = 16: wave f owns the 16-row fragment f.  TT = 32: the
// 2 F fragments (F row fragments, two column fragments each) go to the waves
// round-robin, so each SIMD carries the same share; the results stay in
// registers until every wave has finished reading the halo, whose LDS Z then
// takes over.  The second contraction is one fragment per 16 x 16 output
// block, its k range cut into 16-wide (FP32) or 32-wide (split) chunks spread
// over the waves; the per-wave partial sums are added in a fixed order.
template <int TT, int EK, bool COH = false, bool SPLIT = false>
__device__ __forceinline__ void contract_tile(const EpiArgs& E, const Tile<TT>& T,
                                              const EpiIn (&ein)[Geom<TT>::kOut], Smem<TT, SPLIT>& S, int slot) {
    constexpr int kS = Smem<TT, SPLIT>::S, kS2 = Smem<TT, SPLIT>::S2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int koff = 4 * (lane >> 4);
    const int LIp = T.LIp, LJp = T.LJp;
    float* const Zs = S.Z();
    __syncthreads();

    // ---- Z = X K1_1^T over the halo rows
    const int F = LIp / 16;
    // one 16 x 16 fragment of Z: halo rows 16 f.., output columns 16 c..
    auto zfrag = [&](int f, int c) -> f4 {
        if (SPLIT) {
            const int k8 = 8 * (lane >> 4);
            f4 acc = f4{0.f, 0.f, 0.f, 0.f};
            const float* xr = &S.Xs[(16 * f + (lane & 15)) * kS + k8];
            const uint16_t* khr = &S.Kjh[(16 * c + (lane & 15)) * kS2 + k8];
            const uint16_t* klr = &S.Kjl[(16 * c + (lane & 15)) * kS2 + k8];
            for (int c0 = 0; c0 < LJp; c0 += 32) {
                bf8 ah, al;
                split_bf16(*reinterpret_cast<const f4*>(xr + c0), *reinterpret_cast<const f4*>(xr + c0 + 4), ah, al);
                const bf8 bh = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(khr + c0));
                const bf8 bl = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(klr + c0));
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
            }
            return acc;
        } else {
            // even and odd k-chunks go to two accumulators (independent MFMA chains)
            f4 acc0 = f4{0.f, 0.f, 0.f, 0.f}, acc1 = f4{0.f, 0.f, 0.f, 0.f};
            const float* xr = &S.Xs[(16 * f + (lane & 15)) * kS + koff];
            const float* kr = &S.Kj[(16 * c + (lane & 15)) * kS + koff];
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
            return acc0 + acc1;
        }
    };
    // acc holds Z[ib = 16 f + koff + e][j = 16 c + (lane & 15)]
    if (TT == 16) {
        if (wave < F) {
            const f4 acc = zfrag(wave, 0);
            *reinterpret_cast<f4*>(&Zs[(lane & 15) * kS + 16 * wave + koff]) = acc;
        }
    } else {
        constexpr int kMaxFr = 3;   // 2 F <= 20 fragments over 8 waves
        f4 zacc[kMaxFr];
#pragma unroll
        for (int q = 0; q < kMaxFr; ++q) {
            const int t = wave + 8 * q;
            if (t < 2 * F) zacc[q] = zfrag(t >> 1, t & 1);
        }
        __syncthreads();   // every wave is done with the halo: Z takes over its LDS
#pragma unroll
        for (int q = 0; q < kMaxFr; ++q) {
            const int t = wave + 8 * q;
            if (t < 2 * F)
                *reinterpret_cast<f4*>(&Zs[(16 * (t & 1) + (lane & 15)) * kS + 16 * (t >> 1) + koff]) = zacc[q];
        }
    }
    __syncthreads();

    // ---- Y^T = Z^T K1_0^T: each 16 x 16 output block (column fragment jf,
    // row fragment if) over its k-chunks
    auto yfrag = [&](int jf, int ifr, int c0, f4 acc) -> f4 {
        if (SPLIT) {
            const int k = c0 + 8 * (lane >> 4);
            bf8 ah, al;
            const float* zr = &Zs[(16 * jf + (lane & 15)) * kS + k];
            split_bf16(*reinterpret_cast<const f4*>(zr), *reinterpret_cast<const f4*>(zr + 4), ah, al);
            const bf8 bh = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&S.Kih[(16 * ifr + (lane & 15)) * kS2 + k]));
            const bf8 bl = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&S.Kil[(16 * ifr + (lane & 15)) * kS2 + k]));
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
        } else {
            const f4 a = *reinterpret_cast<const f4*>(&Zs[(16 * jf + (lane & 15)) * kS + c0 + koff]);
            const f4 b = *reinterpret_cast<const f4*>(&S.Ki[(16 * ifr + (lane & 15)) * kS + c0 + koff]);
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], acc, 0, 0, 0);
        }
        return acc;
    };
    constexpr int KC = SPLIT ? 32 : 16;   // k per chunk
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    if (TT == 16) {
        // one fragment, chunk w for wave w (at most 8 chunks)
        if (KC * wave < LIp) acc = yfrag(0, 0, KC * wave, acc);
    } else {
        // four fragments; wave w takes fragment w & 3 and every other chunk
        // from w >> 2 on, accumulated in increasing k
        const int fr = wave & 3;
        for (int c0 = KC * (wave >> 2); c0 < LIp; c0 += 2 * KC) acc = yfrag(fr & 1, fr >> 1, c0, acc);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) S.red[(wave * 4 + e) * kRS + lane] = acc[e];
    __syncthreads();
    EpiAcc ea;
#pragma unroll
    for (int u = 0; u < Geom<TT>::kOut; ++u) {
        // Y[i][j] sits in element j & 3 of MFMA lane (i & 15) + 16 ((j & 15) >> 2)
        // of its fragment's waves
        int il, jl;
        if (TT == 16) {
            il = 4 * wave + (lane >> 4);
            jl = lane & 15;
        } else {
            const int o = tid + kThr * u;
            il = o / TT;
            jl = o % TT;
        }
        const int src = (il & 15) + 16 * ((jl & 15) >> 2), e = jl & 3;
        float y;
        if (TT == 16) {
            if (wave >= 4) continue;
            y = S.red[e * kRS + src];
#pragma unroll
            for (int w = 1; w < 8; ++w) y += S.red[(w * 4 + e) * kRS + src];
        } else {
            const int fr = (jl >> 4) + 2 * (il >> 4);
            y = S.red[(fr * 4 + e) * kRS + src] + S.red[((fr + 4) * 4 + e) * kRS + src];
        }
        epi_apply<EK, COH, 1>(E, T.eidx[u], T.ecnt[u], f4{y, 0.f, 0.f, 0.f}, false, ein[u], ea);
    }
    epi_finish<COH>(E, ea, slot, S.shd);
}

template <int TT, int EK, bool SPLIT>
__global__ void __launch_bounds__(kThr)
gibbs2d_kernel(Band2D B, EpiArgs E) {
    __shared__ __attribute__((aligned(16))) Smem<TT, SPLIT> S;

    // The control flags are read here but acted on only after the halo loads
    // are in flight, so their latencies overlap.
    int done = 0;
    if (E.ctl) done = E.ctl->done | E.ctl->logmode;
    const int lane = threadIdx.x & 63;
    const Tile<TT> T = tile_of<TT, SPLIT>(B, xcd_block(), lane);
    B.X += (int64_t)T.fld * B.n0 * B.n1;   // this block's field of a batch

    // The finishing threads' epilogue inputs are fetched now, ahead of the
    // contraction.
    EpiIn ein[Geom<TT>::kOut];
#pragma unroll
    for (int u = 0; u < Geom<TT>::kOut; ++u) ein[u] = epi_prefetch<EK>(E, T.eidx[u], T.ecnt[u]);

    // the staging loads are issued before the LDS stores
    f4 bx[halo_units<TT>()];
    load_halo<TT>(B, T, bx);
    stage_bands<TT>(B, T, S);
    store_halo<TT, SPLIT>(S, T, bx);
    if (done) return;   // the step has stopped: nothing to compute (uniform)
    contract_tile<TT, EK, false, SPLIT>(E, T, ein, S, (int)blockIdx.x);
}

// ------------------------------------------------------------ resident kernel
//
// Synchronisation between the blocks of one launch: resident_sync.h.

// The blocks whose tiles lie within a tile's halo reach (and itself); returns
// their number (at most kMaxNeighbours).
template <int TT>
__device__ __forceinline__ int neighbours_of(const Band2D& B, int logical, int nb, int* nbr) {
    const int tiles_i = (B.n0 + TT - 1) / TT, tiles_j = (B.n1 + TT - 1) / TT;
    const int ri = (B.W0 + 3 + TT - 1) / TT, rj = (B.W1 + 3 + TT - 1) / TT;
    const int ti = logical / tiles_j, tj = logical % tiles_j;
    int m = 0;
    for (int a = max(0, ti - ri); a <= min(tiles_i - 1, ti + ri); ++a)
        for (int b = max(0, tj - rj); b <= min(tiles_j - 1, tj + rj); ++b) {
            const int lg = a * tiles_j + b;   // logical tile -> block index (inverse of xcd_block)
            nbr[m++] = (nb % 8 != 0) ? lg : (lg % (nb / 8)) * 8 + lg / (nb / 8);
        }
    return m;
}

template <int TT, int PK, bool SPLIT>
__global__ void __launch_bounds__(kThr)
resident2d(Resident2D R) {
    constexpr int NO = Geom<TT>::kOut;
    __shared__ __attribute__((aligned(16))) Smem<TT, SPLIT> S;
    __shared__ Ctl C;                // this block's copy of the control state
    __shared__ int nbr[kMaxNeighbours];
    __shared__ int all[kFusedMaxBlocks];
    __shared__ int n_nbr;
    __shared__ uint32_t okw, word;

    const int tid = threadIdx.x, lane = tid & 63;
    const int nb = (int)gridDim.x;
    const int slot = (int)blockIdx.x;
    Band2D B = R.B;
    const int logical = xcd_block();
    const Tile<TT> T = tile_of<TT, SPLIT>(B, logical, lane);

    if (tid == 0) {
        n_nbr = neighbours_of<TT>(B, logical, nb, nbr);
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
    stage_bands<TT>(B, T, S);
    // epilogue inputs that do not change over the iteration (q; the energy's fields)
    EpiIn inq[NO], inp[NO];
#pragma unroll
    for (int u = 0; u < NO; ++u) {
        inq[u] = epi_prefetch<EK_BUPDATE>(eb, T.eidx[u], T.ecnt[u]);
        inp[u] = epi_prefetch<PK>(ep, T.eidx[u], T.ecnt[u]);
    }
    __syncthreads();
    const int nn = n_nbr;
    uint32_t count = 0;   // phases this block has published

    // One phase: stage the halo of X, contract, epilogue.  Specialised at
    // compile time on whether the epilogue accumulates the stop-test
    // partials, so the common iteration runs straight-line code.
    using yes = std::true_type;
    using no = std::false_type;
    auto phase = [&](auto ek, auto chkc, EpiArgs& E, const EpiIn (&in)[NO], const float* X) {
        constexpr int EKv = decltype(ek)::value;
        constexpr bool CHK = decltype(chkc)::value;
        E.check = CHK ? 1 : 0;
        if (EKv >= EK_PROX) E.write_p = CHK ? 1 : 0;
        B.X = X;
        f4 bx[halo_units<TT>()];
        load_halo<TT, true>(B, T, bx);
        store_halo<TT, SPLIT>(S, T, bx);
        contract_tile<TT, EKv, true, SPLIT>(E, T, in, S, slot);
    };
    const std::integral_constant<int, EK_BUPDATE> ekb;
    const std::integral_constant<int, PK> ekp;

    for (int k = 1; k <= R.K; ++k) {
        // ---- t = xi^T a, b = q / t (and the violation of the previous iterate at checks)
        const bool chk = R.checks && k > 1 && (k - 1) % R.ce == 0;
        eb.t_out = R.hist ? R.hist + (2 * (int64_t)(k - 1)) * R.hist_stride : nullptr;
        EpiIn ia[NO];
#pragma unroll
        for (int u = 0; u < NO; ++u) {
            ia[u] = inq[u];
            if (chk) ia[u].v = ld4_coh(R.b, T.eidx[u], T.ecnt[u], 0.f);
        }
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
                if ((tid >> 6) == 0) ctl_update<true>(&C, R.part, nb, k, R.tol, 1, R.absorb, R.a_only);
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
template <int TT, int AK, bool SPLIT>
__global__ void __launch_bounds__(kThr)
resident_adj(ResidentAdj R) {
    constexpr int NO = Geom<TT>::kOut;
    __shared__ __attribute__((aligned(16))) Smem<TT, SPLIT> S;
    __shared__ int nbr[kMaxNeighbours];
    __shared__ int n_nbr;

    const int tid = threadIdx.x, lane = tid & 63;
    const int nb = (int)gridDim.x;
    const int slot = (int)blockIdx.x;
    Band2D B = R.B;
    const int logical = xcd_block();
    const Tile<TT> T = tile_of<TT, SPLIT>(B, logical, lane);
    if (tid == 0) n_nbr = neighbours_of<TT>(B, logical, nb, nbr);
    stage_bands<TT>(B, T, S);
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
        EpiIn ia[NO];
#pragma unroll
        for (int u = 0; u < NO; ++u) ia[u] = epi_prefetch<EK_ADJ_B, true>(eb, T.eidx[u], T.ecnt[u]);
        if (!wait_for(R.sync, nn, nbr, count, R.spin_limit)) return;
        {
            B.X = R.sbar;
            f4 bx[halo_units<TT>()];
            load_halo<TT, true>(B, T, bx);
            store_halo<TT, SPLIT>(S, T, bx);
        }
        contract_tile<TT, EK_ADJ_B, true, SPLIT>(eb, T, ia, S, slot);
        publish(R.sync, slot, ++count);
        if (k == 1) break;
        ep.hin = R.hist + (2 * (int64_t)(k - 2) + 1) * R.hist_stride;
        EpiIn ip[NO];
#pragma unroll
        for (int u = 0; u < NO; ++u) ip[u] = epi_prefetch<AK, true>(ep, T.eidx[u], T.ecnt[u]);
        if (!wait_for(R.sync, nn, nbr, count, R.spin_limit)) return;
        {
            B.X = R.tbar;
            f4 bx[halo_units<TT>()];
            load_halo<TT, true>(B, T, bx);
            store_halo<TT, SPLIT>(S, T, bx);
        }
        contract_tile<TT, AK, true, SPLIT>(ep, T, ip, S, slot);
        publish(R.sync, slot, ++count);
    }
}

template <int TT, bool SPLIT>
const void* adjoint_kernel_of(int prox_kind) {
    switch (prox_kind) {
        case JKO_F_ZERO: return reinterpret_cast<const void*>(&resident_adj<TT, EK_ADJ_PROX + JKO_F_ZERO, SPLIT>);
        case JKO_F_CONGESTION:
            return reinterpret_cast<const void*>(&resident_adj<TT, EK_ADJ_PROX + JKO_F_CONGESTION, SPLIT>);
        case JKO_F_POROUS: return reinterpret_cast<const void*>(&resident_adj<TT, EK_ADJ_PROX + JKO_F_POROUS, SPLIT>);
        case JKO_F_GEN_ENTROPY:
            return reinterpret_cast<const void*>(&resident_adj<TT, EK_ADJ_PROX + JKO_F_GEN_ENTROPY, SPLIT>);
        default: return reinterpret_cast<const void*>(&resident_adj<TT, EK_ADJ_PROX + JKO_F_ENTROPY, SPLIT>);
    }
}

const void* adjoint_kernel(int tile, int prox_kind, bool split) {
    if (tile == 32) return split ? adjoint_kernel_of<32, true>(prox_kind) : adjoint_kernel_of<32, false>(prox_kind);
    return split ? adjoint_kernel_of<16, true>(prox_kind) : adjoint_kernel_of<16, false>(prox_kind);
}

template <int TT, bool SPLIT>
const void* resident_kernel_of(int prox_kind) {
    switch (prox_kind) {
        case JKO_F_ZERO: return reinterpret_cast<const void*>(&resident2d<TT, EK_PROX + JKO_F_ZERO, SPLIT>);
        case JKO_F_CONGESTION:
            return reinterpret_cast<const void*>(&resident2d<TT, EK_PROX + JKO_F_CONGESTION, SPLIT>);
        case JKO_F_CONGESTION_BINARY:
            return reinterpret_cast<const void*>(&resident2d<TT, EK_PROX + JKO_F_CONGESTION_BINARY, SPLIT>);
        case JKO_F_GEN_ENTROPY:
            return reinterpret_cast<const void*>(&resident2d<TT, EK_PROX + JKO_F_GEN_ENTROPY, SPLIT>);
        case JKO_F_POROUS: return reinterpret_cast<const void*>(&resident2d<TT, EK_PROX + JKO_F_POROUS, SPLIT>);
        default: return reinterpret_cast<const void*>(&resident2d<TT, EK_PROX + JKO_F_ENTROPY, SPLIT>);
    }
}

const void* resident_kernel(int tile, int prox_kind, bool split) {
    if (tile == 32) return split ? resident_kernel_of<32, true>(prox_kind) : resident_kernel_of<32, false>(prox_kind);
    return split ? resident_kernel_of<16, true>(prox_kind) : resident_kernel_of<16, false>(prox_kind);
}

template <int TT, bool SPLIT>
void launch_g2(int ek, dim3 grid, dim3 block, const Band2D& b, const EpiArgs& epi, hipStream_t stream) {
#define JKO_G2(EKV) hipLaunchKernelGGL((gibbs2d_kernel<TT, EKV, SPLIT>), grid, block, 0, stream, b, epi); break
    switch (ek) {
        case EK_STORE: JKO_G2(EK_STORE);
        case EK_BUPDATE: JKO_G2(EK_BUPDATE);
        case EK_MONITOR: JKO_G2(EK_MONITOR);
        case EK_PROX + JKO_F_ZERO: JKO_G2(EK_PROX + JKO_F_ZERO);
        case EK_PROX + JKO_F_CONGESTION: JKO_G2(EK_PROX + JKO_F_CONGESTION);
        case EK_PROX + JKO_F_CONGESTION_BINARY: JKO_G2(EK_PROX + JKO_F_CONGESTION_BINARY);
        case EK_PROX + JKO_F_GEN_ENTROPY: JKO_G2(EK_PROX + JKO_F_GEN_ENTROPY);
        case EK_PROX + JKO_F_POROUS: JKO_G2(EK_PROX + JKO_F_POROUS);
        case EK_PROX + JKO_F_ENTROPY: JKO_G2(EK_PROX + JKO_F_ENTROPY);
        case EK_ADJ_B: JKO_G2(EK_ADJ_B);
        case EK_ADJ_PROX + JKO_F_ZERO: JKO_G2(EK_ADJ_PROX + JKO_F_ZERO);
        case EK_ADJ_PROX + JKO_F_CONGESTION: JKO_G2(EK_ADJ_PROX + JKO_F_CONGESTION);
        case EK_ADJ_PROX + JKO_F_GEN_ENTROPY: JKO_G2(EK_ADJ_PROX + JKO_F_GEN_ENTROPY);
        case EK_ADJ_PROX + JKO_F_POROUS: JKO_G2(EK_ADJ_PROX + JKO_F_POROUS);
        default: JKO_G2(EK_ADJ_PROX + JKO_F_ENTROPY);
    }
#undef JKO_G2
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

// Neighbour lists fit, and at most one block per CU of tiles.
bool resident_shape_fits(int n0, int n1, int W0, int W1, int tile) {
    const int ti = (n0 + tile - 1) / tile, tj = (n1 + tile - 1) / tile;
    const int ri = (W0 + 3 + tile - 1) / tile, rj = (W1 + 3 + tile - 1) / tile;
    if ((int64_t)std::min(ti, 2 * ri + 1) * std::min(tj, 2 * rj + 1) > kMaxNeighbours) return false;
    return gibbs2d_blocks(n0, n1, tile) <= kFusedMaxBlocks;
}

}  // namespace

int band_halfwidth(int n, double gamma) {
    // distances d with (d/n)^2/gamma > 152 ln 2 give exp(.) < 2^-152: zero in float32
    const double dmax = sqrt(152.0 * log(2.0) * gamma) * (double)n;
    const int W = (int)floor(dmax) + 1;
    return std::min(W, n - 1);
}

int64_t gibbs2d_blocks(int n0, int n1, int tile) {
    return (int64_t)((n0 + tile - 1) / tile) * ((n1 + tile - 1) / tile);
}

bool gibbs2d_fits(int n0, int n1, int W0, int W1, int32_t precision, int tile) {
    // halo = tile + 2 W + 3 (alignment), rounded up to 16 (32 for split)
    if (tile != 16 && tile != 32) return false;
    const int cap = tile == 16 ? Geom<16>::kHalo : Geom<32>::kHalo;
    const int rnd = precision == JKO_SPLIT_BF16 ? 31 : 15;
    const int h0 = ((std::min(n0, tile + 2 * W0 + 3)) + rnd) & ~rnd;
    const int h1 = ((std::min(n1, tile + 2 * W1 + 3)) + rnd) & ~rnd;
    return h0 <= cap && h1 <= cap;
}

hipError_t launch_gibbs2d(const Band2D& b, int32_t precision, const EpiArgs& epi, int* nblocks,
                          hipStream_t stream) {
    const int64_t nb = gibbs2d_blocks(b.n0, b.n1, b.tile) * std::max(1, b.batch);
    if (nblocks) *nblocks = (int)nb;
    const dim3 grid((unsigned)nb), block(kThr);
    const bool split = precision == JKO_SPLIT_BF16;
    if (b.tile == 32) {
        if (split) launch_g2<32, true>(ek_of(epi), grid, block, b, epi, stream);
        else launch_g2<32, false>(ek_of(epi), grid, block, b, epi, stream);
    } else {
        if (split) launch_g2<16, true>(ek_of(epi), grid, block, b, epi, stream);
        else launch_g2<16, false>(ek_of(epi), grid, block, b, epi, stream);
    }
    return hipGetLastError();
}

bool resident_adj_fits(int n0, int n1, int W0, int W1, int prox_kind, int32_t precision, int tile) {
    if (!resident_shape_fits(n0, n1, W0, W1, tile)) return false;
    return grid_fits(adjoint_kernel(tile, prox_kind, precision == JKO_SPLIT_BF16), gibbs2d_blocks(n0, n1, tile));
}

hipError_t launch_resident_adj(const ResidentAdj& r, hipStream_t stream) {
    const int64_t nb = gibbs2d_blocks(r.B.n0, r.B.n1, r.B.tile);
    ResidentAdj arg = r;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(adjoint_kernel(r.B.tile, r.prox.kind, r.split != 0), dim3((unsigned)nb),
                                      dim3(kThr), args, 0, stream);
}

bool resident2d_fits(int n0, int n1, int W0, int W1, int prox_kind, int32_t precision, int tile) {
    if (!resident_shape_fits(n0, n1, W0, W1, tile)) return false;
    return grid_fits(resident_kernel(tile, prox_kind, precision == JKO_SPLIT_BF16), gibbs2d_blocks(n0, n1, tile));
}

hipError_t launch_resident2d(const Resident2D& r, hipStream_t stream) {
    const int64_t nb = gibbs2d_blocks(r.B.n0, r.B.n1, r.B.tile);
    Resident2D arg = r;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(resident_kernel(r.B.tile, r.prox.kind, r.split != 0), dim3((unsigned)nb),
                                      dim3(kThr), args, 0, stream);
}

}  // namespace jko
