// Building blocks of the panel-form axis contractions, shared by the
// launch-per-pass kernels (contract.hip) and the resident pass kernel
// (respass.hip).
//
// A pass contracts the contiguous axis of its input X (R rows of n) with the
// one-axis factor K1 and writes the contracted axis first:
//     Y[i][r] = sum_k K1[i][k] X[r][k]
// An output tile of TR rows r and TI positions i multiplies over the tile's
// band of k, [kb0, kb1) aligned to 32, staged in LDS as panels of 32 k:
//   X            [panel][TR rows][32 floats]   (128-byte rows)
//   K1 (FP32)    [panel][TI rows][32 floats]
//   K1 (split)   hi and lo, [panel][TI rows][32 bf16]   (64-byte rows)
// by buffer loads that write LDS directly (16 bytes per lane, no registers on
// the way, rows past the buffer's range read as zeros), all issued at once:
// one memory round trip per tile, and every index a shift or mask.  Within a
// row the 16-byte chunks are XOR-swizzled so the operand reads of 16
// consecutive rows fall in distinct banks:
//   128-byte rows: chunk c of row r is stored at c ^ ((r >> 1) & 7)
//    64-byte rows: chunk c of row r is stored at c ^ ((r >> 2) & 3)
// Split path: X is staged in FP32 and split into bfloat16 hi + lo (hardware
// round-to-nearest-even) as each wave reads its operand.
#pragma once

#include "epilogue.h"

namespace jko {

constexpr int kPanelMax = 5;      // panels per tile band (160 k): 64-row tiles, 3D passes
constexpr int kPanelMaxRot = 7;   // panels per tile band of 32 x 32 tiles (224 k, 56 KiB of LDS)
constexpr int kBufRsrcWord3 = 0x00020000;
constexpr int kCpolCoherent = 16;   // SC1: loads and stores coherent across the XCDs

// Dynamic LDS bytes of the panel form for a tile of TR + TI rows and NP panels
// (the staged epilogue tile reuses it).
constexpr int panel_lds_bytes(int TR, int TI, int NP) { return NP * (TR + TI) * 128; }

// The k range [kb0, kb1) a 32-aligned chunk of outputs [i0, i0 + TI) of an
// axis of n cells multiplies with band half-width W, rounded out to 32.
__device__ __forceinline__ int panel_k0(int i0, int W) { return max(0, i0 - W) & ~31; }
__device__ __forceinline__ int panel_k1(int i0, int TI, int W, int n) { return min(n, (i0 + TI + W + 31) & ~31); }

// The hardware hands consecutive blocks to the 8 XCDs in turn; give each XCD
// a contiguous range of tiles so that tiles sharing an X row strip share an L2.
__device__ __forceinline__ int xcd_logical_block() {
    const int nb = gridDim.x, bid = blockIdx.x;
    if (nb % 8 != 0) return bid;
    return (bid % 8) * (nb / 8) + bid / 8;
}

// Output offset of row r, position i of a rotating pass: the (R, n) input
// becomes (n, R), or, with stacked fields of Rb rows, each field's (Rb, n)
// block becomes its own (n, Rb) block.  Runs of 4 rows never straddle two
// fields (Rb is a multiple of 4).
__device__ __forceinline__ int out_index(int i, int r, int n, int Rb) {
    const int f = r / Rb;
    return f * n * Rb + i * Rb + (r - f * Rb);
}

// Paired tiles (two stacked fields, B = 2): rows [0, TH) of a TR-row tile
// are rows r0 .. r0 + TH of field 0, rows [TH, TR) the same rows of field 1,
// so that the epilogue holds both fields' values of its cells.  X row of
// tile row d:
__device__ __forceinline__ int pair_row(int d, int r0, int Rb, int TH) {
    return d < TH ? r0 + d : Rb + r0 + d - TH;
}

// The epilogue units of a tile: unit u of the block finishes 4 consecutive
// rows rl of output position il.  Unpaired tiles: eidx is the output offset
// of the run, ecnt its length within the R rows.  Paired tiles: each of the
// first TH / 4 units of an output position finishes 4 consecutive cells of
// both fields, eidx is the field-0 offset i * Rb + r.
template <int TR, int TI, int UE, bool PAIR>
__device__ __forceinline__ void tile_units(int tid, int i0, int r0, int n, int R, int Rb, int* eidx, int* ecnt) {
    constexpr int TH = TR / 2;
#pragma unroll
    for (int u = 0; u < UE; ++u) {
        const int unit = tid + u * kThreads;
        const int il = unit / (TR / 4), rl = 4 * (unit % (TR / 4));
        const int i = i0 + il, r = r0 + rl;
        if (PAIR) {
            ecnt[u] = (unit < TI * TR / 4 && rl < TH && i < n) ? max(0, min(4, Rb - r)) : 0;
            eidx[u] = i * Rb + r;
        } else {
            ecnt[u] = (unit < TI * TR / 4 && i < n) ? max(0, min(4, R - r)) : 0;
            eidx[u] = out_index(i, r, n, Rb);
        }
    }
}

// The capacity of each paired unit's cells (kappa, or kappa_scalar).
template <int UE>
__device__ __forceinline__ void attr_capacity(const EpiArgs& E, const int* eidx, const int* ecnt, f4* kap) {
#pragma unroll
    for (int u = 0; u < UE; ++u) {
        kap[u] = f4{E.prox.kappa_s, E.prox.kappa_s, E.prox.kappa_s, E.prox.kappa_s};
        if (E.prox.kappa && ecnt[u] > 0) {
            if (ecnt[u] == 4 && E.vec_ok) kap[u] = *reinterpret_cast<const f4*>(E.prox.kappa + eidx[u]);
            else
                for (int e = 0; e < ecnt[u]; ++e) kap[u][e] = E.prox.kappa[eidx[u] + e];
        }
    }
}

// The attraction's proximal step (Section 5.2) on a paired tile staged in LDS
// as [i][TS] rows: p = min(s_1^alpha s_2^(1 - alpha), kappa), a_m = p / s_m
// (0/0 = 0).  COH: a is stored at device scope.
template <int TR, int TS, int UE, bool COH = false>
__device__ __forceinline__ void attr_finish(const EpiArgs& E, const float* tile, int tid, int n, int Rb,
                                            const int* eidx, const int* ecnt, const f4* kap) {
    constexpr int TH = TR / 2;
    const float al = E.alpha;
    const int64_t N = (int64_t)n * Rb;
#pragma unroll
    for (int u = 0; u < UE; ++u) {
        const int unit = tid + u * kThreads;
        const int il = unit / (TR / 4), rl = 4 * (unit % (TR / 4));
        if (ecnt[u] == 0) continue;
        const f4 s1 = *reinterpret_cast<const f4*>(&tile[il * TS + rl]);
        const f4 s2 = *reinterpret_cast<const f4*>(&tile[il * TS + TH + rl]);
        f4 pv, a1, a2;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float g = (s1[e] > 0.f && s2[e] > 0.f) ? expf(al * logf(s1[e]) + (1.f - al) * logf(s2[e])) : 0.f;
            pv[e] = fminf(g, kap[u][e]);
            a1[e] = pv[e] == 0.f ? 0.f : pv[e] / s1[e];
            a2[e] = pv[e] == 0.f ? 0.f : pv[e] / s2[e];
        }
        const int o = eidx[u];
        if (COH) {
            const bool v4 = E.vec_ok && ((o & 3) == 0);
            st4_coh(E.a, o, ecnt[u], v4, a1);
            st4_coh(E.a + N, o, ecnt[u], v4, a2);
            if (E.write_p) st4(E.p_out, o, ecnt[u], v4, pv);
        } else if (ecnt[u] == 4 && E.vec_ok) {
            *reinterpret_cast<f4*>(E.p_out + o) = pv;
            *reinterpret_cast<f4*>(E.a + o) = a1;
            *reinterpret_cast<f4*>(E.a + N + o) = a2;
        } else {
            for (int e = 0; e < ecnt[u]; ++e) {
                E.p_out[o + e] = pv[e];
                E.a[o + e] = a1[e];
                E.a[N + o + e] = a2[e];
            }
        }
    }
}

// Wait until at most `n` (0 .. 31) of this wave's vector memory operations are
// outstanding; they complete in issue order.  The count is split over the
// immediate's bits 3:0 and 15:14; expcnt and lgkmcnt are left unwaited.
template <int N>
__device__ __forceinline__ void wait_vm_n() {
    __builtin_amdgcn_s_waitcnt((N & 0xF) | (((N >> 4) & 3) << 14) | (0x7 << 4) | (0xF << 8));
}
__device__ __forceinline__ void wait_vm(int n) {
    // n is the same in every lane; read it as a scalar so the switch is a
    // uniform branch (a wait in a case skipped under exec would still run)
    switch (__builtin_amdgcn_readfirstlane(n)) {
#define JKO_VM(N) case N: wait_vm_n<N>(); break;
        JKO_VM(0) JKO_VM(1) JKO_VM(2) JKO_VM(3) JKO_VM(4) JKO_VM(5) JKO_VM(6) JKO_VM(7)
        JKO_VM(8) JKO_VM(9) JKO_VM(10) JKO_VM(11) JKO_VM(12) JKO_VM(13) JKO_VM(14) JKO_VM(15)
        JKO_VM(16) JKO_VM(17) JKO_VM(18) JKO_VM(19) JKO_VM(20) JKO_VM(21) JKO_VM(22) JKO_VM(23)
        JKO_VM(24) JKO_VM(25) JKO_VM(26) JKO_VM(27) JKO_VM(28) JKO_VM(29) JKO_VM(30)
#undef JKO_VM
        default: wait_vm_n<31>(); break;
    }
}

// A 16-byte copy from a buffer to LDS; CPOL: cache policy (kCpolCoherent for
// data another block wrote at device scope during the launch).
template <int CPOL = 0>
__device__ __forceinline__ void lds_copy16(__amdgpu_buffer_rsrc_t rs, void* lds, int voff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)lds, 16, voff, 0, 0, CPOL);
}

// The same copy as an instruction the compiler does not track.  The compiler
// makes every LDS read wait for all the LDS copies it knows to be in flight
// (it cannot tell which LDS they write), so with tracked copies a read of a
// landed panel still waits for the whole band; issued this way, the caller
// alone waits for them (vmcnt, then a barrier) before any access to their
// destination.  The buffer descriptor is built by hand (base, no stride,
// range in bytes); the s_nop covers the wait states between writing M0 or the
// descriptor and the load that reads them.
typedef int i4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ i4v buffer_desc(const void* base, int nbytes) {
    const uint64_t a = reinterpret_cast<uint64_t>(base);
    return i4v{(int)(uint32_t)a, (int)(uint32_t)((a >> 32) & 0xFFFF), nbytes, kBufRsrcWord3};
}

__device__ __forceinline__ void lds_copy16_untracked(i4v rs, void* lds, int voff) {
    const uint32_t m0 = (uint32_t)reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) void*)lds);
    asm volatile("s_nop 4\n\tbuffer_load_dwordx4 %0, %1, 0 offen lds" ::"v"(voff), "s"(rs), "{m0}"(m0) : "memory");
}

// Copies of one X panel (TR rows of 32 k from column kc) into xs, this wave's
// share: 8 rows of 128 bytes per wave-wide copy.  row_of(d) is the X row of
// tile row d.
template <int TR, int CPOL, typename RowOf>
__device__ __forceinline__ void panel_copy_x(__amdgpu_buffer_rsrc_t rx, float* xs, int n, int kc, int wave, int lane,
                                             RowOf row_of) {
    constexpr int XPP = TR / 8;
    const int xrow = lane >> 3, xch = lane & 7;
#pragma unroll
    for (int q = wave; q < XPP; q += kThreads / 64) {
        const int row = q * 8 + xrow;
        const int col = kc + 4 * (xch ^ ((row >> 1) & 7));
        lds_copy16<CPOL>(rx, xs + q * 256, 4 * (row_of(row) * n + col));
    }
}

// Copies of one K1 panel (rows i0 .. i0 + TI of 32 k from column kc), this
// wave's share: FP32 rows into kf, or bf16 hi and lo rows into kh and kl.
template <int TI, bool SPLIT>
__device__ __forceinline__ void panel_copy_k(__amdgpu_buffer_rsrc_t rk, __amdgpu_buffer_rsrc_t rkl, float* kf,
                                             uint16_t* kh, uint16_t* kl, int n, int i0, int kc, int wave, int lane) {
    if (SPLIT) {
        // 16 rows of one bf16 panel (hi, then lo) per wave-wide copy
        constexpr int KPP = TI / 16;
        constexpr int KQ = 2 * KPP;
        const int krow = lane >> 2, kch = lane & 3;
#pragma unroll
        for (int q = wave; q < KQ; q += kThreads / 64) {
            const int qq = q < KPP ? q : q - KPP;
            const int row = qq * 16 + krow;
            const int col = kc + 8 * (kch ^ ((row >> 2) & 3));
            const int voff = 2 * ((i0 + row) * n + col);
            if (q < KPP) lds_copy16(rk, kh + qq * 512, voff);
            else lds_copy16(rkl, kl + qq * 512, voff);
        }
    } else {
        constexpr int KQ = TI / 8;
        const int xrow = lane >> 3, xch = lane & 7;
#pragma unroll
        for (int q = wave; q < KQ; q += kThreads / 64) {
            const int row = q * 8 + xrow;
            const int col = kc + 4 * (xch ^ ((row >> 1) & 7));
            lds_copy16(rk, kf + q * 256, 4 * ((i0 + row) * n + col));
        }
    }
}

// One panel's products: acc[a][b] += (this wave's FM 16-row fragments of the
// panel's X rows) x (its FN 16-row fragments of the panel's K1 rows), over the
// panel's 32 k.  xp, kf / kh, kl: the panel's X and K1 rows in LDS.
template <int TR, int TI, int WR, int WI, bool SPLIT>
__device__ __forceinline__ void panel_mma(f4 (&acc)[TR / WR / 16][TI / WI / 16], const float* xpanel,
                                          const float* kf, const uint16_t* kh, const uint16_t* kl, int lane, int wr,
                                          int wi) {
    constexpr int FM = TR / WR / 16;
    constexpr int FN = TI / WI / 16;
    const int s8 = (lane >> 1) & 7;   // 128-byte row swizzle of every row this lane reads
    const int g = lane >> 4;
    const float* xp = xpanel + (wr * 16 * FM + (lane & 15)) * 32;
    if (SPLIT) {
        const int s4 = (lane >> 2) & 3;
        bf8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) {
            const float* xr = xp + a * 16 * 32;
            const f4 v0 = *reinterpret_cast<const f4*>(xr + 4 * ((2 * g) ^ s8));
            const f4 v1 = *reinterpret_cast<const f4*>(xr + 4 * ((2 * g + 1) ^ s8));
            split_bf16(v0, v1, ah[a], al[a]);
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int o = (wi * 16 * FN + b * 16 + (lane & 15)) * 32 + 8 * (g ^ s4);
            bh[b] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(kh + o));
            bl[b] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(kl + o));
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
            const int ch = 4 * ((4 * h + g) ^ s8);
            f4 av[FM], bv[FN];
#pragma unroll
            for (int a = 0; a < FM; ++a) av[a] = *reinterpret_cast<const f4*>(xp + a * 16 * 32 + ch);
#pragma unroll
            for (int b = 0; b < FN; ++b)
                bv[b] = *reinterpret_cast<const f4*>(kf + (wi * 16 * FN + b * 16 + (lane & 15)) * 32 + ch);
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

// The accumulator tile into LDS as [i][TS] rows (TS = TR + 4), for the
// epilogue units.
template <int TR, int TI, int WR, int WI>
__device__ __forceinline__ void panel_stage_acc(float* tile, const f4 (&acc)[TR / WR / 16][TI / WI / 16], int lane,
                                                int wr, int wi) {
    constexpr int FM = TR / WR / 16;
    constexpr int FN = TI / WI / 16;
    constexpr int TS = TR + 4;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int rl = wr * 16 * FM + a * 16 + 4 * (lane >> 4);
            const int il = wi * 16 * FN + b * 16 + (lane & 15);
            *reinterpret_cast<f4*>(&tile[il * TS + rl]) = acc[a][b];
        }
}

}  // namespace jko
