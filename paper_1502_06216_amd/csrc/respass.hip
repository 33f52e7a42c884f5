// The resident pass kernel: a whole 2D JKO step (every iteration, the stop
// test, the absorption decision) in one cooperative launch, for bands too
// wide for the fused tile kernel's halo.
//
// Each application of xi is the pair of rotating panel passes (panel.h):
//   pass 0: U[j][r] = sum_k K1_1[j][k] X[r][k]   (axis 1; U is the field
//           transposed, rows along axis 1)
//   pass 1: Y[i][j] = sum_k K1_0[i][k] U[j][k]   (axis 0, back to row-major,
//           with the b-update or proximal epilogue)
// so one iteration is four passes: a -> u0 -> (t, b), b -> u1 -> (s, p, a).
// Block t owns one 32 x 32 output tile of each pass and keeps both axes'
// factor panels of its tiles in LDS for the whole launch; between passes it
// waits only for the blocks whose outputs its next pass reads (the blocks
// sharing its rows whose outputs fall in its band of k), instead of at a
// launch boundary.  The products, in the same panel order as the launched
// passes, give the same bits.
//
// With two stacked fields (the attraction's couplings) every tile is paired:
// 16 rows of field 0 and the same 16 rows of field 1, so the proximal step,
// which couples the fields cell by cell, finishes inside the tile.
//
// Ordering: values a pass writes for other blocks (u, b, a, the partials) are
// stored at device scope and read with device-scope loads; a block publishes
// its pass count once its stores have completed (resident_sync.h).  The
// wait lists are symmetric (a block also waits for the blocks that read its
// outputs) and u has one buffer per half-step, so a block never overwrites a
// value another block still has to read:
//   a (written by the s pass 1, read by the next t pass 0 of its readers):
//     before its next s pass 1 the block's s pass 0 waited for those readers
//     to finish their t pass 1, hence their t pass 0;
//   b: likewise one half-step later;
//   u0 (written by the t pass 0, read by the t pass 1 of its readers):
//     before its next t pass 0 the block's s pass 1 waited for those readers
//     to finish their s pass 0, hence their t pass 1; u1 likewise.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "control.h"
#include "epilogue.h"
#include "panel.h"
#include "resident_sync.h"

namespace jko {

namespace {

constexpr int kRT = 32;                  // tile: 32 rows x 32 outputs per pass
constexpr int kRPanels = kPanelMaxRot;   // band of each axis: at most 7 panels (224 k)
constexpr int kRMaxNbr = 64;             // wait-list entries per pass

// Geometry of the grid's tiles.  Pass 0 of block t: rows [r0, r0 + rows) of
// each field (axis 0), outputs [i0, i0 + 32) (axis 1); pass 1: rows along
// axis 1, outputs along axis 0.  Unpaired tiles (one field): both passes of
// a block cover the same 32 x 32 cells.  Paired tiles: 16 rows of each field.
struct RGeo {
    int n0, n1, W0, W1;
    bool pair;
};

__device__ __forceinline__ void tile_of(const RGeo& g, int t, int pass, int* r0, int* i0) {
    const int T0 = g.n0 / kRT, T1 = g.n1 / kRT;
    if (!g.pair) {
        // the launched axis-0 pass orders its tiles (axis-1 block, axis-0
        // block); so do the blocks here, so that partial slot t holds the
        // same cells in both
        const int I = t % T0, J = t / T0;
        *r0 = pass == 0 ? kRT * I : kRT * J;
        *i0 = pass == 0 ? kRT * J : kRT * I;
    } else {
        const int I1 = t / T1, J1 = t % T1;   // pass 0: 16 rows of axis 0, 32 outputs of axis 1
        *r0 = pass == 0 ? 16 * I1 : 16 * (2 * J1 + (I1 & 1));
        *i0 = pass == 0 ? kRT * J1 : kRT * (I1 >> 1);
    }
}

// Cells [a0, a1) x [b0, b1) (axis 0 x axis 1) that pass `pass` of block t
// writes (out) or reads (in).
struct Box {
    int a0, a1, b0, b1;
};
__device__ __forceinline__ bool meets(const Box& x, const Box& y) {
    return x.a0 < y.a1 && y.a0 < x.a1 && x.b0 < y.b1 && y.b0 < x.b1;
}
__device__ __forceinline__ Box box_of(const RGeo& g, int t, int pass, bool out) {
    int r0, i0;
    tile_of(g, t, pass, &r0, &i0);
    const int rows = g.pair ? 16 : kRT;
    if (pass == 0) {
        // rows along axis 0, outputs (or the band of k read) along axis 1
        const int c0 = out ? i0 : panel_k0(i0, g.W1), c1 = out ? i0 + kRT : panel_k1(i0, kRT, g.W1, g.n1);
        return Box{r0, r0 + rows, c0, c1};
    }
    const int c0 = out ? i0 : panel_k0(i0, g.W0), c1 = out ? i0 + kRT : panel_k1(i0, kRT, g.W0, g.n0);
    return Box{c0, c1, r0, r0 + rows};
}

// The blocks pass `pass` of block t waits for: those whose outputs it reads
// (pass 0 reads what pass 1 wrote, pass 1 what pass 0 wrote) and those that
// read its outputs; block indices (inverse of the XCD order).  Thread 0 only.
__device__ int wait_list(const RGeo& g, int t, int pass, int nb, int* list) {
    const int other = 1 - pass;
    const Box in = box_of(g, t, pass, false), out = box_of(g, t, other, true);
    int m = 0;
    for (int y = 0; y < nb; ++y) {
        // y's outputs of the other pass meet this pass's input, or this
        // block's outputs of the other pass meet y's input of this pass
        const bool feeds = meets(box_of(g, y, other, true), in);
        const bool reads = meets(out, box_of(g, y, pass, false));
        if (!(feeds || reads)) continue;
        if (m < kRMaxNbr) list[m] = (nb % 8 != 0) ? y : (y % (nb / 8)) * 8 + y / (nb / 8);
        ++m;
    }
    return m;
}

template <bool SPLIT, int PK, bool PAIR>
__global__ void __launch_bounds__(kThreads)
resident_pass2d(ResidentPass2D R) {
    constexpr int TR = kRT, TI = kRT, WR = 2, WI = 2;
    constexpr int TH = TR / 2;
    constexpr int TS = TR + 4;
    constexpr int UE = (TI * TR / 4 + kThreads - 1) / kThreads;
    constexpr int PAN = TR * 32;   // floats of one X or K panel
    static_assert(TI * TS <= kRPanels * PAN, "the staged tile fits in the X panels");
    __shared__ __attribute__((aligned(16))) float Xs[kRPanels * PAN];
    __shared__ __attribute__((aligned(16))) float Kf[SPLIT ? 1 : 2 * kRPanels * PAN];
    __shared__ __attribute__((aligned(16))) uint16_t Kh[SPLIT ? 2 * kRPanels * PAN : 1];
    __shared__ __attribute__((aligned(16))) uint16_t Kl[SPLIT ? 2 * kRPanels * PAN : 1];
    __shared__ Ctl C;
    __shared__ int nbr[2][kRMaxNbr];
    __shared__ int n_nbr[2];
    __shared__ int all[kFusedMaxBlocks];
    __shared__ uint32_t okw, word;
    __shared__ double shd[8];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave % WR, wi = wave / WR;
    const int nb = (int)gridDim.x;
    const int slot = (int)blockIdx.x;
    const int t = xcd_logical_block();
    const RGeo g{R.n0, R.n1, R.W0, R.W1, PAIR};
    const int64_t N = (int64_t)R.n0 * R.n1;

    // per pass: contracted length, rows per field, tile origin, k range
    int r0[2], i0[2], kb0[2], np[2];
    const int nlen[2] = {R.n1, R.n0};
    const int Rb[2] = {R.n0, R.n1};
    const int W[2] = {R.W1, R.W0};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        tile_of(g, t, s, &r0[s], &i0[s]);
        kb0[s] = panel_k0(i0[s], W[s]);
        np[s] = (panel_k1(i0[s], TI, W[s], nlen[s]) - kb0[s]) >> 5;
    }
    if (tid == 0) {
        n_nbr[0] = wait_list(g, t, 0, nb, nbr[0]);
        n_nbr[1] = wait_list(g, t, 1, nb, nbr[1]);
        C = *R.ctl;
    }
    for (int i = tid; i < nb; i += kThreads) all[i] = i;

    // both passes' factor panels, once for the whole launch
    {
        const float* Kp[2] = {R.K1, R.K0};
        const uint16_t* Khp[2] = {R.K1hi, R.K0hi};
        const uint16_t* Klp[2] = {R.K1lo, R.K0lo};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int n = nlen[s];
            const __amdgpu_buffer_rsrc_t rk = __builtin_amdgcn_make_buffer_rsrc(
                SPLIT ? (void*)const_cast<uint16_t*>(Khp[s]) : (void*)const_cast<float*>(Kp[s]), (short)0,
                SPLIT ? n * n * 2 : n * n * 4, kBufRsrcWord3);
            const __amdgpu_buffer_rsrc_t rkl = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<uint16_t*>(SPLIT ? Klp[s] : Khp[s]), (short)0, n * n * 2, kBufRsrcWord3);
            for (int p = 0; p < np[s]; ++p) {
                const int o = (s * kRPanels + p) * PAN;
                panel_copy_k<TI, SPLIT>(rk, rkl, Kf + (SPLIT ? 0 : o), Kh + (SPLIT ? o : 0), Kl + (SPLIT ? o : 0),
                                        n, i0[s], kb0[s] + 32 * p, wave, lane);
            }
        }
    }

    // epilogue units of pass 0 (the store of u) and pass 1 (b-update and
    // proximal step), and the inputs of pass 1's epilogues that do not change
    int eidx[2][UE], ecnt[2][UE];
    tile_units<TR, TI, UE, PAIR>(tid, i0[0], r0[0], nlen[0], R.B * Rb[0], Rb[0], eidx[0], ecnt[0]);
    tile_units<TR, TI, UE, PAIR>(tid, i0[1], r0[1], nlen[1], R.B * Rb[1], Rb[1], eidx[1], ecnt[1]);

    EpiArgs eb{};
    eb.kind = EpiKind::BUPDATE;
    eb.q = R.q;
    eb.b = R.b;
    eb.vec_ok = R.vec_ok;
    eb.part = R.part;
    EpiArgs ep{};
    ep.kind = PAIR ? EpiKind::ATTR_PROX : EpiKind::PROX;
    ep.a = R.a;
    ep.p_out = R.p_out;
    ep.prox = R.prox;
    ep.alpha = R.alpha;
    ep.vec_ok = R.vec_ok;
    ep.part = R.part;
    constexpr int NF = PAIR ? 2 : 1;   // fields each epilogue unit finishes
    EpiIn inq[NF][UE], inp[UE];
    f4 kap[UE];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int u = 0; u < UE; ++u) inq[f][u] = epi_prefetch<EK_BUPDATE>(eb, eidx[1][u] + f * (int)N, ecnt[1][u]);
    if (PAIR) {
        attr_capacity<UE>(ep, eidx[1], ecnt[1], kap);
    } else {
#pragma unroll
        for (int u = 0; u < UE; ++u) inp[u] = epi_prefetch<PK>(ep, eidx[1][u], ecnt[1][u]);
    }
    wait_vm_n<0>();
    __syncthreads();
    const int nn0 = n_nbr[0], nn1 = n_nbr[1];
    if (nn0 > kRMaxNbr || nn1 > kRMaxNbr) {
        // a wait list that does not fit: abort the launch (every waiting
        // block sees the abort word and returns; the host reports it)
        if (tid == 0) __hip_atomic_store(R.sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    uint32_t count = 0;   // passes this block has published

    // One pass: stage the rows' band of X in LDS (device-scope copies), the
    // panel products, the accumulator tile to LDS, the epilogue.
    using yes = std::true_type;
    using no = std::false_type;
    auto run_pass = [&](auto passc, auto ekc, auto chkc, const float* X, float* Y, EpiArgs& E, const EpiIn(&ein)[NF][UE]) {
        constexpr int s = decltype(passc)::value;
        constexpr int EK = decltype(ekc)::value;
        constexpr bool CHK = decltype(chkc)::value;
        const int n = nlen[s];
        const int rows_total = R.B * Rb[s];
        {
            const __amdgpu_buffer_rsrc_t rx =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(X), (short)0, rows_total * n * 4, kBufRsrcWord3);
            auto row_of = [&](int d) { return PAIR ? pair_row(d, r0[s], Rb[s], TH) : r0[s] + d; };
            for (int p = 0; p < np[s]; ++p)
                panel_copy_x<TR, kCpolCoherent>(rx, Xs + p * PAN, n, kb0[s] + 32 * p, wave, lane, row_of);
        }
        wait_vm_n<0>();
        __syncthreads();
        f4 acc[1][1] = {{f4{0.f, 0.f, 0.f, 0.f}}};
        const int ko = s * kRPanels * PAN;
        for (int p = 0; p < np[s]; ++p)
            panel_mma<TR, TI, WR, WI, SPLIT>(acc, Xs + p * PAN, Kf + (SPLIT ? 0 : ko + p * PAN),
                                             Kh + (SPLIT ? ko + p * PAN : 0), Kl + (SPLIT ? ko + p * PAN : 0), lane,
                                             wr, wi);
        __syncthreads();
        float* tile = Xs;
        panel_stage_acc<TR, TI, WR, WI>(tile, acc, lane, wr, wi);
        __syncthreads();
        if (EK == EK_STORE) {
#pragma unroll
            for (int u = 0; u < UE; ++u) {
                const int unit = tid + u * kThreads;
                const int il = unit / (TR / 4), rl = 4 * (unit % (TR / 4));
                const int c = ecnt[s][u];
                if (c == 0) continue;
                const bool v4 = R.vec_ok && ((eidx[s][u] & 3) == 0);
                st4_coh(Y, eidx[s][u], c, v4, *reinterpret_cast<const f4*>(&tile[il * TS + rl]));
                if (PAIR) st4_coh(Y, eidx[s][u] + (int)N, c, v4, *reinterpret_cast<const f4*>(&tile[il * TS + TH + rl]));
            }
        } else if (EK == EK_ATTR) {
            E.write_p = (CHK && E.p_out) ? 1 : 0;
            attr_finish<TR, TS, UE, true>(E, tile, tid, nlen[1], Rb[1], eidx[1], ecnt[1], kap);
        } else {
            E.check = CHK ? 1 : 0;
            if (EK >= EK_PROX) E.write_p = (CHK && E.p_out) ? 1 : 0;
            EpiAcc ea;
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int u = 0; u < UE; ++u) {
                    const int unit = tid + u * kThreads;
                    const int il = unit / (TR / 4), rl = 4 * (unit % (TR / 4));
                    if (ecnt[s][u] == 0) continue;
                    const f4 v = *reinterpret_cast<const f4*>(&tile[il * TS + f * TH + rl]);
                    epi_apply<EK, true>(E, eidx[s][u] + f * (int)N, ecnt[s][u], v, false, ein[f][u], ea);
                }
            epi_finish<true>(E, ea, slot, shd);
        }
    };
    const std::integral_constant<int, 0> p0;
    const std::integral_constant<int, 1> p1;
    const std::integral_constant<int, EK_STORE> eks;
    const std::integral_constant<int, EK_BUPDATE> ekb;
    const std::integral_constant<int, PK> ekp;
    EpiIn inpp[NF][UE];
#pragma unroll
    for (int u = 0; u < UE; ++u) inpp[0][u] = inp[u];

    for (int k = 1; k <= R.K; ++k) {
        // ---- t = xi^T a, b = q / t (and the violation of the previous iterate at checks)
        const bool chk = R.checks && k > 1 && (k - 1) % R.ce == 0;
        EpiIn ia[NF][UE];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int u = 0; u < UE; ++u) {
                ia[f][u] = inq[f][u];
                if (chk) ia[f][u].v = ld4_coh(R.b, eidx[1][u] + f * (int)N, ecnt[1][u], 0.f);
            }
        if (!wait_for(R.sync, nn0, nbr[0], count, R.spin_limit)) return;
        run_pass(p0, eks, no(), R.a, R.u0, eb, ia);
        publish(R.sync, slot, ++count);
        if (!wait_for(R.sync, nn1, nbr[1], count, R.spin_limit)) return;
        if (chk) run_pass(p1, ekb, yes(), R.u0, nullptr, eb, ia);
        else run_pass(p1, ekb, no(), R.u0, nullptr, eb, ia);
        publish(R.sync, slot, ++count);

        // Stop test: block 0 waits for every block's partials, takes the
        // decision and publishes it (as in the resident tile kernel).
        const bool spec = chk && R.ce >= 2 && k < R.K;
        const uint32_t chk_count = count;
        uint32_t decision = 0;
        if (chk) {
            if (slot == 0) {
                if (!wait_for(R.sync, nb, all, count, R.spin_limit)) return;
                if ((tid >> 6) == 0) ctl_update<true>(&C, R.part, nb, k, R.tol, R.check_mass, R.absorb, R.a_only);
                __syncthreads();
                if (tid == 0) {
                    Ctl* gc = R.ctl;
                    gc->done = C.done;
                    gc->stop_iter = C.stop_iter;
                    gc->nonfinite = C.nonfinite;
                    gc->absorptions = C.absorptions;
                    gc->absorb_pending = C.absorb_pending;
                    gc->logmode = C.logmode;
                    gc->exit_iter = C.absorb_pending ? k : 0;
                    gc->err = C.err;
                    gc->mass = C.mass;
                    gc->maxloga = C.maxloga;
                    gc->maxlogb = C.maxlogb;
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
        if (!wait_for(R.sync, nn0, nbr[0], count, R.spin_limit)) return;
        run_pass(p0, eks, no(), R.b, R.u1, ep, inpp);
        publish(R.sync, slot, ++count);
        if (!wait_for(R.sync, nn1, nbr[1], count, R.spin_limit)) return;
        if (cand) run_pass(p1, ekp, yes(), R.u1, nullptr, ep, inpp);
        else run_pass(p1, ekp, no(), R.u1, nullptr, ep, inpp);
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
            // an absorption switch takes effect after this proximal
            // half-step: the launch returns here (every block) and the host
            // runs the rest of the step on the log-domain passes
            if (decision & 2u) return;
        }
    }
}

template <bool SPLIT>
const void* rp_kernel_of(int kind, bool pair) {
    if (pair) return reinterpret_cast<const void*>(&resident_pass2d<SPLIT, EK_ATTR, true>);
    switch (kind) {
        case JKO_F_ZERO: return reinterpret_cast<const void*>(&resident_pass2d<SPLIT, EK_PROX + JKO_F_ZERO, false>);
        case JKO_F_CONGESTION:
            return reinterpret_cast<const void*>(&resident_pass2d<SPLIT, EK_PROX + JKO_F_CONGESTION, false>);
        case JKO_F_CONGESTION_BINARY:
            return reinterpret_cast<const void*>(&resident_pass2d<SPLIT, EK_PROX + JKO_F_CONGESTION_BINARY, false>);
        case JKO_F_POROUS: return reinterpret_cast<const void*>(&resident_pass2d<SPLIT, EK_PROX + JKO_F_POROUS, false>);
        case JKO_F_ENTROPY:
            return reinterpret_cast<const void*>(&resident_pass2d<SPLIT, EK_PROX + JKO_F_ENTROPY, false>);
        case JKO_F_GEN_ENTROPY:
            return reinterpret_cast<const void*>(&resident_pass2d<SPLIT, EK_PROX + JKO_F_GEN_ENTROPY, false>);
        default: return nullptr;
    }
}

const void* rp_kernel(int kind, bool pair, bool split) {
    return split ? rp_kernel_of<true>(kind, pair) : rp_kernel_of<false>(kind, pair);
}

int band_panels32(int n, int W) {
    int np = 0;
    for (int i0 = 0; i0 < n; i0 += kRT) {
        const int kb0 = std::max(0, i0 - W) & ~31;
        const int kb1 = std::min(n, (i0 + kRT + W + 31) & ~31);
        np = std::max(np, (kb1 - kb0) >> 5);
    }
    return np;
}

}  // namespace

// One block per 32 x 32 tile of each field (paired tiles: 16 rows of each of
// the two fields).
int64_t resident_pass2d_blocks(int n0, int n1, int B) { return (int64_t)B * (n0 / kRT) * (n1 / kRT); }

bool resident_pass2d_shape_fits(int n0, int n1, int W0, int W1, int B) {
    if (n0 % kRT != 0 || n1 % kRT != 0 || (B != 1 && B != 2)) return false;
    if (resident_pass2d_blocks(n0, n1, B) > kFusedMaxBlocks) return false;
    if (band_panels32(n0, W0) > kRPanels || band_panels32(n1, W1) > kRPanels) return false;
    return (int64_t)B * n0 * n1 * 4 < ((int64_t)1 << 31);
}

bool resident_pass2d_fits(int n0, int n1, int W0, int W1, int B, int prox_kind, int32_t precision) {
    if (!resident_pass2d_shape_fits(n0, n1, W0, W1, B)) return false;
    const void* fn = rp_kernel(prox_kind, B == 2, precision == JKO_SPLIT_BF16);
    if (!fn) return false;
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, 0) != hipSuccess) return false;
    return (int64_t)per_cu * cus >= resident_pass2d_blocks(n0, n1, B);
}

hipError_t launch_resident_pass2d(const ResidentPass2D& r, hipStream_t stream) {
    const void* fn = rp_kernel(r.prox.kind, r.B == 2, r.split != 0);
    if (!fn) return hipErrorInvalidValue;
    ResidentPass2D arg = r;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)resident_pass2d_blocks(r.n0, r.n1, r.B)), dim3(kThreads),
                                      args, 0, stream);
}

}  // namespace jko
