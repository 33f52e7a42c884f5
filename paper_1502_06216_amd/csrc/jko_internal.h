// Internal declarations of libjko: device control block, epilogue records and
// the host-side launchers of the kernels (each defined in the translation unit
// that holds its kernels, so no relocatable device code is needed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jko.h"

namespace jko {

// ---------------------------------------------------------------------------
// Device control block, one per workspace.  Written by the single-block
// control kernels (or by block 0 of the resident 2D kernel); every iteration
// kernel reads `done` first and returns when it is set, so that the host can
// queue iterations ahead of the stop test.
// ---------------------------------------------------------------------------
struct Ctl {
    int32_t done;          // 1 once the stop test passed or a non-finite value was met
    int32_t stop_iter;     // iterations whose p is returned (valid when done by tolerance)
    int32_t nonfinite;     // 1 if the monitor saw NaN/inf
    int32_t absorptions;
    int32_t absorb_pending;  // 1 when the last check asked for the log domain: a, b are
                             //    converted after that iteration's proximal half-step
    int32_t logmode;         // 1: the scalings a, b are stored as log a, log b and every
                             //    contraction runs log-in / log-out (exact log-sum-exp passes)
    int32_t exit_iter;       // resident 2D kernel: the iteration after whose proximal half-step
                             //    it returned because an absorption switch is pending (0: none)
    int32_t pad;
    double err;            // last ||b * xi^T a - q||_1
    double mass;           // last sum p
    double maxloga;        // last max |log a| over a > 0
    double maxlogb;        // last max |log b| over b > 0
    double aux[4];
};

// Per-block partial results of the fused epilogues (FP64, one slot per block).
struct Partials {
    double* err;
    double* mass;
    double* maxloga;
    double* maxlogb;
    int32_t cap;           // slots per array
};

// Energy parameters as the kernels see them (fields precomputed per call).
struct ProxArgs {
    int32_t kind;          // jko_energy_kind
    const float* g;        // congestion (both kinds): exp(-sigma w) per cell, or NULL for 1
    const float* kappa;    // congestion capacity field or NULL
    float kappa_s;         // scalar capacity when kappa == NULL
    const float* kf;       // porous: log((m-1) k) per cell; entropy: 1/(1 + sigma c) per cell;
                           // gen. entropy: sigma b m per cell (g then holds m - 1)
    float kf_s;            // scalar value when kf == NULL
    float eps_s;           // gen. entropy: m - 1 when g == NULL
    float lD;              // gen. entropy: log of the density scale
    float m;               // porous exponent
    int32_t newton;        // porous Newton steps
};

// ---------------------------------------------------------------------------
// Contraction pass: contract the contiguous axis of X (R rows of length n)
// with the factor K1 (n x n, symmetric) and write the result with that axis
// first:   Y[i][r] = sum_k K1[i][k] X[r][k].
// K1[i][k] == 0 exactly for |i - k| > W, so each output tile only runs over
// its band of k.  The result goes to one of the epilogues below.
// ---------------------------------------------------------------------------
struct Pass {
    int64_t R;             // rows of X (product of the other axes)
    int32_t n;             // contracted length (= output length along the axis)
    int32_t W;             // band half-width of K1
    const float* K1;       // n x n float32 factor
    const uint16_t* K1hi;  // bfloat16 split of K1 (split precision only)
    const uint16_t* K1lo;
    const float* X;        // input field
    int32_t B;             // 0 or 1: one field; B > 1: B stacked fields of R / B rows each,
                           // rotated separately (R / B must be a multiple of 4)
};

enum class EpiKind : int {
    STORE = 0,      // y = v
    BUPDATE = 1,    // t = v; [err += |b t - q|]; b = q / t
    PROX = 2,       // s = v; p = prox(s); a = p / s; [p_out = p]
    MONITOR = 3,    // t = v; err += |b t - q| (no write)
    ADJ_B = 4,      // bbar = v; y = tbar; acc (qbar) += bbar / t         (reverse of b = q / t)
    ADJ_PROX = 5,   // abar = v; y = sbar; acc (wbar) += ...               (reverse of p = prox(s), a = p / s)
    ATTR_PROX = 6,  // the attraction's two couplings (a pass over B = 2 stacked fields):
                    // p = min(s_1^alpha s_2^(1 - alpha), kappa), a_m = p / s_m, p_out = p
};

struct EpiArgs {
    EpiKind kind;
    float* y;              // STORE destination
    const float* q;        // BUPDATE/MONITOR: old density q
    float* b;              // BUPDATE: scaling b, updated in place; MONITOR: read
    float* a;              // PROX: scaling a, written
    float* p_out;          // PROX: density written when write_p
    float* s_out;          // PROX: optional copy of s (adjoint recomputation)
    float* t_out;          // BUPDATE: optional copy of t (adjoint recomputation)
    const float* hin;      // ADJ_B: t of the iteration; ADJ_PROX: s of the iteration
    float* acc;            // ADJ_B: qbar (accumulated); ADJ_PROX: wbar (accumulated) or NULL
    float sigma;           // ADJ_PROX: tau / gamma
    float alpha;           // ATTR_PROX: 1 / (1 + tau)
    int32_t check;         // BUPDATE: accumulate err with the old b; PROX: mass + max|log a|
    int32_t write_p;
    int32_t vec_ok;        // every field pointer above is 16-byte aligned (vector access)
    ProxArgs prox;
    Partials part;
    const Ctl* ctl;        // kernels return early when ctl->done (the plain-domain
                           // contractions also when ctl->logmode)
};

// Launch one contraction pass; returns the number of blocks (partials slots
// used by the epilogue) through *nblocks.
hipError_t launch_contract(const Pass& pass, int32_t precision, const EpiArgs& epi,
                           int* nblocks, hipStream_t stream);

// Upper bound of the blocks launch_contract may use for a pass of this shape.
int64_t contract_max_blocks(const Pass& pass, int32_t precision);

// 3D application in two launches that keep the layout [a][b][c] (c contiguous):
//   plane pass:  Y[a][b'][c'] = sum_b K1_1[b'][b] sum_c K1_2[c'][c] X[a][b][c]
//   slow pass:   Y[a'][r] = sum_a K1_0[a'][a] X[a][r]   (r = b n2 + c), + epilogue
// Same arithmetic, in the same order, as the three axis passes.
struct Plane3D {
    int n0, n1, n2;        // grid
    int W1, W2;            // band half-widths of the axis-1 and axis-2 factors
    const float* K1;       // n1 x n1 axis-1 factor (and its bfloat16 split)
    const uint16_t* K1hi;
    const uint16_t* K1lo;
    const float* K2;       // n2 x n2 axis-2 factor
    const uint16_t* K2hi;
    const uint16_t* K2lo;
    const float* X;        // input field
    float* Y;              // output field (not X)
    const Ctl* ctl;        // kernels return early when ctl->done
};
bool plane3d_fits(int n0, int n1, int n2, int W0, int W1, int W2);
hipError_t launch_plane3d(const Plane3D& p, int32_t precision, int* nblocks, hipStream_t stream);
// Slow-axis pass: Pass.R = n1 n2 columns, Pass.n = n0, X is n0 x R (rows contiguous in r).
hipError_t launch_contract_slow(const Pass& pass, int32_t precision, const EpiArgs& epi, int* nblocks,
                                hipStream_t stream);
int64_t contract_slow_blocks(const Pass& pass);

// Fused 2D application Y = K1_0 X K1_1 restricted to the float32 band of the
// factors (|i - j| > W => K1[i][j] == 0 exactly), one block per output tile of
// tile x tile cells (16 or 32).
struct Band2D {
    int n0, n1;            // grid
    int W0, W1;            // band half-widths of K1_0, K1_1
    const float* K0;       // n0 x n0
    const float* K1;       // n1 x n1
    const float* X;        // n0 x n1 input
    const uint16_t* K0hi;  // split precision: bfloat16 hi / lo of the factors
    const uint16_t* K0lo;
    const uint16_t* K1hi;
    const uint16_t* K1lo;
    int tile;              // output tile edge: 16 or 32
    int batch;             // per-application kernel only: this many n0 x n1 fields stacked in X and in
                           // the epilogue's fields, one block per (field, tile); 0 or 1: one field
};
// The tile's halo (tile + 2 W, aligned) fits the kernel's LDS.
bool gibbs2d_fits(int n0, int n1, int W0, int W1, int32_t precision, int tile);
int64_t gibbs2d_blocks(int n0, int n1, int tile);
constexpr int64_t kFusedMaxBlocks = 256;   // one block per CU of the chip
hipError_t launch_gibbs2d(const Band2D& b, int32_t precision, const EpiArgs& epi, int* nblocks,
                          hipStream_t stream);

// Synchronisation words of the resident kernel (uint32): an abort word, then
// one 64-byte line per block holding the count of phases it has published.
constexpr int64_t resident_sync_words(int64_t nblocks) { return 64 + 16 * nblocks; }

// One JKO step's iteration on a 2D grid in one cooperative launch (one block
// per 16 x 16 output tile, all resident).  Same arithmetic, order of
// operations, partials and control decisions as the launch-per-application
// path with the fused 2D kernel.  Plain domain only: at a check that asks for
// the absorption switch the launch returns after that iteration's proximal
// half-step (ctl->exit_iter) and the host continues on the log-domain passes.
struct Resident2D {
    Band2D B;              // geometry and factors (B.X unused)
    const float* q;        // old density
    float* a;              // scalings, in/out (a starts at 1, or 0 = log 1)
    float* b;
    float* p_out;          // density written at candidate iterations
    float* hist;           // adjoint recomputation: t_k, s_k at hist + (2(k-1)) stride, +stride; or NULL
    int64_t hist_stride;   // floats
    ProxArgs prox;
    Partials part;
    Ctl* ctl;
    uint32_t* sync;        // resident_sync_words(blocks), zeroed before the launch
    int32_t K;             // iterations
    int32_t ce;            // check cadence
    int32_t checks;        // stop test / absorption checks on
    int32_t vec_ok;        // all field pointers 16-byte aligned
    int32_t spin_limit;    // polls before a wait gives up
    int32_t split;         // split-BF16 contractions
    int32_t a_only;        // the absorption trigger watches max|log a| alone
    double tol;
    double absorb;
};
// The reverse sweep of one step in one cooperative launch (the adjoint of
// the above, on the same tiles).
struct ResidentAdj {
    Band2D B;              // geometry and factors (B.X unused)
    const float* q;        // the step's input density
    const float* hist;     // t_k at hist + (2(k-1)) stride, s_k at + stride
    int64_t hist_stride;   // floats
    float* sbar;           // in: sbar_K; exchanged between blocks
    float* tbar;           // exchanged between blocks
    float* qbar;           // accumulated (zeroed before the launch)
    float* wbar;           // accumulated, or NULL
    ProxArgs prox;
    float sigma;
    uint32_t* sync;        // resident_sync_words(blocks), zeroed before the launch
    int32_t K;
    int32_t vec_ok;
    int32_t spin_limit;
    int32_t split;
};
bool resident_adj_fits(int n0, int n1, int W0, int W1, int prox_kind, int32_t precision, int tile);
hipError_t launch_resident_adj(const ResidentAdj& r, hipStream_t stream);

// True when all blocks of the resident kernel fit on the device at once.
bool resident2d_fits(int n0, int n1, int W0, int W1, int prox_kind, int32_t precision, int tile);
hipError_t launch_resident2d(const Resident2D& r, hipStream_t stream);

// A whole 2D step in one cooperative launch with every application of xi
// as the two rotating panel passes (axis 1 into the transposed intermediate
// u, then axis 0 with the epilogue), for bands up to seven 32-k panels: block
// t owns one 32 x 32 output tile of each pass (paired tiles, 16 rows of each
// field, for the attraction's two couplings) and waits only for the blocks
// whose outputs its pass reads.  Same arithmetic as the launched passes.
struct ResidentPass2D {
    int32_t n0, n1;        // grid, both multiples of 32
    int32_t W0, W1;        // band half-widths
    const float* K0;       // axis-0 factor (n0 x n0) and its bfloat16 split
    const uint16_t* K0hi;
    const uint16_t* K0lo;
    const float* K1;       // axis-1 factor (n1 x n1)
    const uint16_t* K1hi;
    const uint16_t* K1lo;
    int32_t B;             // stacked fields: 1, or 2 (the attraction's couplings)
    const float* q;        // marginals, B fields
    float* a;              // scalings, B fields each (a starts at 1)
    float* b;
    float* u0;             // transposed intermediates, B fields each: t half-step
    float* u1;             //                                          s half-step
    float* p_out;          // density written at candidate iterations
    ProxArgs prox;
    float alpha;           // attraction: 1 / (1 + tau)
    Partials part;
    Ctl* ctl;
    uint32_t* sync;        // resident_sync_words(blocks), zeroed before the launch
    int32_t K;             // iterations
    int32_t ce;            // check cadence
    int32_t checks;        // stop test / absorption checks on
    int32_t vec_ok;        // all field pointers 16-byte aligned
    int32_t spin_limit;    // polls before a wait gives up
    int32_t split;         // split-BF16 contractions
    int32_t a_only;        // the absorption trigger watches max|log a| alone
    int32_t check_mass;    // the proximal epilogue accumulates mass and max|log a| partials
    double tol;
    double absorb;
};
int64_t resident_pass2d_blocks(int n0, int n1, int B);
// The grid and bands suit the kernel (axes of a multiple of 32, at most 256
// blocks, bands of at most seven panels); _fits also asks the device.
bool resident_pass2d_shape_fits(int n0, int n1, int W0, int W1, int B);
bool resident_pass2d_fits(int n0, int n1, int W0, int W1, int B, int prox_kind, int32_t precision);
hipError_t launch_resident_pass2d(const ResidentPass2D& r, hipStream_t stream);

// Largest |i - j| at which the float32 factor exp(-((i-j)/n)^2/gamma) can be
// non-zero (entries below 2^-150 round to zero).
int band_halfwidth(int n, double gamma);

// ----------------------------------------------------------------- pointwise
hipError_t launch_build_factor(float* K1, uint16_t* hi, uint16_t* lo, int n, double gamma,
                               hipStream_t s);
hipError_t launch_fill(float* x, float v, int64_t n, hipStream_t s);
hipError_t launch_copy(float* dst, const float* src, int64_t n, hipStream_t s);
hipError_t launch_copy_scaled(float* dst, const float* src, double f, int64_t n, hipStream_t s);
hipError_t launch_attraction_prox(const float* s, float* a, float* p, const float* kappa, float kappa_s,
                                  double alpha, int64_t N, const Ctl* ctl, hipStream_t st);
hipError_t launch_prepare_energy(const jko_energy* en, double sigma, int64_t N, float* g,
                                 float* kf, hipStream_t s);
hipError_t launch_ctl_reset(Ctl* ctl, int logmode, hipStream_t s);
// Sum of the per-block err partials -> ctl->err; stop / non-finite decision;
// switch to the log domain when max|log a| or max|log b| > absorb (absorb > 0;
// a_only: max|log a| alone).  plain: a check of plain-domain iterations, a
// no-op once the switch has been committed.
hipError_t launch_ctl_check(Ctl* ctl, Partials part, int nparts, int iter, double tol,
                            int check_mass, double absorb, int a_only, int plain, hipStream_t s);
// a <- log a, b <- log b when the last check asked for the switch.
hipError_t launch_absorb(Ctl* ctl, float* a, float* b, int64_t N, hipStream_t s);
// After launch_absorb: logmode <- 1 and exit_iter <- iter if the switch was
// pending; pending <- 0.
hipError_t launch_ctl_commit(Ctl* ctl, int iter, hipStream_t s);
// FP64 sums of p_in, of kappa (or kappa_s * N) and non-finite / negative
// detection of p_in; results to out[0..3] (device doubles).
hipError_t launch_input_check(const float* p_in, const float* kappa, float kappa_s, int64_t N,
                              int congestion, double* part, int part_cap, double* out,
                              hipStream_t s);

// ------------------------------------------------------------------ adjoint
hipError_t launch_adj_prox(const float* s, const float* pbar_ext, const float* abar,
                           float* sbar, float* wbar, const ProxArgs& px, double sigma,
                           int64_t N, hipStream_t st);
hipError_t launch_adj_b(const float* t, const float* q, const float* bbar, float* tbar,
                        float* qbar, int64_t N, hipStream_t st);
hipError_t launch_axpy_inplace(float* y, const float* x, int64_t N, hipStream_t st);

}  // namespace jko
