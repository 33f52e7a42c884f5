// Heat-kernel Gibbs operator on a masked 2D grid (Section 4.1, eq. heat-kernel):
// host-side launchers of the kernels in heat.hip.
//
// xi~ = (Id - (gamma/L) Delta_M)^{-L} with Delta_M the no-flux five-point
// Laplacian of the free cells (spacing 1/n_k along axis k), i.e.
// Id + nu_0 G_0 + nu_1 G_1 with nu_k = gamma n_k^2 / L and G_k the graph
// Laplacian of the free axis-k neighbour pairs.  The operator acts on the
// free cells only: they are numbered in row-major order (gidx: free index ->
// grid cell, cidx: grid cell -> free index or -1), and xi~ is stored over
// those Nf indices.  xi~ is symmetric; the library stores its upper triangle
// of kHeatTile x kHeatTile float32 tiles: tile (I, J), I <= J, of the ld x ld
// matrix (ld = Nf rounded up to the tile) at
// packed index I*nT - I*(I-1)/2 + (J - I), each tile row-major.  Rows and
// columns of the padding are zero.
#pragma once

#include "jko_internal.h"

namespace jko {

constexpr int kHeatTile = 128;

inline int64_t heat_ld(int64_t N) { return (N + kHeatTile - 1) / kHeatTile * kHeatTile; }
inline int64_t heat_ntiles(int64_t N) { return heat_ld(N) / kHeatTile; }
// floats of the packed upper-triangular tiles
inline int64_t heat_operator_floats(int64_t N) {
    const int64_t nT = heat_ntiles(N);
    return nT * (nT + 1) / 2 * kHeatTile * kHeatTile;
}
// floats of the per-pass partial sums (one row block per tile pair)
inline int64_t heat_partial_floats(int64_t N) {
    const int64_t nT = heat_ntiles(N);
    return nT * nT * kHeatTile;
}

// One application of the stored operator, y = A x, with the result of each
// row finished by a pointwise epilogue (EK_STORE, EK_BUPDATE, EK_MONITOR or
// EK_PROX + energy kind, as in the band contractions).
// Row r of the pass is free cell gidx[r]: x, b, a and errrow are indexed by
// r (free-cell vectors), y, q, p and the energy fields by the grid cell.
struct HeatGemv {
    const float* A;          // packed upper-triangular tiles
    float* part;             // heat_partial_floats(N) scratch
    int32_t nT;              // tiles per side
    int64_t ld;              // nT * kHeatTile
    int64_t N;               // rows: free cells
    const int32_t* gidx;     // free index -> grid cell
    const float* x;          // ld floats, padding zero
    float* y;                // STORE: result (grid)
    const float* q;          // BUPDATE / MONITOR: the step's input density (grid)
    float* b;                // BUPDATE: b = q / y (0/0 = 0); MONITOR: read
    double* errrow;          // BUPDATE (when check) / MONITOR: |b_old y - q| per row
    int32_t check;
    float* a;                // PROX: a = p / y (0/0 = 0)
    float* p;                // PROX: p = Prox(y) (grid)
    ProxArgs px;             // fields indexed by grid cell
};

// Numbers the free cells in row-major order: cidx (N), gidx (first Nf
// entries), *count (device int64) = Nf.  One block.
hipError_t launch_heat_compact(const uint8_t* mask, int64_t N, int32_t* cidx, int32_t* gidx, int64_t* count,
                               hipStream_t st);

// x[r] = src[gidx[r]] for r < nf, 0 up to ld.
hipError_t launch_heat_gather(float* x, const float* src, const int32_t* gidx, int64_t nf, int64_t ld,
                              hipStream_t st);

// Chebyshev iterations per implicit step that bring the error of each solve
// below tol of the right-hand side for the spectrum [1, beta].
int heat_cheb_iters(double beta, double tol);

// Per-product form: the L solves of one product stop at this error relative
// to the right-hand side's norm.  A product's far tail lies many orders below
// its norm, and the scaling iteration divides by it (b = q / t), so the bound
// sits far below float32 resolution.
constexpr double kHeatSolveTol = 1e-13;

// One product y = xi~ x by L solves on the grid (the paper's form of the
// operator): x (free-cell vector of g) is scattered to the grid vector X,
// solved in place, and each free row finished by the epilogue `ek` of g
// (codes of launch_heat_gemv).  R, R1, D0, D1: grid scratch (N doubles
// each; the residual and the direction alternate between their pairs).
struct HeatSolve {
    const uint8_t* mask;     // NULL = no obstacle
    const int32_t* cidx;     // grid cell -> free index or -1
    int n0, n1, L;
    double gamma;
    double* X;
    double* R;
    double* R1;
    double* D0;
    double* D1;
};

// Coefficients of up to 8 consecutive Chebyshev iterations (one launch).
struct HeatChebSteps {
    double c1[8], c2[8];
    int steps;
};
hipError_t launch_heat_solve(int ek, const HeatGemv& g, const HeatSolve& h, hipStream_t st);

// Scratch doubles heat_build_operator needs for an N-cell grid (4 N C).
int64_t heat_build_scratch(int64_t N);

// Writes the packed tiles of xi~ over the nf free cells (heat_operator_floats(nf)
// floats).  scratch: heat_build_scratch(N) doubles.
hipError_t heat_build_operator(const uint8_t* mask, int n0, int n1, double gamma, int L, const int32_t* cidx,
                               const int32_t* gidx, int64_t nf, float* A, double* scratch, hipStream_t st);

// Epilogue codes of launch_heat_gemv: store, b-update, monitor, and the
// proximal epilogue HEAT_EK_PROX + energy kind (the band contractions' codes).
enum : int { HEAT_EK_STORE = 0, HEAT_EK_BUPDATE = 1, HEAT_EK_MONITOR = 2, HEAT_EK_PROX = 3 };

hipError_t launch_heat_gemv(int ek, const HeatGemv& g, hipStream_t st);

// x[0..n) = v, x[n..ld) = 0
hipError_t launch_heat_fill(float* x, float v, int64_t n, int64_t ld, hipStream_t st);


// out[0] = sum of errrow[0..ne) (when errrow != NULL), out[1] = sum of
// p[0..np) (when p != NULL), out[2] = number of non-finite errrow entries.
// One block, fixed order.
hipError_t launch_heat_sums(const double* errrow, int64_t ne, const float* p, int64_t np, double* out,
                            hipStream_t st);

// Input check of a step's density: out[0] = mass, out[1] = capacity over the
// free cells (kappa field or kappa_s; +inf allowed), out[2] = number of
// cells that are negative or non-finite, hold mass on an obstacle, or have a
// negative/NaN capacity.
hipError_t launch_heat_input(const float* p, const uint8_t* mask, const float* kappa, float kappa_s, int64_t N,
                             double* out, hipStream_t st);

}  // namespace jko
