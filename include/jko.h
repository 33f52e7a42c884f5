/*
 * jko.h -- C ABI of the MI355X (gfx950) entropic JKO library (libjko.so).
 *
 * The library computes entropic Wasserstein gradient-flow (JKO) steps
 *     p_{t+1} = argmin_{p in simplex} W_gamma(p, p_t) + tau f(p)
 * (Peyre 2015, Section 2.2, eq. def-jko-operator and eq. smooth-jko) on a
 * uniform cell-centred grid of [0,1]^d, d in {1,2,3}, with squared Euclidean
 * ground cost c_ij = |x_i - x_j|^2 (Section 2.1, alpha = 2).  Cell centres
 * along an axis of length n are (i + 1/2)/n.
 *
 * Each step is solved by KL Dykstra in diagonal-scaling form (Section 3.4,
 * Proposition 3.3, Listing 1): pi = diag(a) xi diag(b) with the Gibbs kernel
 * xi = exp(-c/gamma) (Section 3.1).  The correction factors u, v of
 * Proposition 3.3 are identically 1 (u = 1/a after even half-steps), so one
 * iteration is
 *     b = q / (xi^T a);  s = xi b;  p = Prox^KL_{(tau/gamma) f}(s);  a = p / s
 * with q = p_t, a cold-started at 1 at every step (Listing 1, step 2), and the
 * stopping test of Listing 1 on || b * xi^T a - q ||_1 after an even
 * half-step (JKO_F_ATTRACTION keeps two such couplings, described with the
 * energies).  xi is applied as per-axis dense contractions with the factor
 * K1[i][j] = exp(-(x_i - x_j)^2 / gamma) (the separable Gaussian kernel of
 * Section 4.1), exactly (no truncation, no boundary condition).  On a
 * non-convex 2D domain (a grid with obstacles) the jko_heat_* calls replace
 * xi by the heat kernel of Section 4.1 (eq. heat-kernel), described with
 * them below.
 *
 * Conventions shared by every entry point:
 *  - Fields are contiguous float32 arrays in row-major order
 *    n[0] x ... x n[ndim-1] (last axis fastest), N = prod n[k] cells.
 *  - Every float / double pointer argument named as a field, and the
 *    workspace, is a DEVICE pointer on the current HIP device; pointers to
 *    jko_grid / jko_heat_domain / jko_energy / jko_params / jko_stats
 *    structs, and the
 *    iters_per_step array of jko_backward, are HOST pointers.
 *  - The caller owns every buffer.  The library never allocates device
 *    memory: all scratch lives in the caller's workspace, whose size is given
 *    by jko_workspace_bytes() (jko_heat_workspace_bytes() for the heat
 *    kernel).  It keeps one small pinned host buffer and one
 *    event per process for its stop-test read-back.
 *  - All work is ordered on `stream` (a hipStream_t; NULL = default stream).
 *    jko_gibbs_apply, jko_heat_apply and jko_backward return before their
 *    kernels finish.  The calls that run steps wait for a device result at
 *    a few points: the check of the input density (mass, capacity,
 *    finiteness) before the iteration is queued; the stop tests of a
 *    tolerance-mode step (read back one check interval behind the queue);
 *    the end of a step whose absorb_threshold is finite and positive (the
 *    host must know which domain the step ended in); and a non-NULL host
 *    stats pointer.
 *  - Arguments are validated before any launch; on error nothing is launched
 *    and a status < 0 is returned.  jko_last_error() describes the last
 *    failure of the calling thread.
 *  - Calls that share a workspace must not overlap in time.
 */
#ifndef JKO_H
#define JKO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    JKO_OK = 0,
    JKO_ERR_INVALID = -1,     /* bad argument (sizes, parameters, null pointer) */
    JKO_ERR_WORKSPACE = -2,   /* workspace missing or smaller than required */
    JKO_ERR_HIP = -3,         /* a HIP runtime call failed (see jko_last_error) */
    JKO_ERR_NONFINITE = -4,   /* NaN/inf met by the FP64 monitor; outputs are still written */
    JKO_ERR_INFEASIBLE = -5   /* capacity sum(kappa) < sum(p_t) (congestion, binary congestion,
                                 attraction) */
} jko_status;

/* Arithmetic of the Gibbs contractions.  Accumulation is float32 in both;
 * JKO_SPLIT_BF16 splits each operand x = hi + lo (bfloat16, round to nearest
 * even) and sums the three MFMA products hi*hi + hi*lo + lo*hi. */
typedef enum { JKO_FP32 = 0, JKO_SPLIT_BF16 = 1 } jko_precision;

/* Energy f (Section 4).  sigma = tau / gamma below.
 *  JKO_F_ZERO        f = 0; prox is the identity.
 *  JKO_F_CONGESTION  f = iota_{[0,kappa]}(p) + <w, p>; prox min(s e^{-sigma w}, kappa)
 *                    (Section 4.2, Proposition 4.1; kappa may vary in space,
 *                    kappa = +inf means no cap).
 *  JKO_F_POROUS      f = sum_i c_i (D p_i)^m / ((m - 1) D), m > 1, density scale D;
 *                    prox psi solves log psi + k psi^{m-1} = log s with
 *                    k = sigma c m D^{m-1} / (m - 1) (first-order condition as in
 *                    Section 4.4, Proposition 4.2), by Newton steps on log psi.
 *  JKO_F_ENTROPY     f = sum_i c_i p_i (log p_i - 1); prox s^{1/(1 + sigma c)}
 *                    (Section 4.4, Proposition 4.2 with m = 1).
 *  JKO_F_CONGESTION_BINARY
 *                    f = iota_{{0,kappa}^N}(p) + <w, p>, the non-convex functional
 *                    of Section 4.5 (eq. dfn-congestion-noncvx); prox kappa where
 *                    s e^{-sigma w} >= kappa / e (e = exp 1), else 0: the prox of the
 *                    section with the linear term folded into the divergence.  At
 *                    the tie the prox is two-valued and kappa is taken.  Same fields
 *                    as JKO_F_CONGESTION, but kappa must be finite.  The iteration
 *                    is the paper's non-convex Dykstra (no convergence guarantee);
 *                    jko_backward refuses this energy (the prox is piecewise
 *                    constant).
 *  JKO_F_GEN_ENTROPY f = sum_i b_i e_{m_i}(D p_i) / D, the generalised entropies of
 *                    Section 4.4 (eq. defn-gen-entropies): e_1(x) = x (log x - 1),
 *                    e_m(x) = x (x^{m-1} - m) / (m - 1); weights b_i = coef (or
 *                    coef_scalar) >= 0, exponents m_i = m_field (or m) >= 1 per
 *                    cell, density scale D = density_scale (1 = the paper's form).
 *                    Prox (Proposition 4.2): psi = D p solves
 *                    log psi + sigma b m (psi^{m-1} - 1) / (m - 1) = log(D s)
 *                    (the m = 1 limit is psi = (D s)^{1/(1 + sigma b)}), by
 *                    Newton steps on log psi (at most newton_steps); jko_backward
 *                    differentiates it through the implicit derivative
 *                    d log psi / d log s = 1 / (1 + sigma b m psi^{m-1}).
 *  JKO_F_ATTRACTION  f = W_gamma(r, p) + iota_[0,kappa](p), the Wasserstein
 *                    attraction towards target (r, N cells, device; a shape,
 *                    scaled to the mass of each step's input) with
 *                    congestion of Section 5.2, solved by the two-coupling
 *                    scaling of Proposition 5.2 (marginals first; the proximal
 *                    half-step is eq. prox-psi-attraction).  The workspace is
 *                    sized by JKO_OP_ATTRACTION_STEP / _FLOW.  1D and 2D grids
 *                    with every axis >= 3; absorption as for the other
 *                    energies, the switch triggered by max|log b| alone; a
 *                    step runs on the resident pass kernel where the shape
 *                    allows (see the execution flags); no backward. */
typedef enum {
    JKO_F_ZERO = 0,
    JKO_F_CONGESTION = 1,
    JKO_F_POROUS = 2,
    JKO_F_ENTROPY = 3,
    JKO_F_CONGESTION_BINARY = 4,
    JKO_F_GEN_ENTROPY = 5,
    JKO_F_ATTRACTION = 6
} jko_energy_kind;

typedef struct {
    int32_t ndim;        /* 1, 2 or 3 */
    int32_t n[3];        /* axis lengths, 1 <= n[k] <= 1024; unused entries ignored */
} jko_grid;

typedef struct {
    int32_t kind;            /* jko_energy_kind */
    const float* w;          /* congestion / binary congestion potential, N cells, device; NULL = 0 */
    const float* kappa;      /* capacity (congestion, binary congestion, attraction), N cells,
                                device; NULL = kappa_scalar */
    float kappa_scalar;      /* used when kappa == NULL; may be +inf */
    const float* coef;       /* porous / entropy / gen. entropy weight, N cells, device; NULL = coef_scalar */
    float coef_scalar;
    float m;                 /* porous exponent, > 1; gen. entropy exponent when m_field == NULL, >= 1 */
    float density_scale;     /* porous / gen. entropy D, > 0 (1 = per-cell mass) */
    int32_t newton_steps;    /* porous / gen. entropy: cap on the Newton steps per cell, 1..32
                                (0 = default 8); a cell stops earlier, once its update is
                                within 2^-20 of its scale (below float32 rounding after it) */
    const float* m_field;    /* gen. entropy exponents m_i >= 1, N cells, device; NULL = m */
    const float* target;     /* attraction target density r, N cells, device */
} jko_energy;

typedef struct {
    double gamma;            /* entropic regularisation, > 0 */
    double tau;              /* JKO time step, > 0 */
    double tol_l1;           /* stop when ||b * xi^T a - q||_1 <= tol_l1; <= 0: run max_iters */
    int32_t max_iters;       /* iteration cap per step, >= 1 */
    int32_t check_every;     /* stop-test cadence in iterations, >= 1 */
    int32_t precision;       /* jko_precision */
    int32_t flags;           /* jko_flags bits (0 = defaults) */
    double absorb_threshold; /* log-domain absorption: at the first stop-test check where
                                max|log a| or max|log b| exceeds it, a and b are absorbed
                                (carried as logs) after that iteration's proximal
                                half-step, and every later Gibbs product is an exact
                                log-sum-exp (each output shifted by its own largest term,
                                no band assumed; float32 arithmetic in both precisions);
                                <= 0: log domain from the first iteration; +inf or NaN:
                                never.  With a finite threshold the checks also run in
                                fixed-count mode; their results are read back without
                                stalling the queue (the plain-domain kernels queued after
                                a switch return at once and the step resumes after the
                                switch iteration in the log domain); the attraction
                                reads each check back synchronously. */
} jko_params;

/* Execution flags of jko_params.flags.
 * 2D applications of xi run as the fused tile kernel (16 x 16 tiles) where at
 * most 256 tiles cover the grid; else, on axes of a multiple of 32 with at
 * most 256 tiles of 32 x 32 and bands of at most seven 32-cell panels, as
 * two per-axis passes; else as the fused kernel with 32 x 32 tiles where it
 * fits, else as the passes.  A step whose applications are fused tiles or
 * such passes normally runs whole in one cooperative launch (the resident
 * tile kernel, or the resident pass kernel, which runs the passes without
 * launch boundaries); so does the attraction's pair of couplings on the
 * passes' shapes.
 * JKO_FLAG_NO_RESIDENT: one launch per Gibbs application (per pass) instead
 *   of the resident kernels.  Both paths give the same bits.
 * JKO_FLAG_AXIS_PASSES: on 3D grids whose axes are multiples of 32 (the
 *   second at most 128), an application of xi normally runs as a plane pass
 *   (axes 1 and 2 of each plane, the intermediate kept on chip) and an axis-0
 *   pass; this flag runs three axis passes instead.  Both give the same bits.
 *   On 2D grids it runs every application as per-axis passes instead of the
 *   fused tile kernel (and a step on the resident pass kernel where its
 *   shape allows).
 * JKO_FLAG_ABSORB_ON_A: the absorption switch (finite absorb_threshold)
 *   watches max|log a| alone instead of max(max|log a|, max|log b|).  Ignored
 *   by JKO_F_ATTRACTION, which watches max|log b|. */
typedef enum { JKO_FLAG_NO_RESIDENT = 1, JKO_FLAG_AXIS_PASSES = 2, JKO_FLAG_ABSORB_ON_A = 4 } jko_flags;

typedef enum { JKO_STOP_TOL = 0, JKO_STOP_CAP = 1 } jko_stop_reason;

typedef struct {
    int32_t iters;           /* iterations whose p was returned */
    int32_t absorptions;     /* number of log-domain absorptions performed */
    int32_t stop_reason;     /* jko_stop_reason */
    int32_t status;          /* jko_status of this step */
    double marginal_l1;      /* ||b * xi^T a - q||_1 of the returned iterate (FP64 sum;
                                attraction: summed over both couplings) */
    double mass;             /* sum of the returned p (FP64 sum) */
    double max_abs_log_a;    /* max |log a| over cells with a > 0, last check (0 for the
                                attraction, which does not monitor it) */
    double max_abs_log_b;    /* max |log b| over cells with b > 0, last check */
} jko_stats;

/* Operation codes for jko_workspace_bytes. */
typedef enum {
    JKO_OP_GIBBS = 0,
    JKO_OP_STEP = 1,
    JKO_OP_FLOW = 2,
    JKO_OP_BACKWARD = 3,
    JKO_OP_ATTRACTION_STEP = 4,   /* jko_step with JKO_F_ATTRACTION */
    JKO_OP_ATTRACTION_FLOW = 5    /* jko_flow with JKO_F_ATTRACTION */
} jko_op;

/* Bytes of device workspace `op` needs for this grid and these parameters
 * (for JKO_OP_BACKWARD, n_steps is the largest iteration count of one step).
 * Returns 0 when the grid is invalid. */
size_t jko_workspace_bytes(const jko_grid* grid, const jko_params* params, int32_t op,
                           int32_t n_steps);

/* y = xi x: the Gibbs kernel of Section 3.1 applied to one field (the
 * operation Section 3.4 notes the whole method reduces to).  xi is symmetric
 * on this grid, so this is also xi^T x.  x and y are N-cell device fields
 * and may not alias.  precision: jko_precision. */
jko_status jko_gibbs_apply(const jko_grid* grid, double gamma, int32_t precision,
                           const float* x, float* y, void* workspace, size_t workspace_bytes,
                           void* stream);

/* Doubles in the device statistics record of jko_step. */
#define JKO_STATS_DEV_DOUBLES 8

/* One JKO step p_out = Prox^{W_gamma}_{tau f}(p_in) (eq. def-jko-operator) by
 * the iteration of Listing 1.  p_in >= 0 (any mass); p_out may not alias
 * p_in.  Returns JKO_ERR_INFEASIBLE before launching the iteration when a
 * congestion capacity cannot hold the mass of p_in.
 * stats (host, nullable) receives the step's statistics and makes the call
 * wait for the step to finish.
 * stats_dev (device, nullable, 8-byte aligned, JKO_STATS_DEV_DOUBLES doubles,
 * aliasing neither p_in nor p_out) receives the same record, ordered on
 * `stream` after p_out, without a read-back: the fields of jko_stats in their
 * order (iters, absorptions, stop_reason, status, marginal_l1, mass,
 * max_abs_log_a, max_abs_log_b), each as a double.  With stats NULL the call
 * then does not wait for it, and a non-finite value met by the monitor
 * appears only as status JKO_ERR_NONFINITE in the record, not as the return
 * value.  Either pointer, when given, costs one more t = xi^T a on a step
 * that ends at max_iters (the violation of the returned iterate). */
jko_status jko_step(const jko_grid* grid, const jko_energy* energy, const jko_params* params,
                    const float* p_in, float* p_out, jko_stats* stats, double* stats_dev,
                    void* workspace, size_t workspace_bytes, void* stream);

/* n_steps JKO steps from p0 (eq. smooth-jko with fixed gamma, tau).
 * pT (device, N cells) receives p_{n_steps}.  checkpoints (device, nullable,
 * n_steps * N floats) receives p_0 ... p_{n_steps-1}, the inputs of each step,
 * for jko_backward.  stats (host, nullable) is an array of n_steps records. */
jko_status jko_flow(const jko_grid* grid, const jko_energy* energy, const jko_params* params,
                    int32_t n_steps, const float* p0, float* pT, float* checkpoints,
                    jko_stats* stats, void* workspace, size_t workspace_bytes, void* stream);

/* Reverse-mode derivative of L(p_T) through the unrolled flow: given the
 * checkpoints p_0..p_{n_steps-1} written by jko_flow and the iteration count
 * of every step (host array, stats[t].iters of the forward), and dL/dp_T,
 * writes dL/dw (nullable) and dL/dp0 (nullable).  dL/dw is the derivative
 * with respect to the energy's per-cell field: the potential w for
 * CONGESTION (w required), the weights coef for GEN_ENTROPY (coef required).
 * Each step's iterations are recomputed from its checkpoint, their
 * intermediate Gibbs products are kept in the workspace, then swept in
 * reverse.  The derivative is that of the map at the given iteration counts
 * (tol_l1 is ignored).  Energies: ZERO, CONGESTION, ENTROPY, POROUS,
 * GEN_ENTROPY (dL/dp0 only for ENTROPY and POROUS); CONGESTION_BINARY and
 * ATTRACTION are refused. */
jko_status jko_backward(const jko_grid* grid, const jko_energy* energy, const jko_params* params,
                        int32_t n_steps, const int32_t* iters_per_step, const float* checkpoints,
                        const float* dL_dpT, float* dL_dw, float* dL_dp0,
                        void* workspace, size_t workspace_bytes, void* stream);

/* jko_step without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, semantics and results as jko_step;
 * the workspace is a static device array of JKO_STATIC_WORKSPACE_BYTES inside
 * the library, one per GPU, held from the first call on that GPU until the
 * process ends.  The call allocates nothing: no device or pinned host memory
 * and no event (its stop-test and statistics read-backs are synchronous
 * copies to pageable host memory).  Grids whose step needs more workspace
 * than the array holds (jko_workspace_bytes with JKO_OP_STEP, or
 * JKO_OP_ATTRACTION_STEP) are refused with JKO_ERR_WORKSPACE before any
 * launch; 2D grids up to 512 x 512 fit.  Every call on one GPU shares that
 * GPU's array, so calls that overlap in time on one GPU (any streams, any
 * threads) race and must not be made. */
#define JKO_STATIC_WORKSPACE_BYTES ((size_t)16 << 20)
jko_status jko_step_static(const jko_grid* grid, const jko_energy* energy, const jko_params* params,
                           const float* p_in, float* p_out, jko_stats* stats, void* stream);

/* Measurement aid (not part of the method): sets up one step of p_in as
 * jko_step does, then times its kernel launches `reps` times on `stream` with
 * HIP events.  Where a step runs on a resident kernel (the tile kernel or
 * the pass kernel; see the execution flags), that is one launch running
 * params->max_iters iterations with no stop test.  Otherwise it is each launch of one
 * iteration -- those of t = xi^T a ending in the b-update epilogue, then those
 * of s = xi b ending in the proximal epilogue (one launch per application for
 * 2D grids on the fused tile kernel, else one per axis) -- back to back.
 * ms_per_launch (host, room for 2*ndim doubles) receives the mean duration of
 * one launch of each, in launch order; *n_launches (host, nullable) their
 * number.  The scalings are set to 1 first; p_in is not modified.
 * Synchronous.  JKO_F_ATTRACTION is refused. */
jko_status jko_time_iteration(const jko_grid* grid, const jko_energy* energy, const jko_params* params,
                              const float* p_in, int32_t reps, double* ms_per_launch, int32_t* n_launches,
                              void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Heat-kernel Gibbs operator on a masked 2D grid (Section 4.1, eq.
 * heat-kernel).  On a non-convex domain M (the free cells of an n0 x n1 grid
 * of [0,1]^2; obstacles carry no mass) xi is replaced by
 *
 *     xi~ = (Id - (gamma / L) Delta_M)^{-L},
 *
 * L implicit Euler steps of the heat equation up to time gamma, with
 * Delta_M the five-point Laplacian of the free cells, spacing 1/n_k along
 * axis k and no flux across the grid's edge or into an obstacle.  xi~ is
 * symmetric, non-negative and conserves mass on each connected part of M;
 * transport through it follows the domain's geodesics.
 *
 * The paper applies xi~ by L sparse back-substitutions per product.  Up to
 * 65536 cells this library builds xi~ once per (domain, gamma, L) as a dense
 * float32 matrix in the workspace (over the Nf free cells, the upper triangle
 * of 128 x 128 tiles, about Nf^2 * 2 bytes: 187 MB for the 9556 free cells of
 * a 100 x 100 room) by FP64 Chebyshev solves on the device, then runs every
 * product of the scaling iteration as one pass over it.  Above 65536 cells
 * (or with per_product = 1) it applies xi~ the paper's way instead: each
 * product is L solves of (Id - (gamma/L) Delta_M) y = rhs on the grid, each a
 * Chebyshev iteration in FP64 (one five-point stencil sweep per iteration,
 * eight iterations per launch on tiles with a halo of eight cells, to 1e-13
 * of the right-hand side; linear in the grid's size), rounded to float32; no
 * operator is stored.  The flow uses the iteration and stop test
 * of jko_step with xi replaced by xi~; float32 only, no log domain, no
 * backward.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n0, n1;          /* grid, n0 x n1 cells (row-major, n1 fastest; n0 = 1: a 1D grid),
                                n0 * n1 <= 2^20 */
    const uint8_t* mask;     /* device, n0*n1 bytes, nonzero = free cell; NULL = no obstacle.
                                Read by every call below: keep it alive and unchanged while the
                                workspace's operator is in use */
    int32_t L;               /* implicit heat steps, 1..1000 (the paper uses 10) */
    int32_t per_product;     /* 0: the stored dense operator while n0 * n1 <= 65536, the
                                per-product solves above; 1: the per-product solves always */
} jko_heat_domain;

/* Bytes of device workspace the calls below need for this domain (the dense
 * operator, its construction scratch, and the iteration's fields); 0 when
 * the domain is invalid. */
size_t jko_heat_workspace_bytes(const jko_heat_domain* domain);

/* Builds xi~ for this domain and gamma into the workspace (which then holds
 * it for jko_heat_apply and jko_heat_flow with the same domain and gamma).
 * Each column is L solves of (Id - (gamma/L) Delta_M) x = rhs by Chebyshev
 * iteration in FP64 to 1e-14 of the right-hand side, rounded to float32.
 * Synchronous.  Cost: L * (about 3 sqrt(1 + 4 gamma (n0^2 + n1^2) / L) + 1)
 * stencil sweeps over N x min(N, 1024) doubles per 1024 columns. */
jko_status jko_heat_build(const jko_heat_domain* domain, double gamma, void* workspace,
                          size_t workspace_bytes, void* stream);

/* y = xi~ x (= xi~^T x) for an N-cell device field x (values on obstacles
 * ignored; y is 0 there).  x and y may not alias.  Refuses a workspace
 * whose operator was built for another domain (synchronous check). */
jko_status jko_heat_apply(const jko_heat_domain* domain, const float* x, float* y,
                          void* workspace, size_t workspace_bytes, void* stream);

/* n_steps JKO steps from p0 with xi~ in place of xi (the crowd-motion
 * examples of Section 4.3 on obstacle domains).  energy: every kind but
 * JKO_F_ATTRACTION.  params: gamma must equal the gamma of jko_heat_build;
 * precision JKO_FP32; absorb_threshold +inf or NaN; flags ignored.  p0
 * (device, N cells) must be zero on obstacles.  stats (host, nullable): one
 * record per step (max_abs_log_a/b are 0: not monitored).  Synchronous:
 * the stop test and the statistics read device sums back. */
jko_status jko_heat_flow(const jko_heat_domain* domain, const jko_energy* energy, const jko_params* params,
                         int32_t n_steps, const float* p0, float* pT, jko_stats* stats,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Static description of a status code. */
const char* jko_status_string(int32_t status);

/* Message of the last failure in the calling thread ("" if none). */
const char* jko_last_error(void);

/* Library version, for the binding's compatibility check. */
int32_t jko_version(void);

#ifdef __cplusplus
}
#endif

#endif /* JKO_H */
