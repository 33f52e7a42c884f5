// Host driver and C ABI of libjko (see include/jko.h).
//
// One JKO step runs Listing 1 of the paper in the reduced scaling form of
// Proposition 3.3:  per iteration  t = xi^T a -> b = q / t  and
// s = xi b -> p = Prox(s), a = p / s, each Gibbs application being d per-axis
// contraction passes whose last pass carries the pointwise update.  After an
// absorption switch (a, b carried as logs) every application runs on the
// exact log-sum-exp passes instead; the host always knows which domain the
// device is in before it queues an application.  The stop
// test of Listing 1 (|| b * xi^T a - q ||_1 <= tol after an even half-step) is
// computed on the device every `check_every` iterations from the t of the next
// iteration; the host queues iterations one check interval ahead of the test
// it has read back, and every kernel returns at once when the device control
// block says the step is done, so the GPU never idles on the read-back.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "jko_internal.h"
#include "heat.h"
#include "logpass.h"

using namespace jko;

namespace {

thread_local std::string g_err;

jko_status fail(jko_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(x)                                                                  \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess)                                                       \
            return fail(JKO_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_));   \
    } while (0)

constexpr int kMaxN = 1024;
constexpr size_t kAlign = 256;
// Polls of one grid-barrier wait of the resident kernel before it gives up
// (each poll sleeps ~64 cycles: far beyond any legitimate wait).
constexpr int kBarrierSpinLimit = 1 << 22;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Geo {
    int d = 0;
    int n[3] = {1, 1, 1};
    int64_t N = 0;
};

bool geo_of(const jko_grid* g, Geo* out) {
    if (!g || g->ndim < 1 || g->ndim > 3) return false;
    Geo r;
    r.d = g->ndim;
    r.N = 1;
    for (int k = 0; k < r.d; ++k) {
        if (g->n[k] < 1 || g->n[k] > kMaxN) return false;
        r.n[k] = g->n[k];
        r.N *= g->n[k];
    }
    *out = r;
    return true;
}

// The passes of one application of xi, in order: axis d-1 (contiguous) first,
// then d-2, ..., 0.  Each pass moves its axis to the front of the memory
// order, so pass p contracts the contiguous axis of pass p-1's output, and
// after all d passes the field is back in row-major order.
struct PassShape {
    int64_t R;
    int n;
    int axis;
};

struct PassList {
    PassShape p[3];
    int count = 0;
    const PassShape* begin() const { return p; }
    const PassShape* end() const { return p + count; }
    size_t size() const { return (size_t)count; }
    const PassShape& operator[](size_t i) const { return p[i]; }
};

PassList passes_of(const Geo& g) {
    PassList v;
    for (int k = g.d - 1; k >= 0; --k) v.p[v.count++] = PassShape{g.N / g.n[k], g.n[k], k};
    return v;
}

Pass make_pass(const PassShape& ps) {
    Pass p{};
    p.R = ps.R;
    p.n = ps.n;
    return p;
}

// ---------------------------------------------------------------- workspace

enum : int { OP_GIBBS = 0, OP_STEP = 1, OP_FLOW = 2, OP_BACKWARD = 3, OP_ATTR_STEP = 4, OP_ATTR_FLOW = 5 };

// The Wasserstein attraction keeps two couplings; their scalings are stacked
// as one field of shape (2, n...) whose first axis has the identity as factor.
Geo stacked_of(const Geo& g) {
    Geo s;
    s.d = g.d + 1;
    s.n[0] = 2;
    for (int k = 0; k < g.d; ++k) s.n[k + 1] = g.n[k];
    s.N = 2 * g.N;
    return s;
}

struct Layout {
    size_t ctl = 0, sync = 0, hostout = 0, part = 0, factors = 0, fields = 0, hist = 0, stats = 0, total = 0;
    int part_cap = 0;
    size_t factor_off[3] = {0, 0, 0};
    int nfields = 0;
    int64_t hist_fields = 0;
};

int part_cap_of(const Geo& g) {
    int64_t cap = 768;   // input check uses 3 x 256
    if (g.d == 2) cap = std::max<int64_t>(cap, gibbs2d_blocks(g.n[0], g.n[1], 16));
    for (const PassShape& ps : passes_of(g)) {
        const int64_t b = contract_max_blocks(make_pass(ps), 0);
        if (b > cap) cap = b;
    }
    if (g.d == 3) {
        Pass s{};
        s.R = (int64_t)g.n[1] * g.n[2];
        s.n = g.n[0];
        cap = std::max<int64_t>(cap, contract_slow_blocks(s));
    }
    if (g.d == 3 && g.n[0] == 2)      // the attraction's two couplings on a batched 2D kernel
        cap = std::max<int64_t>(cap, 2 * gibbs2d_blocks(g.n[1], g.n[2], 16));
    for (int k = 0; k < g.d; ++k) {   // log-domain passes
        int64_t outer = 1, inner = 1;
        for (int j = 0; j < k; ++j) outer *= g.n[j];
        for (int j = k + 1; j < g.d; ++j) inner *= g.n[j];
        cap = std::max<int64_t>(cap, log_pass_blocks(make_log_pass(outer, g.n[k], inner, 0, 1.0, nullptr)));
    }
    return (int)cap;
}

Layout layout_of(const Geo& g, int op, int64_t iters_or_steps) {
    Layout L;
    size_t off = 0;
    L.ctl = off;
    off += align_up(sizeof(Ctl));
    L.sync = off;
    off += align_up(4 * (size_t)resident_sync_words(kFusedMaxBlocks));
    L.hostout = off;
    off += align_up(8 * sizeof(double));
    L.part_cap = part_cap_of(g);
    L.part = off;
    off += align_up(4 * (size_t)L.part_cap * sizeof(double));
    L.factors = off;
    for (int k = 0; k < g.d; ++k) {
        int same = -1;
        for (int j = 0; j < k; ++j)
            if (g.n[j] == g.n[k]) same = j;
        if (same >= 0) {
            L.factor_off[k] = L.factor_off[same];
            continue;
        }
        const size_t nn = (size_t)g.n[k] * g.n[k];
        L.factor_off[k] = off;
        off += align_up(nn * sizeof(float)) + 2 * align_up(nn * sizeof(uint16_t));
    }
    // fields: z1, z2 (all ops); a, b, g, kf (step+); p ping-pong x2 (flow+);
    // backward: q, abar, sbar, bbar, tbar, qbar, pbar, wacc, tmp
    int nf = 2;
    if (op >= OP_STEP) nf += 4;
    if (op >= OP_FLOW) nf += 2;
    if (op == OP_BACKWARD) nf += 9;
    L.nfields = nf;
    L.fields = off;
    off += (size_t)nf * align_up((size_t)g.N * sizeof(float));
    if (op == OP_BACKWARD) {
        L.hist_fields = 2 * std::max<int64_t>(iters_or_steps, 1);
        L.hist = off;
        off += (size_t)L.hist_fields * align_up((size_t)g.N * sizeof(float));
    }
    if (op == OP_FLOW) {
        L.stats = off;
        off += align_up((size_t)std::max<int64_t>(iters_or_steps, 1) * 8 * sizeof(double));
    }
    L.total = off;
    return L;
}

struct Plan {
    Geo g;
    Layout L;
    char* base = nullptr;
    Ctl* ctl = nullptr;
    uint32_t* sync = nullptr;
    double* hostout = nullptr;
    Partials part{};
    const float* K1[3] = {};
    const uint16_t* K1hi[3] = {};
    const uint16_t* K1lo[3] = {};
    float* field[24] = {};
    hipStream_t st = nullptr;
    int prec = 0;
    double gamma = 0.0;
    bool ident[3] = {false, false, false};   // axis whose factor is the identity (the attraction's stacking axis)
    int W[3] = {0, 0, 0};        // float32 band half-widths of the factors
    bool fused2d = false;        // 2D applications use the fused band kernel
    int tile = 0;                // ... with output tiles of this edge (16 or 32)
    bool batch2d = false;        // stacked (2, n0, n1) applications: the fused kernel on both fields
    bool batch_pass = false;     // stacked (2, n0, n1) applications: per-field rotating passes, no pass over
                                 // the identity axis
    bool resident = false;       // ... and a step may run in one resident launch
    bool respass = false;        // a step may run in one launch of the resident pass kernel
    bool plane3d = false;        // 3D applications run as a plane pass and a slow-axis pass

    float* F(int i) const { return field[i]; }
    float* hist(int64_t i) const {
        return reinterpret_cast<float*>(base + L.hist + (size_t)i * align_up((size_t)g.N * sizeof(float)));
    }
};

enum : int { F_Z1 = 0, F_Z2, F_A, F_B, F_G, F_KF, F_P0, F_P1, F_Q, F_ABAR, F_SBAR, F_BBAR, F_TBAR, F_QBAR,
             F_PBAR, F_WACC, F_TMP };

jko_status carve(Plan* P, const Geo& g, int op, int64_t extra, void* ws, size_t ws_bytes, int prec,
                 hipStream_t st) {
    P->g = g;
    P->L = layout_of(g, op, extra);
    if (!ws) return fail(JKO_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", P->L.total);
    if (ws_bytes < P->L.total)
        return fail(JKO_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, P->L.total);
    if (((uintptr_t)ws) % 16 != 0) return fail(JKO_ERR_WORKSPACE, "workspace must be 16-byte aligned");
    P->base = static_cast<char*>(ws);
    P->ctl = reinterpret_cast<Ctl*>(P->base + P->L.ctl);
    P->sync = reinterpret_cast<uint32_t*>(P->base + P->L.sync);
    P->hostout = reinterpret_cast<double*>(P->base + P->L.hostout);
    double* pd = reinterpret_cast<double*>(P->base + P->L.part);
    const int cap = P->L.part_cap;
    P->part = Partials{pd, pd + cap, pd + 2 * cap, pd + 3 * cap, cap};
    for (int k = 0; k < g.d; ++k) {
        const size_t nn = (size_t)g.n[k] * g.n[k];
        char* f = P->base + P->L.factor_off[k];
        P->K1[k] = reinterpret_cast<const float*>(f);
        P->K1hi[k] = reinterpret_cast<const uint16_t*>(f + align_up(nn * sizeof(float)));
        P->K1lo[k] = reinterpret_cast<const uint16_t*>(f + align_up(nn * sizeof(float)) +
                                                       align_up(nn * sizeof(uint16_t)));
    }
    for (int i = 0; i < P->L.nfields; ++i)
        P->field[i] = reinterpret_cast<float*>(P->base + P->L.fields +
                                               (size_t)i * align_up((size_t)g.N * sizeof(float)));
    P->st = st;
    P->prec = prec;
    return JKO_OK;
}

jko_status build_factors(Plan& P, double gamma, int32_t flags = 0) {
    P.gamma = gamma;
    for (int k = 0; k < P.g.d; ++k) P.W[k] = band_halfwidth(P.g.n[k], gamma);
    P.plane3d = P.g.d == 3 && !(flags & JKO_FLAG_AXIS_PASSES) &&
                plane3d_fits(P.g.n[0], P.g.n[1], P.g.n[2], P.W[0], P.W[1], P.W[2]);
    // A 2D application runs as the fused tile kernel, which trades redundant
    // halo work for one launch, with 16 x 16 tiles where at most one block
    // per CU covers the grid.  Otherwise, for axes of a multiple of 32 whose
    // bands span at most seven 32-k panels and at most 256 tiles of 32 x 32,
    // as the two panel passes (and a step on the resident pass kernel, which
    // runs them without launch boundaries); else as the fused kernel with
    // 32 x 32 tiles where it fits, else as the passes.
    P.tile = 0;
    const bool passes2d =
        P.g.d == 2 && resident_pass2d_shape_fits(P.g.n[0], P.g.n[1], P.W[0], P.W[1], 1);
    if (P.g.d == 2 && !(flags & JKO_FLAG_AXIS_PASSES))
        for (int tt : {16, 32}) {
            if (tt == 32 && passes2d) break;
            if (gibbs2d_fits(P.g.n[0], P.g.n[1], P.W[0], P.W[1], P.prec, tt) &&
                gibbs2d_blocks(P.g.n[0], P.g.n[1], tt) <= kFusedMaxBlocks) {
                P.tile = tt;
                break;
            }
        }
    P.fused2d = P.tile != 0;
    P.resident = P.fused2d;
    P.respass = !P.fused2d && passes2d;
    for (int k = 0; k < P.g.d; ++k) {
        bool done = false;
        for (int j = 0; j < k; ++j)
            if (P.g.n[j] == P.g.n[k]) done = true;
        if (done) continue;
        HIP_TRY(launch_build_factor(const_cast<float*>(P.K1[k]), const_cast<uint16_t*>(P.K1hi[k]),
                                    const_cast<uint16_t*>(P.K1lo[k]), P.g.n[k], gamma, P.st));
    }
    return JKO_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Vector (16-byte) epilogue access is allowed when every field pointer is aligned.
void set_vec(EpiArgs& e) {
    const void* ps[] = {e.y, e.q, e.b, e.a, e.p_out, e.s_out, e.t_out, e.hin, e.acc,
                        e.prox.g, e.prox.kappa, e.prox.kf};
    bool ok = true;
    for (const void* p : ps) ok = ok && aligned16(p);
    e.vec_ok = ok ? 1 : 0;
}

// The plane pass of a 3D application (x -> z1) and its slow-axis pass (z1 -> epilogue).
Plane3D plane_of(const Plan& P, const float* x, const Ctl* ctl) {
    return Plane3D{P.g.n[0], P.g.n[1], P.g.n[2], P.W[1], P.W[2], P.K1[1], P.K1hi[1], P.K1lo[1],
                   P.K1[2], P.K1hi[2], P.K1lo[2], x, P.F(F_Z1), ctl};
}
Pass slow_of(const Plan& P) {
    Pass s{};
    s.R = (int64_t)P.g.n[1] * P.g.n[2];
    s.n = P.g.n[0];
    s.W = P.W[0];
    s.K1 = P.K1[0];
    s.K1hi = P.K1hi[0];
    s.K1lo = P.K1lo[0];
    s.X = P.F(F_Z1);
    return s;
}

// y = xi x with the last pass's result handed to `epi`.  Uses z1, z2 as
// intermediates; x must not alias them.  *nblocks = blocks of the last pass.
jko_status apply_xi(const Plan& P, const float* x, EpiArgs epi, int* nblocks) {
    set_vec(epi);
    if (P.batch2d) {
        Band2D b{P.g.n[1], P.g.n[2], P.W[1],   P.W[2],   P.K1[1], P.K1[2],
                 x,        P.K1hi[1], P.K1lo[1], P.K1hi[2], P.K1lo[2], P.tile, P.g.n[0]};
        int nb = 0;
        HIP_TRY(launch_gibbs2d(b, P.prec, epi, &nb, P.st));
        if (nblocks) *nblocks = nb;
        return JKO_OK;
    }
    if (P.fused2d) {
        Band2D b{P.g.n[0], P.g.n[1], P.W[0],   P.W[1],   P.K1[0], P.K1[1],
                 x,        P.K1hi[0], P.K1lo[0], P.K1hi[1], P.K1lo[1], P.tile};
        int nb = 0;
        HIP_TRY(launch_gibbs2d(b, P.prec, epi, &nb, P.st));
        if (nblocks) *nblocks = nb;
        return JKO_OK;
    }
    if (P.plane3d) {
        HIP_TRY(launch_plane3d(plane_of(P, x, epi.ctl), P.prec, nullptr, P.st));
        int nb = 0;
        HIP_TRY(launch_contract_slow(slow_of(P), P.prec, epi, &nb, P.st));
        if (nblocks) *nblocks = nb;
        return JKO_OK;
    }
    PassList ps = passes_of(P.g);
    if (P.batch_pass) ps.count = P.g.d - 1;   // axes d-1 .. 1; axis 0 stacks the fields
    const float* in = x;
    for (size_t i = 0; i < ps.size(); ++i) {
        Pass pass = make_pass(ps[i]);
        if (P.batch_pass) pass.B = P.g.n[0];
        pass.K1 = P.K1[ps[i].axis];
        pass.K1hi = P.K1hi[ps[i].axis];
        pass.K1lo = P.K1lo[ps[i].axis];
        pass.W = P.W[ps[i].axis];
        pass.X = in;
        const bool last = (i + 1 == ps.size());
        EpiArgs e;
        int nb = 0;
        if (last) {
            e = epi;
        } else {
            e = EpiArgs{};
            e.kind = EpiKind::STORE;
            e.y = P.F((i % 2 == 0) ? F_Z1 : F_Z2);
            e.ctl = epi.ctl;
            e.part = epi.part;
            set_vec(e);
        }
        HIP_TRY(launch_contract(pass, P.prec, e, &nb, P.st));
        if (last && nblocks) *nblocks = nb;
        if (!last) in = e.y;
    }
    return JKO_OK;
}

// y = xi x in the log domain (x, y and the epilogue's scalings hold logs): one
// exact log-sum-exp pass per axis, in the field's own layout, the last one
// handing its values to `epi`; identity axes are skipped.  Uses z1, z2.
jko_status apply_xi_log(const Plan& P, const float* x, EpiArgs epi, int* nblocks) {
    int axes[3], na = 0;
    for (int k = P.g.d - 1; k >= 0; --k)
        if (!P.ident[k]) axes[na++] = k;
    const float* in = x;
    for (int i = 0; i < na; ++i) {
        const int k = axes[i];
        int64_t outer = 1, inner = 1;
        for (int j = 0; j < k; ++j) outer *= P.g.n[j];
        for (int j = k + 1; j < P.g.d; ++j) inner *= P.g.n[j];
        const LogPass L = make_log_pass(outer, P.g.n[k], inner, P.W[k], P.gamma, in);
        const bool last = i + 1 == na;
        EpiArgs e = epi;
        if (!last) {
            e = EpiArgs{};
            e.kind = EpiKind::STORE;
            e.y = P.F(i % 2 == 0 ? F_Z1 : F_Z2);
            e.ctl = epi.ctl;
            e.part = epi.part;
        }
        int nb = 0;
        HIP_TRY(launch_log_pass(L, e, &nb, P.st));
        if (last && nblocks) *nblocks = nb;
        in = e.y;
    }
    return JKO_OK;
}

// Either domain: the plain contractions, or the log-domain passes.
jko_status apply_xi_in(bool logd, const Plan& P, const float* x, const EpiArgs& epi, int* nblocks) {
    return logd ? apply_xi_log(P, x, epi, nblocks) : apply_xi(P, x, epi, nblocks);
}

// Host mirror of the control block for the stop-test read-back.  The calls
// use a pinned buffer and an event (made once per thread), so that the host
// can look at one check while the next interval is queued.  The no-allocation
// entry point uses a pageable buffer and no event instead (every read-back is
// synchronous).
struct Readback {
    Ctl* host = nullptr;
    hipEvent_t ev = nullptr;
    int device = -1;
};
// The pinned one releases its buffer and event when its thread ends; for the
// main thread that is at exit, before the HIP runtime's own teardown (the
// destructors of thread-local objects run before those of static ones).
struct PinnedReadback : Readback {
    PinnedReadback() = default;
    PinnedReadback(const PinnedReadback&) = delete;
    PinnedReadback& operator=(const PinnedReadback&) = delete;
    ~PinnedReadback() {
        if (ev) (void)hipEventDestroy(ev);
        if (host) (void)hipHostFree(host);
    }
};
thread_local PinnedReadback g_rb;        // pinned
thread_local Ctl g_pageable[4];
thread_local Readback g_rb_pageable{g_pageable, nullptr, -1};
thread_local Readback* g_cur = &g_rb;    // the one the current call uses
thread_local bool g_no_alloc = false;    // inside jko_step_static

Readback& rb() { return *g_cur; }

jko_status readback_init() {
    if (g_no_alloc) {
        g_cur = &g_rb_pageable;
        return JKO_OK;
    }
    g_cur = &g_rb;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (g_rb.host && g_rb.device == dev) return JKO_OK;
    if (!g_rb.host) HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&g_rb.host), 4 * sizeof(Ctl), hipHostMallocDefault));
    if (g_rb.ev && g_rb.device != dev) {
        (void)hipEventDestroy(g_rb.ev);
        g_rb.ev = nullptr;
    }
    if (!g_rb.ev) HIP_TRY(hipEventCreateWithFlags(&g_rb.ev, hipEventDisableTiming));
    g_rb.device = dev;
    return JKO_OK;
}

jko_status read_ctl(const Plan& P, Ctl* out) {
    HIP_TRY(hipMemcpyAsync(rb().host, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, P.st));
    HIP_TRY(hipStreamSynchronize(P.st));
    *out = *rb().host;
    return JKO_OK;
}

// ---------------------------------------------------------------- validation

jko_status check_params(const jko_params* pr) {
    if (!pr) return fail(JKO_ERR_INVALID, "params is NULL");
    if (!(pr->gamma > 0.0) || !isfinite(pr->gamma)) return fail(JKO_ERR_INVALID, "gamma must be finite and > 0");
    if (!(pr->tau > 0.0) || !isfinite(pr->tau)) return fail(JKO_ERR_INVALID, "tau must be finite and > 0");
    if (pr->max_iters < 1) return fail(JKO_ERR_INVALID, "max_iters must be >= 1");
    if (pr->check_every < 1) return fail(JKO_ERR_INVALID, "check_every must be >= 1");
    if (pr->precision != JKO_FP32 && pr->precision != JKO_SPLIT_BF16)
        return fail(JKO_ERR_INVALID, "unknown precision %d", pr->precision);
    if (isnan(pr->tol_l1)) return fail(JKO_ERR_INVALID, "tol_l1 is NaN");
    if (pr->flags & ~(JKO_FLAG_NO_RESIDENT | JKO_FLAG_AXIS_PASSES | JKO_FLAG_ABSORB_ON_A))
        return fail(JKO_ERR_INVALID, "unknown flags 0x%x", pr->flags);
    return JKO_OK;
}

// Both congestion kinds share the potential, capacity, preparation and
// capacity check; they differ only in the prox.
bool is_congestion(const jko_energy* en) {
    return en->kind == JKO_F_CONGESTION || en->kind == JKO_F_CONGESTION_BINARY;
}

jko_status check_energy(const jko_energy* en) {
    if (!en) return fail(JKO_ERR_INVALID, "energy is NULL");
    switch (en->kind) {
        case JKO_F_ZERO:
            return JKO_OK;
        case JKO_F_CONGESTION:
            if (!en->kappa && (isnan(en->kappa_scalar) || en->kappa_scalar < 0.f))
                return fail(JKO_ERR_INVALID, "kappa_scalar must be >= 0 (or +inf)");
            return JKO_OK;
        case JKO_F_CONGESTION_BINARY:
            if (!en->kappa && !(en->kappa_scalar >= 0.f && isfinite(en->kappa_scalar)))
                return fail(JKO_ERR_INVALID, "binary congestion: kappa_scalar must be finite and >= 0");
            return JKO_OK;
        case JKO_F_ENTROPY:
            if (!en->coef && !(en->coef_scalar >= 0.f)) return fail(JKO_ERR_INVALID, "coef_scalar must be >= 0");
            return JKO_OK;
        case JKO_F_ATTRACTION:
            if (!en->target) return fail(JKO_ERR_INVALID, "attraction: target is NULL");
            if (!en->kappa && (isnan(en->kappa_scalar) || en->kappa_scalar < 0.f))
                return fail(JKO_ERR_INVALID, "kappa_scalar must be >= 0 (or +inf)");
            return JKO_OK;
        case JKO_F_GEN_ENTROPY:
            if (!en->m_field && (!(en->m >= 1.f) || !isfinite(en->m)))
                return fail(JKO_ERR_INVALID, "generalised entropy exponent m must be >= 1");
            if (!(en->density_scale > 0.f) || !isfinite(en->density_scale))
                return fail(JKO_ERR_INVALID, "density_scale must be > 0");
            if (!en->coef && !(en->coef_scalar >= 0.f)) return fail(JKO_ERR_INVALID, "coef_scalar must be >= 0");
            if (en->newton_steps < 0 || en->newton_steps > 32)
                return fail(JKO_ERR_INVALID, "newton_steps must be in 0..32");
            return JKO_OK;
        case JKO_F_POROUS:
            if (!(en->m > 1.f) || !isfinite(en->m)) return fail(JKO_ERR_INVALID, "porous exponent m must be > 1");
            if (!(en->density_scale > 0.f)) return fail(JKO_ERR_INVALID, "density_scale must be > 0");
            if (!en->coef && !(en->coef_scalar >= 0.f)) return fail(JKO_ERR_INVALID, "coef_scalar must be >= 0");
            if (en->newton_steps < 0 || en->newton_steps > 32)
                return fail(JKO_ERR_INVALID, "newton_steps must be in 0..32");
            return JKO_OK;
        default:
            return fail(JKO_ERR_INVALID, "unknown energy kind %d", en->kind);
    }
}

ProxArgs prox_args_fields(const jko_energy* en, double sigma, float* fg, float* fkf) {
    ProxArgs px{};
    px.kind = en->kind;
    px.m = en->m;
    px.newton = en->newton_steps > 0 ? en->newton_steps : 8;
    if (is_congestion(en)) {
        px.g = en->w ? fg : nullptr;
        px.kappa = en->kappa;
        px.kappa_s = en->kappa_scalar;
    } else if (en->kind == JKO_F_ENTROPY) {
        if (en->coef) px.kf = fkf;
        else px.kf_s = (float)(1.0 / (1.0 + sigma * (double)en->coef_scalar));
    } else if (en->kind == JKO_F_GEN_ENTROPY) {
        // c = sigma b m and eps = m - 1 per cell when either b or m is a field
        if (en->coef || en->m_field) {
            px.kf = fkf;
            px.g = fg;
        } else {
            px.kf_s = (float)(sigma * (double)en->coef_scalar * (double)en->m);
            px.eps_s = en->m - 1.f;
        }
        px.lD = (float)log((double)en->density_scale);
    } else if (en->kind == JKO_F_POROUS) {
        if (en->coef) px.kf = fkf;
        else {
            const double m = en->m;
            px.kf_s = (float)log(sigma * (double)en->coef_scalar * m * pow((double)en->density_scale, m - 1.0));
        }
    }
    return px;
}

ProxArgs prox_args(const Plan& P, const jko_energy* en, double sigma) {
    return prox_args_fields(en, sigma, P.F(F_G), P.F(F_KF));
}

jko_status prepare_energy(const Plan& P, const jko_energy* en, double sigma) {
    const bool need = (is_congestion(en) && en->w) ||
                      ((en->kind == JKO_F_ENTROPY || en->kind == JKO_F_POROUS) && en->coef) ||
                      (en->kind == JKO_F_GEN_ENTROPY && (en->coef || en->m_field));
    if (!need) return JKO_OK;
    HIP_TRY(launch_prepare_energy(en, sigma, P.g.N, P.F(F_G), P.F(F_KF), P.st));
    return JKO_OK;
}

// Capacity / finiteness check of a density (synchronous).
jko_status input_check(const Plan& P, const jko_energy* en, const float* p) {
    HIP_TRY(launch_input_check(p, en->kappa, en->kappa_scalar, P.g.N, is_congestion(en),
                               P.part.err, 3 * 256, P.hostout, P.st));
    double h[3];
    HIP_TRY(hipMemcpyAsync(rb().host, P.hostout, 3 * sizeof(double), hipMemcpyDeviceToHost, P.st));
    HIP_TRY(hipStreamSynchronize(P.st));
    memcpy(h, rb().host, sizeof h);
    if (h[2] > 0.0) return fail(JKO_ERR_NONFINITE, "input density or capacity has %g negative/non-finite cells", h[2]);
    if (is_congestion(en) && h[1] < h[0] * (1.0 - 1e-6))
        return fail(JKO_ERR_INFEASIBLE, "capacity sum %.9g < mass %.9g", h[1], h[0]);
    return JKO_OK;
}

// ------------------------------------------------------------ device stats

// Writes a step's statistics, in the field order of jko_stats and all as
// doubles, to `out` (device) from the control block the step left, so that a
// caller can keep them on the device without a read-back.  `mass` (device,
// nullable) replaces the control block's mass; `attr`: the attraction, which
// does not monitor max|log a|.
__global__ void k_stats_export(const Ctl* c, const double* mass, double* out, int32_t K, int32_t tolmode,
                               int32_t attr) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const bool bytol = tolmode && c->done && !c->nonfinite;
    out[0] = bytol ? c->stop_iter : K;
    out[1] = c->absorptions;
    out[2] = bytol ? JKO_STOP_TOL : JKO_STOP_CAP;
    out[3] = c->nonfinite ? JKO_ERR_NONFINITE : JKO_OK;
    out[4] = c->err;
    out[5] = mass ? mass[0] : c->mass;
    out[6] = attr ? 0.0 : c->maxloga;
    out[7] = c->maxlogb;
}

hipError_t launch_stats_export(const Ctl* c, const double* mass, double* out, int K, bool tolmode, bool attr,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_stats_export, dim3(1), dim3(64), 0, s, c, mass, out, K, tolmode ? 1 : 0, attr ? 1 : 0);
    return hipGetLastError();
}

// ----------------------------------------------------------------- resident

bool use_resident(const Plan& P, const jko_params* pr, const ProxArgs& px) {
    return P.resident && !(pr->flags & JKO_FLAG_NO_RESIDENT) &&
           resident2d_fits(P.g.n[0], P.g.n[1], P.W[0], P.W[1], px.kind, P.prec, P.tile);
}

// The resident pass kernel (no history for the adjoint's recomputation).
bool use_respass(const Plan& P, const jko_params* pr, const ProxArgs& px, bool record_hist) {
    return P.respass && !record_hist && !(pr->flags & JKO_FLAG_NO_RESIDENT) &&
           resident_pass2d_fits(P.g.n[0], P.g.n[1], P.W[0], P.W[1], 1, px.kind, P.prec);
}

// Queue the resident pass kernel for K iterations of a step on B stacked
// fields (the scalings and control block initialised); q holds the B
// marginals.  *launched as for launch_resident.
jko_status launch_respass(const Plan& P, int B, int W0, int W1, int k0, int k1, const float* q, float* p_out,
                          const ProxArgs& px, float alpha, int K, int ce, bool checks, double tol, double absorb,
                          int a_only, bool* launched) {
    *launched = false;
    ResidentPass2D r{};
    const int n0 = P.g.n[k0], n1 = P.g.n[k1];
    r.n0 = n0;
    r.n1 = n1;
    r.W0 = W0;
    r.W1 = W1;
    r.K0 = P.K1[k0];
    r.K0hi = P.K1hi[k0];
    r.K0lo = P.K1lo[k0];
    r.K1 = P.K1[k1];
    r.K1hi = P.K1hi[k1];
    r.K1lo = P.K1lo[k1];
    r.B = B;
    r.q = q;
    r.a = P.F(F_A);
    r.b = P.F(F_B);
    r.u0 = P.F(F_Z1);
    r.u1 = P.F(F_Z2);
    r.p_out = p_out;
    r.prox = px;
    r.alpha = alpha;
    r.part = P.part;
    r.ctl = P.ctl;
    r.sync = P.sync;
    r.K = K;
    r.ce = ce;
    r.checks = checks ? 1 : 0;
    r.split = P.prec == JKO_SPLIT_BF16 ? 1 : 0;
    r.a_only = a_only;
    r.check_mass = B == 1 ? 1 : 0;
    r.tol = tol;
    r.absorb = absorb;
    r.spin_limit = kBarrierSpinLimit;
    EpiArgs al{};
    al.q = q;
    al.b = r.b;
    al.a = r.a;
    al.y = r.u0;
    al.acc = r.u1;
    al.p_out = p_out;
    al.prox = px;
    set_vec(al);
    r.vec_ok = al.vec_ok;
    HIP_TRY(launch_fill(reinterpret_cast<float*>(P.sync), 0.f,
                        resident_sync_words(resident_pass2d_blocks(n0, n1, B)), P.st));
    const hipError_t e = launch_resident_pass2d(r, P.st);
    if (e == hipErrorCooperativeLaunchTooLarge) {
        (void)hipGetLastError();
        return JKO_OK;
    }
    HIP_TRY(e);
    *launched = true;
    return JKO_OK;
}

// Queue the resident kernel for K iterations of a step (scalings and control
// block already initialised).  *launched is false (and nothing is queued but
// the sync-word reset) when the runtime refuses the cooperative grid, e.g.
// because part of the device is unavailable: the caller then runs the launch
// path instead.
jko_status launch_resident(const Plan& P, const float* q, float* p_out, const ProxArgs& px, int K, int ce,
                           bool checks, double tol, double absorb, int a_only, bool record_hist, bool* launched) {
    *launched = false;
    Resident2D r{};
    r.B = Band2D{P.g.n[0], P.g.n[1], P.W[0], P.W[1], P.K1[0], P.K1[1], nullptr,
                 P.K1hi[0], P.K1lo[0], P.K1hi[1], P.K1lo[1], P.tile};
    r.split = P.prec == JKO_SPLIT_BF16 ? 1 : 0;
    r.q = q;
    r.a = P.F(F_A);
    r.b = P.F(F_B);
    r.p_out = p_out;
    r.hist = record_hist ? P.hist(0) : nullptr;
    r.hist_stride = record_hist ? (int64_t)(P.hist(1) - P.hist(0)) : 0;
    r.prox = px;
    r.part = P.part;
    r.ctl = P.ctl;
    r.sync = P.sync;
    r.K = K;
    r.ce = ce;
    r.checks = checks ? 1 : 0;
    r.tol = tol;
    r.absorb = absorb;
    r.a_only = a_only;
    r.spin_limit = kBarrierSpinLimit;
    EpiArgs al{};
    al.q = q;
    al.b = r.b;
    al.a = r.a;
    al.p_out = p_out;
    al.prox = px;
    al.t_out = r.hist;
    set_vec(al);
    r.vec_ok = al.vec_ok && (r.hist_stride % 4 == 0);
    HIP_TRY(launch_fill(reinterpret_cast<float*>(P.sync), 0.f,
                        resident_sync_words(gibbs2d_blocks(P.g.n[0], P.g.n[1], P.tile)), P.st));
    const hipError_t e = launch_resident2d(r, P.st);
    if (e == hipErrorCooperativeLaunchTooLarge) {
        (void)hipGetLastError();
        return JKO_OK;
    }
    HIP_TRY(e);
    *launched = true;
    return JKO_OK;
}

// Synchronous: fails if a wait of the last resident launch ran out.
jko_status resident_check(const Plan& P) {
    uint32_t w = 0;
    HIP_TRY(hipMemcpyAsync(rb().host, P.sync, sizeof w, hipMemcpyDeviceToHost, P.st));
    HIP_TRY(hipStreamSynchronize(P.st));
    memcpy(&w, rb().host, sizeof w);
    if (w) return fail(JKO_ERR_HIP, "resident kernel: a wait for another block timed out");
    return JKO_OK;
}

// ----------------------------------------------------------------- one step

struct StepOut {
    jko_stats st{};
};

// Runs the iteration of one step with q (device) -> p_out (device).  When
// `record_hist` is set, iteration k stores t_k and s_k into
// P.hist(2(k-1)) and P.hist(2(k-1)+1) (adjoint recomputation, fixed count).
// `st_out` (host) and `st_dev` (device, 8 doubles) receive the statistics;
// only the host record makes the step wait for them.
jko_status run_step(const Plan& P, const jko_params* pr, const ProxArgs& px, const float* q, float* p_out,
                    bool want_stats, bool record_hist, jko_stats* st_out, double* st_dev = nullptr) {
    const int K = pr->max_iters;
    const int ce = pr->check_every;
    const bool tolmode = pr->tol_l1 > 0.0;
    float* a = P.F(F_A);
    float* b = P.F(F_B);

    // Absorption: threshold <= 0 runs the log domain from the start (log a = 0),
    // +inf never switches, otherwise the check that sees max|log a|, max|log b|
    // above it switches.
    const double thr = pr->absorb_threshold;
    const bool log_from_start = thr <= 0.0;
    const double absorb = (log_from_start || !(thr < INFINITY)) ? 0.0 : thr;
    const int a_only = (pr->flags & JKO_FLAG_ABSORB_ON_A) ? 1 : 0;
    HIP_TRY(launch_fill(a, log_from_start ? 0.f : 1.f, P.g.N, P.st));
    HIP_TRY(launch_ctl_reset(P.ctl, log_from_start ? 1 : 0, P.st));
    // Checks (monitor, absorption trigger) every `ce` iterations in tolerance
    // mode, and in fixed-count mode when absorption may trigger.
    const bool checks = tolmode || absorb > 0.0;
    // The domain the next application runs in.  A switch is decided on the
    // device at a check; the host reads that check back before it queues
    // anything after it, so it always launches the right kernels.
    bool logd = log_from_start;

    EpiArgs eb{};
    eb.kind = EpiKind::BUPDATE;
    eb.q = q;
    eb.b = b;
    eb.part = P.part;
    eb.ctl = P.ctl;
    EpiArgs ep{};
    ep.kind = EpiKind::PROX;
    ep.a = a;
    ep.p_out = p_out;
    ep.prox = px;
    ep.part = P.part;
    ep.ctl = P.ctl;

    int k0 = 1;   // first iteration left to the launch path
    bool resident = false;
    const bool respass = !logd && use_respass(P, pr, px, record_hist);
    if (!logd && (respass || use_resident(P, pr, px))) {
        jko_status s = respass ? launch_respass(P, 1, P.W[0], P.W[1], 0, 1, q, p_out, px, 0.f, K, ce, checks,
                                                pr->tol_l1, absorb, a_only, &resident)
                               : launch_resident(P, q, p_out, px, K, ce, checks, pr->tol_l1, absorb, a_only,
                                                 record_hist, &resident);
        if (s) return s;
        if (resident && (s = resident_check(P))) return s;
        if (resident && absorb > 0.0) {
            // The kernel returns after the proximal half-step of an iteration
            // whose check asked for the switch: convert the scalings and run
            // the rest of the step on the log-domain passes.
            Ctl c{};
            if ((s = read_ctl(P, &c))) return s;
            if (c.exit_iter > 0 && !c.done) {
                HIP_TRY(launch_absorb(P.ctl, a, b, P.g.N, P.st));
                HIP_TRY(launch_ctl_commit(P.ctl, c.exit_iter, P.st));
                logd = true;
                k0 = c.exit_iter + 1;
                resident = false;
            }
        }
    }

    // Each check's control block is read back asynchronously after the
    // iteration's proximal half-step (and, in the plain domain, the
    // absorption commit), and looked at when the next check's kernels are
    // queued, so the GPU does not idle on the read-back.  A stop makes every
    // later kernel return at once.  A switch to the log domain makes the
    // plain-domain kernels queued after it return at once too: when the host
    // sees it, it resumes at the iteration after the switch in the log domain
    // (the state is exactly the one the switch left).  Without an event
    // (the allocation-free entry point) every check is read back at once.
    const bool async_rb = rb().ev != nullptr;
    bool pending = false;   // a read-back of the control block is in flight
    bool stopped = false;
    int nb = 0;
    int k = k0;
    for (;;) {
        for (; k <= (resident ? 0 : K); ++k) {
            eb.check = (checks && k > 1 && (k - 1) % ce == 0) ? 1 : 0;
            eb.t_out = record_hist ? P.hist(2 * (int64_t)(k - 1)) : nullptr;
            jko_status s = apply_xi_in(logd, P, a, eb, &nb);
            if (s) return s;
            if (eb.check) {
                HIP_TRY(launch_ctl_check(P.ctl, P.part, nb, k, pr->tol_l1, 1, absorb, a_only, logd ? 0 : 1, P.st));
                if (pending) {
                    HIP_TRY(hipEventSynchronize(rb().ev));
                    pending = false;
                    const Ctl h = *rb().host;
                    if (h.done) {
                        stopped = true;
                        break;
                    }
                    if (h.logmode && !logd) {   // resume after the switch iteration
                        logd = true;
                        k = h.exit_iter;
                        continue;
                    }
                }
            }
            const bool cand = (checks && k % ce == 0) || k == K;
            ep.check = cand ? 1 : 0;
            ep.write_p = cand ? 1 : 0;
            ep.s_out = record_hist ? P.hist(2 * (int64_t)(k - 1) + 1) : nullptr;
            s = apply_xi_in(logd, P, b, ep, &nb);
            if (s) return s;
            if (eb.check && absorb > 0.0 && !logd) {
                // a switch decided at this iteration's check takes effect now
                HIP_TRY(launch_absorb(P.ctl, a, b, P.g.N, P.st));
                HIP_TRY(launch_ctl_commit(P.ctl, k, P.st));
            }
            if (eb.check) {
                if (async_rb) {
                    HIP_TRY(hipMemcpyAsync(rb().host, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, P.st));
                    HIP_TRY(hipEventRecord(rb().ev, P.st));
                    pending = true;
                } else {
                    Ctl c{};
                    if ((s = read_ctl(P, &c))) return s;
                    if (c.done) {
                        stopped = true;
                        break;
                    }
                    if (c.logmode) logd = true;
                }
            }
        }
        if (stopped || resident || logd || !(absorb > 0.0)) break;
        // a switch after the last check that was looked at voided the
        // iterations queued after it: resume there
        HIP_TRY(hipStreamSynchronize(P.st));
        pending = false;
        Ctl c{};
        jko_status s = read_ctl(P, &c);
        if (s) return s;
        if (c.logmode && !logd && !c.done) {
            logd = true;
            k = c.exit_iter + 1;
            continue;
        }
        break;
    }
    // Cap reached: the violation of the returned iterate takes one more
    // t = xi^T a (its kernels and check return at once on a stopped step).
    auto monitor = [&]() -> jko_status {
        EpiArgs em{};
        em.kind = EpiKind::MONITOR;
        em.q = q;
        em.b = b;
        em.part = P.part;
        em.ctl = P.ctl;
        jko_status s = apply_xi_in(logd, P, a, em, &nb);
        if (s) return s;
        HIP_TRY(launch_ctl_check(P.ctl, P.part, nb, K + 1, -1.0, 1, 0.0, 0, 0, P.st));
        return JKO_OK;
    };
    Ctl c{};
    if (tolmode || want_stats) {
        HIP_TRY(hipStreamSynchronize(P.st));
        jko_status s = read_ctl(P, &c);
        if (s) return s;
        if (!c.done && (want_stats || st_dev)) {
            if ((s = monitor())) return s;
            if ((s = read_ctl(P, &c))) return s;
            c.done = 0;
        }
    } else if (st_dev) {
        jko_status s = monitor();   // queued without a read-back
        if (s) return s;
    }
    if (st_dev) HIP_TRY(launch_stats_export(P.ctl, nullptr, st_dev, K, tolmode, false, P.st));
    if (st_out) {
        jko_stats& o = *st_out;
        const bool bytol = tolmode && c.done && !c.nonfinite;
        o.iters = bytol ? c.stop_iter : K;
        o.absorptions = c.absorptions;
        o.stop_reason = bytol ? JKO_STOP_TOL : JKO_STOP_CAP;
        o.status = c.nonfinite ? JKO_ERR_NONFINITE : JKO_OK;
        o.marginal_l1 = c.err;
        o.mass = c.mass;
        o.max_abs_log_a = c.maxloga;
        o.max_abs_log_b = c.maxlogb;
    }
    if (c.nonfinite) return fail(JKO_ERR_NONFINITE, "non-finite value in the marginal monitor");
    return JKO_OK;
}

// Mass of a density of N cells (synchronous).
jko_status mass_of(const Plan& P, const float* p, int64_t N, double* out) {
    HIP_TRY(launch_input_check(p, nullptr, INFINITY, N, 0, P.part.err, 3 * 256, P.hostout, P.st));
    HIP_TRY(hipMemcpyAsync(rb().host, P.hostout, sizeof(double), hipMemcpyDeviceToHost, P.st));
    HIP_TRY(hipStreamSynchronize(P.st));
    memcpy(out, rb().host, sizeof(double));
    return JKO_OK;
}

// One JKO step of the Wasserstein attraction with congestion (Section 5.2) on
// the stacked plan P (shape (2, n...)): the scaling of Proposition 5.2 with the
// marginals first and the corrections dropped.  Iteration k:
//   t_m = xi^T a_m, b_m = (q, r)_m / t_m          (b-update epilogue, stacked)
//   s_m = xi b_m                                    (store epilogue)
//   p = min(s_1^{1/(1+tau)} s_2^{tau/(1+tau)}, kappa), a_m = p / s_m
// with the monitor, stop rule and statistics of run_step (the monitor is the
// violation of both couplings' right marginals).  N cells per field; the
// target is scaled by rscale to the mass of q (both couplings need one mass).
jko_status run_attraction(const Plan& P, const jko_params* pr, const jko_energy* en, const float* q, float* p_out,
                          int64_t N, double rscale, bool want_stats, jko_stats* st_out, double* st_dev = nullptr) {
    // Absorption as in run_step: <= 0 runs the log domain from the start, +inf
    // (or NaN) never switches, otherwise the check that sees max|log b| above
    // the threshold switches a and b to logs after that iteration's proximal
    // half-step (max|log a| is not monitored here).
    const double thr = pr->absorb_threshold;
    const bool logmode = thr <= 0.0;
    const double absorb = (logmode || !(thr < INFINITY)) ? 0.0 : thr;
    const int K = pr->max_iters;
    const int ce = pr->check_every;
    const bool tolmode = pr->tol_l1 > 0.0;
    const bool checks = tolmode || absorb > 0.0;
    float* a = P.F(F_A);
    float* b = P.F(F_B);
    float* sv = P.F(F_G);    // s_1, s_2
    float* qs = P.F(F_KF);   // q, r
    HIP_TRY(launch_copy(qs, q, N, P.st));
    HIP_TRY(launch_copy_scaled(qs + N, en->target, rscale, N, P.st));   // r at the mass of q
    HIP_TRY(launch_fill(a, logmode ? 0.f : 1.f, 2 * N, P.st));
    HIP_TRY(launch_ctl_reset(P.ctl, logmode ? 1 : 0, P.st));
    EpiArgs eb{};
    eb.kind = EpiKind::BUPDATE;
    eb.q = qs;
    eb.b = b;
    eb.part = P.part;
    eb.ctl = P.ctl;
    EpiArgs es{};
    es.kind = EpiKind::STORE;
    es.y = sv;
    es.part = P.part;
    es.ctl = P.ctl;
    const double alpha = 1.0 / (1.0 + pr->tau);
    // per-field rotating passes: the last pass of s = xi b finishes the
    // proximal step itself (it pairs both couplings' rows of its cells)
    EpiArgs ex{};
    ex.kind = EpiKind::ATTR_PROX;
    ex.a = a;
    ex.p_out = p_out;
    ex.prox.kappa = en->kappa;
    ex.prox.kappa_s = en->kappa_scalar;
    ex.alpha = (float)alpha;
    ex.part = P.part;
    ex.ctl = P.ctl;
    bool logd = logmode;   // the domain of the next application (as in run_step)
    bool pending = false, stopped = false;
    int nb = 0;
    int k_first = 1;   // first iteration left to the launch path
    if (!logd && P.respass && resident_pass2d_fits(P.g.n[1], P.g.n[2], P.W[1], P.W[2], 2, 0, P.prec)) {
        // the whole step in one launch of the resident pass kernel (paired tiles)
        bool launched = false;
        jko_status s = launch_respass(P, 2, P.W[1], P.W[2], 1, 2, qs, p_out, ex.prox, ex.alpha, K, ce, checks,
                                      pr->tol_l1, absorb, 0, &launched);
        if (s) return s;
        if (launched) {
            if ((s = resident_check(P))) return s;
            k_first = K + 1;
            if (absorb > 0.0) {
                // returned after the proximal half-step of the iteration whose
                // check asked for the log domain: convert and go on there
                Ctl c{};
                if ((s = read_ctl(P, &c))) return s;
                if (c.exit_iter > 0 && !c.done) {
                    HIP_TRY(launch_absorb(P.ctl, a, b, 2 * N, P.st));
                    HIP_TRY(launch_ctl_commit(P.ctl, c.exit_iter, P.st));
                    logd = true;
                    k_first = c.exit_iter + 1;
                }
            }
        }
    }
    for (int k = k_first; k <= K; ++k) {
        eb.check = (checks && k > 1 && (k - 1) % ce == 0) ? 1 : 0;
        jko_status s = apply_xi_in(logd, P, a, eb, &nb);
        if (s) return s;
        if (eb.check) HIP_TRY(launch_ctl_check(P.ctl, P.part, nb, k, pr->tol_l1, 0, absorb, 0, 0, P.st));
        if (eb.check && tolmode && rb().ev) {
            if (pending) {
                HIP_TRY(hipEventSynchronize(rb().ev));
                if (rb().host->done) stopped = true;
            }
            if (stopped) break;
            HIP_TRY(hipMemcpyAsync(rb().host, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, P.st));
            HIP_TRY(hipEventRecord(rb().ev, P.st));
            pending = true;
        } else if (eb.check && tolmode) {
            Ctl c{};
            if ((s = read_ctl(P, &c))) return s;
            if (c.done) break;
        }
        if (!logd && P.batch_pass) {
            if ((s = apply_xi(P, b, ex, &nb))) return s;
        } else {
            if ((s = apply_xi_in(logd, P, b, es, &nb))) return s;
            HIP_TRY(launch_attraction_prox(sv, a, p_out, en->kappa, en->kappa_scalar, alpha, N, P.ctl, P.st));
        }
        if (eb.check && absorb > 0.0 && !logd) {   // a switch decided at this iteration's check takes effect now
            HIP_TRY(launch_absorb(P.ctl, a, b, 2 * N, P.st));
            HIP_TRY(launch_ctl_commit(P.ctl, k, P.st));
            Ctl c{};
            if ((s = read_ctl(P, &c))) return s;
            if (c.logmode) logd = true;
        }
    }
    auto monitor = [&]() -> jko_status {
        EpiArgs em{};
        em.kind = EpiKind::MONITOR;
        em.q = qs;
        em.b = b;
        em.part = P.part;
        em.ctl = P.ctl;
        jko_status s = apply_xi_in(logd, P, a, em, &nb);
        if (s) return s;
        HIP_TRY(launch_ctl_check(P.ctl, P.part, nb, K + 1, -1.0, 0, 0.0, 0, 0, P.st));
        return JKO_OK;
    };
    Ctl c{};
    if (tolmode || want_stats) {
        HIP_TRY(hipStreamSynchronize(P.st));
        jko_status s = read_ctl(P, &c);
        if (s) return s;
        if (!c.done && (want_stats || st_dev)) {
            if ((s = monitor())) return s;
            if ((s = read_ctl(P, &c))) return s;
            c.done = 0;
        }
    } else if (st_dev) {
        jko_status s = monitor();   // queued without a read-back
        if (s) return s;
    }
    if (st_dev) {
        // the mass of the returned density (the control block holds the
        // coupling sums), then the record
        HIP_TRY(launch_input_check(p_out, nullptr, INFINITY, N, 0, P.part.err, 3 * 256, P.hostout, P.st));
        HIP_TRY(launch_stats_export(P.ctl, P.hostout, st_dev, K, tolmode, true, P.st));
    }
    if (st_out) {
        double mass = 0.0;
        jko_status s = mass_of(P, p_out, N, &mass);
        if (s) return s;
        jko_stats& o = *st_out;
        const bool bytol = tolmode && c.done && !c.nonfinite;
        o.iters = bytol ? c.stop_iter : K;
        o.absorptions = c.absorptions;
        o.stop_reason = bytol ? JKO_STOP_TOL : JKO_STOP_CAP;
        o.status = c.nonfinite ? JKO_ERR_NONFINITE : JKO_OK;
        o.marginal_l1 = c.err;
        o.mass = mass;
        o.max_abs_log_a = 0.0;
        o.max_abs_log_b = c.maxlogb;
    }
    if (c.nonfinite) return fail(JKO_ERR_NONFINITE, "non-finite value in the marginal monitor");
    return JKO_OK;
}

// jko_step (n_steps = 1, no checkpoints) and jko_flow for the attraction.
jko_status attraction_flow(const Geo& g, const jko_energy* en, const jko_params* pr, int n_steps, const float* p0,
                           float* pT, float* checkpoints, jko_stats* stats, double* stats_dev, void* ws,
                           size_t ws_bytes, hipStream_t st, bool flow) {
    if (g.d > 2) return fail(JKO_ERR_INVALID, "attraction: 1D and 2D grids only");
    for (int k = 0; k < g.d; ++k)
        if (g.n[k] < 3) return fail(JKO_ERR_INVALID, "attraction: every axis needs at least 3 cells");
    Plan P;
    jko_status s = carve(&P, stacked_of(g), flow ? OP_FLOW : OP_STEP, n_steps, ws, ws_bytes, pr->precision, st);
    if (s) return s;
    if ((s = readback_init())) return s;
    if ((s = build_factors(P, pr->gamma, pr->flags))) return s;
    // the stacking axis: gamma -> 0 rounds every off-diagonal entry to zero
    HIP_TRY(launch_build_factor(const_cast<float*>(P.K1[0]), const_cast<uint16_t*>(P.K1hi[0]),
                                const_cast<uint16_t*>(P.K1lo[0]), 2, 1e-30, P.st));
    P.ident[0] = true;
    // 2D grids: both couplings in one launch of the fused 2D kernel per
    // application (axis 0 of the stacked field is the identity)
    // the resident pass kernel (paired tiles) where the grid and bands suit it
    const bool respass2 = g.d == 2 && !(pr->flags & JKO_FLAG_NO_RESIDENT) &&
                          resident_pass2d_shape_fits(g.n[0], g.n[1], P.W[1], P.W[2], 2);
    if (g.d == 2 && !respass2 && !(pr->flags & JKO_FLAG_AXIS_PASSES))
        for (int tt : {16, 32})
            if (gibbs2d_fits(g.n[0], g.n[1], P.W[1], P.W[2], P.prec, tt) &&
                gibbs2d_blocks(g.n[0], g.n[1], tt) <= kFusedMaxBlocks) {
                P.tile = tt;
                P.batch2d = true;
                break;
            }
    // bands too wide for the fused kernel: each field rotates through its own
    // two passes (rows of a field a multiple of 4), so no pass runs over the
    // identity axis
    if (g.d == 2 && !P.batch2d && g.n[0] % 4 == 0 && g.n[1] % 4 == 0) P.batch_pass = true;
    P.respass = respass2;
    // capacity of the initial density, and a target of the same mass
    double h[3], hr[3];
    HIP_TRY(launch_input_check(p0, en->kappa, en->kappa_scalar, g.N, 1, P.part.err, 3 * 256, P.hostout, P.st));
    HIP_TRY(hipMemcpyAsync(rb().host, P.hostout, 3 * sizeof(double), hipMemcpyDeviceToHost, P.st));
    HIP_TRY(hipStreamSynchronize(P.st));
    memcpy(h, rb().host, sizeof h);
    HIP_TRY(launch_input_check(en->target, nullptr, INFINITY, g.N, 0, P.part.err, 3 * 256, P.hostout, P.st));
    HIP_TRY(hipMemcpyAsync(rb().host, P.hostout, 3 * sizeof(double), hipMemcpyDeviceToHost, P.st));
    HIP_TRY(hipStreamSynchronize(P.st));
    memcpy(hr, rb().host, sizeof hr);
    if (h[2] > 0.0 || hr[2] > 0.0) return fail(JKO_ERR_NONFINITE, "input density, capacity or target has negative/non-finite cells");
    if (h[1] < h[0] * (1.0 - 1e-6)) return fail(JKO_ERR_INFEASIBLE, "capacity sum %.9g < mass %.9g", h[1], h[0]);
    if (!(hr[0] > 0.0)) return fail(JKO_ERR_INVALID, "attraction: the target has no mass");
    const float* q = p0;
    double mq = h[0];
    jko_status worst = JKO_OK;
    for (int t = 0; t < n_steps; ++t) {
        if (checkpoints) HIP_TRY(launch_copy(checkpoints + (int64_t)t * g.N, q, g.N, P.st));
        float* out = (t == n_steps - 1) ? pT : P.F((t % 2 == 0) ? F_P0 : F_P1);
        if (t > 0 && (s = mass_of(P, q, g.N, &mq))) return s;
        s = run_attraction(P, pr, en, q, out, g.N, mq / hr[0], stats != nullptr, stats ? &stats[t] : nullptr,
                           t == n_steps - 1 ? stats_dev : nullptr);
        if (s == JKO_ERR_NONFINITE) {
            worst = s;
        } else if (s) {
            return s;
        }
        q = out;
    }
    if (worst) return fail(worst, "non-finite value in the marginal monitor");
    return JKO_OK;
}

// ------------------------------------------------------------ no-allocation step
//
// Workspace of jko_step_static: one file-scope device array, of which each
// GPU the library runs on holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel or copy (on the host it is
// only a stand-in for the symbol): it takes the device address once per
// device with hipGetSymbolAddress and uses that.
constexpr size_t kStaticWorkspaceBytes = JKO_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

jko_status scratch_of(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(JKO_ERR_HIP, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(JKO_ERR_HIP, "hipGetSymbolAddress returned NULL for the static workspace");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return JKO_OK;
}

// While alive, read-backs use the pageable buffer (no pinned allocation, no event).
struct NoAllocScope {
    NoAllocScope() { g_no_alloc = true; }
    ~NoAllocScope() {
        g_no_alloc = false;
        g_cur = &g_rb;
    }
};

jko_status common_checks(const jko_grid* grid, Geo* g) {
    if (!geo_of(grid, g)) return fail(JKO_ERR_INVALID, "grid: ndim must be 1..3 and 1 <= n[k] <= %d", kMaxN);
    return JKO_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

int32_t jko_version(void) { return 2; }

const char* jko_last_error(void) { return g_err.c_str(); }

const char* jko_status_string(int32_t s) {
    switch (s) {
        case JKO_OK: return "ok";
        case JKO_ERR_INVALID: return "invalid argument";
        case JKO_ERR_WORKSPACE: return "workspace missing or too small";
        case JKO_ERR_HIP: return "HIP runtime error";
        case JKO_ERR_NONFINITE: return "non-finite value";
        case JKO_ERR_INFEASIBLE: return "capacity cannot hold the mass";
        default: return "unknown status";
    }
}

size_t jko_workspace_bytes(const jko_grid* grid, const jko_params* params, int32_t op, int32_t n) {
    Geo g;
    if (!geo_of(grid, &g)) return 0;
    if (op < OP_GIBBS || op > OP_ATTR_FLOW) return 0;
    if (op == OP_ATTR_STEP || op == OP_ATTR_FLOW) {
        if (g.d > 2) return 0;
        return layout_of(stacked_of(g), op == OP_ATTR_STEP ? OP_STEP : OP_FLOW, n).total;
    }
    int64_t extra = n;
    if (op == OP_BACKWARD && params && n <= 0) extra = params->max_iters;
    return layout_of(g, op, extra).total;
}

jko_status jko_gibbs_apply(const jko_grid* grid, double gamma, int32_t precision, const float* x, float* y,
                           void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    Geo g;
    jko_status s = common_checks(grid, &g);
    if (s) return s;
    if (!(gamma > 0.0) || !isfinite(gamma)) return fail(JKO_ERR_INVALID, "gamma must be finite and > 0");
    if (precision != JKO_FP32 && precision != JKO_SPLIT_BF16) return fail(JKO_ERR_INVALID, "unknown precision");
    if (!x || !y) return fail(JKO_ERR_INVALID, "x and y must be non-NULL");
    if (x == y) return fail(JKO_ERR_INVALID, "x and y may not alias");
    Plan P;
    s = carve(&P, g, OP_GIBBS, 0, ws, ws_bytes, precision, static_cast<hipStream_t>(stream));
    if (s) return s;
    s = build_factors(P, gamma);
    if (s) return s;
    EpiArgs e{};
    e.kind = EpiKind::STORE;
    e.y = y;
    return apply_xi(P, x, e, nullptr);
}

jko_status jko_step(const jko_grid* grid, const jko_energy* energy, const jko_params* params, const float* p_in,
                    float* p_out, jko_stats* stats, double* stats_dev, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    Geo g;
    jko_status s = common_checks(grid, &g);
    if (s) return s;
    if ((s = check_params(params)) || (s = check_energy(energy))) return s;
    if (!p_in || !p_out) return fail(JKO_ERR_INVALID, "p_in and p_out must be non-NULL");
    if (p_in == p_out) return fail(JKO_ERR_INVALID, "p_in and p_out may not alias");
    if (stats_dev && (reinterpret_cast<uintptr_t>(stats_dev) % alignof(double) != 0 ||
                      static_cast<const void*>(stats_dev) == static_cast<const void*>(p_in) ||
                      static_cast<const void*>(stats_dev) == static_cast<const void*>(p_out)))
        return fail(JKO_ERR_INVALID, "stats_dev must be 8-byte aligned and may not alias p_in or p_out");
    if (energy->kind == JKO_F_ATTRACTION)
        return attraction_flow(g, energy, params, 1, p_in, p_out, nullptr, stats, stats_dev, ws, ws_bytes,
                               static_cast<hipStream_t>(stream), false);
    Plan P;
    s = carve(&P, g, OP_STEP, 0, ws, ws_bytes, params->precision, static_cast<hipStream_t>(stream));
    if (s) return s;
    if ((s = readback_init())) return s;
    const double sigma = params->tau / params->gamma;
    if ((s = build_factors(P, params->gamma, params->flags))) return s;
    if ((s = prepare_energy(P, energy, sigma))) return s;
    if ((s = input_check(P, energy, p_in))) return s;
    const ProxArgs px = prox_args(P, energy, sigma);
    return run_step(P, params, px, p_in, p_out, stats != nullptr, false, stats, stats_dev);
}

jko_status jko_step_static(const jko_grid* grid, const jko_energy* energy, const jko_params* params,
                           const float* p_in, float* p_out, jko_stats* stats, void* stream) {
    g_err.clear();
    Geo g;
    jko_status s = common_checks(grid, &g);
    if (s) return s;
    if ((s = check_params(params)) || (s = check_energy(energy))) return s;
    const bool attr = energy->kind == JKO_F_ATTRACTION;
    if (attr && g.d > 2) return fail(JKO_ERR_INVALID, "attraction: 1D and 2D grids only");
    const size_t need = layout_of(attr ? stacked_of(g) : g, OP_STEP, 0).total;
    if (need > kStaticWorkspaceBytes)
        return fail(JKO_ERR_WORKSPACE, "jko_step_static: this grid needs %zu bytes of workspace; the static one holds %zu",
                    need, kStaticWorkspaceBytes);
    void* ws = nullptr;
    if ((s = scratch_of(&ws))) return s;
    NoAllocScope scope;
    return jko_step(grid, energy, params, p_in, p_out, stats, nullptr, ws, kStaticWorkspaceBytes, stream);
}

jko_status jko_flow(const jko_grid* grid, const jko_energy* energy, const jko_params* params, int32_t n_steps,
                    const float* p0, float* pT, float* checkpoints, jko_stats* stats, void* ws, size_t ws_bytes,
                    void* stream) {
    g_err.clear();
    Geo g;
    jko_status s = common_checks(grid, &g);
    if (s) return s;
    if ((s = check_params(params)) || (s = check_energy(energy))) return s;
    if (n_steps < 1) return fail(JKO_ERR_INVALID, "n_steps must be >= 1");
    if (!p0 || !pT) return fail(JKO_ERR_INVALID, "p0 and pT must be non-NULL");
    if (p0 == pT) return fail(JKO_ERR_INVALID, "p0 and pT may not alias");
    if (energy->kind == JKO_F_ATTRACTION)
        return attraction_flow(g, energy, params, n_steps, p0, pT, checkpoints, stats, nullptr, ws, ws_bytes,
                               static_cast<hipStream_t>(stream), true);
    Plan P;
    s = carve(&P, g, OP_FLOW, n_steps, ws, ws_bytes, params->precision, static_cast<hipStream_t>(stream));
    if (s) return s;
    if ((s = readback_init())) return s;
    const double sigma = params->tau / params->gamma;
    if ((s = build_factors(P, params->gamma, params->flags))) return s;
    if ((s = prepare_energy(P, energy, sigma))) return s;
    if ((s = input_check(P, energy, p0))) return s;
    const ProxArgs px = prox_args(P, energy, sigma);
    const float* q = p0;
    jko_status worst = JKO_OK;
    for (int t = 0; t < n_steps; ++t) {
        if (checkpoints) HIP_TRY(launch_copy(checkpoints + (int64_t)t * g.N, q, g.N, P.st));
        float* out = (t == n_steps - 1) ? pT : P.F((t % 2 == 0) ? F_P0 : F_P1);
        s = run_step(P, params, px, q, out, stats != nullptr, false, stats ? &stats[t] : nullptr);
        if (s == JKO_ERR_NONFINITE) {
            worst = s;
        } else if (s) {
            return s;
        }
        q = out;
    }
    if (worst) return fail(worst, "non-finite value in the marginal monitor");
    return JKO_OK;
}

jko_status jko_time_iteration(const jko_grid* grid, const jko_energy* energy, const jko_params* params,
                              const float* p_in, int32_t reps, double* ms_per_launch, int32_t* n_launches,
                              void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    Geo g;
    jko_status s = common_checks(grid, &g);
    if (s) return s;
    if ((s = check_params(params)) || (s = check_energy(energy))) return s;
    if (!p_in || !ms_per_launch || reps < 1) return fail(JKO_ERR_INVALID, "bad timing arguments");
    if (energy->kind == JKO_F_ATTRACTION) return fail(JKO_ERR_INVALID, "attraction: no iteration timing");
    Plan P;
    s = carve(&P, g, OP_STEP, 0, ws, ws_bytes, params->precision, static_cast<hipStream_t>(stream));
    if (s) return s;
    const double sigma = params->tau / params->gamma;
    if ((s = build_factors(P, params->gamma, params->flags))) return s;
    if ((s = prepare_energy(P, energy, sigma))) return s;
    const ProxArgs px = prox_args(P, energy, sigma);
    float* a = P.F(F_A);
    float* b = P.F(F_B);
    HIP_TRY(launch_fill(a, 1.f, g.N, P.st));
    HIP_TRY(launch_fill(b, 1.f, g.N, P.st));
    HIP_TRY(launch_ctl_reset(P.ctl, 0, P.st));
    for (int i = 0; i < 2 * g.d; ++i) ms_per_launch[i] = 0.0;

    EpiArgs eb{};
    eb.kind = EpiKind::BUPDATE;
    eb.q = p_in;
    eb.b = b;
    eb.part = P.part;
    eb.ctl = P.ctl;
    EpiArgs ep{};
    ep.kind = EpiKind::PROX;
    ep.a = a;
    ep.p_out = nullptr;   // write_p = 0
    ep.prox = px;
    ep.part = P.part;
    ep.ctl = P.ctl;
    set_vec(eb);
    set_vec(ep);

    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto timed = [&](auto&& launch, double* out) -> jko_status {
        jko_status r = launch();   // warm-up
        if (r) return r;
        HIP_TRY(hipEventRecord(e0, P.st));
        for (int k = 0; k < reps; ++k)
            if ((r = launch())) return r;
        HIP_TRY(hipEventRecord(e1, P.st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        *out = (double)ms / reps;
        return JKO_OK;
    };
    int slot = 0;
    const bool respass = use_respass(P, params, px, false);
    if (respass || use_resident(P, params, px)) {
        // one launch of the resident kernel running max_iters iterations (the
        // resident pass kernel writes no density here)
        if ((s = readback_init())) return s;
        double tot = 0.0;
        for (int k = 0; k <= reps && !s; ++k) {   // k = 0: warm-up
            HIP_TRY(launch_fill(a, 1.f, g.N, P.st));
            HIP_TRY(launch_ctl_reset(P.ctl, 0, P.st));
            HIP_TRY(hipEventRecord(e0, P.st));
            bool launched = false;
            s = respass ? launch_respass(P, 1, P.W[0], P.W[1], 0, 1, p_in, nullptr, px, 0.f, params->max_iters, 1,
                                         false, 0.0, 0.0, 0, &launched)
                        : launch_resident(P, p_in, P.F(F_Z1), px, params->max_iters, 1, false, 0.0, 0.0, 0, false,
                                          &launched);
            if (s) break;
            if (!launched) {
                s = fail(JKO_ERR_HIP, "the cooperative grid of the resident kernel was refused");
                break;
            }
            HIP_TRY(hipEventRecord(e1, P.st));
            if ((s = resident_check(P))) break;
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (k > 0) tot += ms;
        }
        ms_per_launch[slot++] = tot / reps;
    } else if (P.fused2d) {
        // one launch per application
        s = timed([&]() { return apply_xi(P, a, eb, nullptr); }, &ms_per_launch[slot++]);
        if (!s) s = timed([&]() { return apply_xi(P, b, ep, nullptr); }, &ms_per_launch[slot++]);
    } else if (P.plane3d) {
        // per application: the plane pass, then the axis-0 pass with the epilogue
        for (int app = 0; app < 2 && !s; ++app) {
            const float* x = app == 0 ? a : b;
            s = timed([&]() -> jko_status {
                HIP_TRY(launch_plane3d(plane_of(P, x, P.ctl), P.prec, nullptr, P.st));
                return JKO_OK;
            }, &ms_per_launch[slot++]);
            if (s) break;
            const EpiArgs e = app == 0 ? eb : ep;
            s = timed([&]() -> jko_status {
                int nb = 0;
                HIP_TRY(launch_contract_slow(slow_of(P), P.prec, e, &nb, P.st));
                return JKO_OK;
            }, &ms_per_launch[slot++]);
        }
    } else {
        const PassList ps = passes_of(g);
        for (int app = 0; app < 2 && !s; ++app) {
            for (size_t i = 0; i < ps.size() && !s; ++i) {
                Pass pass = make_pass(ps[i]);
                pass.K1 = P.K1[ps[i].axis];
                pass.K1hi = P.K1hi[ps[i].axis];
                pass.K1lo = P.K1lo[ps[i].axis];
                pass.W = P.W[ps[i].axis];
                const bool last = (i + 1 == ps.size());
                pass.X = (i == 0) ? (app == 0 ? a : b) : P.F((i % 2 == 1) ? F_Z1 : F_Z2);
                EpiArgs e = app == 0 ? eb : ep;
                if (!last) {
                    e = EpiArgs{};
                    e.kind = EpiKind::STORE;
                    e.y = P.F(i % 2 == 0 ? F_Z1 : F_Z2);
                    e.ctl = P.ctl;
                    e.part = P.part;
                    set_vec(e);
                }
                s = timed([&]() -> jko_status {
                    int nb = 0;
                    HIP_TRY(launch_contract(pass, P.prec, e, &nb, P.st));
                    return JKO_OK;
                }, &ms_per_launch[slot++]);
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_launches) *n_launches = slot;
    return s;
}

jko_status jko_backward(const jko_grid* grid, const jko_energy* energy, const jko_params* params,
                        int32_t n_steps, const int32_t* iters_per_step, const float* checkpoints,
                        const float* dL_dpT, float* dL_dw, float* dL_dp0, void* ws, size_t ws_bytes,
                        void* stream) {
    g_err.clear();
    Geo g;
    jko_status s = common_checks(grid, &g);
    if (s) return s;
    if ((s = check_params(params)) || (s = check_energy(energy))) return s;
    if (energy->kind == JKO_F_CONGESTION_BINARY)
        return fail(JKO_ERR_INVALID, "binary congestion: the prox is piecewise constant, no gradient");
    if (energy->kind == JKO_F_ATTRACTION) return fail(JKO_ERR_INVALID, "attraction: no adjoint is built");
    if (n_steps < 1) return fail(JKO_ERR_INVALID, "n_steps must be >= 1");
    if (!iters_per_step || !checkpoints || !dL_dpT) return fail(JKO_ERR_INVALID, "missing input");
    if (dL_dw && energy->kind != JKO_F_CONGESTION && energy->kind != JKO_F_GEN_ENTROPY)
        return fail(JKO_ERR_INVALID, "dL/dw exists only for the congestion and generalised entropy energies");
    if (dL_dw && energy->kind == JKO_F_CONGESTION && !energy->w)
        return fail(JKO_ERR_INVALID, "dL/dw needs the potential w");
    if (dL_dw && energy->kind == JKO_F_GEN_ENTROPY && !energy->coef)
        return fail(JKO_ERR_INVALID, "dL/dcoef needs the weight field coef");
    int kmax = 0;
    for (int t = 0; t < n_steps; ++t) {
        if (iters_per_step[t] < 1) return fail(JKO_ERR_INVALID, "iters_per_step[%d] < 1", t);
        kmax = std::max(kmax, iters_per_step[t]);
    }
    Plan P;
    s = carve(&P, g, OP_BACKWARD, kmax, ws, ws_bytes, params->precision, static_cast<hipStream_t>(stream));
    if (s) return s;
    if ((s = readback_init())) return s;
    const double sigma = params->tau / params->gamma;
    if ((s = build_factors(P, params->gamma, params->flags))) return s;
    if ((s = prepare_energy(P, energy, sigma))) return s;
    const ProxArgs px = prox_args(P, energy, sigma);
    const int64_t N = g.N;
    float* pbar = P.F(F_PBAR);    // adjoint of the current step's output
    float* qbar = P.F(F_QBAR);    // adjoint of the current step's input
    float* wacc = P.F(F_WACC);
    HIP_TRY(launch_copy(pbar, dL_dpT, N, P.st));
    if (dL_dw) HIP_TRY(launch_fill(wacc, 0.f, N, P.st));
    jko_params fixed = *params;
    fixed.tol_l1 = 0.0;
    fixed.absorb_threshold = INFINITY;   // the adjoint differentiates the plain iteration
    for (int t = n_steps - 1; t >= 0; --t) {
        const float* q = checkpoints + (int64_t)t * N;
        const int K = iters_per_step[t];
        fixed.max_iters = K;
        // Recompute the step, keeping t_k and s_k.
        s = run_step(P, &fixed, px, q, P.F(F_TMP), false, true, nullptr);
        if (s) return s;
        HIP_TRY(launch_fill(qbar, 0.f, N, P.st));
        float* sbar = P.F(F_SBAR);
        float* tbar = P.F(F_TBAR);
        // k = K: the external pbar enters; afterwards each reverse step is two
        // Gibbs applications whose epilogues carry the pointwise reverse steps:
        //   bbar = xi sbar_k  -> tbar_k, qbar += ...          (reverse of b = q / t)
        //   abar = xi tbar_k  -> sbar_{k-1}, wbar += ...      (reverse of the prox at k - 1)
        // in one resident launch where the 2D tiles fit the chip, else one
        // launch per application.
        HIP_TRY(launch_adj_prox(P.hist(2 * (int64_t)(K - 1) + 1), pbar, nullptr, sbar, dL_dw ? wacc : nullptr, px,
                                sigma, N, P.st));
        bool resident = false;
        if (P.resident && !(params->flags & JKO_FLAG_NO_RESIDENT) &&
            resident_adj_fits(g.n[0], g.n[1], P.W[0], P.W[1], px.kind, P.prec, P.tile)) {
            ResidentAdj r{};
            r.B = Band2D{g.n[0], g.n[1], P.W[0], P.W[1], P.K1[0], P.K1[1], nullptr,
                         P.K1hi[0], P.K1lo[0], P.K1hi[1], P.K1lo[1], P.tile};
            r.q = q;
            r.hist = P.hist(0);
            r.hist_stride = (int64_t)(P.hist(1) - P.hist(0));
            r.sbar = sbar;
            r.tbar = tbar;
            r.qbar = qbar;
            r.wbar = dL_dw ? wacc : nullptr;
            r.prox = px;
            r.sigma = (float)sigma;
            r.sync = P.sync;
            r.K = K;
            r.spin_limit = kBarrierSpinLimit;
            r.split = P.prec == JKO_SPLIT_BF16 ? 1 : 0;
            EpiArgs al{};
            al.q = q;
            al.y = tbar;
            al.acc = qbar;
            al.hin = r.hist;
            al.prox = px;
            set_vec(al);
            r.vec_ok = al.vec_ok && aligned16(sbar) && aligned16(wacc) && (r.hist_stride % 4 == 0);
            HIP_TRY(launch_fill(reinterpret_cast<float*>(P.sync), 0.f,
                                resident_sync_words(gibbs2d_blocks(g.n[0], g.n[1], P.tile)),
                                P.st));
            const hipError_t e = launch_resident_adj(r, P.st);
            if (e == hipErrorCooperativeLaunchTooLarge) {
                (void)hipGetLastError();
            } else {
                HIP_TRY(e);
                resident = true;
                if ((s = resident_check(P))) return s;
            }
        }
        for (int k = K; k >= 1 && !resident; --k) {
            EpiArgs eb{};
            eb.kind = EpiKind::ADJ_B;
            eb.hin = P.hist(2 * (int64_t)(k - 1));
            eb.q = q;
            eb.y = tbar;
            eb.acc = qbar;
            if ((s = apply_xi(P, sbar, eb, nullptr))) return s;
            if (k > 1) {
                EpiArgs ea{};
                ea.kind = EpiKind::ADJ_PROX;
                ea.hin = P.hist(2 * (int64_t)(k - 2) + 1);
                ea.y = sbar;
                ea.acc = dL_dw ? wacc : nullptr;
                ea.prox = px;
                ea.sigma = (float)sigma;
                if ((s = apply_xi(P, tbar, ea, nullptr))) return s;
            }
        }
        HIP_TRY(launch_copy(pbar, qbar, N, P.st));
    }
    if (dL_dp0) HIP_TRY(launch_copy(dL_dp0, pbar, N, P.st));
    if (dL_dw) HIP_TRY(launch_copy(dL_dw, wacc, N, P.st));
    return JKO_OK;
}

}  // extern "C"

// ------------------------------------------------------------ heat kernel
// The heat-kernel Gibbs operator of Section 4.1 on a masked 2D grid, stored
// densely in the workspace (heat.hip), and the scaling iteration on it.

namespace {

constexpr int32_t kHeatMagic = 0x48454154;   // "HEAT"
constexpr int64_t kHeatMaxCells = 65536;         // the stored dense operator
constexpr int64_t kHeatMaxCellsSolve = 1 << 20;  // the per-product solves

struct HeatHdr {
    int32_t magic, n0, n1, L;
    int32_t solve, pad;      // 1: products by L solves (no stored operator)
    double gamma;
    int64_t nf;              // free cells (the operator's order)
};

struct HeatLayout {
    int64_t N = 0, ld = 0;
    bool solve = false;      // products by L solves on the grid, no stored operator
    size_t hdr = 0, A = 0, part = 0, scratch = 0, cidx = 0, gidx = 0, a = 0, b = 0, x = 0, p0 = 0, p1 = 0, g = 0,
           kf = 0, err = 0, out = 0;
    size_t total = 0;
};

// The dense stored operator up to 2^16 cells unless the domain asks for the
// per-product solves; the solves above.
bool heat_solve_mode(const jko_heat_domain* d) {
    return d->per_product != 0 || (int64_t)d->n0 * d->n1 > kHeatMaxCells;
}

HeatLayout heat_layout(int n0, int n1, bool solve) {
    HeatLayout H;
    H.N = (int64_t)n0 * n1;
    H.ld = heat_ld(H.N);
    H.solve = solve;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes); return at; };
    H.hdr = take(sizeof(HeatHdr));
    H.A = take(solve ? 0 : (size_t)heat_operator_floats(H.N) * sizeof(float));
    H.part = take(solve ? 0 : (size_t)heat_partial_floats(H.N) * sizeof(float));
    H.scratch = take((size_t)(solve ? 5 * H.N : heat_build_scratch(H.N)) * sizeof(double));
    H.cidx = take(H.N * sizeof(int32_t));
    H.gidx = take(H.N * sizeof(int32_t));
    H.a = take(H.ld * sizeof(float));
    H.b = take(H.ld * sizeof(float));
    H.x = take(H.ld * sizeof(float));
    H.p0 = take(H.N * sizeof(float));
    H.p1 = take(H.N * sizeof(float));
    H.g = take(H.N * sizeof(float));
    H.kf = take(H.N * sizeof(float));
    H.err = take(H.N * sizeof(double));
    H.out = take(8 * sizeof(double));
    H.total = o;
    return H;
}

jko_status heat_domain_check(const jko_heat_domain* d) {
    if (!d) return fail(JKO_ERR_INVALID, "heat domain is NULL");
    if (d->n0 < 1 || d->n1 < 1 || (int64_t)d->n0 * d->n1 > kHeatMaxCellsSolve)
        return fail(JKO_ERR_INVALID, "heat domain: need n0, n1 >= 1 and n0 * n1 <= %lld",
                    (long long)kHeatMaxCellsSolve);
    if (d->L < 1 || d->L > 1000) return fail(JKO_ERR_INVALID, "heat domain: L must be in 1..1000");
    return JKO_OK;
}

jko_status heat_ws_check(const HeatLayout& H, void* ws, size_t ws_bytes) {
    if (!ws) return fail(JKO_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", H.total);
    if (ws_bytes < H.total) return fail(JKO_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, H.total);
    if (((uintptr_t)ws) % 16 != 0) return fail(JKO_ERR_WORKSPACE, "workspace must be 16-byte aligned");
    return JKO_OK;
}

// Reads the operator's record back and checks that it was built for this
// domain (and, when gamma > 0, this gamma).  Synchronous.
jko_status heat_hdr_check(const jko_heat_domain* d, const char* ws, double gamma, hipStream_t st, int64_t* nf) {
    HIP_TRY(hipMemcpyAsync(rb().host, ws, sizeof(HeatHdr), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    HeatHdr h;
    memcpy(&h, rb().host, sizeof h);
    if (h.magic != kHeatMagic || h.n0 != d->n0 || h.n1 != d->n1 || h.L != d->L || h.solve != (heat_solve_mode(d) ? 1 : 0))
        return fail(JKO_ERR_INVALID, "heat: the workspace holds no operator of this domain (call jko_heat_build)");
    if (gamma > 0.0 && h.gamma != gamma)
        return fail(JKO_ERR_INVALID, "heat: operator built for gamma %.17g, params ask %.17g", h.gamma, gamma);
    *nf = h.nf;
    return JKO_OK;
}

// The gamma the workspace's operator was built for (synchronous).
jko_status heat_hdr_gamma(const char* ws, hipStream_t st, double* gamma) {
    HIP_TRY(hipMemcpyAsync(rb().host, ws, sizeof(HeatHdr), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    HeatHdr h;
    memcpy(&h, rb().host, sizeof h);
    *gamma = h.gamma;
    return JKO_OK;
}

jko_status heat_sums(const double* err, int64_t ne, const float* p, int64_t np, double* dev_out, hipStream_t st,
                     double h[3]) {
    HIP_TRY(launch_heat_sums(err, ne, p, np, dev_out, st));
    HIP_TRY(hipMemcpyAsync(rb().host, dev_out, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    memcpy(h, rb().host, 3 * sizeof(double));
    return JKO_OK;
}

// One product of the iteration with the epilogue `ek`: a pass over the stored
// operator, or the L solves of the per-product form (hs.X != NULL).
jko_status heat_product(int ek, const HeatGemv& g, const HeatSolve& hs, hipStream_t st) {
    if (hs.X) HIP_TRY(launch_heat_solve(ek, g, hs, st));
    else HIP_TRY(launch_heat_gemv(ek, g, st));
    return JKO_OK;
}

// The per-product solves' context of a domain (X = NULL for the stored operator).
HeatSolve heat_solve_of(const HeatLayout& H, const jko_heat_domain* d, char* base, double gamma) {
    HeatSolve hs{};
    if (!H.solve) return hs;
    double* sc = reinterpret_cast<double*>(base + H.scratch);
    hs.mask = d->mask;
    hs.cidx = reinterpret_cast<const int32_t*>(base + H.cidx);
    hs.n0 = d->n0;
    hs.n1 = d->n1;
    hs.L = d->L;
    hs.gamma = gamma;
    hs.X = sc;
    hs.R = sc + H.N;
    hs.R1 = sc + 2 * H.N;
    hs.D0 = sc + 3 * H.N;
    hs.D1 = sc + 4 * H.N;
    return hs;
}

// One step q -> p_out by the reduced iteration (t = xi~ a; b = q / t;
// s = xi~ b; p = Prox(s); a = p / s) with the stop test of the band path:
// at iteration k > 1 with (k - 1) % check_every == 0 and tol > 0 the
// violation ||b t - q||_1 of iteration k - 1 is summed, and the step returns
// that iterate when it is at most tol.
jko_status heat_step(const HeatLayout& H, char* base, int64_t nf, const HeatSolve& hs, const jko_params* pr,
                     const ProxArgs& px, int kind, const float* q, float* p_out, jko_stats* st_out,
                     hipStream_t st) {
    const float* A = reinterpret_cast<const float*>(base + H.A);
    float* a = reinterpret_cast<float*>(base + H.a);
    float* b = reinterpret_cast<float*>(base + H.b);
    double* err = reinterpret_cast<double*>(base + H.err);
    double* dout = reinterpret_cast<double*>(base + H.out);
    const int64_t ldf = heat_ld(nf);
    HIP_TRY(launch_heat_fill(a, 1.f, nf, ldf, st));
    HIP_TRY(launch_heat_fill(b, 0.f, nf, ldf, st));
    HIP_TRY(launch_heat_fill(p_out, 0.f, 0, H.N, st));   // obstacles: never written by the passes
    HeatGemv gt{};
    gt.A = A;
    gt.part = reinterpret_cast<float*>(base + H.part);
    gt.nT = (int32_t)heat_ntiles(nf);
    gt.ld = ldf;
    gt.N = nf;
    gt.gidx = reinterpret_cast<const int32_t*>(base + H.gidx);
    gt.x = a;
    gt.q = q;
    gt.b = b;
    gt.errrow = err;
    HeatGemv gs = gt;
    gs.x = b;
    gs.a = a;
    gs.p = p_out;
    gs.px = px;
    const bool tolmode = pr->tol_l1 > 0.0;
    int iters = pr->max_iters;
    bool bytol = false;
    double h[3] = {0.0, 0.0, 0.0};
    for (int k = 1; k <= pr->max_iters; ++k) {
        gt.check = tolmode && k > 1 && (k - 1) % pr->check_every == 0;
        jko_status s = heat_product(HEAT_EK_BUPDATE, gt, hs, st);
        if (s) return s;
        if (gt.check) {
            s = heat_sums(err, nf, nullptr, 0, dout, st, h);
            if (s) return s;
            if (h[2] > 0.0) break;
            if (h[0] <= pr->tol_l1) {
                iters = k - 1;
                bytol = true;
                break;
            }
        }
        if ((s = heat_product(HEAT_EK_PROX + kind, gs, hs, st))) return s;
    }
    if (!bytol && h[2] == 0.0) {
        jko_status s = heat_product(HEAT_EK_MONITOR, gt, hs, st);
        if (s) return s;
    }
    jko_status s = heat_sums(err, nf, p_out, H.N, dout, st, h);
    if (s) return s;
    const bool bad = h[2] > 0.0 || !isfinite(h[0]) || !isfinite(h[1]);
    if (st_out) {
        jko_stats& o = *st_out;
        o.iters = iters;
        o.absorptions = 0;
        o.stop_reason = bytol ? JKO_STOP_TOL : JKO_STOP_CAP;
        o.status = bad ? JKO_ERR_NONFINITE : JKO_OK;
        o.marginal_l1 = bad ? NAN : h[0];
        o.mass = h[1];
        o.max_abs_log_a = 0.0;
        o.max_abs_log_b = 0.0;
    }
    if (bad) return fail(JKO_ERR_NONFINITE, "non-finite value in the marginal monitor");
    return JKO_OK;
}

}  // namespace

extern "C" {

size_t jko_heat_workspace_bytes(const jko_heat_domain* domain) {
    if (!domain || domain->n0 < 1 || domain->n1 < 1 || (int64_t)domain->n0 * domain->n1 > kHeatMaxCellsSolve)
        return 0;
    return heat_layout(domain->n0, domain->n1, heat_solve_mode(domain)).total;
}

jko_status jko_heat_build(const jko_heat_domain* domain, double gamma, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    jko_status s = heat_domain_check(domain);
    if (s) return s;
    if (!(gamma > 0.0) || !isfinite(gamma)) return fail(JKO_ERR_INVALID, "gamma must be finite and > 0");
    const HeatLayout H = heat_layout(domain->n0, domain->n1, heat_solve_mode(domain));
    if ((s = heat_ws_check(H, ws, ws_bytes))) return s;
    if ((s = readback_init())) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    int32_t* cidx = reinterpret_cast<int32_t*>(base + H.cidx);
    int32_t* gidx = reinterpret_cast<int32_t*>(base + H.gidx);
    int64_t* dcount = reinterpret_cast<int64_t*>(base + H.out);
    HIP_TRY(launch_heat_compact(domain->mask, H.N, cidx, gidx, dcount, st));
    HIP_TRY(hipMemcpyAsync(rb().host, dcount, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int64_t nf = 0;
    memcpy(&nf, rb().host, sizeof nf);
    if (!H.solve)
        HIP_TRY(heat_build_operator(domain->mask, domain->n0, domain->n1, gamma, domain->L, cidx, gidx, nf,
                                    reinterpret_cast<float*>(base + H.A), reinterpret_cast<double*>(base + H.scratch),
                                    st));
    HeatHdr h{kHeatMagic, domain->n0, domain->n1, domain->L, H.solve ? 1 : 0, 0, gamma, nf};
    memcpy(rb().host, &h, sizeof h);
    HIP_TRY(hipMemcpyAsync(base + H.hdr, rb().host, sizeof h, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return JKO_OK;
}

jko_status jko_heat_apply(const jko_heat_domain* domain, const float* x, float* y, void* ws, size_t ws_bytes,
                          void* stream) {
    g_err.clear();
    jko_status s = heat_domain_check(domain);
    if (s) return s;
    if (!x || !y) return fail(JKO_ERR_INVALID, "x and y must be non-NULL");
    if (x == y) return fail(JKO_ERR_INVALID, "x and y may not alias");
    const HeatLayout H = heat_layout(domain->n0, domain->n1, heat_solve_mode(domain));
    if ((s = heat_ws_check(H, ws, ws_bytes))) return s;
    if ((s = readback_init())) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    int64_t nf = 0;
    if ((s = heat_hdr_check(domain, base + H.hdr, 0.0, st, &nf))) return s;
    double gamma = 0.0;   // the gamma the workspace was built for
    if ((s = heat_hdr_gamma(base + H.hdr, st, &gamma))) return s;
    const int32_t* gidx = reinterpret_cast<const int32_t*>(base + H.gidx);
    float* xp = reinterpret_cast<float*>(base + H.x);
    HIP_TRY(launch_heat_gather(xp, x, gidx, nf, heat_ld(nf), st));
    HIP_TRY(launch_heat_fill(y, 0.f, 0, H.N, st));        // obstacles
    HeatGemv g{};
    g.A = reinterpret_cast<const float*>(base + H.A);
    g.part = reinterpret_cast<float*>(base + H.part);
    g.nT = (int32_t)heat_ntiles(nf);
    g.ld = heat_ld(nf);
    g.N = nf;
    g.gidx = gidx;
    g.x = xp;
    g.y = y;
    return heat_product(HEAT_EK_STORE, g, heat_solve_of(H, domain, base, gamma), st);
}

jko_status jko_heat_flow(const jko_heat_domain* domain, const jko_energy* energy, const jko_params* params,
                         int32_t n_steps, const float* p0, float* pT, jko_stats* stats, void* ws, size_t ws_bytes,
                         void* stream) {
    g_err.clear();
    jko_status s = heat_domain_check(domain);
    if (s) return s;
    if ((s = check_params(params)) || (s = check_energy(energy))) return s;
    if (energy->kind == JKO_F_ATTRACTION) return fail(JKO_ERR_INVALID, "heat: the attraction is not supported");
    if (params->precision != JKO_FP32) return fail(JKO_ERR_INVALID, "heat: the stored operator is float32 only");
    if (!(isnan(params->absorb_threshold) || (isinf(params->absorb_threshold) && params->absorb_threshold > 0)))
        return fail(JKO_ERR_INVALID, "heat: no log domain (absorb_threshold must be +inf or NaN)");
    if (n_steps < 1) return fail(JKO_ERR_INVALID, "n_steps must be >= 1");
    if (!p0 || !pT) return fail(JKO_ERR_INVALID, "p0 and pT must be non-NULL");
    if (p0 == pT) return fail(JKO_ERR_INVALID, "p0 and pT may not alias");
    const HeatLayout H = heat_layout(domain->n0, domain->n1, heat_solve_mode(domain));
    if ((s = heat_ws_check(H, ws, ws_bytes))) return s;
    if ((s = readback_init())) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    int64_t nf = 0;
    if ((s = heat_hdr_check(domain, base + H.hdr, params->gamma, st, &nf))) return s;
    const double sigma = params->tau / params->gamma;
    float* fg = reinterpret_cast<float*>(base + H.g);
    float* fkf = reinterpret_cast<float*>(base + H.kf);
    const bool need = (is_congestion(energy) && energy->w) ||
                      ((energy->kind == JKO_F_ENTROPY || energy->kind == JKO_F_POROUS) && energy->coef) ||
                      (energy->kind == JKO_F_GEN_ENTROPY && (energy->coef || energy->m_field));
    if (need) HIP_TRY(launch_prepare_energy(energy, sigma, H.N, fg, fkf, st));
    double* dout = reinterpret_cast<double*>(base + H.out);
    HIP_TRY(launch_heat_input(p0, domain->mask, is_congestion(energy) ? energy->kappa : nullptr,
                              is_congestion(energy) ? energy->kappa_scalar : INFINITY, H.N, dout, st));
    double h[3];
    HIP_TRY(hipMemcpyAsync(rb().host, dout, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    memcpy(h, rb().host, sizeof h);
    if (h[2] > 0.0)
        return fail(JKO_ERR_NONFINITE, "heat: %g cells of p0 are negative, non-finite or on an obstacle, "
                    "or have a negative capacity", h[2]);
    if (is_congestion(energy) && h[1] < h[0] * (1.0 - 1e-6))
        return fail(JKO_ERR_INFEASIBLE, "capacity sum %.9g < mass %.9g", h[1], h[0]);
    const ProxArgs px = prox_args_fields(energy, sigma, fg, fkf);
    const float* q = p0;
    jko_status worst = JKO_OK;
    for (int t = 0; t < n_steps; ++t) {
        float* out = (t == n_steps - 1) ? pT : reinterpret_cast<float*>(base + ((t % 2 == 0) ? H.p0 : H.p1));
        s = heat_step(H, base, nf, heat_solve_of(H, domain, base, params->gamma), params, px, energy->kind, q, out,
                      stats ? &stats[t] : nullptr, st);
        if (s == JKO_ERR_NONFINITE) worst = s;
        else if (s) return s;
        q = out;
    }
    if (worst) return fail(worst, "non-finite value in the marginal monitor");
    return JKO_OK;
}

}  // extern "C"
