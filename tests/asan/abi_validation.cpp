// Host driver for the AddressSanitizer build of the library's host code.
//
// Every call below is refused by the argument checks of the C ABI before any
// HIP call or kernel launch, so the program needs no GPU: it exercises the
// validation, workspace sizing, error-message and status-string paths of the
// host driver under AddressSanitizer (heap, stack and global bounds, use after
// free), together with the thread-local error message.  The device pointers
// passed are placeholders that the refused calls never dereference.
// Prints "ok <checks>" and returns 0 when every call returned what it should.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <thread>
#include <vector>

#include "jko.h"

namespace {

int g_checks = 0;
int g_failed = 0;

void expect_status(int line, jko_status got, jko_status want, const char* msg_part) {
    ++g_checks;
    const char* msg = jko_last_error();
    if (got != want) {
        fprintf(stderr, "line %d: status %d, expected %d (%s)\n", line, (int)got, (int)want, msg);
        ++g_failed;
        return;
    }
    if (msg_part && !strstr(msg, msg_part)) {
        fprintf(stderr, "line %d: message \"%s\" lacks \"%s\"\n", line, msg, msg_part);
        ++g_failed;
    }
}

void expect_true(int line, bool ok, const char* what) {
    ++g_checks;
    if (!ok) {
        fprintf(stderr, "line %d: %s\n", line, what);
        ++g_failed;
    }
}

#define EXPECT(call, want, part) expect_status(__LINE__, (call), (want), (part))
#define CHECK(cond) expect_true(__LINE__, (cond), #cond)

// placeholders for device buffers: never dereferenced by a refused call
float* dev(uintptr_t k) { return reinterpret_cast<float*>(uintptr_t(0x7000000000) + k * 0x100000); }

jko_grid grid2(int n0, int n1) {
    jko_grid g{};
    g.ndim = 2;
    g.n[0] = n0;
    g.n[1] = n1;
    return g;
}

jko_params params_ok() {
    jko_params p{};
    p.gamma = 2e-4;
    p.tau = 2e-3;
    p.tol_l1 = 0.0;
    p.max_iters = 10;
    p.check_every = 5;
    p.precision = JKO_FP32;
    p.flags = 0;
    p.absorb_threshold = 50.0;
    return p;
}

jko_energy congestion() {
    jko_energy e{};
    e.kind = JKO_F_CONGESTION;
    e.kappa_scalar = 1.0f;
    return e;
}

void workspace_sizes() {
    jko_params p = params_ok();
    jko_grid g = grid2(256, 256);
    const size_t step = jko_workspace_bytes(&g, &p, JKO_OP_STEP, 0);
    CHECK(step > 256u * 256u * sizeof(float));
    CHECK(jko_workspace_bytes(&g, &p, JKO_OP_FLOW, 10) >= step);
    CHECK(jko_workspace_bytes(&g, &p, JKO_OP_BACKWARD, 300) > jko_workspace_bytes(&g, &p, JKO_OP_BACKWARD, 10));
    CHECK(jko_workspace_bytes(&g, &p, JKO_OP_ATTRACTION_STEP, 0) > step);
    CHECK(jko_workspace_bytes(&g, &p, -1, 0) == 0);
    CHECK(jko_workspace_bytes(&g, &p, 6, 0) == 0);
    CHECK(jko_workspace_bytes(nullptr, &p, JKO_OP_STEP, 0) == 0);
    jko_grid bad = grid2(0, 8);
    CHECK(jko_workspace_bytes(&bad, &p, JKO_OP_STEP, 0) == 0);
    bad = grid2(8, 1025);
    CHECK(jko_workspace_bytes(&bad, &p, JKO_OP_STEP, 0) == 0);
    bad.ndim = 4;
    CHECK(jko_workspace_bytes(&bad, &p, JKO_OP_STEP, 0) == 0);
    jko_grid g3{3, {64, 64, 64}};
    CHECK(jko_workspace_bytes(&g3, &p, JKO_OP_STEP, 0) > 0);
    CHECK(jko_workspace_bytes(&g3, &p, JKO_OP_ATTRACTION_STEP, 0) == 0);   // attraction: 1D and 2D only
    jko_grid g1{1, {1024, 0, 0}};
    CHECK(jko_workspace_bytes(&g1, &p, JKO_OP_GIBBS, 0) > 0);
    // the largest grids: sizes must not overflow
    jko_grid gmax{3, {1024, 1024, 1024}};
    CHECK(jko_workspace_bytes(&gmax, &p, JKO_OP_STEP, 0) > (size_t)1024 * 1024 * 1024 * sizeof(float));
}

void step_arguments() {
    jko_grid g = grid2(64, 64);
    jko_params p = params_ok();
    jko_energy e = congestion();
    const size_t ws_need = jko_workspace_bytes(&g, &p, JKO_OP_STEP, 0);
    void* ws = dev(100);
    EXPECT(jko_step(nullptr, &e, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID, nullptr);
    jko_grid bad = grid2(64, 2048);
    EXPECT(jko_step(&bad, &e, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID, nullptr);
    EXPECT(jko_step(&g, nullptr, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
           "energy is NULL");
    EXPECT(jko_step(&g, &e, nullptr, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
           "params is NULL");
    for (double gamma : {0.0, -1.0, (double)NAN, (double)INFINITY}) {
        jko_params q = params_ok();
        q.gamma = gamma;
        EXPECT(jko_step(&g, &e, &q, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID, "gamma");
    }
    {
        jko_params q = params_ok();
        q.tau = 0.0;
        EXPECT(jko_step(&g, &e, &q, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID, "tau");
        q = params_ok();
        q.max_iters = 0;
        EXPECT(jko_step(&g, &e, &q, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "max_iters");
        q = params_ok();
        q.check_every = 0;
        EXPECT(jko_step(&g, &e, &q, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "check_every");
        q = params_ok();
        q.precision = 7;
        EXPECT(jko_step(&g, &e, &q, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "unknown precision 7");
        q = params_ok();
        q.tol_l1 = NAN;
        EXPECT(jko_step(&g, &e, &q, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID, "NaN");
        q = params_ok();
        q.flags = 64;
        EXPECT(jko_step(&g, &e, &q, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "unknown flags 0x40");
    }
    {
        jko_energy f = e;
        f.kind = 99;
        EXPECT(jko_step(&g, &f, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "unknown energy kind 99");
        f = e;
        f.kappa_scalar = -1.f;
        EXPECT(jko_step(&g, &f, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "kappa_scalar");
        f = e;
        f.kind = JKO_F_CONGESTION_BINARY;
        f.kappa_scalar = INFINITY;
        EXPECT(jko_step(&g, &f, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "binary congestion");
        f = jko_energy{};
        f.kind = JKO_F_POROUS;
        f.m = 1.f;
        f.density_scale = 1.f;
        EXPECT(jko_step(&g, &f, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "porous exponent");
        f.m = 2.f;
        f.newton_steps = 33;
        EXPECT(jko_step(&g, &f, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "newton_steps");
        f = jko_energy{};
        f.kind = JKO_F_GEN_ENTROPY;
        f.m = 0.5f;
        f.density_scale = 1.f;
        EXPECT(jko_step(&g, &f, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "exponent m");
        f = jko_energy{};
        f.kind = JKO_F_ATTRACTION;
        EXPECT(jko_step(&g, &f, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "target is NULL");
        f.target = dev(3);
        jko_grid g3{3, {32, 32, 32}};
        EXPECT(jko_step(&g3, &f, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "1D and 2D");
        jko_grid thin = grid2(2, 64);
        EXPECT(jko_step(&thin, &f, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID,
               "at least 3 cells");
        // the attraction needs its own, larger workspace
        EXPECT(jko_step(&g, &f, &p, dev(1), dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_WORKSPACE,
               "needed");
    }
    EXPECT(jko_step(&g, &e, &p, nullptr, dev(2), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID, "non-NULL");
    EXPECT(jko_step(&g, &e, &p, dev(1), dev(1), nullptr, nullptr, ws, ws_need, nullptr), JKO_ERR_INVALID, "alias");
    double* sd = reinterpret_cast<double*>(dev(4));
    EXPECT(jko_step(&g, &e, &p, dev(1), dev(2), nullptr, reinterpret_cast<double*>(dev(2)), ws, ws_need, nullptr),
           JKO_ERR_INVALID, "stats_dev");
    EXPECT(jko_step(&g, &e, &p, dev(1), dev(2), nullptr, reinterpret_cast<double*>(reinterpret_cast<char*>(sd) + 4), ws,
                    ws_need, nullptr),
           JKO_ERR_INVALID, "stats_dev");
    EXPECT(jko_step(&g, &e, &p, dev(1), dev(2), nullptr, sd, nullptr, ws_need, nullptr), JKO_ERR_WORKSPACE, "NULL");
    EXPECT(jko_step(&g, &e, &p, dev(1), dev(2), nullptr, sd, ws, ws_need - 1, nullptr), JKO_ERR_WORKSPACE, "needed");
    EXPECT(jko_step(&g, &e, &p, dev(1), dev(2), nullptr, sd, reinterpret_cast<char*>(ws) + 8, ws_need, nullptr),
           JKO_ERR_WORKSPACE, "aligned");
    // the static workspace holds no 1024 x 1024 step
    jko_grid big = grid2(1024, 1024);
    EXPECT(jko_step_static(&big, &e, &p, dev(1), dev(2), nullptr, nullptr), JKO_ERR_WORKSPACE, "static");
}

void flow_and_backward_arguments() {
    jko_grid g = grid2(64, 64);
    jko_params p = params_ok();
    jko_energy e = congestion();
    void* ws = dev(100);
    const size_t flow_need = jko_workspace_bytes(&g, &p, JKO_OP_FLOW, 4);
    EXPECT(jko_flow(&g, &e, &p, 0, dev(1), dev(2), nullptr, nullptr, ws, flow_need, nullptr), JKO_ERR_INVALID,
           "n_steps");
    EXPECT(jko_flow(&g, &e, &p, 4, dev(1), dev(1), nullptr, nullptr, ws, flow_need, nullptr), JKO_ERR_INVALID, "alias");
    EXPECT(jko_flow(&g, &e, &p, 4, dev(1), dev(2), nullptr, nullptr, ws, flow_need - 16, nullptr), JKO_ERR_WORKSPACE,
           "needed");

    const int n_steps = 3;
    std::vector<int32_t> iters(n_steps, 300);   // exactly n_steps entries: the checks read no further
    const size_t bw_need = jko_workspace_bytes(&g, &p, JKO_OP_BACKWARD, 300);
    jko_energy bin = e;
    bin.kind = JKO_F_CONGESTION_BINARY;
    EXPECT(jko_backward(&g, &bin, &p, n_steps, iters.data(), dev(1), dev(2), nullptr, dev(3), ws, bw_need, nullptr),
           JKO_ERR_INVALID, "no gradient");
    jko_energy att{};
    att.kind = JKO_F_ATTRACTION;
    att.target = dev(5);
    EXPECT(jko_backward(&g, &att, &p, n_steps, iters.data(), dev(1), dev(2), nullptr, dev(3), ws, bw_need, nullptr),
           JKO_ERR_INVALID, "no adjoint");
    EXPECT(jko_backward(&g, &e, &p, 0, iters.data(), dev(1), dev(2), nullptr, dev(3), ws, bw_need, nullptr),
           JKO_ERR_INVALID, "n_steps");
    EXPECT(jko_backward(&g, &e, &p, n_steps, nullptr, dev(1), dev(2), nullptr, dev(3), ws, bw_need, nullptr),
           JKO_ERR_INVALID, "missing input");
    iters[n_steps - 1] = 0;
    EXPECT(jko_backward(&g, &e, &p, n_steps, iters.data(), dev(1), dev(2), nullptr, dev(3), ws, bw_need, nullptr),
           JKO_ERR_INVALID, "iters_per_step[2]");
    iters[n_steps - 1] = 300;
    jko_energy ent{};
    ent.kind = JKO_F_ENTROPY;
    ent.coef_scalar = 1.f;
    EXPECT(jko_backward(&g, &ent, &p, n_steps, iters.data(), dev(1), dev(2), dev(4), nullptr, ws, bw_need, nullptr),
           JKO_ERR_INVALID, "dL/dw exists only");
    EXPECT(jko_backward(&g, &e, &p, n_steps, iters.data(), dev(1), dev(2), dev(4), nullptr, ws, bw_need, nullptr),
           JKO_ERR_INVALID, "potential w");
    // a longest step beyond the workspace's history
    iters[1] = 301;
    EXPECT(jko_backward(&g, &e, &p, n_steps, iters.data(), dev(1), dev(2), nullptr, dev(3), ws, bw_need, nullptr),
           JKO_ERR_WORKSPACE, "needed");

    EXPECT(jko_gibbs_apply(&g, 0.0, JKO_FP32, dev(1), dev(2), ws, 1 << 30, nullptr), JKO_ERR_INVALID, "gamma");
    EXPECT(jko_gibbs_apply(&g, 1e-3, 3, dev(1), dev(2), ws, 1 << 30, nullptr), JKO_ERR_INVALID, "precision");
    EXPECT(jko_gibbs_apply(&g, 1e-3, JKO_FP32, dev(1), dev(1), ws, 1 << 30, nullptr), JKO_ERR_INVALID, "alias");
    EXPECT(jko_gibbs_apply(&g, 1e-3, JKO_FP32, dev(1), dev(2), ws, 64, nullptr), JKO_ERR_WORKSPACE, "needed");

    double ms[6];
    int32_t nl = 0;
    EXPECT(jko_time_iteration(&g, &e, &p, dev(1), 0, ms, &nl, ws, 1 << 30, nullptr), JKO_ERR_INVALID, "timing");
    EXPECT(jko_time_iteration(&g, &att, &p, dev(1), 3, ms, &nl, ws, 1 << 30, nullptr), JKO_ERR_INVALID, "attraction");
}

void heat_arguments() {
    jko_heat_domain d{};
    d.n0 = 100;
    d.n1 = 100;
    d.mask = nullptr;
    d.L = 10;
    const size_t dense = jko_heat_workspace_bytes(&d);
    CHECK(dense > (size_t)100 * 100 * 100 * 100 / 2 * sizeof(float) / 2);
    d.per_product = 1;
    const size_t solve = jko_heat_workspace_bytes(&d);
    CHECK(solve > 0 && solve < dense);
    d.per_product = 0;
    jko_heat_domain big = d;
    big.n0 = 1024;
    big.n1 = 1024;
    CHECK(jko_heat_workspace_bytes(&big) > 0);   // solves above 2^16 cells
    big.n0 = 1025;
    CHECK(jko_heat_workspace_bytes(&big) == 0);
    CHECK(jko_heat_workspace_bytes(nullptr) == 0);
    void* ws = dev(200);
    jko_heat_domain badL = d;
    badL.L = 0;
    EXPECT(jko_heat_build(&badL, 1e-3, ws, dense, nullptr), JKO_ERR_INVALID, "L must be");
    badL.L = 1001;
    EXPECT(jko_heat_build(&badL, 1e-3, ws, dense, nullptr), JKO_ERR_INVALID, "L must be");
    EXPECT(jko_heat_build(&d, -1.0, ws, dense, nullptr), JKO_ERR_INVALID, "gamma");
    EXPECT(jko_heat_build(&d, 1e-3, ws, dense - 1, nullptr), JKO_ERR_WORKSPACE, "needed");
    EXPECT(jko_heat_build(nullptr, 1e-3, ws, dense, nullptr), JKO_ERR_INVALID, "NULL");
    EXPECT(jko_heat_apply(&d, dev(1), dev(1), ws, dense, nullptr), JKO_ERR_INVALID, "alias");
    EXPECT(jko_heat_apply(&d, dev(1), dev(2), nullptr, dense, nullptr), JKO_ERR_WORKSPACE, "NULL");
    jko_params p = params_ok();
    p.gamma = 1e-3;
    p.tau = 2e-2;
    jko_energy e = congestion();
    EXPECT(jko_heat_flow(&d, &e, &p, 3, dev(1), dev(2), nullptr, ws, dense, nullptr), JKO_ERR_INVALID, "log domain");
    p.absorb_threshold = INFINITY;
    jko_params ps = p;
    ps.precision = JKO_SPLIT_BF16;
    EXPECT(jko_heat_flow(&d, &e, &ps, 3, dev(1), dev(2), nullptr, ws, dense, nullptr), JKO_ERR_INVALID, "float32");
    jko_energy att{};
    att.kind = JKO_F_ATTRACTION;
    att.target = dev(5);
    EXPECT(jko_heat_flow(&d, &att, &p, 3, dev(1), dev(2), nullptr, ws, dense, nullptr), JKO_ERR_INVALID, "attraction");
    EXPECT(jko_heat_flow(&d, &e, &p, 0, dev(1), dev(2), nullptr, ws, dense, nullptr), JKO_ERR_INVALID, "n_steps");
    EXPECT(jko_heat_flow(&d, &e, &p, 3, dev(1), dev(2), nullptr, ws, 1024, nullptr), JKO_ERR_WORKSPACE, "needed");
}

void strings_and_threads() {
    for (int s = 0; s >= -5; --s) CHECK(strlen(jko_status_string(s)) > 0 && strcmp(jko_status_string(s), "unknown status") != 0);
    CHECK(strcmp(jko_status_string(-99), "unknown status") == 0);
    CHECK(jko_version() == 2);
    // the last error is per thread: a failure on another thread leaves this one's message alone
    jko_grid g = grid2(8, 8);
    jko_params p = params_ok();
    jko_energy e = congestion();
    EXPECT(jko_step(&g, &e, &p, dev(1), dev(1), nullptr, nullptr, dev(100), 1 << 30, nullptr), JKO_ERR_INVALID, "alias");
    std::string other;
    std::thread t([&] {
        jko_params q = params_ok();
        q.max_iters = -3;
        jko_step(&g, &e, &q, dev(1), dev(2), nullptr, nullptr, dev(100), 1 << 30, nullptr);
        other = jko_last_error();
    });
    t.join();
    CHECK(other.find("max_iters") != std::string::npos);
    CHECK(strstr(jko_last_error(), "alias") != nullptr);
    // the message carries the refused value
    jko_energy f = e;
    f.kind = 2147483647;
    EXPECT(jko_step(&g, &f, &p, dev(1), dev(2), nullptr, nullptr, dev(100), 1 << 30, nullptr), JKO_ERR_INVALID,
           "2147483647");
}

}  // namespace

int main() {
    workspace_sizes();
    step_arguments();
    flow_and_backward_arguments();
    heat_arguments();
    strings_and_threads();
    if (g_failed) {
        fprintf(stderr, "%d of %d checks failed\n", g_failed, g_checks);
        return 1;
    }
    printf("ok %d\n", g_checks);
    return 0;
}
