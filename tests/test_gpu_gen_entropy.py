"""Generalised entropies (Section 4.4, per-cell weights b_i and exponents
m_i >= 1) on the HIP path against the FP64 oracle, through the C ABI.

The two set-ups of the paper's nonlinear-diffusion example stand in for its
figure: a fixed exponent with weights growing from 1 at the boundary to 20 in
the centre, and unit weights with exponents growing from 1 to 2.  Densities
are in density units (D = N) so that the nonlinearity matters.  Tolerances
(rel-L1 of the density) are those of the other energies: 1e-5 for FP32,
1e-4 for split-BF16.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1502_06216_amd as jk
from workloads import make_workload, small_case

from _util import banner, dev, energies, f32, host64, rel_l1

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_bf16": 1e-4}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _centre_bump(shape):
    """1 in the centre, exactly 0 on the outermost cells."""
    out = np.ones(shape)
    for ax, n in enumerate(shape):
        x = np.arange(n)
        prof = np.sin(np.pi * x / max(n - 1, 1))
        prof[0] = prof[-1] = 0.0
        out = out * prof.reshape([n if k == ax else 1 for k in range(len(shape))])
    return out


def _case(shape, setup, seed=4):
    wl = small_case(shape, "porous", seed=seed)
    wl.kind = "gen_entropy"
    wl.density_scale = float(np.prod(shape))
    bump = _centre_bump(shape)
    if setup == "weights":
        wl.coef = 1.0 + 19.0 * bump
        wl.m = 1.4
        wl.m_field = None
    else:
        wl.coef = None
        wl.coef_scalar = 1.0
        wl.m_field = 1.0 + bump          # exactly 1 on the boundary cells
    return wl


def _flow_errors(wl, precision, n_steps, iters, absorb=float("inf")):
    g_en, o_en = energies(wl)
    pT, stats, ck = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, n_steps, max_iters=iters, precision=precision,
                            absorb_threshold=absorb, checkpoints=True)
    q = f32(wl.p0).astype(np.float64)
    for _ in range(n_steps):
        q, st = O.jko_step(q, o_en, wl.gamma, wl.tau, iters)
    return rel_l1(host64(pT), q), stats, st


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("setup", ["weights", "exponents"])
@pytest.mark.parametrize("shape", [(48, 40), (100,), (20, 24, 36), (64, 64, 64)])
def test_flow_matches_oracle(shape, setup, precision):
    banner(f"gen entropy {shape} {setup} {precision}")
    wl = _case(shape, setup)
    err, stats, st = _flow_errors(wl, precision, 2, 30)
    print(f"[gpu-test] gen entropy {shape} {setup} {precision}: rel-L1 {err:.2e}", flush=True)
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_log_domain_matches_oracle(precision):
    banner(f"gen entropy log domain {precision}")
    wl = _case((48, 40), "exponents")
    err, _, _ = _flow_errors(wl, precision, 2, 30, absorb=0.0)
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_resident_and_launch_paths_agree_bitwise(precision):
    banner(f"gen entropy resident vs launch {precision}")
    wl = _case((96, 80), "exponents")
    g_en, _ = energies(wl)
    for absorb in (float("inf"), 0.0):
        outs = []
        for resident in (True, False):
            p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=40, tol=0.0, precision=precision,
                            absorb_threshold=absorb, resident=resident)
            outs.append(host64(p))
        np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_plane_and_axis_passes_agree_bitwise(precision):
    banner(f"gen entropy planes vs axis passes {precision}")
    wl = _case((64, 64, 64), "weights")
    g_en, _ = energies(wl)
    outs = []
    for planes in (True, False):
        p, _ = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=20, tol=0.0, precision=precision,
                       planes=planes)
        outs.append(host64(p))
    np.testing.assert_array_equal(outs[0], outs[1])


def test_unit_exponent_is_the_entropy_energy():
    """m = 1 everywhere with weights c is the entropy energy (Proposition 4.2,
    m = 1): both kinds take the same steps to float32 rounding."""
    banner("gen entropy m = 1 vs entropy")
    wl = small_case((48, 40), "entropy", seed=4)
    g_en, _ = energies(wl)
    a, _ = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=30, tol=0.0)
    wl.kind = "gen_entropy"
    wl.m = 1.0
    g_gen, _ = energies(wl)
    b, _ = jk.step(dev(wl.p0), g_gen, wl.gamma, wl.tau, max_iters=30, tol=0.0)
    assert rel_l1(host64(b), host64(a)) <= 1e-6


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_gen512_one_step_full_size(precision):
    """The benchmarked configuration (512^2, exponents 1 to 2, same launches)
    for one step of 100 iterations against the oracle."""
    banner(f"gen512 one step {precision}")
    wl = make_workload("gen512")
    err, stats, st = _flow_errors(wl, precision, 1, 100)
    print(f"[gpu-test] gen512 {precision}: rel-L1 {err:.2e}", flush=True)
    assert err <= TOL[precision]


@pytest.mark.parametrize("shape,setup", [((48, 40), "exponents"), ((48, 40), "weights"), ((20, 24, 36), "exponents"),
                                         ((20, 24, 36), "weights")])
def test_adjoint_matches_fp64_autograd(shape, setup):
    """dL/dp0 (and, where the weights are a field, dL/db) of
    L = ||p_T - target||^2 from the hand-written adjoint (its prox step
    through the implicit derivatives) against torch float64 autograd through
    the oracle's unrolled iteration, 2 steps x 30 iterations."""
    from oracle.grad import loss_and_grads
    banner(f"gen entropy adjoint {shape} {setup}")
    wl = _case(shape, setup)
    g_en, o_en = energies(wl)
    rng = np.random.default_rng(9)
    target = rng.uniform(size=shape)
    target /= target.sum()
    pT, _, ck = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, 2, max_iters=30, checkpoints=True)
    dL = 2.0 * (pT - dev(target))
    want_b = wl.coef is not None
    gw, gp = jk.backward(ck, [30, 30], dL.contiguous(), g_en, wl.gamma, wl.tau, want_w=want_b)
    assert (gw is not None) == want_b
    loss, rb, rp, _ = loss_and_grads(f32(wl.p0).astype(np.float64), np.zeros(shape), np.inf, wl.gamma, wl.tau,
                                    [30, 30], target, kind="gen_entropy", coef=o_en._coef(shape), m=o_en._m(shape),
                                    density_scale=wl.density_scale)
    ep = np.linalg.norm(host64(gp) - rp) / np.linalg.norm(rp)
    eb = np.linalg.norm(host64(gw) - rb) / np.linalg.norm(rb) if want_b else 0.0
    print(f"[gpu-test] gen entropy adjoint {shape} {setup}: rel err dL/dp0 {ep:.2e}, dL/db {eb:.2e}", flush=True)
    assert ep <= 1e-3 and eb <= 1e-3


@pytest.mark.parametrize("resident", [True, False])
def test_tolerance_mode_stops_like_the_oracle(resident):
    """Tolerance mode (stop test every 10 iterations, in the resident kernel
    or on the host-driven path): the step stops within one check interval
    of the oracle and returns the oracle's iterate at that count."""
    banner(f"gen entropy tolerance mode resident={resident}")
    wl = _case((48, 40), "exponents")
    g_en, o_en = energies(wl)
    tol, ce = 1e-6, 10
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=3000, tol=tol, check_every=ce,
                    resident=resident)
    q = f32(wl.p0).astype(np.float64)
    ref, ost = O.jko_step(q, o_en, wl.gamma, wl.tau, 3000, tol=tol, check_every=ce)
    print(f"[gpu-test] gen entropy tolerance: device {st['iters']} iterations, oracle {ost['iters']}", flush=True)
    assert st["stop"] == "tol" and ost["stop"] == "tol"
    assert st["iters"] % ce == 0 and abs(st["iters"] - ost["iters"]) <= ce
    assert st["marginal_l1"] <= tol
    assert st["mass"] == pytest.approx(float(host64(p).sum()), rel=1e-5)
    ref_same, _ = O.jko_step(q, o_en, wl.gamma, wl.tau, st["iters"])
    assert rel_l1(host64(p), ref_same) <= TOL["fp32"]

