"""Wasserstein attraction with congestion (Section 5.2, two couplings) on the
HIP path against the FP64 oracle, through the C ABI.

The device stacks the two couplings' scalings as one field of shape
(2, n...) and runs the reduced scaling of Proposition 5.2 (marginals first,
corrections dropped), which the oracle pins against the verbatim iteration.
Tolerances (rel-L1 of the density): 1e-5 for FP32, 1e-4 for split-BF16.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1502_06216_amd as jk
from workloads import gaussian_bumps, make_workload, small_case

from _util import banner, dev, energies, f32, host64, rel_l1

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_bf16": 1e-4}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _case(shape, seed=5, gamma=None):
    wl = small_case(shape, "congestion", seed=seed, gamma=gamma)
    wl.kind = "attraction"
    wl.w = None
    d = len(shape)
    r = gaussian_bumps(shape, [tuple([0.25] * d), tuple([0.7] + [0.3] * (d - 1))], 0.1, [0.5, 0.5])
    # the same mass as the float32 density the device receives
    r32 = f32(r).astype(np.float64)
    wl.target = r32 * (f32(wl.p0).astype(np.float64).sum() / r32.sum())
    return wl


def _oracle(wl, steps, iters, tol=0.0, check_every=1):
    r = f32(wl.target).astype(np.float64)
    kappa = f32(wl.kappa_field()).astype(np.float64)
    q = f32(wl.p0).astype(np.float64)
    for _ in range(steps):
        q, st = O.attraction_step(q, r, kappa, wl.gamma, wl.tau, iters, tol=tol, check_every=check_every)
    return q, st


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("shape", [(48, 40), (100,), (33, 29)])
def test_flow_matches_oracle(shape, precision):
    banner(f"attraction {shape} {precision}")
    wl = _case(shape)
    g_en, _ = energies(wl)
    pT, stats, ck = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, 2, max_iters=30, precision=precision,
                            checkpoints=True)
    ref, rst = _oracle(wl, 2, 30)
    err = rel_l1(host64(pT), ref)
    print(f"[gpu-test] attraction {shape} {precision}: rel-L1 {err:.2e}, marginal {stats[-1]['marginal_l1']:.3e} "
          f"vs {rst['marginal_l1']:.3e}", flush=True)
    assert err <= TOL[precision]
    assert (host64(pT) <= f32(wl.kappa_field()) + 0).all()
    assert stats[-1]["marginal_l1"] == pytest.approx(rst["marginal_l1"], rel=0.05, abs=3e-6)
    assert stats[-1]["mass"] == pytest.approx(float(host64(pT).sum()), rel=1e-5)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("shape", [(200, 160), (224, 100), (192, 160), (201, 161)])
def test_wide_band_matches_oracle(shape, precision):
    """gamma = 1e-3: bands of about a third of each axis, too wide for the
    fused 2D kernel.  (200, 160) runs the two couplings through per-field
    rotating passes (rows a multiple of 4), the paired proximal pass in the
    chunked form (axis 0 not a multiple of 32); (224, 100) runs that pass in
    the panel form, with 100 rows per field (the last paired tile's field-0
    half reads past its field); (192, 160) runs the whole step on the
    resident pass kernel; (201, 161) runs the stacked field's three
    passes."""
    banner(f"attraction wide band {shape} {precision}")
    wl = _case(shape, gamma=1e-3)
    wl.tau = 1e-2
    # the density moved by 3 rows, off the obstacles (scalings within float32)
    kappa = f32(wl.kappa_field()).astype(np.float64)
    r = np.roll(f32(wl.p0).astype(np.float64), -3, axis=0)
    r[-3:, :] = 0.0
    r[kappa <= 0] = 0.0
    wl.target = r * (f32(wl.p0).astype(np.float64).sum() / r.sum())
    g_en, _ = energies(wl)
    pT, stats, _ = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, 2, max_iters=30, precision=precision)
    ref, rst = _oracle(wl, 2, 30)
    err = rel_l1(host64(pT), ref)
    print(f"[gpu-test] attraction wide band {shape} {precision}: rel-L1 {err:.2e}", flush=True)
    assert err <= TOL[precision]
    assert stats[-1]["marginal_l1"] == pytest.approx(rst["marginal_l1"], rel=0.05, abs=3e-6)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_wide_band_scalar_capacity(precision):
    """The per-field rotating passes with a scalar capacity (the fused
    proximal epilogue reads no capacity field), and without capacity."""
    banner(f"attraction wide band, scalar capacity {precision}")
    for kap in (1.5 / (200 * 160), float("inf")):
        wl = _case((200, 160), gamma=1e-3)
        wl.tau = 1e-2
        wl.kappa = None
        wl.kappa_scalar = kap
        r = np.roll(f32(wl.p0).astype(np.float64), -3, axis=0)
        r[-3:, :] = 0.0
        wl.target = r * (f32(wl.p0).astype(np.float64).sum() / r.sum())
        g_en, _ = energies(wl)
        pT, stats, _ = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, 2, max_iters=30, precision=precision)
        ref, _ = _oracle(wl, 2, 30)
        err = rel_l1(host64(pT), ref)
        print(f"[gpu-test] attraction wide band kappa={kap:.3g} {precision}: rel-L1 {err:.2e}", flush=True)
        assert err <= TOL[precision]


def test_wide_band_absorption_switch():
    """A wide band (per-field rotating passes with the fused proximal step)
    and a target beyond float32's reach: the step switches to the log domain
    once and matches the oracle's exact log-sum-exp step."""
    banner("attraction wide band absorption switch")
    wl = _case((200, 160), gamma=1e-3)
    g_en, _ = energies(wl)
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=30, check_every=1, absorb_threshold=20.0)
    r = f32(wl.target).astype(np.float64)
    kappa = f32(wl.kappa_field()).astype(np.float64)
    ref, _ = O.attraction_step_log(f32(wl.p0).astype(np.float64), r, kappa, wl.gamma, wl.tau, 30)
    err = rel_l1(host64(p), ref)
    print(f"[gpu-test] attraction wide band switch: absorptions {st['absorptions']}, rel-L1 {err:.2e}", flush=True)
    assert st["absorptions"] == 1
    assert np.isfinite(host64(p)).all() and err <= TOL["fp32"]


def test_attraction_to_its_own_density_is_one_blur():
    """r = q without capacity: every iteration returns the blur xi (q / xi^T 1)."""
    banner("attraction r = q")
    wl = _case((48, 40))
    wl.target = f32(wl.p0).astype(np.float64)
    wl.kappa = None
    wl.kappa_scalar = float("inf")
    g_en, _ = energies(wl)
    p, _ = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=5, tol=0.0)
    q = f32(wl.p0).astype(np.float64)
    ref = O.gibbs_apply(q / O.gibbs_apply(np.ones_like(q), wl.gamma, transpose=True), wl.gamma)
    assert rel_l1(host64(p), ref) <= 1e-6


def test_tolerance_mode_stops_like_the_oracle():
    banner("attraction tolerance mode")
    wl = _case((48, 40))
    g_en, _ = energies(wl)
    tol, ce = 1e-6, 10
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=3000, tol=tol, check_every=ce)
    ref, ost = _oracle(wl, 1, 3000, tol=tol, check_every=ce)
    print(f"[gpu-test] attraction tolerance: device {st['iters']} iterations, oracle {ost['iters']}", flush=True)
    assert st["stop"] == "tol" and ost["stop"] == "tol"
    assert st["iters"] % ce == 0 and abs(st["iters"] - ost["iters"]) <= ce
    assert st["marginal_l1"] <= tol
    same, _ = _oracle(wl, 1, st["iters"])
    assert rel_l1(host64(p), same) <= TOL["fp32"]


def test_target_is_a_shape():
    """The target is scaled to the density's mass: a target of twice the mass
    gives the same step."""
    banner("attraction target scale, errors")
    wl = _case((48, 40))
    g_en, _ = energies(wl)
    p1, _ = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=20)
    twice = jk.EnergySpec(kind="attraction", kappa=g_en.kappa, target=g_en.target * 2.0)
    p2, _ = jk.step(dev(wl.p0), twice, wl.gamma, wl.tau, max_iters=20)
    assert rel_l1(host64(p2), host64(p1)) <= 1e-6


def test_absorption_switch():
    """A finite threshold: below it the step is the plain one bit for bit;
    with a target beyond float32's reach max|log b| crosses it, the step
    switches to the log domain once and matches the oracle's exact
    log-sum-exp step."""
    banner("attraction absorption switch")
    wl = _case((48, 40))
    g_en, _ = energies(wl)
    plain, s0 = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=30, check_every=1)
    thr, s1 = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=30, check_every=1, absorb_threshold=1e6)
    assert torch.equal(plain, thr) and s1["absorptions"] == 0
    wl.gamma *= 0.25
    wl.tau *= 0.25
    g_en, o_en = energies(wl)
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=30, check_every=1, absorb_threshold=20.0)
    r = f32(wl.target).astype(np.float64)
    kappa = f32(wl.kappa_field()).astype(np.float64)
    ref, _ = O.attraction_step_log(f32(wl.p0).astype(np.float64), r, kappa, wl.gamma, wl.tau, 30)
    err = rel_l1(host64(p), ref)
    print(f"[gpu-test] attraction switch: absorptions {st['absorptions']}, rel-L1 {err:.2e}", flush=True)
    assert st["absorptions"] == 1
    assert np.isfinite(host64(p)).all() and err <= TOL["fp32"]


def _log_run(precision, gamma_scale):
    wl = _case((48, 40))
    wl.gamma *= gamma_scale
    wl.tau *= gamma_scale
    g_en, _ = energies(wl)
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=30, tol=0.0, precision=precision,
                    absorb_threshold=0.0)
    r = f32(wl.target).astype(np.float64)
    kappa = f32(wl.kappa_field()).astype(np.float64)
    ref, _ = O.attraction_step_log(f32(wl.p0).astype(np.float64), r, kappa, wl.gamma, wl.tau, 30)
    return host64(p), ref, kappa


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_log_domain_matches_oracle(precision):
    """absorb_threshold = 0: the whole step in log form against the oracle's
    exact log-sum-exp form (every log-domain product shifts each output by
    its own largest term)."""
    banner(f"attraction log domain {precision}")
    p, ref, _ = _log_run(precision, 1.0)
    err = rel_l1(p, ref)
    print(f"[gpu-test] attraction log {precision}: rel-L1 {err:.2e}", flush=True)
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_log_domain_far_target_matches_oracle(precision):
    """A target beyond the float32 reach of the kernel (gamma a quarter of the
    default, where the plain domain fails): the log domain stays within
    capacity and matches the exact log-sum-exp step."""
    banner(f"attraction log domain far target {precision}")
    p, ref, kappa = _log_run(precision, 0.25)
    err = rel_l1(p, ref)
    print(f"[gpu-test] attraction log far target {precision}: rel-L1 {err:.2e}", flush=True)
    assert np.isfinite(p).all() and (p <= kappa * (1 + 1e-6)).all()
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_crowd256_attraction_one_step_full_size(precision):
    """The benchmarked configuration (256^2, capacity with obstacles) for one
    step of 300 iterations against the oracle."""
    banner(f"crowd256_attraction one step {precision}")
    wl = make_workload("crowd256_attraction")
    g_en, _ = energies(wl)
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=wl.max_iters, tol=0.0, precision=precision)
    ref, rst = _oracle(wl, 1, wl.max_iters)
    err = rel_l1(host64(p), ref)
    print(f"[gpu-test] crowd256_attraction {precision}: rel-L1 {err:.2e}", flush=True)
    assert err <= TOL[precision]
