"""The 3D plane path (a plane pass over axes 1 and 2 with the intermediate on
chip, then an axis-0 pass with the epilogue) against the three axis passes:
both run the same arithmetic in the same order, so densities, checkpoints,
gradients and the statistics' counts and maxima must agree bit for bit (the
FP64 sums of per-block partials to rounding).  Gibbs products on shapes
that take the plane path are also checked against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1502_06216_amd as jk
from workloads import make_workload, small_case

from _util import banner, dev, energies, f32, host64, rel_l1

pytestmark = pytest.mark.gpu

GIBBS_TOL = {"fp32": 1e-6, "split_bf16": 2e-5}
STAT_KEYS = ("iters", "absorptions", "stop", "status", "marginal_l1", "mass", "max_abs_log_a", "max_abs_log_b")
FP64_SUMS = ("marginal_l1", "mass")
PRECISIONS = ["fp32", "split_bf16"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _same_stats(s1, s2):
    """Counts, decisions and maxima exactly; the FP64 sums of per-block
    partials to rounding (the axis-0 pass may tile differently from the last
    axis pass, which regroups the sum)."""
    for k in STAT_KEYS:
        if k in FP64_SUMS:
            assert s1[k] == pytest.approx(s2[k], rel=1e-12, abs=1e-300), (k, s1[k], s2[k])
        else:
            assert s1[k] == s2[k], (k, s1[k], s2[k])


def _same_step(wl, **kw):
    g_en, _ = energies(wl)
    out = [jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, planes=planes, **kw) for planes in (True, False)]
    (p1, s1), (p2, s2) = out
    assert torch.equal(p1, p2), f"max |diff| {float((p1 - p2).abs().max()):.3e}"
    _same_stats(s1, s2)
    return p1, s1


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("shape,gamma", [((32, 64, 96), 4e-3), ((64, 32, 32), 2e-2), ((96, 128, 64), 1e-3),
                                         ((32, 64, 160), 3e-2), ((160, 32, 32), 3e-2)])
def test_gibbs_apply_plane_path_matches_oracle(shape, gamma, precision):
    """Shapes with every axis a multiple of 32 (bands from one panel up to the
    widest the plane pass takes) against the plain separable FP64 product."""
    banner(f"plane gibbs {shape} gamma={gamma} {precision}")
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 1.0, size=shape) * np.exp(rng.normal(0, 2, size=shape))
    y = jk.gibbs_apply(dev(x), gamma, precision)
    ref = O.gibbs_apply(f32(x).astype(np.float64), gamma)
    err = rel_l1(host64(y), ref)
    print(f"[gpu-test] plane gibbs {shape} {precision}: rel-L1 {err:.2e}", flush=True)
    assert err <= GIBBS_TOL[precision]


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("shape,kind", [((64, 96, 96), "congestion"), ((32, 64, 64), "entropy"),
                                        ((32, 64, 64), "porous"), ((64, 32, 96), "zero"),
                                        ((96, 128, 32), "congestion")])
def test_step_same_bits_as_axis_passes(shape, kind, precision):
    banner(f"plane step {shape} {kind} {precision}")
    wl = small_case(shape, kind, seed=6)
    if kind == "porous":
        wl.density_scale = float(np.prod(wl.shape))
    _same_step(wl, max_iters=40, tol=1e-7, check_every=7, precision=precision)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("threshold", [0.0, 50.0])
def test_log_domain_same_bits_as_axis_passes(threshold, precision):
    """Log-domain contractions (from the start, or after a switch at a check):
    per-row shifts in the first stage, per-column shifts over each chunk's
    band in the second, per-column shifts in the axis-0 pass."""
    banner(f"plane log domain thr={threshold} {precision}")
    wl = small_case((64, 64, 64), "congestion", seed=8, projected=False)
    p, st = _same_step(wl, max_iters=120, check_every=10, absorb_threshold=threshold, precision=precision)
    assert st["absorptions"] == 1


@pytest.mark.parametrize("precision", PRECISIONS)
def test_crowd128c_full_step_same_bits(precision):
    """The 128^3 crowd workload, one full 300-iteration step."""
    banner(f"plane crowd128c {precision}")
    wl = make_workload("crowd128c")
    _same_step(wl, max_iters=300, check_every=10, precision=precision)


def test_flow_and_adjoint_same_bits():
    """Checkpointed flow, recomputation and reverse sweep (the adjoint
    epilogues on the axis-0 pass) against the axis passes."""
    banner("plane flow + adjoint")
    wl = small_case((32, 64, 64), "congestion", seed=9)
    g_en, _ = energies(wl)
    outs = []
    for planes in (True, False):
        pT, st, ck = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, 3, max_iters=30, checkpoints=True, planes=planes)
        dL = (2.0 * pT).contiguous()
        gw, gp = jk.backward(ck, [30] * 3, dL, g_en, wl.gamma, wl.tau, planes=planes)
        outs.append((pT, ck, gw, gp, st))
    for a, b in zip(outs[0][:4], outs[1][:4]):
        assert torch.equal(a, b)
    for s1, s2 in zip(outs[0][4], outs[1][4]):
        _same_stats(s1, s2)


def test_time_iteration_launch_counts():
    """Four launches per iteration on the plane path, six with axis passes."""
    banner("plane timing")
    wl = small_case((64, 64, 64), "congestion", seed=1)
    g_en, _ = energies(wl)
    ms = jk.time_iteration(dev(wl.p0), g_en, wl.gamma, wl.tau, reps=3)
    ms_axis = jk.time_iteration(dev(wl.p0), g_en, wl.gamma, wl.tau, reps=3, planes=False)
    assert len(ms) == 4 and len(ms_axis) == 6
    assert all(t > 0 for t in ms + ms_axis)
