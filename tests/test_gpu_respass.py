"""The resident pass kernel (a 2D step's per-axis panel passes in one
cooperative launch, each block waiting only for the blocks whose outputs its
next pass reads) against the same passes launched one by one: the products
are the same, so densities must agree bit for bit; with one field the
statistics too (the partial sums are taken over the same tiles in the same
order).  The launched passes are pinned to the FP64 oracle by the parity
tests, and the 512^2 configurations, which run on this kernel by default,
by the configuration tests; one case here checks the oracle directly."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1502_06216_amd as jk
from workloads import make_workload, small_case

from _util import banner, dev, energies, f32, host64, rel_l1

pytestmark = pytest.mark.gpu

STAT_KEYS = ("iters", "absorptions", "stop", "status", "marginal_l1", "mass", "max_abs_log_a", "max_abs_log_b")
TOL = {"fp32": 1e-5, "split_bf16": 1e-4}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _both(wl, planes=False, **kw):
    """(resident pass kernel, launched passes)."""
    g_en, _ = energies(wl)
    return [jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, resident=r, planes=planes, **kw) for r in (True, False)]


def _same(res, ref, keys=STAT_KEYS):
    (p1, s1), (p2, s2) = res, ref
    assert torch.equal(p1, p2), f"max |diff| {float((p1 - p2).abs().max()):.3e}"
    for k in keys:
        assert s1[k] == s2[k], (k, s1[k], s2[k])


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("name,kw", [
    ("porous512_scaled", dict(max_iters=300, tol=1e-6, check_every=10, planes=True)),
    ("gen512", dict(max_iters=120, tol=0.0, check_every=10, planes=True)),
    ("crowd256", dict(max_iters=100, tol=0.0, check_every=10)),
    ("crowd256_binary", dict(max_iters=60, tol=0.0, check_every=10)),
])
def test_named_workloads_same_bits(name, kw, precision):
    """512^2 nonlinear diffusion (tolerance mode) and generalised entropies run
    on the pass kernel by default; 256^2 crowd motion and binary congestion
    with the per-axis passes asked for."""
    banner(f"respass {name} {precision}")
    _same(*_both(make_workload(name), precision=precision, **kw))


@pytest.mark.parametrize("kind", ["congestion", "entropy", "porous", "zero"])
def test_energies_same_bits(kind):
    banner(f"respass 96x64 {kind}")
    wl = small_case((96, 64), kind, seed=4)
    _same(*_both(wl, max_iters=80, tol=0.0, check_every=5))


def test_one_block_grid():
    """32 x 32: one block, whose waits are on itself."""
    banner("respass 32x32")
    wl = make_workload("crowd32", projected=True)
    _same(*_both(wl, max_iters=300, tol=1e-6, check_every=10))


@pytest.mark.parametrize("ce", [1, 7])
def test_tolerance_stop_same_bits(ce):
    """Every check cadence, stopping on the tolerance (the 512^2 case above
    stops on it with 256 blocks)."""
    banner(f"respass tolerance stop ce={ce}")
    wl = make_workload("crowd32", projected=True)
    res, ref = _both(wl, max_iters=3000, tol=1e-6, check_every=ce)
    _same(res, ref)
    assert res[1]["stop"] == "tol"


def test_absorption_switch_same_bits():
    """A switch to the log domain at a check: the kernel returns after that
    iteration's proximal half-step and the step goes on on the log passes."""
    banner("respass absorption switch")
    wl = make_workload("crowd32", projected=False)
    res, ref = _both(wl, max_iters=300, check_every=10, absorb_threshold=50.0)
    _same(res, ref)
    assert res[1]["absorptions"] == 1


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_flow_matches_oracle(precision):
    banner(f"respass 96x128 flow vs oracle {precision}")
    wl = small_case((96, 128), "congestion", seed=8, gamma=1e-3, tau=5e-3, n_boxes=3)
    g_en, o_en = energies(wl)
    pT, stats, _ = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, 2, max_iters=60, precision=precision, planes=False)
    q = f32(wl.p0).astype(np.float64)
    for _ in range(2):
        q, ost = O.jko_step(q, o_en, wl.gamma, wl.tau, 60)
    err = rel_l1(host64(pT), q)
    print(f"[gpu-test] respass flow {precision}: rel-L1 {err:.2e}", flush=True)
    assert err <= TOL[precision]
    assert stats[-1]["marginal_l1"] == pytest.approx(ost["marginal_l1"], rel=1e-3)


ATTR_KEYS = ("iters", "absorptions", "stop", "status")


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_attraction_same_bits(precision):
    """The attraction's two couplings on paired tiles against the per-field
    rotating passes launched one by one."""
    banner(f"respass attraction {precision}")
    wl = make_workload("crowd256_attraction")
    res, ref = _both(wl, max_iters=100, tol=0.0, check_every=10, precision=precision)
    _same(res, ref, ATTR_KEYS)
    assert res[1]["marginal_l1"] == pytest.approx(ref[1]["marginal_l1"], rel=1e-9)


def _attraction_case(shape, gamma=1e-3):
    wl = small_case(shape, "congestion", seed=5, gamma=gamma)
    wl.kind = "attraction"
    wl.w = None
    wl.tau = 1e-2
    kappa = f32(wl.kappa_field()).astype(np.float64)
    r = np.roll(f32(wl.p0).astype(np.float64), -3, axis=0)
    r[-3:, :] = 0.0
    r[kappa <= 0] = 0.0
    wl.target = r * (f32(wl.p0).astype(np.float64).sum() / r.sum())
    return wl


def test_attraction_tolerance_and_switch_same_bits():
    banner("respass attraction tolerance stop and absorption switch")
    wl = _attraction_case((192, 160))
    # a tolerance the iteration reaches: twice the violation after 300 iterations
    g_en, _ = energies(wl)
    _, s300 = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=300, tol=0.0, check_every=10)
    res, ref = _both(wl, max_iters=2000, tol=2.0 * s300["marginal_l1"], check_every=10)
    _same(res, ref, ATTR_KEYS)
    assert res[1]["stop"] == "tol" and res[1]["iters"] <= 300
    res, ref = _both(wl, max_iters=60, tol=0.0, check_every=10, absorb_threshold=5.0)
    _same(res, ref, ATTR_KEYS)
    assert res[1]["absorptions"] == 1


@pytest.mark.parametrize("name,steps,kw", [
    ("porous512_scaled", 10, dict(max_iters=300, tol=1e-6, check_every=10)),
    ("crowd256_attraction", 3, dict(max_iters=300, tol=0.0, check_every=10)),
])
def test_flows_repeat_bit_for_bit(name, steps, kw):
    """Whole flows (every step one launch of the pass kernel): two runs give
    the same bits, and so do the launched passes."""
    banner(f"respass flow {name} x {steps}")
    wl = make_workload(name)
    g_en, _ = energies(wl)
    outs = [jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, steps, resident=r, **kw) for r in (True, True, False)]
    (p1, s1, _), (p2, s2, _), (p3, s3, _) = outs
    assert torch.equal(p1, p2) and torch.equal(p1, p3)
    assert [s["iters"] for s in s1] == [s["iters"] for s in s2] == [s["iters"] for s in s3]
