"""Binary congestion (the non-convex {0, kappa} constraint of Section 4.5)
on the HIP path against the FP64 oracle, through the C ABI.

Its prox is a threshold on z = s e^{-sigma w} at kappa/e.  The device decides
in float32 on its own float32 s, the oracle in float64, so a cell whose z
lies within the float32 error of s from the threshold may go either way.
The first iteration is compared cell by cell away from those near-ties
(computed from the oracle's own z).  In longer runs a flipped decision feeds
the next products and moves z elsewhere by a little more than rounding, so
there every cell decided differently must be a near-tie of the oracle's last
prox argument within a wider band (NEAR_RUN), and few cells may differ; the
paths of the library that share their arithmetic (resident and launch, plane
and axis passes) must agree bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1502_06216_amd as jk
from workloads import make_workload, small_case

from _util import banner, dev, energies, f32, host64

pytestmark = pytest.mark.gpu

# half-width, in log z, of the band around the threshold left out of the
# cell-by-cell comparison: a few times the relative error of the device's s
NEAR = {"fp32": 1e-4, "split_bf16": 1e-3}
# the same after many iterations, where earlier flips have moved z
NEAR_RUN = 2e-2


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _case(shape, seed=3):
    wl = small_case(shape, "congestion", seed=seed)
    wl.kind = "binary_congestion"
    return wl


def _oracle_run(q, o_en, wl, n_steps, iters):
    """The oracle's flow and the log-gap of its last prox argument to the
    threshold, log z - (log kappa - 1) with z = s e^{-sigma w}."""
    last = {}

    def observe(k, s_, p_):
        last["s"] = s_

    for _ in range(n_steps):
        q, _ = O.jko_step(q, o_en, wl.gamma, wl.tau, iters, observe=observe)
    sigma = wl.tau / wl.gamma
    with np.errstate(divide="ignore", invalid="ignore"):
        gap = np.log(last["s"]) - sigma * o_en._w(q.shape) - (np.log(o_en._kappa(q.shape)) - 1.0)
    return q, gap


def _check_differing_cells(p, ref, gap, label, max_frac):
    """Cells decided differently: few, and each a near-tie of the oracle."""
    differ = (p > 0) != (ref > 0)
    worst = float(np.abs(gap[differ]).max()) if differ.any() else 0.0
    print(f"[gpu-test] {label}: {differ.mean():.2e} of cells decided differently, largest oracle "
          f"log-gap among them {worst:.2e}", flush=True)
    assert differ.mean() <= max_frac
    assert worst <= NEAR_RUN


def _binary_values(p, kappa, rtol=0.0):
    """Every cell is 0 or its (float32) capacity; rtol allows the last bits
    of exp(log kappa) that the log domain returns."""
    return bool(np.all((p == 0.0) | (np.abs(p - kappa) <= rtol * kappa)))


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("shape", [(48, 40), (100,), (20, 24, 36), (64, 64, 64)])
def test_first_iteration_decisions_match_the_oracle(shape, precision):
    banner(f"binary first iteration {shape} {precision}")
    wl = _case(shape)
    g_en, o_en = energies(wl)
    q = f32(wl.p0).astype(np.float64)
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=1, tol=0.0, precision=precision)
    p = host64(p)
    ref, _ = O.jko_step(q, o_en, wl.gamma, wl.tau, 1)
    # the oracle's own prox argument after one iteration (a = 1): s = xi (q / xi^T 1)
    sigma = wl.tau / wl.gamma
    t = O.gibbs_apply(np.ones(q.shape), wl.gamma)
    s = O.gibbs_apply(q / t, wl.gamma)
    kappa = o_en._kappa(q.shape)
    with np.errstate(divide="ignore"):
        gap = np.log(s) - sigma * o_en._w(q.shape) - (np.log(kappa) - 1.0)
    far = ~(np.abs(gap) < NEAR[precision])
    assert far.mean() > 0.98, far.mean()
    np.testing.assert_array_equal(p[far], ref[far])
    assert _binary_values(p, kappa)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_steps_stay_binary_and_close_to_the_oracle(precision):
    """Two steps of 30 iterations: binary values, and few cells decided
    differently from the FP64 oracle."""
    banner(f"binary flow {precision}")
    wl = _case((48, 40))
    g_en, o_en = energies(wl)
    pT, stats, ck = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, 2, max_iters=30, precision=precision,
                            checkpoints=True)
    q, gap = _oracle_run(f32(wl.p0).astype(np.float64), o_en, wl, 2, 30)
    p = host64(pT)
    kappa = o_en._kappa(q.shape)
    assert _binary_values(p, kappa) and _binary_values(q, kappa)
    _check_differing_cells(p, q, gap, f"binary flow {precision}", 0.005)
    assert all(s["iters"] == 30 for s in stats)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_resident_and_launch_paths_agree_bitwise(precision):
    banner(f"binary resident vs launch {precision}")
    wl = _case((96, 80))
    g_en, _ = energies(wl)
    for absorb in (float("inf"), 0.0):
        outs = []
        for resident in (True, False):
            p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=40, tol=0.0, precision=precision,
                            absorb_threshold=absorb, resident=resident)
            outs.append((host64(p), st["marginal_l1"]))
        np.testing.assert_array_equal(outs[0][0], outs[1][0])
        assert outs[0][1] == pytest.approx(outs[1][1], rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_plane_and_axis_passes_agree_bitwise(precision):
    banner(f"binary planes vs axis passes {precision}")
    wl = _case((64, 64, 64))
    g_en, _ = energies(wl)
    outs = []
    for planes in (True, False):
        p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=20, tol=0.0, precision=precision,
                        planes=planes)
        outs.append(host64(p))
    np.testing.assert_array_equal(outs[0], outs[1])


def test_log_domain_decides_like_the_plain_domain():
    """The log-domain prox tests log z >= log kappa - 1 instead of z >= kappa/e:
    after 20 iterations the two differ in a handful of near-tie cells at most."""
    banner("binary log vs plain")
    wl = _case((96, 80))
    g_en, o_en = energies(wl)
    outs = []
    for absorb in (float("inf"), 0.0):
        p, _ = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=20, tol=0.0, absorb_threshold=absorb)
        outs.append(host64(p))
    kappa = o_en._kappa(outs[0].shape)
    assert _binary_values(outs[0], kappa) and _binary_values(outs[1], kappa, rtol=1e-6)
    _, gap = _oracle_run(f32(wl.p0).astype(np.float64), o_en, wl, 1, 20)
    _check_differing_cells(outs[0], outs[1], gap, "binary log vs plain", 0.005)


def test_collapsed_step_is_reported():
    """Where sigma w > 1 over the whole support the prox empties every cell,
    xi^T a vanishes under positive mass and the step is undefined (the
    oracle's marginal is NaN there): the library reports JKO_ERR_NONFINITE."""
    banner("binary collapse")
    wl = _case((48, 40))
    wl.w = wl.w * 0.0 + 2.0 * wl.gamma / wl.tau     # sigma w = 2 everywhere
    g_en, o_en = energies(wl)
    with np.errstate(all="ignore"):
        _, st = O.jko_step(f32(wl.p0).astype(np.float64), o_en, wl.gamma, wl.tau, 3)
    assert not np.isfinite(st["marginal_l1"])
    with pytest.raises(jk.JKOError) as err:
        jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=3, tol=0.0)
    assert err.value.status == jk.JKO_ERR_NONFINITE


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_crowd256_binary_full_size(precision):
    """The benchmarked configuration (256^2, 300 iterations) for one step:
    binary values, the decisions of the FP64 oracle in all but a few cells,
    and the reported marginal violation close to the oracle's."""
    banner(f"crowd256_binary one step {precision}")
    wl = make_workload("crowd256_binary")
    g_en, o_en = energies(wl)
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=wl.max_iters, tol=0.0, precision=precision)
    q = f32(wl.p0).astype(np.float64)
    ref, gap = _oracle_run(q, o_en, wl, 1, wl.max_iters)
    _, rst = O.jko_step(q, o_en, wl.gamma, wl.tau, wl.max_iters)
    p = host64(p)
    kappa = o_en._kappa(ref.shape)
    assert _binary_values(p, kappa) and _binary_values(ref, kappa)
    _check_differing_cells(p, ref, gap, f"crowd256_binary {precision}", 0.001)
    print(f"[gpu-test] crowd256_binary {precision}: marginal {st['marginal_l1']:.4e} vs "
          f"{rst['marginal_l1']:.4e}", flush=True)
    assert st["marginal_l1"] == pytest.approx(rst["marginal_l1"], rel=0.01)


def test_stats_of_a_binary_step():
    """The reported mass is the sum of the returned binary density, and the
    reported violation is the oracle's at the same count."""
    banner("binary stats")
    wl = _case((48, 40))
    g_en, o_en = energies(wl)
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=40, tol=0.0)
    _, ost = O.jko_step(f32(wl.p0).astype(np.float64), o_en, wl.gamma, wl.tau, 40)
    assert st["mass"] == pytest.approx(float(host64(p).sum()), rel=1e-5)
    assert st["marginal_l1"] == pytest.approx(ost["marginal_l1"], rel=1e-3)

