"""The resident 2D kernel (one cooperative launch per step; between the Gibbs
applications each block waits for the blocks its halo reaches) against the
launch-per-application path:
both run the same tile arithmetic, partial sums and control decisions, so the
densities and statistics must agree bit for bit.  The launch path itself is
pinned to the FP64 oracle by the parity tests."""
import numpy as np
import pytest
import torch

import paper_1502_06216_amd as jk
from workloads import make_workload, small_case

from _util import banner, dev, energies, host64

pytestmark = pytest.mark.gpu

STAT_KEYS = ("iters", "absorptions", "stop", "status", "marginal_l1", "mass", "max_abs_log_a", "max_abs_log_b")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _both(wl, **kw):
    g_en, _ = energies(wl)
    out = []
    for resident in (True, False):
        p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, resident=resident, **kw)
        out.append((p, st))
    return out


def _same(res, ref):
    (p1, s1), (p2, s2) = res, ref
    assert torch.equal(p1, p2), f"max |diff| {float((p1 - p2).abs().max()):.3e}"
    for k in STAT_KEYS:
        assert s1[k] == s2[k], (k, s1[k], s2[k])


@pytest.mark.parametrize("tol", [0.0, 1e-6])
def test_crowd32_same_bits(tol):
    banner(f"resident crowd32 tol={tol}")
    wl = make_workload("crowd32", projected=True)
    res, ref = _both(wl, max_iters=3000 if tol else 300, tol=tol, check_every=10)
    _same(res, ref)
    if tol:
        assert res[1]["stop"] == "tol"


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("tol,cap", [(0.0, 300), (1e-6, 2000)])
def test_crowd256_same_bits(tol, cap, precision):
    """The 256x256 crowd workload at full size (256 resident blocks)."""
    banner(f"resident crowd256 tol={tol} cap={cap} {precision}")
    wl = make_workload("crowd256")
    res, ref = _both(wl, max_iters=cap, tol=tol, check_every=10, precision=precision)
    _same(res, ref)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("shape,kind", [((45, 70), "congestion"), ((48, 40), "entropy"), ((48, 40), "porous"),
                                        ((48, 40), "zero"), ((17, 130), "congestion")])
def test_ragged_and_other_energies_same_bits(shape, kind, precision):
    banner(f"resident {shape} {kind} {precision}")
    wl = small_case(shape, kind, seed=4)
    if kind == "porous":
        wl.density_scale = float(np.prod(wl.shape))
    _same(*_both(wl, max_iters=60, tol=1e-7, check_every=7, precision=precision))


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("threshold", [0.0, 50.0])
def test_log_domain_same_bits(threshold, precision):
    """Absorption inside the resident launch (from the start, or switched at a
    check) matches the launch path's separate absorb kernel."""
    banner(f"resident log domain thr={threshold} {precision}")
    wl = make_workload("crowd32", projected=False)
    res, ref = _both(wl, max_iters=300, check_every=10, absorb_threshold=threshold, precision=precision)
    _same(res, ref)
    assert res[1]["absorptions"] == 1


def test_nonfinite_is_reported_the_same():
    banner("resident non-finite")
    wl = small_case((64, 64), "congestion", seed=1, gamma=2e-4, tau=2e-3, n_boxes=3, projected=False,
                    cap_factor=1.2)
    g_en, _ = energies(wl)
    for resident in (True, False):
        with pytest.raises(jk.JKOError) as e:
            jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=60, resident=resident)
        assert e.value.status == jk.JKO_ERR_NONFINITE


@pytest.mark.parametrize("name,steps,iters", [("crowd32", 3, 50), ("crowd256_fixed", 2, 60)])
def test_flow_and_adjoint_same_bits(name, steps, iters):
    """Checkpointed flow, the adjoint's recomputation (t_k, s_k recorded by
    the resident kernel) and the resident reverse sweep against the launch
    path."""
    banner(f"resident flow + adjoint {name}")
    wl = make_workload(name, projected=True) if name == "crowd32" else make_workload(name)
    g_en, _ = energies(wl)
    outs = []
    for resident in (True, False):
        pT, st, ck = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, steps, max_iters=iters, checkpoints=True,
                             resident=resident)
        dL = (2.0 * pT).contiguous()
        gw, gp = jk.backward(ck, [iters] * steps, dL, g_en, wl.gamma, wl.tau, resident=resident)
        outs.append((pT, ck, gw, gp, st))
    for a, b in zip(outs[0][:4], outs[1][:4]):
        assert torch.equal(a, b)
    for s1, s2 in zip(outs[0][4], outs[1][4]):
        for k in STAT_KEYS:
            assert s1[k] == s2[k]


def test_repeated_calls_reset_the_sync_words():
    """Back-to-back resident steps (the published phase counts start from zero
    each launch) give the same bits every time."""
    banner("resident repeated")
    wl = make_workload("crowd32", projected=True)
    g_en, _ = energies(wl)
    q = dev(wl.p0)
    first = [jk.step(q, g_en, wl.gamma, wl.tau, max_iters=100)[0] for _ in range(3)]
    for p in first[1:]:
        assert torch.equal(p, first[0])


def test_time_iteration_reports_one_resident_launch():
    banner("resident timing")
    wl = make_workload("crowd256")
    g_en, _ = energies(wl)
    ms = jk.time_iteration(dev(wl.p0), g_en, wl.gamma, wl.tau, reps=2, iters=100)
    assert len(ms) == 1 and ms[0] > 0
    ms2 = jk.time_iteration(dev(wl.p0), g_en, wl.gamma, wl.tau, reps=2, resident=False)
    assert len(ms2) == 2


def test_crowd256_flow_many_steps_same_bits():
    """Six checkpointed steps of the 256x256 flow (3600 resident phases with
    neighbour waits): every checkpoint identical to the launch path's."""
    banner("resident crowd256 flow 6 x 300")
    wl = make_workload("crowd256_fixed")
    g_en, _ = energies(wl)
    outs = []
    for resident in (True, False):
        pT, st, ck = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, 6, max_iters=300, tol=1e-7, check_every=10,
                             checkpoints=True, resident=resident)
        outs.append((pT, ck, st))
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    for s1, s2 in zip(outs[0][2], outs[1][2]):
        for k in STAT_KEYS:
            assert s1[k] == s2[k]


@pytest.mark.parametrize("ce,tol,thr", [(1, 1e-6, float("inf")), (2, 1e-6, float("inf")), (3, 0.0, 50.0),
                                        (1, 0.0, 50.0), (7, 1e-7, 50.0)])
def test_check_cadences_same_bits(ce, tol, thr):
    """Every check cadence: checks every iteration (the decision is awaited
    before the proximal half-step), and cadences >= 2 (the half-step overlaps
    the decision), with and without an absorption switch, stopping early or
    at the cap."""
    banner(f"resident cadence ce={ce} tol={tol} thr={thr}")
    wl = make_workload("crowd32", projected=False)
    res, ref = _both(wl, max_iters=400, tol=tol, check_every=ce, absorb_threshold=thr)
    _same(res, ref)


def test_switch_after_the_last_iteration_same_bits():
    """An absorption switch decided at the check of the last iteration takes
    effect after its proximal half-step, where the capped step's closing
    monitor reads the log-domain scalings: the resident kernel converts b
    there once its neighbours are done with it.  The cap is the first one at
    which the switch happens (found by bisection on the launch path)."""
    banner("resident switch after the last iteration")
    wl = make_workload("crowd32", projected=False)
    g_en, _ = energies(wl)
    q = dev(wl.p0)

    def switched(k):
        _, st = jk.step(q, g_en, wl.gamma, wl.tau, max_iters=k, check_every=1, absorb_threshold=50.0,
                        resident=False)
        return st["absorptions"] == 1

    lo, hi = 1, 300
    assert switched(hi) and not switched(lo)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if switched(mid):
            hi = mid
        else:
            lo = mid
    res, ref = _both(wl, max_iters=hi, check_every=1, absorb_threshold=50.0)
    _same(res, ref)
    assert res[1]["absorptions"] == 1 and res[1]["stop"] == "cap"
