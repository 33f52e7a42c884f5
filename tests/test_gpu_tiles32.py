"""The 32 x 32 output tiles of the fused 2D kernels (grids with more than 256
tiles of 16 x 16 and at most 256 of 32 x 32, such as 512 x 512): Gibbs
products and flows against the FP64 oracle, the resident kernels against the
launch-per-application path bit for bit, and the adjoint against FP64
autograd."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1502_06216_amd as jk
from oracle.grad import loss_and_grads
from workloads import make_workload, small_case

from _util import banner, dev, energies, f32, host64, rel_l1

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_bf16": 1e-4}
GIBBS_TOL = {"fp32": 1e-6, "split_bf16": 2e-5}
STAT_KEYS = ("iters", "absorptions", "stop", "status", "marginal_l1", "mass", "max_abs_log_a", "max_abs_log_b")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _both(wl, **kw):
    g_en, _ = energies(wl)
    return [jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, resident=r, **kw) for r in (True, False)]


def _same(res, ref):
    (p1, s1), (p2, s2) = res, ref
    assert torch.equal(p1, p2), f"max |diff| {float((p1 - p2).abs().max()):.3e}"
    for k in STAT_KEYS:
        assert s1[k] == s2[k], (k, s1[k], s2[k])


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("shape,gamma", [((512, 512), 1e-4), ((300, 280), 2e-4), ((270, 512), 1e-4),
                                         ((512, 300), 1.5e-4)])
def test_gibbs_apply_matches_oracle(shape, gamma, precision):
    banner(f"tiles32 gibbs {shape} gamma={gamma} {precision}")
    rng = np.random.default_rng(21)
    x = rng.uniform(0.0, 1.0, size=shape) * np.exp(rng.normal(0, 2, size=shape))
    y = jk.gibbs_apply(dev(x), gamma, precision)
    ref = O.gibbs_apply(f32(x).astype(np.float64), gamma)
    err = rel_l1(host64(y), ref)
    print(f"[gpu-test] tiles32 gibbs {shape} {precision}: rel-L1 {err:.2e}", flush=True)
    assert err <= GIBBS_TOL[precision]


def _case(shape, seed=6):
    return small_case(shape, "congestion", seed=seed, gamma=2e-4, tau=2e-3, n_boxes=3)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_flow_matches_oracle(precision):
    """Congestion with obstacles on a ragged 300 x 280 grid, 2 steps x 60
    iterations (resident kernel)."""
    banner(f"tiles32 flow 300x280 {precision}")
    wl = _case((300, 280))
    g_en, o_en = energies(wl)
    pT, stats, _ = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, 2, max_iters=60, precision=precision)
    q = f32(wl.p0).astype(np.float64)
    for _ in range(2):
        q, ost = O.jko_step(q, o_en, wl.gamma, wl.tau, 60)
    err = rel_l1(host64(pT), q)
    print(f"[gpu-test] tiles32 flow {precision}: rel-L1 {err:.2e}", flush=True)
    assert err <= TOL[precision]
    assert stats[-1]["marginal_l1"] == pytest.approx(ost["marginal_l1"], rel=1e-3)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("name,kw", [("porous512_scaled", dict(max_iters=300, tol=1e-6, check_every=10)),
                                     ("gen512", dict(max_iters=120, tol=0.0, check_every=10)),
                                     ("ragged", dict(max_iters=200, tol=1e-7, check_every=7))])
def test_resident_same_bits_as_launch_path(name, kw, precision):
    """512^2 nonlinear diffusion (tolerance mode) and the generalised
    entropies (both on the resident pass kernel against the launched passes:
    512 is a multiple of 32), and ragged congestion (32 x 32 tiles): resident
    and launch paths give the same bits and statistics."""
    banner(f"tiles32 resident vs launch {name} {precision}")
    wl = _case((300, 280)) if name == "ragged" else make_workload(name)
    _same(*_both(wl, precision=precision, **kw))


def test_absorption_switch_hands_over_the_same_bits():
    """A switch to the log domain at a check: the resident kernel returns and
    the step continues on the log-domain passes, as the launch path does."""
    banner("tiles32 absorption switch")
    wl = small_case((300, 280), "congestion", seed=6, gamma=2e-4, tau=2e-3, n_boxes=3, projected=False)
    res, ref = _both(wl, max_iters=120, check_every=10, absorb_threshold=50.0)
    _same(res, ref)
    assert res[1]["absorptions"] == 1


def test_adjoint_matches_autograd_and_launch_path():
    """dL/dw and dL/dp0 through 2 steps x 30 iterations on the 300 x 280 grid:
    the resident reverse sweep equals the launch path's bit for bit, and both
    match FP64 autograd."""
    banner("tiles32 adjoint")
    wl = _case((300, 280))
    g_en, o_en = energies(wl)
    rng = np.random.default_rng(3)
    target = rng.uniform(size=wl.shape)
    target /= target.sum()
    outs = []
    for resident in (True, False):
        pT, _, ck = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, 2, max_iters=30, checkpoints=True,
                            resident=resident)
        dL = (2.0 * (pT - dev(target))).contiguous()
        outs.append(jk.backward(ck, [30, 30], dL, g_en, wl.gamma, wl.tau, resident=resident))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    _, rw, rp, _ = loss_and_grads(f32(wl.p0).astype(np.float64), o_en._w(wl.shape), o_en._kappa(wl.shape),
                                  wl.gamma, wl.tau, [30, 30], target)
    ew = np.linalg.norm(host64(outs[0][0]) - rw) / np.linalg.norm(rw)
    ep = np.linalg.norm(host64(outs[0][1]) - rp) / np.linalg.norm(rp)
    print(f"[gpu-test] tiles32 adjoint: rel err dL/dw {ew:.2e}, dL/dp0 {ep:.2e}", flush=True)
    assert ew <= 1e-3 and ep <= 1e-3
