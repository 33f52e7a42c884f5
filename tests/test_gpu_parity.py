"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances (relative L1 on densities): 1e-5 for FP32 contractions, 1e-4 for
split-BF16; Gibbs products alone: 1e-6 / 2e-5 (rel-L1).  Whole flows also
meet a per-cell bound (1e-4 / 2e-3 of each cell's value, cells under 1e-3
of the largest measured against that floor), so that an error concentrated
on a few cells (an obstacle's edge) cannot hide in the aggregate.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_1502_06216_amd as jk
from workloads import make_workload, small_case, gaussian_bumps

from _util import CELL_TOL, banner, cell_err, dev, energies, f32, host64, rel_l1

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_bf16": 1e-4}
# absolute slack on the reported marginal violation near its rounding floor
MONITOR_ABS = {"fp32": 2e-7, "split_bf16": 3e-6}
GIBBS_TOL = {"fp32": 1e-6, "split_bf16": 2e-5}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


# ------------------------------------------------------------- Gibbs products

@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("shape,gamma", [((37,), 4e-3), ((50, 70), 2e-3), ((64, 64), 1e-3),
                                         ((20, 24, 36), 5e-3), ((33, 17, 40), 1e-2), ((256, 256), 2e-4),
                                         ((130, 6), 3e-2), ((1, 96), 1e-3), ((96, 1), 1e-3)])
def test_gibbs_apply_matches_oracle(shape, gamma, precision):
    banner(f"gibbs {shape} gamma={gamma} {precision}")
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 1.0, size=shape) * np.exp(rng.normal(0, 2, size=shape))
    y = jk.gibbs_apply(dev(x), gamma, precision)
    ref = O.gibbs_apply(f32(x).astype(np.float64), gamma)
    assert rel_l1(host64(y), ref) <= GIBBS_TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_gibbs_apply_structured_inputs(precision):
    """Bumps with exact zeros and tiny tails."""
    shape = (96, 80)
    x = gaussian_bumps(shape, [(0.3, 0.4), (0.7, 0.6)], 0.05, [0.5, 0.5])
    x[x < 1e-30] = 0.0
    x[10:20, :] = 0.0
    y = jk.gibbs_apply(dev(x), 1e-3, precision)
    ref = O.gibbs_apply(f32(x).astype(np.float64), 1e-3)
    assert rel_l1(host64(y), ref) <= GIBBS_TOL[precision]
    assert (host64(y) >= 0).all()


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_gibbs_apply_128cube_sampled(precision):
    """Full-size 3D grid: sampled outputs against the plain sum over all cells."""
    shape = (128, 128, 128)
    gamma = 5e-4
    banner(f"gibbs 128^3 sampled {precision}")
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 1.0, size=shape).astype(np.float32).astype(np.float64)
    y = host64(jk.gibbs_apply(dev(x), gamma, precision)).ravel()
    idx = rng.choice(x.size, size=48, replace=False)
    ref = O.gibbs_rows(shape, gamma, idx, x)
    assert rel_l1(y[idx], ref) <= GIBBS_TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_gibbs_apply_largest_axes(precision):
    """The largest axis the boundary accepts (1024): a full 1D product, and
    sampled outputs of a 1024 x 1024 grid against the plain sum."""
    banner(f"gibbs largest axes {precision}")
    rng = np.random.default_rng(21)
    x1 = rng.uniform(0.0, 1.0, size=(1024,)) * np.exp(rng.normal(0, 2, size=(1024,)))
    y1 = jk.gibbs_apply(dev(x1), 1e-4, precision)
    assert rel_l1(host64(y1), O.gibbs_apply(f32(x1).astype(np.float64), 1e-4)) <= GIBBS_TOL[precision]
    shape = (1024, 1024)
    x = rng.uniform(0.0, 1.0, size=shape).astype(np.float32).astype(np.float64)
    y = host64(jk.gibbs_apply(dev(x), 2e-5, precision)).ravel()
    idx = np.concatenate([[0, 1023, 1024 * 1023, x.size - 1], rng.choice(x.size, size=28, replace=False)])
    ref = O.gibbs_rows(shape, 2e-5, idx, x)
    assert rel_l1(y[idx], ref) <= GIBBS_TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_step_on_the_largest_2d_grid(precision):
    """A few iterations of a congestion step on 1024 x 1024 against the oracle.
    At this gamma the bumps' tails leave scalings in the float32 denormal
    range, which the split-BF16 products do not keep (s rounds to 0, a to 0,
    t to 0 and b = q / t overflows: reported as non-finite); the split run
    therefore uses the log domain, whose result equals the plain iteration's."""
    banner(f"step 1024^2 {precision}")
    wl = small_case((1024, 1024), "congestion", seed=12)
    g_en, o_en = energies(wl)
    thr = 0.0 if precision == "split_bf16" else float("inf")
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=6, precision=precision, absorb_threshold=thr)
    ref, _ = O.jko_step(f32(wl.p0).astype(np.float64), o_en, wl.gamma, wl.tau, 6)
    err = rel_l1(host64(p), ref)
    print(f"[gpu-test] accuracy 1024^2 6 it {precision}: rel-L1 vs FP64 oracle {err:.3e}", flush=True)
    assert err <= TOL[precision]


def test_gibbs_apply_deterministic():
    x = dev(np.random.default_rng(0).uniform(size=(130, 70)))
    y1 = jk.gibbs_apply(x, 2e-3)
    y2 = jk.gibbs_apply(x, 2e-3)
    assert torch.equal(y1, y2)


# ------------------------------------------------------------- whole flows

def _flow_parity(wl, precision, n_steps, iters, tol=None):
    g_en, o_en = energies(wl)
    p0 = f32(wl.p0).astype(np.float64)
    pT, stats, ck = jk.flow(dev(wl.p0), g_en, wl.gamma, wl.tau, n_steps, max_iters=iters,
                            precision=precision, checkpoints=True)
    ck = host64(ck)
    q = p0
    errs = []
    for t in range(n_steps):
        # the device checkpoints are the inputs of each step
        if t > 0:
            errs.append(rel_l1(ck[t], q))
        q, st = O.jko_step(q, o_en, wl.gamma, wl.tau, iters)
        assert stats[t]["iters"] == iters
        assert stats[t]["marginal_l1"] == pytest.approx(st["marginal_l1"], rel=0.05, abs=MONITOR_ABS[precision])
    errs.append(rel_l1(host64(pT), q))
    return errs, stats, host64(pT), q


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("projected", [True, False])
def test_crowd32_flow_matches_oracle(precision, projected):
    """32x32 crowd motion, 10 JKO steps x 300 iterations (paper Listing 1)."""
    banner(f"crowd32 projected={projected} {precision}")
    wl = make_workload("crowd32", projected=projected)
    errs, stats, p, ref = _flow_parity(wl, precision, wl.n_steps, wl.max_iters)
    ce = cell_err(p, ref)
    print(f"[gpu-test] crowd32 projected={projected} {precision}: rel-L1 {max(errs):.2e}, per cell {ce:.2e}",
          flush=True)
    assert max(errs) <= TOL[precision], errs
    assert ce <= CELL_TOL[precision]
    assert (p <= np.float32(wl.kappa_scalar)).all()


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("shape", [(45, 70), (20, 24, 36), (100,)])
def test_ragged_congestion_matches_oracle(shape, precision):
    banner(f"ragged congestion {shape} {precision}")
    wl = small_case(shape, "congestion", seed=2)
    errs, stats, p, ref = _flow_parity(wl, precision, 2, 60)
    ce = cell_err(p, ref)
    print(f"[gpu-test] ragged congestion {shape} {precision}: rel-L1 {max(errs):.2e}, per cell {ce:.2e}", flush=True)
    assert max(errs) <= TOL[precision], errs
    assert ce <= CELL_TOL[precision]
    assert (p <= f32(wl.kappa_field()) + 0).all()


@pytest.mark.parametrize("kind", ["entropy", "porous", "zero"])
@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_other_energies_match_oracle(kind, precision):
    banner(f"energy {kind} {precision}")
    wl = small_case((48, 40), kind, seed=4)
    if kind == "porous":
        wl.density_scale = float(np.prod(wl.shape))   # Newton regime k s^{m-1} >> 1
    errs, stats, p, ref = _flow_parity(wl, precision, 2, 40)
    ce = cell_err(p, ref)
    print(f"[gpu-test] energy {kind} {precision}: rel-L1 {max(errs):.2e}, per cell {ce:.2e}", flush=True)
    assert max(errs) <= TOL[precision], errs
    assert ce <= CELL_TOL[precision]


def test_porous512_literal_and_scaled_one_step():
    for name in ("porous512", "porous512_scaled"):
        banner(name)
        wl = make_workload(name)
        g_en, o_en = energies(wl)
        p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=20)
        ref, ost = O.jko_step(f32(wl.p0).astype(np.float64), o_en, wl.gamma, wl.tau, 20)
        assert rel_l1(host64(p), ref) <= TOL["fp32"]


def test_tolerance_mode_stops_like_the_oracle():
    wl = make_workload("crowd32", projected=True)
    g_en, o_en = energies(wl)
    tol, ce = 1e-6, 10
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=3000, tol=tol, check_every=ce)
    ref, ost = O.jko_step(f32(wl.p0).astype(np.float64), o_en, wl.gamma, wl.tau, 3000, tol=tol,
                          check_every=ce)
    assert st["stop"] == "tol" and ost["stop"] == "tol"
    assert st["iters"] % ce == 0
    assert abs(st["iters"] - ost["iters"]) <= ce
    assert st["marginal_l1"] <= tol
    ref_same, _ = O.jko_step(f32(wl.p0).astype(np.float64), o_en, wl.gamma, wl.tau, st["iters"])
    assert rel_l1(host64(p), ref_same) <= TOL["fp32"]


def test_mass_and_capacity_invariants():
    wl = make_workload("crowd32", projected=False)
    g_en, _ = energies(wl)
    q = dev(wl.p0)
    for _ in range(3):
        p, st = jk.step(q, g_en, wl.gamma, wl.tau, max_iters=300)
        ph = host64(p)
        assert ph.min() >= 0.0
        assert (ph <= np.float32(wl.kappa_scalar)).all()
        assert abs(ph.sum() - host64(q).sum()) <= st["marginal_l1"] + 1e-6
        assert st["mass"] == pytest.approx(ph.sum(), rel=1e-6)
        q = p


def test_errors_are_reported():
    wl = make_workload("crowd32", projected=True)
    g_en, _ = energies(wl)
    g_en.kappa_scalar = 0.5 / 1024          # capacity holds half the mass
    with pytest.raises(jk.JKOError) as e:
        jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=10)
    assert e.value.status == jk.JKO_ERR_INFEASIBLE
    g_en, _ = energies(wl)
    p = dev(wl.p0)
    p[3, 4] = float("nan")
    with pytest.raises(jk.JKOError) as e:
        jk.step(p, g_en, wl.gamma, wl.tau, max_iters=10)
    assert e.value.status == jk.JKO_ERR_NONFINITE


# ------------------------------------------------------------- closed forms

def _moments(p, x):
    m = (p * x).sum() / p.sum()
    return m, (p * (x - m) ** 2).sum() / p.sum()


@pytest.mark.parametrize("absorb", [math.inf, 0.0])
def test_heat_flow_gaussian_on_gpu(absorb):
    """Entropy energy on a 256x256 product Gaussian (plain scalings, and the log
    domain from the first iteration): parity with the FP64 oracle at the same
    iteration count, and each axis's variance against the closed-form heat-flow
    recursion (within the truncation of the bounded domain, 1e-3)."""
    n, gamma, tau, S0 = 256, 1e-3, 2e-3, 1e-2
    x = (np.arange(n) + 0.5) / n
    g1 = np.exp(-(x - 0.5) ** 2 / (2 * S0))
    p = np.outer(g1, g1)
    p /= p.sum()
    ref = f32(p).astype(np.float64)
    S = _moments(ref.sum(1), x)[1]
    q = dev(p)
    en = jk.EnergySpec(kind="entropy")
    oen = O.Energy(kind="entropy")
    for _ in range(2):
        q, st = jk.step(q, en, gamma, tau, max_iters=600, absorb_threshold=absorb)
        ref, _ = O.jko_step(ref, oen, gamma, tau, 600)
        u = ((gamma + 2 * S) + math.sqrt((gamma + 2 * S) ** 2 + 8 * tau * S)) / 2
        S = (u + tau) / 2
        ph = host64(q)
        assert rel_l1(ph, ref) <= TOL["fp32"]
        assert _moments(ph.sum(1), x)[1] == pytest.approx(S, rel=1e-3)
        assert _moments(ph.sum(0), x)[1] == pytest.approx(S, rel=1e-3)


def test_ornstein_uhlenbeck_on_gpu():
    n, gamma, tau, lam, c = 512, 2e-4, 2e-3, 1.0, 0.7
    x = (np.arange(n) + 0.5) / n
    p = np.exp(-(x - 0.4) ** 2 / (2 * 2e-3))
    p /= p.sum()
    mu, S = _moments(f32(p).astype(np.float64), x)
    en = jk.EnergySpec(kind="congestion", w=dev(lam * (x - c) ** 2))
    q = dev(p)
    for _ in range(4):
        q, st = jk.step(q, en, gamma, tau, max_iters=3)
        mu = (mu + tau * lam * c) / (1 + tau * lam)
        S = S / (1 + tau * lam) ** 2 + gamma / (2 * (1 + tau * lam))
        m_, v_ = _moments(host64(q), x)
        assert m_ == pytest.approx(mu, rel=1e-5)
        assert v_ == pytest.approx(S, rel=1e-4)


# ------------------------------------------------------------- full sizes

@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_crowd256_one_step_full_size(precision):
    """The 256x256 crowd workload at its full size, one step of 300 iterations."""
    banner(f"crowd256 full {precision}")
    wl = make_workload("crowd256_fixed")
    g_en, o_en = energies(wl)
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=300, precision=precision)
    ref, ost = O.jko_step(f32(wl.p0).astype(np.float64), o_en, wl.gamma, wl.tau, 300)
    err = rel_l1(host64(p), ref)
    print(f"[gpu-test] accuracy crowd256 300 it {precision}: rel-L1 vs FP64 oracle {err:.3e}", flush=True)
    assert err <= TOL[precision]
    assert st["marginal_l1"] == pytest.approx(ost["marginal_l1"], rel=0.05)


_REF128 = {}


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_crowd128c_few_iterations_full_size(precision):
    """The 128^3 workload at full size (panel-form passes), 8 iterations."""
    banner(f"crowd128c full, 8 iterations, {precision}")
    wl = make_workload("crowd128c")
    g_en, o_en = energies(wl)
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=8, precision=precision)
    if "ref" not in _REF128:
        _REF128["ref"] = O.jko_step(f32(wl.p0).astype(np.float64), o_en, wl.gamma, wl.tau, 8)[0]
    err = rel_l1(host64(p), _REF128["ref"])
    print(f"[gpu-test] accuracy crowd128c 8 it {precision}: rel-L1 vs FP64 oracle {err:.3e}", flush=True)
    assert err <= TOL[precision]


# ------------------------------------------------------------- log domain

@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("threshold", [0.0, 50.0])
def test_log_domain_matches_plain_oracle(threshold, precision):
    """Absorbing the scalings (from the start, or at the first check above 50)
    gives the plain iteration's result where that one stays finite."""
    banner(f"log domain thr={threshold} {precision}")
    wl = make_workload("crowd32", projected=False)
    g_en, o_en = energies(wl)
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=300, check_every=10,
                    absorb_threshold=threshold, precision=precision)
    ref, _ = O.jko_step(f32(wl.p0).astype(np.float64), o_en, wl.gamma, wl.tau, 300)
    assert st["absorptions"] == 1
    assert rel_l1(host64(p), ref) <= TOL[precision]
    ph = host64(p)
    assert (ph <= np.float32(wl.kappa_scalar)).all() and ph.min() >= 0


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_log_domain_survives_where_plain_fp32_overflows(precision):
    """Small gamma, literal bump mixture far above the capacity: the plain FP32
    scalings overflow.  The absorbed iteration stays finite, keeps the
    invariants and matches the exact log-sum-exp oracle (each log-domain
    product shifts every output by its own largest term and assumes no
    band)."""
    banner(f"log domain stress {precision}")
    wl = small_case((64, 64), "congestion", seed=1, gamma=2e-4, tau=2e-3, n_boxes=3, projected=False,
                    cap_factor=1.2)
    g_en, o_en = energies(wl)
    iters = 60
    with pytest.raises(jk.JKOError):
        jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=iters)   # NONFINITE in plain FP32
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=iters, check_every=5, absorb_threshold=0.0,
                    precision=precision)
    ph = host64(p)
    assert np.isfinite(ph).all() and np.isfinite(st["marginal_l1"])
    assert ph.min() >= 0 and (ph <= f32(wl.kappa_field())).all()
    ref, ost = O.jko_step_log(f32(wl.p0).astype(np.float64), o_en, wl.gamma, wl.tau, iters)
    err = rel_l1(ph, ref)
    print(f"[gpu-test] log-domain stress {precision}: rel-L1 vs exact LSE oracle {err:.3e}, "
          f"marginal {st['marginal_l1']:.3e} (oracle {ost['marginal_l1']:.3e})", flush=True)
    assert err <= TOL[precision]
    assert st["marginal_l1"] == pytest.approx(ost["marginal_l1"], rel=1e-3)


# ------------------------------------------------------------- adjoint

def _adjoint_case(shape_name, n_steps, iters):
    if shape_name == "crowd32":
        wl = make_workload("crowd32", projected=True)
    else:
        wl = make_workload("crowd256_fixed")
    rng = np.random.default_rng(7)
    N = wl.N
    ex = wl.extras["exit"]
    from workloads import gaussian_bumps as gb
    target = gb(wl.shape, [ex - np.array([0.1, 0.0])], 0.05, [1.0])
    mask = wl.extras["mask"]
    target[mask] = 0.0
    target /= target.sum()
    return wl, target


@pytest.mark.parametrize("name,n_steps,iters", [("crowd32", 3, 50), ("crowd256", 2, 60)])
def test_adjoint_matches_fp64_autograd(name, n_steps, iters):
    """dL/dw and dL/dp0 of L = ||p_T - target||^2 from the hand-written adjoint
    (recompute from per-step checkpoints, reverse sweep) against torch float64
    autograd through the oracle's unrolled iteration."""
    from oracle.grad import loss_and_grads
    banner(f"adjoint {name} {n_steps}x{iters}")
    wl, target = _adjoint_case(name, n_steps, iters)
    g_en, o_en = energies(wl)
    p0 = dev(wl.p0)
    pT, _, ck = jk.flow(p0, g_en, wl.gamma, wl.tau, n_steps, max_iters=iters, checkpoints=True)
    dL = 2.0 * (pT - dev(target))
    gw, gp = jk.backward(ck, [iters] * n_steps, dL.contiguous(), g_en, wl.gamma, wl.tau)
    kap = wl.kappa_field()
    loss, rw, rp, _ = loss_and_grads(f32(wl.p0).astype(np.float64), f32(wl.w).astype(np.float64),
                                     f32(kap).astype(np.float64), wl.gamma, wl.tau, [iters] * n_steps, target)
    ew = np.linalg.norm(host64(gw) - rw) / np.linalg.norm(rw)
    ep = np.linalg.norm(host64(gp) - rp) / np.linalg.norm(rp)
    print(f"[gpu-test] adjoint {name}: rel err dL/dw {ew:.2e}, dL/dp0 {ep:.2e}", flush=True)
    assert ew <= 1e-3 and ep <= 1e-3


def test_autograd_function_and_directional_derivative():
    """JKOFlowFn.backward equals the library gradient, and <grad, d> matches a
    central difference of the GPU forward along a random direction d (no
    capacity, so the flow is smooth in w)."""
    banner("autograd fn")
    wl, target = _adjoint_case("crowd32", 2, 40)
    g_en, _ = energies(wl)
    g_en.kappa_scalar = math.inf
    w = dev(wl.w).requires_grad_(True)
    p0 = dev(wl.p0).requires_grad_(True)
    kap = torch.full(wl.shape, math.inf, dtype=torch.float32, device="cuda")
    tgt = dev(target)
    pT = jk.JKOFlowFn.apply(p0, w, kap, wl.gamma, wl.tau, 2, 40, "fp32")
    loss = ((pT - tgt) ** 2).sum()
    loss.backward()
    d = torch.from_numpy(np.random.default_rng(3).standard_normal(wl.shape).astype(np.float32)).cuda()
    h = 2e-3

    def L(wv):
        with torch.no_grad():
            out = jk.JKOFlowFn.apply(p0.detach(), wv, kap, wl.gamma, wl.tau, 2, 40, "fp32")
            return float(((out.double() - tgt.double()) ** 2).sum())

    fd = (L(w.detach() + h * d) - L(w.detach() - h * d)) / (2 * h)
    an = float((w.grad.double() * d.double()).sum())
    assert an == pytest.approx(fd, rel=1e-2)
    # the autograd path returns the library's gradient
    ck = jk.flow(p0.detach(), g_en, wl.gamma, wl.tau, 2, max_iters=40, checkpoints=True)[2]
    gw, gp = jk.backward(ck, [40, 40], (2.0 * (pT.detach() - tgt)).contiguous(), g_en, wl.gamma, wl.tau)
    assert torch.allclose(w.grad, gw, rtol=1e-5, atol=1e-12)
    assert torch.allclose(p0.grad, gp, rtol=1e-5, atol=1e-12)


def test_crowd256_literal_log_domain_stress():
    """The literal 256x256 crowd (bump mixture 26x above the capacity): plain
    FP32 scalings overflow (near iteration 43); the log-domain iteration (log
    form from the start) stays finite, keeps 0 <= p <= kappa and, after 300
    iterations, matches the exact FP64 log-sum-exp oracle's step (stored in
    tests/golden/log_references.npz by make_log_references.py, which calls
    only the oracle)."""
    import importlib.util
    import os
    banner("crowd256 literal, log domain, 300 iterations")
    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_log_references", os.path.join(gdir, "make_log_references.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with np.load(os.path.join(gdir, "log_references.npz"), allow_pickle=False) as z:
        ref = z["crowd256_literal_p"]
        iters = int(z["crowd256_literal_iters"])
        ref_marginal = float(z["crowd256_literal_marginal"])
        ref_mass = float(z["crowd256_literal_mass"])
        ref_digest = str(z["crowd256_literal_digest"])
    wl, p0, o_en = mod.inputs()
    assert mod.digest(wl, p0, o_en) == ref_digest, "workload changed since the golden file"
    g_en, _ = energies(wl)
    with pytest.raises(jk.JKOError) as e:
        jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=80)
    assert e.value.status == jk.JKO_ERR_NONFINITE
    p, st = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=iters, check_every=10, absorb_threshold=0.0)
    ph = host64(p)
    assert np.isfinite(ph).all() and np.isfinite(st["marginal_l1"])
    assert ph.min() >= 0 and (ph <= f32(wl.kappa_field())).all()
    err = rel_l1(ph, ref)
    print(f"[gpu-test] crowd256 literal log domain, {iters} iterations: rel-L1 vs exact LSE oracle {err:.3e}, "
          f"marginal {st['marginal_l1']:.4e} (oracle {ref_marginal:.4e}), mass {st['mass']:.6f} "
          f"(oracle {ref_mass:.6f})", flush=True)
    assert err <= TOL["fp32"]
    assert st["marginal_l1"] == pytest.approx(ref_marginal, rel=1e-4)
