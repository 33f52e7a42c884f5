"""The heat-kernel Gibbs operator of Section 4.1 (eq. heat-kernel) on masked
2D grids, on the HIP path against the FP64 oracle (sparse LU solves),
through the C ABI.

Up to 2^16 cells the library stores xi~ as a dense float32 matrix built on
the device by FP64 Chebyshev solves; each product is one matrix-vector pass
in float32.  Above (or on request) each product is the paper's L implicit
solves, by FP64 Chebyshev stencil sweeps on the grid.  Tolerances: the
operator 1e-6 (rel-L1 of a product: float32 entries and float32 sums), the
flows 1e-5 (rel-L1 of the density, as for the Gaussian kernel).
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1502_06216_amd as jk
from workloads import heat_room, make_workload, project_capacity

from _util import banner, dev, energies, f32, host64, rel_l1

pytestmark = pytest.mark.gpu

TOL_OP = 1e-6
TOL_FLOW = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _mask_dev(mask):
    return None if mask is None else torch.from_numpy(np.ascontiguousarray(mask.astype(np.uint8))).cuda()


def _op(wl):
    return jk.HeatOperator(wl.shape, wl.gamma, wl.heat_L, mask=_mask_dev(wl.mask))


def _room(shape, seed=3, kind="congestion", bind=True):
    """A room of the given shape; with bind, the capacity is half the peak of
    the initial density (projected under it) so that congestion is active."""
    wl = heat_room(*shape, seed=seed, n_steps=2, max_iters=30)
    if kind == "congestion" and bind:
        wl.kappa_scalar = 0.5 * wl.p0.max()
        wl.p0 = project_capacity(wl.p0, wl.kappa_scalar)
    elif kind != "congestion":
        # tau = 2.5 gamma as for the Gaussian-kernel small cases: at the crowd's
        # tau = 20 gamma an entropy's prox s^{1/(1 + sigma c)} stays far above
        # the kernel's float32 tail and a = p / s overflows (no log domain here)
        wl.kind = kind
        wl.tau = 2.5 * wl.gamma
        wl.w = None
        wl.kappa_scalar = np.inf
        rng = np.random.default_rng(seed)
        wl.coef = np.where(wl.mask, 1.0 + 0.5 * rng.uniform(size=wl.shape), 1.0)
        wl.m = 2.0
    return wl


@pytest.mark.parametrize("shape,masked", [((24, 20), True), ((48, 40), True), ((33, 29), False), ((1, 37), False),
                                          ((64, 50), True)])
def test_operator_matches_oracle(shape, masked):
    banner(f"heat operator {shape} masked={masked}")
    if masked:
        wl = heat_room(*shape, seed=2)
        mask, gamma, L = wl.mask, wl.gamma, wl.heat_L
    else:
        mask, gamma, L = np.ones(shape, bool), 10.0 / max(shape) ** 2, 10
    op = jk.HeatOperator(shape, gamma, L, mask=_mask_dev(mask) if masked else None)
    H = O.HeatKernel(mask, gamma, L)
    rng = np.random.default_rng(7)
    x = np.where(mask, rng.uniform(size=shape), 0.0)
    y = host64(op.apply(dev(x)))
    ref = H(f32(x).astype(np.float64))
    err = rel_l1(y, ref)
    print(f"[gpu-test] heat operator {shape}: rel-L1 {err:.2e}", flush=True)
    assert err <= TOL_OP
    assert np.abs(y - ref).max() <= TOL_OP * np.abs(ref).max() * 10
    assert not y[~mask].any()
    assert y.sum() == pytest.approx(f32(x).astype(np.float64).sum(), rel=1e-6)


def test_operator_columns_are_the_oracle_matrix():
    """Every column of xi~ on a small room (unit inputs), against the oracle's
    dense matrix entry by entry (absolute 1e-7: float32 entries of size <= 1)."""
    banner("heat operator columns")
    wl = heat_room(12, 10, seed=1)
    op = _op(wl)
    D = O.HeatKernel(wl.mask, wl.gamma, wl.heat_L).dense()
    N = wl.mask.size
    eye = torch.eye(N, dtype=torch.float32, device="cuda")
    cols = np.stack([host64(op.apply(eye[j].reshape(wl.shape).contiguous())).ravel() for j in range(N)], axis=1)
    cols[:, ~wl.mask.ravel()] = 0.0    # columns of obstacles: inputs there are ignored
    np.testing.assert_allclose(cols, D, rtol=0, atol=1e-7)


def _oracle_flow(wl, o_en, steps, iters, tol=0.0, check_every=1):
    H = O.HeatKernel(wl.mask, wl.gamma, wl.heat_L)
    q = f32(wl.p0).astype(np.float64)
    sts = []
    for _ in range(steps):
        q, st = O.jko_step(q, o_en, wl.gamma, wl.tau, iters, tol=tol, check_every=check_every, op=H)
        sts.append(st)
    return q, sts


@pytest.mark.parametrize("kind", ["congestion", "zero", "entropy", "porous"])
@pytest.mark.parametrize("shape", [(24, 20), (48, 40)])
def test_flow_matches_oracle(shape, kind):
    banner(f"heat flow {shape} {kind}")
    wl = _room(shape, kind=kind)
    g_en, o_en = energies(wl)
    op = _op(wl)
    pT, stats = op.flow(dev(wl.p0), g_en, wl.tau, 2, max_iters=30)
    ref, rst = _oracle_flow(wl, o_en, 2, 30)
    err = rel_l1(host64(pT), ref)
    print(f"[gpu-test] heat flow {shape} {kind}: rel-L1 {err:.2e}, marginal {stats[-1]['marginal_l1']:.3e} "
          f"vs {rst[-1]['marginal_l1']:.3e}", flush=True)
    assert err <= TOL_FLOW
    assert not host64(pT)[~wl.mask].any()
    assert stats[-1]["mass"] == pytest.approx(float(host64(pT).sum()), rel=1e-5)
    assert stats[-1]["marginal_l1"] == pytest.approx(rst[-1]["marginal_l1"], rel=0.05, abs=1e-6)
    if kind == "congestion":
        assert (host64(pT) <= np.float32(wl.kappa_scalar) * (1 + 1e-6)).all()


def test_tolerance_mode_stops_like_the_oracle():
    banner("heat tolerance mode")
    wl = _room((48, 40))
    g_en, o_en = energies(wl)
    op = _op(wl)
    tol, ce = 1e-6, 10
    p, st = op.step(dev(wl.p0), g_en, wl.tau, max_iters=3000, tol=tol, check_every=ce)
    ref, ost = _oracle_flow(wl, o_en, 1, 3000, tol=tol, check_every=ce)
    ost = ost[0]
    print(f"[gpu-test] heat tolerance: device {st['iters']} iterations, oracle {ost['iters']}", flush=True)
    assert st["stop"] == "tol" and ost["stop"] == "tol"
    assert st["iters"] % ce == 0 and abs(st["iters"] - ost["iters"]) <= ce
    assert st["marginal_l1"] <= tol
    same, _ = _oracle_flow(wl, o_en, 1, st["iters"])
    assert rel_l1(host64(p), same) <= TOL_FLOW


def test_binary_congestion_on_the_heat_kernel():
    """The non-convex {0, kappa} constraint with xi~: binary values and the
    oracle's decisions in all but a few near-tie cells after one iteration."""
    banner("heat binary congestion")
    wl = _room((48, 40), bind=False)
    wl.kind = "binary_congestion"
    wl.w = wl.w * (0.5 / ((wl.tau / wl.gamma) * float(wl.w.max())))
    g_en, o_en = energies(wl)
    op = _op(wl)
    p, _ = op.step(dev(wl.p0), g_en, wl.tau, max_iters=1)
    ref, _ = _oracle_flow(wl, o_en, 1, 1)
    p = host64(p)
    k = np.float32(wl.kappa_scalar)
    assert np.all((p == 0) | (p == k))
    assert float(np.mean((p > 0) != (ref > 0))) <= 0.01


def test_overflow_is_reported():
    """The plain-domain limit: entropy at sigma c ~ 25 overflows a = p / s in
    float32 on the kernel's tail; the library reports JKO_ERR_NONFINITE."""
    banner("heat overflow reported")
    wl = _room((24, 20), kind="entropy")
    wl.tau = 20.0 * wl.gamma
    g_en, _ = energies(wl)
    op = _op(wl)
    with pytest.raises(jk.JKOError) as e:
        op.flow(dev(wl.p0), g_en, wl.tau, 1, max_iters=30)
    assert e.value.status == jk.JKO_ERR_NONFINITE


def test_refusals():
    banner("heat refusals")
    wl = _room((24, 20))
    g_en, _ = energies(wl)
    op = _op(wl)
    on_wall = wl.p0.copy()
    on_wall[~wl.mask] = 1e-3
    with pytest.raises(jk.JKOError) as e:
        op.flow(dev(on_wall), g_en, wl.tau, 1, max_iters=5)
    assert e.value.status == jk.JKO_ERR_NONFINITE
    tight = jk.EnergySpec(kind="congestion", kappa_scalar=1e-6)
    with pytest.raises(jk.JKOError) as e:
        op.flow(dev(wl.p0), tight, wl.tau, 1, max_iters=5)
    assert e.value.status == jk.JKO_ERR_INFEASIBLE
    other = jk.HeatOperator(wl.shape, wl.gamma, wl.heat_L, mask=_mask_dev(wl.mask))
    other.gamma = 2.0 * wl.gamma             # params ask another gamma than the operator was built for
    with pytest.raises(jk.JKOError) as e:
        other.flow(dev(wl.p0), g_en, wl.tau, 1, max_iters=5)
    assert e.value.status == jk.JKO_ERR_INVALID and "gamma" in str(e.value)


def test_heat100_one_step_full_size():
    """The benchmarked configuration (100^2 room, L = 10, 300 iterations) for
    one step against the oracle."""
    banner("heat100 one step")
    wl = make_workload("heat100")
    g_en, o_en = energies(wl)
    op = _op(wl)
    p, st = op.step(dev(wl.p0), g_en, wl.tau, max_iters=wl.max_iters)
    ref, rst = _oracle_flow(wl, o_en, 1, wl.max_iters)
    err = rel_l1(host64(p), ref)
    print(f"[gpu-test] heat100: rel-L1 {err:.2e}, marginal {st['marginal_l1']:.3e} vs {rst[0]['marginal_l1']:.3e}",
          flush=True)
    assert err <= TOL_FLOW


def test_largest_grid():
    """The largest grid of the stored operator (2^16 cells: a 256 x 256 room,
    512 tiles a side, an 8.6 GB operator): a product and a 10-iteration
    step against the oracle."""
    banner("heat largest grid 256x256")
    wl = heat_room(256, 256, seed=5)
    op = _op(wl)
    H = O.HeatKernel(wl.mask, wl.gamma, wl.heat_L)
    rng = np.random.default_rng(11)
    x = np.where(wl.mask, rng.uniform(size=wl.shape), 0.0)
    y = host64(op.apply(dev(x)))
    err = rel_l1(y, H(f32(x).astype(np.float64)))
    g_en, o_en = energies(wl)
    p, st = op.step(dev(wl.p0), g_en, wl.tau, max_iters=10)
    q = f32(wl.p0).astype(np.float64)
    ref, rst = O.jko_step(q, o_en, wl.gamma, wl.tau, 10, op=H)
    errf = rel_l1(host64(p), ref)
    print(f"[gpu-test] heat 256x256: operator rel-L1 {err:.2e}, step rel-L1 {errf:.2e}", flush=True)
    assert err <= TOL_OP
    assert errf <= TOL_FLOW
    assert st["marginal_l1"] == pytest.approx(rst["marginal_l1"], rel=0.01)


def test_degenerate_domains():
    """A single free cell (xi~ is the identity there: a step keeps the
    density), a grid without obstacles (mask NULL) with L = 1, and a domain
    cut in two by a wall (no mass crosses it), each against the oracle."""
    banner("heat degenerate domains")
    # one free cell
    mask = np.zeros((5, 7), bool)
    mask[2, 3] = True
    op = jk.HeatOperator(mask.shape, 1e-2, 10, mask=_mask_dev(mask))
    x = np.where(mask, 0.7, 0.0)
    assert np.array_equal(host64(op.apply(dev(x))), f32(x).astype(np.float64))
    p0 = np.where(mask, 1.0, 0.0)
    p, st = op.step(dev(p0), jk.EnergySpec(kind="congestion", kappa_scalar=2.0), 1e-2, max_iters=5)
    assert np.array_equal(host64(p), p0) and st["marginal_l1"] == 0.0
    # no obstacles, one implicit step
    shape, gamma = (30, 26), 0.02
    op = jk.HeatOperator(shape, gamma, 1)
    H = O.HeatKernel(np.ones(shape, bool), gamma, 1)
    rng = np.random.default_rng(4)
    q = rng.uniform(size=shape)
    q /= q.sum()
    en = jk.EnergySpec(kind="entropy", coef_scalar=0.5)
    p, _ = op.step(dev(q), en, 2.5 * gamma, max_iters=20)
    ref, _ = O.jko_step(f32(q).astype(np.float64), O.Energy(kind="entropy", coef_scalar=0.5), gamma, 2.5 * gamma,
                        20, op=H)
    assert rel_l1(host64(p), ref) <= TOL_FLOW
    # a closed wall: two rooms, mass only on the left
    mask = np.ones((20, 24), bool)
    mask[:, 11] = False
    wl = heat_room(20, 24, seed=6)
    wl.mask = mask
    wl.w = np.zeros(mask.shape)
    p0 = np.where(mask & (np.arange(24)[None, :] < 11), 1.0, 0.0)
    p0 /= p0.sum()
    wl.p0 = p0
    g_en, o_en = energies(wl)
    op = _op(wl)
    p, _ = op.step(dev(p0), g_en, wl.tau, max_iters=30)
    ref, _ = _oracle_flow(wl, o_en, 1, 30)
    assert host64(p)[:, 12:].max() == 0.0
    assert rel_l1(host64(p), ref) <= TOL_FLOW


def test_per_product_solves_match_the_stored_operator_and_oracle():
    """The per-product form (L solves per product, no stored operator) on a
    48 x 40 room: a product and a 2-step flow against the oracle and against
    the stored dense operator."""
    banner("heat per-product solves vs stored operator")
    wl = _room((48, 40))
    g_en, o_en = energies(wl)
    dense = _op(wl)
    solve = jk.HeatOperator(wl.shape, wl.gamma, wl.heat_L, mask=_mask_dev(wl.mask), per_product=True)
    H = O.HeatKernel(wl.mask, wl.gamma, wl.heat_L)
    rng = np.random.default_rng(8)
    x = np.where(wl.mask, rng.uniform(size=wl.shape), 0.0)
    ys = host64(solve.apply(dev(x)))
    assert rel_l1(ys, H(f32(x).astype(np.float64))) <= TOL_OP
    assert rel_l1(ys, host64(dense.apply(dev(x)))) <= TOL_OP
    ps, sts = solve.flow(dev(wl.p0), g_en, wl.tau, 2, max_iters=30)
    pd, _ = dense.flow(dev(wl.p0), g_en, wl.tau, 2, max_iters=30)
    ref, rst = _oracle_flow(wl, o_en, 2, 30)
    err = rel_l1(host64(ps), ref)
    print(f"[gpu-test] heat per-product 48x40: rel-L1 {err:.2e} (vs stored operator "
          f"{rel_l1(host64(ps), host64(pd)):.2e})", flush=True)
    assert err <= TOL_FLOW
    assert sts[-1]["marginal_l1"] == pytest.approx(rst[-1]["marginal_l1"], rel=0.05, abs=1e-6)


@pytest.mark.timeout(600)
def test_room_above_65536_cells():
    """A 300 x 300 room (90 000 cells, beyond the stored operator's limit):
    the per-product solves for a product and a 2-step x 30-iteration crowd
    flow with the capacity active, against the oracle's sparse LU solves."""
    banner("heat 300x300 room, per-product solves")
    wl = _room((300, 300))
    assert int(wl.mask.sum()) > 65536
    op = _op(wl)
    H = O.HeatKernel(wl.mask, wl.gamma, wl.heat_L)
    rng = np.random.default_rng(12)
    x = np.where(wl.mask, rng.uniform(size=wl.shape), 0.0)
    erra = rel_l1(host64(op.apply(dev(x))), H(f32(x).astype(np.float64)))
    g_en, o_en = energies(wl)
    pT, stats = op.flow(dev(wl.p0), g_en, wl.tau, 2, max_iters=30)
    ref, rst = _oracle_flow(wl, o_en, 2, 30)
    err = rel_l1(host64(pT), ref)
    print(f"[gpu-test] heat 300x300: operator rel-L1 {erra:.2e}, flow rel-L1 {err:.2e}, marginal "
          f"{stats[-1]['marginal_l1']:.3e} vs {rst[-1]['marginal_l1']:.3e}", flush=True)
    assert erra <= TOL_OP
    assert err <= TOL_FLOW
    assert (host64(pT) <= np.float32(wl.kappa_scalar) * (1 + 1e-6)).all()
    assert not host64(pT)[~wl.mask].any()
