"""jko_step's device statistics record (``stats_dev``): the eight fields of
the host record, as doubles, written on the stream after the density with no
read-back.  Each case runs one step three times on the same input: with the
host record alone, with the device record alone, and with both.  The
densities must agree bit for bit and the records field for field (both are
written from the same control block on the device).  The host record itself
is pinned to the oracle by the parity tests."""
import math

import numpy as np
import pytest
import torch

import paper_1502_06216_amd as jk
from workloads import gaussian_bumps, make_workload, small_case

from _util import banner, dev, energies, f32

pytestmark = pytest.mark.gpu

KEYS = ("iters", "absorptions", "stop", "status", "marginal_l1", "mass", "max_abs_log_a", "max_abs_log_b")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _three_ways(wl, **kw):
    en, _ = energies(wl)
    p0 = dev(wl.p0)
    p_h, st_h = jk.step(p0, en, wl.gamma, wl.tau, **kw)
    rec = torch.full((jk.STATS_DEV_DOUBLES,), math.nan, dtype=torch.float64, device=p0.device)
    p_d, none = jk.step(p0, en, wl.gamma, wl.tau, with_stats=False, stats_dev=rec, **kw)
    assert none is None
    rec_b = torch.full_like(rec, math.nan)
    p_b, st_b = jk.step(p0, en, wl.gamma, wl.tau, stats_dev=rec_b, **kw)
    torch.cuda.synchronize()
    st_d = jk.stats_from_device(rec)
    st_bd = jk.stats_from_device(rec_b)
    for p in (p_d, p_b):
        assert torch.equal(p, p_h), f"max |diff| {float((p - p_h).abs().max()):.3e}"
    for k in KEYS:
        assert st_d[k] == st_h[k], (k, st_d[k], st_h[k])
        assert st_b[k] == st_h[k], (k, st_b[k], st_h[k])
        assert st_bd[k] == st_h[k], (k, st_bd[k], st_h[k])
    return st_h


@pytest.mark.parametrize("resident", [True, False])
@pytest.mark.parametrize("tol,cap", [(0.0, 200), (1e-6, 3000), (1e-12, 60)])
def test_crowd32(tol, cap, resident):
    banner(f"stats_dev crowd32 tol={tol} cap={cap} resident={resident}")
    wl = make_workload("crowd32", projected=True)
    st = _three_ways(wl, max_iters=cap, tol=tol, check_every=10, resident=resident)
    assert st["stop"] == ("tol" if tol == 1e-6 else "cap")
    assert st["iters"] <= cap


@pytest.mark.parametrize("resident", [True, False])
def test_crowd32_absorption_switch(resident):
    """The unprojected density switches to the log domain during the step."""
    banner(f"stats_dev crowd32 switch resident={resident}")
    wl = make_workload("crowd32", projected=False)
    st = _three_ways(wl, max_iters=300, check_every=10, absorb_threshold=50.0, resident=resident)
    assert st["absorptions"] == 1


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_crowd256_log_domain(precision):
    banner(f"stats_dev crowd256 log domain {precision}")
    wl = make_workload("crowd256")
    _three_ways(wl, max_iters=100, check_every=10, absorb_threshold=0.0, precision=precision)


def test_crowd256_resident_default_threshold():
    banner("stats_dev crowd256 resident absorb 50")
    wl = make_workload("crowd256")
    _three_ways(wl, max_iters=300, check_every=10, absorb_threshold=50.0)


def test_3d_porous():
    banner("stats_dev 3D porous 32x32x32")
    wl = small_case((32, 32, 32), "porous", seed=3)
    _three_ways(wl, max_iters=80, check_every=10)


@pytest.mark.parametrize("tol", [0.0, 1e-7])
def test_attraction(tol):
    """The attraction's record carries the mass of the returned density and
    max|log a| = 0."""
    banner(f"stats_dev attraction 48x40 tol={tol}")
    wl = small_case((48, 40), "congestion", seed=5)
    wl.kind = "attraction"
    wl.w = None
    r = gaussian_bumps((48, 40), [(0.25, 0.25), (0.7, 0.3)], 0.1, [0.5, 0.5])
    r32 = f32(r).astype(np.float64)
    wl.target = r32 * (f32(wl.p0).astype(np.float64).sum() / r32.sum())
    st = _three_ways(wl, max_iters=400, tol=tol, check_every=10)
    assert st["max_abs_log_a"] == 0.0


def test_record_needs_float64_on_the_device():
    wl = make_workload("crowd32", projected=True)
    en, _ = energies(wl)
    p0 = dev(wl.p0)
    with pytest.raises(TypeError):
        jk.step(p0, en, wl.gamma, wl.tau, stats_dev=torch.zeros(8, dtype=torch.float32, device=p0.device))
    with pytest.raises(TypeError):
        jk.step(p0, en, wl.gamma, wl.tau, stats_dev=torch.zeros(8, dtype=torch.float64))
    with pytest.raises(TypeError):
        jk.step(p0, en, wl.gamma, wl.tau, stats_dev=torch.zeros(7, dtype=torch.float64, device=p0.device))
