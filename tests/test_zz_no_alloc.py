"""jko_step_static (the step on the library's static device workspace, for
callers that cannot allocate) against jko_step with a caller workspace:
the same kernels on the same inputs, so the same bits and statistics.  Each
case makes two calls in a row, the second on a smaller input, so that the
second runs on a workspace the first has left dirty."""
import math

import numpy as np
import pytest
import torch

import paper_1502_06216_amd as jk
from workloads import make_workload, small_case

from _util import banner, dev, energies

pytestmark = pytest.mark.gpu

KEYS = ("iters", "absorptions", "stop", "status", "marginal_l1", "mass", "max_abs_log_a", "max_abs_log_b")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _same(wl, **kw):
    g_en, _ = energies(wl)
    p0 = dev(wl.p0)
    ref, sref = jk.step(p0, g_en, wl.gamma, wl.tau, **kw)
    out = torch.full_like(p0, float("nan"))
    got, sgot = jk.step_static(p0, g_en, wl.gamma, wl.tau, out=out, **kw)
    assert got.data_ptr() == out.data_ptr()
    assert torch.equal(got, ref)
    for k in KEYS:
        assert sgot[k] == sref[k], (k, sgot[k], sref[k])


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_resident_2d_then_smaller(precision):
    """256^2 crowd, 300 iterations on the resident kernel, then the 32^2
    crowd on the same static workspace."""
    banner(f"static workspace: 256^2 then 32^2 {precision}")
    _same(make_workload("crowd256_fixed"), max_iters=300, precision=precision)
    _same(make_workload("crowd32"), max_iters=300, precision=precision)


def test_tolerance_mode_and_launch_path_then_smaller():
    """Tolerance mode (every check read back synchronously) on the launch
    path, then a smaller ragged grid in tolerance mode on the resident
    kernel."""
    banner("static workspace: tolerance mode")
    _same(small_case((96, 80), "congestion", seed=2), max_iters=400, tol=1e-7, check_every=7, resident=False)
    _same(small_case((45, 70), "congestion", seed=3), max_iters=400, tol=1e-7, check_every=7)


def test_3d_and_log_domain_then_smaller():
    """A 64^3 step on the plane and axis-0 passes, then a log-domain step
    (switch at a check) on a 2D grid."""
    banner("static workspace: 3D, then the log domain")
    wl = small_case((64, 64, 64), "congestion", seed=5)
    _same(wl, max_iters=40)
    _same(make_workload("crowd32", projected=False), max_iters=120, check_every=10, absorb_threshold=50.0)


def test_oversized_grid_is_refused():
    banner("static workspace: oversized grid")
    wl = make_workload("crowd128c")
    g_en, _ = energies(wl)
    with pytest.raises(jk.JKOError) as e:
        jk.step_static(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=2)
    assert e.value.status == jk.JKO_ERR_WORKSPACE
    # and the static workspace still serves a grid that fits
    _same(make_workload("crowd32"), max_iters=50)
