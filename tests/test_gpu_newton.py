"""The Newton proxes' stopping rule (porous medium, generalised entropies,
Section 4.4, Proposition 4.2): each cell stops once its update is within
2^-20 of its scale, so a cap above the steps any cell takes changes nothing,
bit for bit, while a cap below them does.  Covers the kernels that step NE
cells per thread (pass kernels) and one (fused tile kernel), in the plain and
the log domain; agreement with the FP64 oracle is the parity tests' part."""
import numpy as np
import pytest
import torch

import paper_1502_06216_amd as jk
import workloads as W
from workloads import make_workload

from _util import banner, dev, energies

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    jk.load()


def _gen(wl):
    X = W._mesh(wl.shape)
    wl.kind = "gen_entropy"
    wl.coef = None
    wl.coef_scalar = 1.0
    wl.m_field = 1.0 + np.sin(np.pi * X[0]) * np.sin(np.pi * X[1])
    return wl


def _cases():
    p256 = W._porous("porous256", (256, 256), 2e-4, 2e-3, 2.0, 0, True, 3, 300, 0.0)
    p3 = W._porous("porous3d", (48, 40, 32), 2e-3, 5e-3, 2.0, 1, True, 3, 300, 0.0)
    return {
        "porous512_scaled": (make_workload("porous512_scaled"), {}),
        "gen512": (make_workload("gen512"), {}),
        "porous512_launched": (make_workload("porous512_scaled"), dict(resident=False)),
        "porous256_tiles": (p256, {}),
        "gen256_tiles_log": (_gen(W._porous("gen256", (256, 256), 2e-4, 2e-3, 2.0, 0, True, 3, 300, 0.0)),
                             dict(absorb_threshold=1.0)),
        "porous3d_planes_log": (p3, dict(absorb_threshold=1.0)),
    }


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_cap_above_settling_changes_nothing(name):
    banner(f"newton cap {name}")
    wl, kw = _cases()[name]
    g_en, _ = energies(wl)
    out = {}
    for cap in (1, 8, 32):
        g_en.newton_steps = cap
        out[cap] = jk.step(dev(wl.p0), g_en, wl.gamma, wl.tau, max_iters=60, tol=0.0, check_every=10, **kw)
    (p8, s8), (p32, s32), (p1, _) = out[8], out[32], out[1]
    assert torch.equal(p8, p32), f"max |diff| {float((p8 - p32).abs().max()):.3e}"
    assert s8["marginal_l1"] == s32["marginal_l1"] and s8["absorptions"] == s32["absorptions"]
    if kw.get("absorb_threshold") is not None:
        assert s8["absorptions"] == 1
    assert not torch.equal(p1, p8), "a cap of one Newton step should change the result"
