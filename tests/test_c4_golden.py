"""Pins of the stored FP64 reference of the differentiation workload
(``tests/golden/c4_gradients.npz``, written by
``tests/golden/make_c4_gradients.py`` from the oracle only): 20 JKO steps x
300 iterations of the congestion flow with the capacity active, at 32 x 32
and 256 x 256.

The stored autograd gradients are checked against the stored central
differences, which come from plain forward runs of the oracle (no
autograd):
* cell by cell where the difference is a derivative: the capped set of
  every iteration is the same at both ends of the interval, and the loss's
  rounding over the step is far below the gradient (cells at a capacity kink
  or of negligible mass are counted, not compared);
* along seeded random directions in p0 (h = 1e-4), to 1e-3.
Along random directions in w the quotient is no derivative: the congestion
prox min(s e^{-sigma w}, kappa) makes the loss piecewise smooth in w, and a
step of 1e-3 changes the capped state of 1.6e4 (32 x 32) to 2.5e6 (256 x 256)
(iteration, cell) pairs (counts stored), so the quotient averages one-sided
slopes (2e-3 to 0.26 from the gradient); those values are printed, not
compared.  At 32 x 32 the stored gradients are also recomputed by the
oracle's autograd.
"""
import importlib.util
import os

import numpy as np
import pytest

from oracle.grad import loss_and_grads

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "c4_gradients.npz")


def _module():
    spec = importlib.util.spec_from_file_location("make_c4_gradients",
                                                  os.path.join(HERE, "golden", "make_c4_gradients.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def gold():
    with np.load(GOLDEN, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


@pytest.fixture(scope="module")
def mod():
    return _module()


@pytest.mark.parametrize("name,tag", [("crowd32", "c32"), ("crowd256_fixed", "c256")])
def test_inputs_unchanged(gold, mod, name, tag):
    _, p0, w, kappa, target = mod.instance(name)
    assert mod.digest(p0, w, kappa, target) == str(gold[f"{tag}_digest"])


def test_cellwise_differences_match_autograd(gold, mod):
    compared = 0
    for name, tag in (("crowd32", "c32"), ("crowd256_fixed", "c256")):
        _, p0, _, _, _ = mod.instance(name)
        for which in ("w", "p"):
            ok = mod.fd_cells_valid(gold, tag, which, p0)
            cells = gold[f"{tag}_cells_{which}"][ok]
            g = np.asarray(gold[f"{tag}_g{which}"], np.float64).ravel()[cells]
            fd = gold[f"{tag}_fd_{which}"][ok]
            assert np.all(np.abs(fd - g) <= 1e-3 * np.abs(g)), (tag, which)
            compared += int(ok.sum())
    assert compared >= 10


@pytest.mark.parametrize("tag", ["c32", "c256"])
def test_directional_differences_match_autograd(gold, mod, tag):
    name = "crowd32" if tag == "c32" else "crowd256_fixed"
    _, p0, _, _, _ = mod.instance(name)
    gw = np.asarray(gold[f"{tag}_gw"], np.float64)
    gp = np.asarray(gold[f"{tag}_gp"], np.float64)
    for k in range(mod.N_DIRS):
        vw = gold[f"{tag}_dir_vw"][k].astype(np.float64)
        vp = gold[f"{tag}_dir_vp"][k].astype(np.float64)
        dw, dp = float((gw * vw).sum()), float((gp * p0 * vp).sum())
        assert abs(gold[f"{tag}_dir_fd_p"][k] - dp) <= 1e-3 * abs(dp)
        print(f"{tag} direction {k}: p0 {abs(gold[f'{tag}_dir_fd_p'][k] - dp) / abs(dp):.1e} "
              f"({int(gold[f'{tag}_dir_flips_p'][k])} flips); w {abs(gold[f'{tag}_dir_fd_w'][k] - dw) / abs(dw):.1e} "
              f"({int(gold[f'{tag}_dir_flips_w'][k])} flips, not compared)")


def test_small_instance_gradients_recompute(gold, mod):
    wl, p0, w, kappa, target = mod.instance("crowd32")
    loss, gw, gp, _ = loss_and_grads(p0, w, kappa, wl.gamma, wl.tau, [mod.ITERS] * mod.N_STEPS, target)
    assert loss == pytest.approx(float(gold["c32_loss"]), rel=1e-12)
    assert np.allclose(gw, gold["c32_gw"], rtol=1e-9, atol=1e-12 * np.abs(gw).max())
    assert np.allclose(gp, gold["c32_gp"], rtol=1e-9, atol=1e-12 * np.abs(gp).max())
