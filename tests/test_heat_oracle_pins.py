"""Pins of the heat-kernel oracle (Section 4.1, eq. heat-kernel) against
facts that do not go through its sparse assembly or its solver:

* on a grid without obstacles the no-flux five-point Laplacian is
  diagonalised by the orthonormal DCT-II, with eigenvalue 2 - 2 cos(pi k/n)
  per axis, so xi~ = C^T diag(prod (1 + sum_k nu_k lambda_k)^{-L}) C in
  closed form;
* on a tiny masked grid the system matrix is rebuilt by plain loops over
  cells and neighbours and inverted densely;
* xi~ is symmetric, non-negative, conserves mass on each connected part of
  the domain, and couples nothing across a closed wall;
* with the zero energy one JKO step is exactly one application of xi~
  (xi~ 1 = 1 on the domain).
"""
import numpy as np
import pytest
from scipy.fft import dctn, idctn

import oracle as O
from workloads import heat_room, project_capacity

TOL = 1e-11


def _dct_heat(x, gamma, L):
    """xi~ x on a full grid through the DCT-II eigenbasis."""
    shape = x.shape
    lam = 0.0
    for ax, n in enumerate(shape):
        nu = gamma * n * n / L
        k = np.arange(n)
        ev = nu * (2.0 - 2.0 * np.cos(np.pi * k / n))
        lam = lam + ev.reshape([n if a == ax else 1 for a in range(len(shape))])
    return idctn(dctn(x, type=2, norm="ortho") * (1.0 + lam) ** (-L), type=2, norm="ortho")


@pytest.mark.parametrize("shape", [(7, 5), (1, 9), (12, 12), (3, 16)])
@pytest.mark.parametrize("gamma,L", [(1e-2, 1), (1e-2, 10), (3e-3, 10), (0.5, 4)])
def test_full_grid_matches_the_dct_closed_form(shape, gamma, L):
    rng = np.random.default_rng(1)
    x = rng.uniform(size=shape)
    H = O.HeatKernel(np.ones(shape, bool), gamma, L)
    ref = _dct_heat(x, gamma, L)
    np.testing.assert_allclose(H(x), ref, rtol=0, atol=TOL * np.abs(ref).max())


def _brute_matrix(mask, gamma, L):
    """Id - (gamma/L) Delta_M over the cells of M, by loops over cells and
    their four neighbours (spacing 1/n_k, no flux into obstacles or out of
    the grid), then its dense inverse raised to the L-th power, expanded to
    all grid cells."""
    n0, n1 = mask.shape
    cells = [(i, j) for i in range(n0) for j in range(n1) if mask[i, j]]
    pos = {c: k for k, c in enumerate(cells)}
    m = len(cells)
    A = np.eye(m)
    for (i, j), r in pos.items():
        for di, dj, n in ((1, 0, n0), (-1, 0, n0), (0, 1, n1), (0, -1, n1)):
            nb = (i + di, j + dj)
            if nb in pos:
                nu = gamma * n * n / L
                A[r, r] += nu
                A[r, pos[nb]] -= nu
    P = np.linalg.matrix_power(np.linalg.inv(A), L)
    full = np.zeros((n0 * n1, n0 * n1))
    flat = [i * n1 + j for (i, j) in cells]
    full[np.ix_(flat, flat)] = P
    return full


def _tiny_mask():
    mask = np.ones((6, 5), bool)
    mask[2, 1:4] = False      # a wall with a gap at each end
    mask[4, 3] = False        # a pillar
    return mask


@pytest.mark.parametrize("gamma,L", [(2e-2, 1), (2e-2, 10), (0.3, 3)])
def test_masked_grid_matches_brute_force(gamma, L):
    mask = _tiny_mask()
    H = O.HeatKernel(mask, gamma, L)
    ref = _brute_matrix(mask, gamma, L)
    np.testing.assert_allclose(H.dense(), ref, rtol=0, atol=TOL)


def test_invariants_on_a_room():
    wl = heat_room(32, 28, seed=2)
    H = O.HeatKernel(wl.mask, wl.gamma, wl.heat_L)
    D = H.dense()
    inside = wl.mask.ravel()
    np.testing.assert_allclose(D, D.T, atol=1e-13)
    assert D.min() >= -1e-15
    # mass conservation: unit column sums on the domain, zero columns elsewhere
    np.testing.assert_allclose(D.sum(axis=0)[inside], 1.0, atol=1e-12)
    assert not D[~inside].any() and not D[:, ~inside].any()


def test_nothing_crosses_a_closed_wall():
    mask = np.ones((10, 12), bool)
    mask[:, 5] = False
    H = O.HeatKernel(mask, 0.5, 10)
    x = np.zeros(mask.shape)
    x[4, 2] = 1.0
    y = H(x)
    assert y[:, 6:].max() == 0.0
    assert y[:, :5].sum() == pytest.approx(1.0, abs=1e-12)
    assert (y[:, :5] > 0).all()      # but it reaches every cell of its own side


def test_zero_energy_step_is_one_heat_application():
    wl = heat_room(24, 20, seed=3)
    H = O.HeatKernel(wl.mask, wl.gamma, wl.heat_L)
    q = wl.p0
    p, st = O.jko_step(q, O.Energy(kind="zero"), wl.gamma, wl.tau, 7, op=H)
    np.testing.assert_allclose(p, H(q), rtol=1e-12, atol=1e-300)
    assert st["marginal_l1"] < 1e-12


def test_congestion_step_with_the_heat_kernel():
    """The crowd-motion step on the room with a binding capacity (half the
    peak, the initial density projected under it): capacity respected,
    marginal violation decreasing, mass conserved as the violation vanishes,
    and the capacity active somewhere."""
    wl = heat_room(24, 20, seed=3)
    kappa = 0.5 * wl.p0.max()
    q = project_capacity(wl.p0, kappa)
    H = O.HeatKernel(wl.mask, wl.gamma, wl.heat_L)
    en = O.Energy(kind="congestion", w=wl.w, kappa_scalar=kappa)
    errs = []
    for it in (10, 40, 400):
        p, st = O.jko_step(q, en, wl.gamma, wl.tau, it, op=H)
        errs.append(st["marginal_l1"])
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6
    assert (p <= kappa * (1 + 1e-12)).all()
    assert (p >= kappa * (1 - 1e-9)).sum() >= 5
    assert p.sum() == pytest.approx(q.sum(), rel=1e-5)
    assert not p[~wl.mask].any()
