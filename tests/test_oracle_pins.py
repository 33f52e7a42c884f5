"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formulas: each compares it with an
independent route to the same number (a direct minimisation, a convex solver,
a closed-form Gaussian solution, the explicit-coupling form of the algorithm,
finite differences).
"""
import math
import warnings

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from oracle.grad import loss_and_grads
from workloads import make_workload, gaussian_bumps


# ---------------------------------------------------------------- Gibbs kernel

@pytest.mark.parametrize("shape", [(7,), (6, 7), (4, 5, 6), (3, 2, 5)])
def test_separable_gibbs_equals_dense_definition(shape):
    """xi = exp(-|x_i - x_j|^2/gamma) over all pairs of grid points (Section 3.1)
    equals the per-axis factorisation used for uniform grids (Section 4.1)."""
    rng = np.random.default_rng(1)
    x = rng.uniform(size=shape)
    for gamma in (0.01, 0.3):
        dense = O.gibbs_apply(x, gamma, "dense")
        sep = O.gibbs_apply(x, gamma, "separable")
        np.testing.assert_allclose(sep, dense, rtol=1e-13, atol=0)


def test_dense_gibbs_entries_by_loops():
    shape = (3, 4)
    gamma = 0.07
    xi = O.gibbs_dense(shape, gamma)
    pts = [((i + 0.5) / 3, (j + 0.5) / 4) for i in range(3) for j in range(4)]
    for I, P in enumerate(pts):
        for J, Q in enumerate(pts):
            assert xi[I, J] == pytest.approx(
                math.exp(-((P[0] - Q[0]) ** 2 + (P[1] - Q[1]) ** 2) / gamma), rel=1e-15)


@pytest.mark.parametrize("shape", [(9,), (7, 5), (3, 6, 5)])
def test_gibbs_rows_equal_dense_products(shape):
    """The single-output form used for spot checks of large grids (each
    output as its own sum over all cells) equals rows of the dense product
    with the N x N matrix built from pairwise distances, on ragged grids and
    at both ends of the grid."""
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 2.0, size=shape)
    N = int(np.prod(shape))
    idx = np.array(sorted({0, N - 1, N // 2, *rng.integers(0, N, size=5).tolist()}))
    for gamma in (0.02, 0.5):
        full = O.gibbs_dense(shape, gamma) @ x.ravel()
        np.testing.assert_allclose(O.gibbs_rows(shape, gamma, idx, x), full[idx], rtol=1e-13, atol=0)


def test_log_gibbs_matches_plain():
    rng = np.random.default_rng(2)
    x = rng.uniform(0.1, 2.0, size=(5, 6, 4))
    gamma = 0.05
    np.testing.assert_allclose(np.exp(O.log_gibbs_apply(np.log(x), gamma)),
                               O.gibbs_apply(x, gamma), rtol=1e-13)


# ---------------------------------------------------------------- proximal maps

def _golden_min(f, lo, hi, iters=400):
    g = (math.sqrt(5) - 1) / 2
    a, b = lo, hi
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(iters):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
    return 0.5 * (a + b)


def _kl(p, s):
    # KL(p|s) without its constant s, which does not move the minimiser
    return (p * math.log(p / s) if p > 0 else 0.0) - p


def _log_golden_min(f, lo, hi):
    """Minimise f over p in [lo, hi] (lo > 0) by golden section on log p."""
    return math.exp(_golden_min(lambda u: f(math.exp(u)), math.log(lo), math.log(hi)))


@pytest.mark.parametrize("s", [1e-6, 3e-3, 0.3, 1.0, 4.0])
@pytest.mark.parametrize("sigma", [0.5, 2.5, 10.0])
def test_prox_congestion_minimises(s, sigma):
    """Proposition 4.1 against a direct minimisation of KL(p|s) + sigma f(p)."""
    for w, kappa in ((0.3, 2.0 * s), (0.01, 0.5 * s), (0.0, math.inf), (0.7, 0.0)):
        got = float(O.prox_congestion(np.array(s), sigma, np.array(w), np.array(kappa)))
        if kappa == 0.0:
            assert got == 0.0
            continue
        hi = min(kappa, 2.0 * s)
        ref = _log_golden_min(lambda p: _kl(p, s) + sigma * w * p, s * 1e-20, hi)
        assert got == pytest.approx(ref, rel=2e-6, abs=1e-300)


def test_prox_binary_congestion_follows_the_threshold_rule():
    """Section 4.5: the KL prox of the binary constraint is 0 below kappa/e and
    kappa above it.  With the potential, the argument is s e^{-sigma w} (the
    linear term folded into the KL divergence, as for Proposition 4.1).  The
    oracle's two-candidate argmin must reproduce that rule cell by cell."""
    rng = np.random.default_rng(5)
    n = 4000
    s = rng.uniform(0, 2, n) * 10.0 ** rng.uniform(-6, 2, n)
    w = rng.uniform(-1, 1, n)
    kappa = rng.uniform(0, 3, n) * 10.0 ** rng.uniform(-6, 2, n)
    for sigma in (0.3, 2.0, 9.0):
        z = s * np.exp(-sigma * w)
        got = O.prox_binary_congestion(s, sigma, w, kappa)
        far = np.abs(z / (kappa / math.e) - 1.0) > 1e-9
        rule = np.where(z > kappa / math.e, kappa, 0.0)
        assert far.mean() > 0.99
        np.testing.assert_array_equal(got[far], rule[far])
        assert np.all((got == kappa) | (got == 0.0))


def test_prox_binary_congestion_tie_and_degenerate_cells():
    """At z = kappa/e exactly the prox is two-valued: kappa is taken.  Built
    exactly in floating point with kappa = s and sigma w = 1; kappa = 0 and
    s = 0 give 0; the log form takes the same decisions."""
    s = np.array([0.3, 2.0, 1e-4])
    assert np.array_equal(O.prox_binary_congestion(s, 1.0, 1.0, s), s)
    en = O.Energy(kind="binary_congestion", w=np.ones(3), kappa=s)
    np.testing.assert_allclose(np.exp(O.log_prox(np.log(s), 1.0, en)), s, rtol=1e-15)
    assert O.prox_binary_congestion(np.array([0.5]), 1.0, 0.0, 0.0)[0] == 0.0
    assert O.prox_binary_congestion(np.array([0.0]), 1.0, 0.0, 2.0)[0] == 0.0
    rng = np.random.default_rng(6)
    s = rng.uniform(1e-4, 3, 500)
    en = O.Energy(kind="binary_congestion", w=rng.uniform(-1, 1, 500), kappa=rng.uniform(0, 2, 500))
    lp, pp = np.exp(O.log_prox(np.log(s), 1.7, en)), O.prox(s, 1.7, en)
    np.testing.assert_array_equal(lp > 0, pp > 0)
    np.testing.assert_allclose(lp, pp, rtol=1e-15)


def test_binary_congestion_step_is_binary_in_both_forms():
    """A binary-congestion JKO step (the non-convex iteration of Section 4.5)
    returns densities in {0, kappa}, and its plain and log forms agree."""
    rng = np.random.default_rng(7)
    shape = (12, 10)
    N = int(np.prod(shape))
    q = rng.uniform(0.2, 1.0, size=shape)
    q /= q.sum()
    en = O.Energy(kind="binary_congestion", w=rng.uniform(0, 1, size=shape), kappa_scalar=2.5 / N)
    p1, st1 = O.jko_step(q, en, 0.01, 0.02, 40)
    p2, st2 = O.jko_step_log(q, en, 0.01, 0.02, 40)
    assert set(np.unique(p1)) <= {0.0, 2.5 / N}
    assert (p1 > 0).any() and (p1 == 0).any()
    # same decisions; the log form's exp(log kappa) may differ from kappa in the last bit
    np.testing.assert_array_equal(p2 > 0, p1 > 0)
    np.testing.assert_allclose(p2, p1, rtol=1e-15)


@pytest.mark.parametrize("s", [1e-5, 0.02, 0.5, 1.0, 3.0])
@pytest.mark.parametrize("sigma,c", [(0.5, 1.0), (2.5, 0.3), (10.0, 2.0)])
def test_prox_entropy_minimises(s, sigma, c):
    """Proposition 4.2 (m = 1) against a direct minimisation."""
    got = float(O.prox_entropy(np.array(s), sigma, np.array(c)))
    ref = _log_golden_min(lambda p: _kl(p, s) + sigma * c * p * (math.log(p) - 1.0),
                          s * 1e-30 if s < 1 else 1e-30, 2.0 * max(s, 1.0))
    assert got == pytest.approx(ref, rel=2e-6)


@pytest.mark.parametrize("m", [1.4, 2.0, 3.0])
@pytest.mark.parametrize("s", [1e-6, 1e-3, 0.2, 1.0, 30.0])
@pytest.mark.parametrize("sigma,c,D", [(10.0, 1.0, 1.0), (1.0, 0.1, 1.0), (10.0, 1.9, 4096.0)])
def test_prox_porous_minimises(m, s, sigma, c, D):
    """Generalised-entropy prox (f = c (D p)^m / ((m-1) D)) against a direct
    minimisation, and the log-form root against the linear-form root."""
    en = O.Energy(kind="porous", coef_scalar=c, m=m, density_scale=D)
    got = float(O.prox(np.array([s]), sigma, en)[0])
    ref = _log_golden_min(lambda p: _kl(p, s) + sigma * c * (D * p) ** m / ((m - 1.0) * D),
                          s * 1e-30, s)
    assert got == pytest.approx(ref, rel=2e-6)
    got_log = float(np.exp(O.log_prox(np.log(np.array([s])), sigma, en)[0]))
    assert got_log == pytest.approx(got, rel=1e-12)


def _e_m(x, m):
    """Section 4.4, eq. defn-gen-entropies: e_1 = x (log x - 1),
    e_m = x (x^{m-1} - m) / (m - 1), the latter evaluated as
    x ((x^{m-1} - 1) / (m - 1) - 1) with expm1, free of cancellation near m = 1."""
    if x == 0.0:
        return 0.0
    if m == 1.0:
        return x * (math.log(x) - 1.0)
    return x * (math.expm1((m - 1.0) * math.log(x)) / (m - 1.0) - 1.0)


@pytest.mark.parametrize("m", [1.0, 1.0 + 1e-6, 1.05, 1.4, 2.0, 3.0])
@pytest.mark.parametrize("s,sigma,b,D", [(0.3, 2.0, 1.0, 1.0), (2.5, 0.7, 4.0, 1.0), (1e-4, 5.0, 0.5, 1e3),
                                         (0.02, 10.0, 20.0, 50.0), (3.0, 1.0, 0.0, 1.0)])
def test_prox_gen_entropy_minimises(m, s, sigma, b, D):
    """Proposition 4.2 with weight b and density scale D against a direct
    minimisation of KL(p|s) + sigma b e_m(D p) / D written from the
    definition of e_m."""
    got = float(np.exp(O.log_prox_gen_entropy(np.log(s), sigma, b, m, D)))
    ref = _log_golden_min(lambda p: _kl(p, s) + sigma * b * _e_m(D * p, m) / D, s * 1e-12, s * 1e6)
    assert got == pytest.approx(ref, rel=2e-6)


def test_prox_gen_entropy_is_continuous_at_m_one_and_matches_porous_shift():
    """As m -> 1 the prox tends to the entropy prox (the -m s term of e_m
    makes the family continuous), and for m > 1 it equals the porous prox
    (no linear term) applied to s e^{sigma b m / (m - 1)}: the linear term
    folded into the divergence."""
    s = np.array([1e-3, 0.2, 1.0, 7.0])
    for sigma, b in ((1.0, 1.0), (3.0, 0.4)):
        at1 = O.log_prox_gen_entropy(np.log(s), sigma, b, 1.0, 1.0)
        near = O.log_prox_gen_entropy(np.log(s), sigma, b, 1.0 + 1e-7, 1.0)
        np.testing.assert_allclose(near, at1, rtol=0, atol=1e-5)
        for m in (1.3, 2.0, 2.7):
            got = np.exp(O.log_prox_gen_entropy(np.log(s), sigma, b, m, 1.0))
            k = sigma * b * m / (m - 1.0)
            ref = O.prox_porous(s * np.exp(k), k, m)
            np.testing.assert_allclose(got, ref, rtol=1e-10)


def test_lambertw_of_log_large_argument():
    for logz in (10.0, 300.0, 690.0):
        w = O.lambertw_of_log(np.array([logz]))[0]
        assert w + math.log(w) == pytest.approx(logz, rel=1e-14)
    w = O.lambertw_of_log(np.array([5000.0]))[0]
    assert w + math.log(w) == pytest.approx(5000.0, rel=1e-14)


# ---------------------------------------------------------------- the iteration

def _tiny_congestion(shape, seed=0, kappa_factor=1.6):
    rng = np.random.default_rng(seed)
    N = int(np.prod(shape))
    q = rng.uniform(0.2, 1.0, size=shape)
    q /= q.sum()
    w = rng.uniform(0, 1, size=shape)
    return q, O.Energy(kind="congestion", w=w, kappa_scalar=kappa_factor / N)


@pytest.mark.parametrize("kind", ["congestion", "entropy", "porous", "gen_entropy"])
def test_three_forms_of_dykstra_agree(kind):
    """Explicit-coupling KL Dykstra (Proposition 3.2 proxes) == Proposition 3.3
    scaling form == the reduced iteration, half-step by half-step."""
    shape = (4, 5)
    gamma, tau = 0.05, 0.1
    q, en = _tiny_congestion(shape)
    if kind == "entropy":
        en = O.Energy(kind="entropy", coef=np.linspace(0.5, 1.5, 20).reshape(shape))
    elif kind == "porous":
        en = O.Energy(kind="porous", coef_scalar=1.3, m=2.0, density_scale=20.0)
    elif kind == "gen_entropy":
        en = O.Energy(kind="gen_entropy", coef=np.linspace(1.0, 5.0, 20).reshape(shape),
                      m_field=np.linspace(1.0, 2.0, 20).reshape(shape), density_scale=20.0)
    for L in (2, 4, 10, 30):
        p1 = O.dykstra_coupling(q, en, gamma, tau, L)
        p2, a, b, u, v = O.dykstra_scaling(q, en, gamma, tau, L)
        p3, _ = O.jko_step(q, en, gamma, tau, L // 2, mode="dense")
        p4, _ = O.jko_step(q, en, gamma, tau, L // 2, mode="separable")
        np.testing.assert_allclose(p2, p1, rtol=1e-11)
        np.testing.assert_allclose(p3, p1, rtol=1e-11)
        np.testing.assert_allclose(p4, p3, rtol=1e-12)
        # the corrections of Proposition 3.3 after an even half-step
        np.testing.assert_allclose(u * a, 1.0, rtol=1e-12)
        np.testing.assert_allclose(v, 1.0, rtol=1e-12)


def _solve_jko_convex(q, en, gamma, tau):
    """Solve eq. prox-step, min <c,pi> + gamma E(pi) + tau f(pi 1) s.t.
    pi^T 1 = q, with SLSQP on the entries of pi (1D grid)."""
    n = q.size
    x = (np.arange(n) + 0.5) / n
    c = (x[:, None] - x[None, :]) ** 2
    if en.kind == "congestion":
        w = en._w(q.shape)
        kappa = en._kappa(q.shape)
    coef = en._coef(q.shape)

    def F(v):
        pi = v.reshape(n, n)
        p = pi.sum(1)
        val = (c * pi).sum() + gamma * (pi * (np.log(pi) - 1)).sum()
        g = c + gamma * np.log(pi)
        if en.kind == "congestion":
            val += tau * (w * p).sum()
            g = g + tau * w[:, None]
        elif en.kind == "entropy":
            val += tau * (coef * p * (np.log(p) - 1)).sum()
            g = g + tau * (coef * np.log(p))[:, None]
        return val, g.ravel()

    cons = [dict(type="eq", fun=lambda v: v.reshape(n, n).sum(0) - q,
                 jac=lambda v: np.kron(np.ones((1, n)), np.eye(n)))]
    if en.kind == "congestion" and np.isfinite(kappa).any():
        cons.append(dict(type="ineq", fun=lambda v: kappa - v.reshape(n, n).sum(1),
                         jac=lambda v: -np.kron(np.eye(n), np.ones((1, n)))))
    v0 = (np.ones((n, n)) * q[None, :] / n).ravel()
    with np.errstate(all="ignore"), warnings.catch_warnings():
        warnings.simplefilter("ignore")
        res = minimize(F, v0, jac=True, method="SLSQP", constraints=cons,
                       bounds=[(1e-14, None)] * (n * n),
                       options=dict(ftol=1e-16, maxiter=2000))
    return res.x.reshape(n, n).sum(1)


@pytest.mark.parametrize("kind", ["congestion", "entropy"])
def test_converged_step_solves_the_jko_problem(kind):
    """The Dykstra fixed point is the minimiser of the KL formulation of one
    entropic JKO step (Section 3.1, Proposition 3.1), found independently by a
    generic constrained solver."""
    n = 6
    rng = np.random.default_rng(3)
    q = rng.uniform(0.3, 1.0, n)
    q /= q.sum()
    gamma, tau = 0.05, 0.1
    if kind == "congestion":
        en = O.Energy(kind="congestion", w=3 * np.linspace(0, 1, n) ** 2, kappa_scalar=0.22)
    else:
        en = O.Energy(kind="entropy", coef=rng.uniform(0.5, 1.5, n))
    p, st = O.jko_step(q, en, gamma, tau, max_iters=20000, tol=1e-14, check_every=1,
                       mode="dense")
    ref = _solve_jko_convex(q, en, gamma, tau)
    np.testing.assert_allclose(p, ref, rtol=2e-5, atol=1e-9)
    if kind == "congestion":
        assert p.max() <= 0.22
        assert (ref > 0.22 - 1e-6).any(), "the capacity should be active in this case"


# ---------------------------------------------------------- Wasserstein attraction

def _attraction_case(seed=12, shape=(6, 5)):
    rng = np.random.default_rng(seed)
    q = rng.uniform(0.2, 1.0, size=shape)
    q /= q.sum()
    r = rng.uniform(0.2, 1.0, size=shape) ** 3
    r /= r.sum()
    return q, r


def test_attraction_reduced_equals_proposition_5_2():
    """Proposition 5.2 verbatim (marginals first) == the reduced iteration,
    half-step by half-step, with u_m a_m = 1 and v_m = 1 after even
    half-steps (the corrections that the reduction drops)."""
    q, r = _attraction_case()
    kappa = 1.2 * max(q.max(), r.max())
    for L in (2, 4, 10, 30):
        pg, a, b, u, v = O.attraction_generic(q, r, kappa, 0.05, 0.1, L, first=2, mode="dense")
        pr, _ = O.attraction_step(q, r, kappa, 0.05, 0.1, L // 2, mode="separable")
        np.testing.assert_allclose(pr, pg, rtol=1e-11)
        for m in range(2):
            np.testing.assert_allclose(u[m] * a[m], 1.0, rtol=1e-12)
            np.testing.assert_allclose(v[m], 1.0, rtol=1e-12)


def test_attraction_limit_does_not_depend_on_the_order():
    """Dykstra's limit is the minimiser whatever function acts first: the
    printed order (psi_1 first) and the marginals-first order agree once
    converged."""
    q, r = _attraction_case(13)
    kappa = 1.1 * q.max()
    p1, *_ = O.attraction_generic(q, r, kappa, 0.05, 0.1, 4001, first=1)
    p2, *_ = O.attraction_generic(q, r, kappa, 0.05, 0.1, 4000, first=2)
    np.testing.assert_allclose(p1, p2, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("p1,p2,tau,kappa", [(0.3, 0.8, 0.1, np.inf), (2.0, 0.05, 1.5, np.inf),
                                             (0.4, 0.9, 0.7, 0.45), (1e-3, 4.0, 3.0, np.inf)])
def test_attraction_prox_minimises(p1, p2, tau, kappa):
    """eq. prox-psi-attraction against a direct minimisation over p of
    KL(p|p1) + tau KL(p|p2) on [0, kappa] (the KL_lambda divergence of (p, p)
    to (p1, p2), lambda = (1, tau))."""
    got = float(O.prox_attraction_psi1(np.array(p1), np.array(p2), tau, kappa))
    hi = min(kappa, 10.0 * max(p1, p2))
    ref = _log_golden_min(lambda p: _kl(p, p1) + tau * _kl(p, p2), 1e-12 * min(p1, p2), hi)
    assert got == pytest.approx(ref, rel=2e-6)


def test_attraction_log_form_matches_plain_where_both_finite():
    """The log form of the attraction step (exact log-sum-exp products) takes
    the plain form's iterates where both are finite."""
    q, r = _attraction_case(16, shape=(12, 10))
    kappa = 1.3 * q.max()
    p1, s1 = O.attraction_step(q, r, kappa, 0.02, 0.2, 40)
    p2, s2 = O.attraction_step_log(q, r, kappa, 0.02, 0.2, 40)
    np.testing.assert_allclose(p2, p1, rtol=1e-10, atol=1e-300)
    assert s2["marginal_l1"] == pytest.approx(s1["marginal_l1"], rel=1e-8)


def test_attraction_to_its_own_density_is_one_blur():
    """r = q without capacity: f = W(q, .) makes the step the minimiser of
    (1 + tau) W_gamma(q, p), the blur xi (q / xi^T 1) of the conclusion."""
    q, _ = _attraction_case(14)
    p, _ = O.attraction_step(q, q, np.inf, 0.05, 0.3, 3)
    ref = O.gibbs_apply(q / O.gibbs_apply(np.ones_like(q), 0.05, transpose=True), 0.05)
    np.testing.assert_allclose(p, ref, rtol=1e-12)


def test_converged_attraction_step_solves_the_two_coupling_problem():
    """The converged scaling solves the problem of Section 5.2 posed on the
    couplings themselves: min <c, pi_1> + gamma E(pi_1) + tau (<c, pi_2> +
    gamma E(pi_2)) s.t. pi_1^T 1 = q, pi_2^T 1 = r, pi_1 1 = pi_2 1 <= kappa,
    found by SLSQP on the entries (1D grid)."""
    n = 6
    rng = np.random.default_rng(15)
    q = rng.uniform(0.3, 1.0, n)
    q /= q.sum()
    r = np.linspace(0.05, 1.0, n) ** 2
    r /= r.sum()
    gamma, tau, kappa = 0.05, 0.4, 0.19
    p, st = O.attraction_step(q, r, kappa, gamma, tau, max_iters=20000, tol=1e-14, check_every=1,
                              mode="dense")
    x = (np.arange(n) + 0.5) / n
    c = (x[:, None] - x[None, :]) ** 2

    def F(v):
        p1, p2 = v[:n * n].reshape(n, n), v[n * n:].reshape(n, n)
        val = (c * p1).sum() + gamma * (p1 * (np.log(p1) - 1)).sum()
        val += tau * ((c * p2).sum() + gamma * (p2 * (np.log(p2) - 1)).sum())
        g = np.concatenate([(c + gamma * np.log(p1)).ravel(), (tau * (c + gamma * np.log(p2))).ravel()])
        return val, g

    col = np.kron(np.ones((1, n)), np.eye(n))
    row = np.kron(np.eye(n), np.ones((1, n)))
    Z = np.zeros((n, n * n))
    cons = [dict(type="eq", fun=lambda v: v[:n * n].reshape(n, n).sum(0) - q, jac=lambda v: np.hstack([col, Z])),
            dict(type="eq", fun=lambda v: v[n * n:].reshape(n, n).sum(0) - r, jac=lambda v: np.hstack([Z, col])),
            # equal left marginals; the last one follows from the others (both
            # couplings carry mass one), and SLSQP needs independent constraints
            dict(type="eq", fun=lambda v: (v[:n * n].reshape(n, n).sum(1) - v[n * n:].reshape(n, n).sum(1))[:-1],
                 jac=lambda v: np.hstack([row, -row])[:-1]),
            dict(type="ineq", fun=lambda v: kappa - v[:n * n].reshape(n, n).sum(1), jac=lambda v: np.hstack([-row, Z]))]
    v0 = np.concatenate([(np.ones((n, n)) * q[None, :] / n).ravel(), (np.ones((n, n)) * r[None, :] / n).ravel()])
    with np.errstate(all="ignore"), warnings.catch_warnings():
        warnings.simplefilter("ignore")
        res = minimize(F, v0, jac=True, method="SLSQP", constraints=cons, bounds=[(1e-14, None)] * (2 * n * n),
                       options=dict(ftol=1e-16, maxiter=3000))
    assert res.success, res.message
    ref = res.x[:n * n].reshape(n, n).sum(1)
    np.testing.assert_allclose(p, ref, rtol=5e-5, atol=1e-9)
    assert p.max() <= kappa and (ref > kappa - 1e-6).any(), "the capacity should be active in this case"


def _heat_recursion(S, gamma, tau):
    u = ((gamma + 2 * S) + math.sqrt((gamma + 2 * S) ** 2 + 8 * tau * S)) / 2
    return (u + tau) / 2


def _moments(p, x):
    m = (p * x).sum() / p.sum()
    return m, (p * (x - m) ** 2).sum() / p.sum()


def test_heat_flow_keeps_gaussian_with_closed_form_variance():
    """f = entropy: a Gaussian stays Gaussian.  With cost |x-y|^2 the JKO step
    maps variance S to (u + tau)/2, u = ((gamma+2S) + sqrt((gamma+2S)^2 +
    8 tau S))/2 (continuous Gaussian solution of the first-order conditions of
    eq. prox-step with a = p^{-tau/gamma})."""
    n, gamma, tau, S0 = 512, 2e-4, 1e-3, 3e-3
    x = (np.arange(n) + 0.5) / n
    p = np.exp(-(x - 0.5) ** 2 / (2 * S0))
    p /= p.sum()
    en = O.Energy(kind="entropy")
    S = _moments(p, x)[1]
    for _ in range(4):
        p, st = O.jko_step(p, en, gamma, tau, max_iters=20000, tol=1e-13, check_every=10)
        S = _heat_recursion(S, gamma, tau)
        mean, var = _moments(p, x)
        assert st["stop"] == "tol"
        assert var == pytest.approx(S, rel=2e-6)
        assert mean == pytest.approx(0.5, abs=1e-12)
        assert p.sum() == pytest.approx(1.0, abs=1e-12)


def test_heat_flow_2d_is_product_of_1d():
    """On a product Gaussian the 2D step factorises: each axis follows the 1D
    variance recursion (ragged 2D grid)."""
    shape = (80, 96)
    gamma, tau, S0 = 1.5e-3, 2e-3, 2e-3
    x0 = (np.arange(shape[0]) + 0.5) / shape[0]
    x1 = (np.arange(shape[1]) + 0.5) / shape[1]
    p = np.exp(-(x0[:, None] - 0.5) ** 2 / (2 * S0)) * np.exp(-(x1[None, :] - 0.5) ** 2 / (2 * S0))
    p /= p.sum()
    en = O.Energy(kind="entropy")
    S = [_moments(p.sum(1), x0)[1], _moments(p.sum(0), x1)[1]]
    for _ in range(2):
        p, st = O.jko_step(p, en, gamma, tau, max_iters=20000, tol=1e-13, check_every=10)
        S = [_heat_recursion(s, gamma, tau) for s in S]
        assert _moments(p.sum(1), x0)[1] == pytest.approx(S[0], rel=2e-5)
        assert _moments(p.sum(0), x1)[1] == pytest.approx(S[1], rel=2e-5)


def test_ornstein_uhlenbeck_closed_form():
    """f = <w, p> with w = lam |x - c|^2 and no capacity: each step maps
    (mean, var) to ((mu + tau lam c)/(1 + tau lam),
    var/(1 + tau lam)^2 + gamma / (2 (1 + tau lam))) (the conditional law of
    pi given the old position is Gaussian); the prox is Proposition 4.1 with
    kappa = +inf, i.e. the linear shift rule of Appendix A."""
    n, gamma, tau, lam, c = 512, 2e-4, 2e-3, 1.0, 0.7
    x = (np.arange(n) + 0.5) / n
    mu, S = 0.4, 2e-3
    p = np.exp(-(x - mu) ** 2 / (2 * S))
    p /= p.sum()
    mu, S = _moments(p, x)
    en = O.Energy(kind="congestion", w=lam * (x - c) ** 2)
    for _ in range(5):
        p, st = O.jko_step(p, en, gamma, tau, max_iters=3)
        mu = (mu + tau * lam * c) / (1 + tau * lam)
        S = S / (1 + tau * lam) ** 2 + gamma / (2 * (1 + tau * lam))
        m_, v_ = _moments(p, x)
        assert m_ == pytest.approx(mu, rel=1e-11)
        assert v_ == pytest.approx(S, rel=1e-10)
        assert st["marginal_l1"] < 1e-13


def test_zero_energy_is_one_blur():
    """f = 0: the step returns a blur of p_t by xi (the small-tau limit in the
    paper's conclusion); on a Gaussian the variance grows by gamma/2, and the
    iteration is at its fixed point after one iteration."""
    n, gamma, S0 = 400, 3e-4, 2e-3
    x = (np.arange(n) + 0.5) / n
    p = np.exp(-(x - 0.5) ** 2 / (2 * S0))
    p /= p.sum()
    S = _moments(p, x)[1]
    p1, st1 = O.jko_step(p, O.Energy(), gamma, 0.01, max_iters=1)
    p5, st5 = O.jko_step(p, O.Energy(), gamma, 0.01, max_iters=5)
    np.testing.assert_allclose(p5, p1, rtol=1e-13)
    assert _moments(p1, x)[1] == pytest.approx(S + gamma / 2, rel=1e-12)
    assert st1["marginal_l1"] < 1e-14


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("projected", [True, False])
def test_congestion_invariants_crowd32(projected):
    """0 <= p <= kappa after every step (Proposition 4.1), and the mass moves by
    at most the monitored violation: sum p_{t+1} = sum_j b_j (xi^T a)_j."""
    wl = make_workload("crowd32", projected=projected, n_steps=4, max_iters=100)
    en = O.Energy(kind="congestion", w=wl.w, kappa=wl.kappa, kappa_scalar=wl.kappa_scalar)
    q = wl.p0
    for _ in range(wl.n_steps):
        p, st = O.jko_step(q, en, wl.gamma, wl.tau, wl.max_iters)
        assert p.min() >= 0.0
        assert (p <= wl.kappa_field()).all()
        assert abs(p.sum() - q.sum()) <= st["marginal_l1"] * (1 + 1e-12) + 1e-15
        q = p


def test_tolerance_stop_returns_the_fixed_count_iterate():
    wl = make_workload("crowd32", projected=True)
    en = O.Energy(kind="congestion", w=wl.w, kappa_scalar=wl.kappa_scalar)
    p, st = O.jko_step(wl.p0, en, wl.gamma, wl.tau, 5000, tol=1e-7, check_every=7)
    assert st["stop"] == "tol"
    assert st["iters"] % 7 == 0
    assert st["marginal_l1"] <= 1e-7
    p2, st2 = O.jko_step(wl.p0, en, wl.gamma, wl.tau, st["iters"])
    np.testing.assert_array_equal(p, p2)
    assert st2["marginal_l1"] == pytest.approx(st["marginal_l1"], rel=1e-12)


def test_log_domain_matches_plain_where_both_finite():
    wl = make_workload("crowd32", projected=False)
    en = O.Energy(kind="congestion", w=wl.w, kappa_scalar=wl.kappa_scalar)
    p1, s1 = O.jko_step(wl.p0, en, wl.gamma, wl.tau, 60)
    p2, s2 = O.jko_step_log(wl.p0, en, wl.gamma, wl.tau, 60)
    np.testing.assert_allclose(p2, p1, rtol=1e-10, atol=1e-300)
    assert s2["marginal_l1"] == pytest.approx(s1["marginal_l1"], rel=1e-8)
    en_p = O.Energy(kind="porous", coef_scalar=1.0, m=2.0, density_scale=1024.0)
    p3, _ = O.jko_step(wl.p0, en_p, wl.gamma, wl.tau, 20)
    p4, _ = O.jko_step_log(wl.p0, en_p, wl.gamma, wl.tau, 20)
    np.testing.assert_allclose(p4, p3, rtol=1e-10)
    x = np.linspace(0, 1, 32)
    en_g = O.Energy(kind="gen_entropy", coef=1.0 + 19.0 * np.outer(np.sin(np.pi * x), np.sin(np.pi * x)),
                    m_field=1.0 + np.outer(np.sin(np.pi * x), np.sin(np.pi * x)), density_scale=1024.0)
    p5, _ = O.jko_step(wl.p0, en_g, wl.gamma, wl.tau, 20)
    p6, _ = O.jko_step_log(wl.p0, en_g, wl.gamma, wl.tau, 20)
    np.testing.assert_allclose(p6, p5, rtol=1e-10)


# ---------------------------------------------------------------- gradients

def test_reference_gradient_gen_entropy_matches_finite_differences():
    """The generalised-entropy flow (per-cell weights and exponents from 1 to
    2, density units): autograd through the implicit derivatives of the prox
    == central differences of the numpy oracle's forward map in p0 and in the
    weights b."""
    shape = (8, 8)
    rng = np.random.default_rng(8)
    gamma, tau = 2e-2, 5e-2
    p0 = gaussian_bumps(shape, rng.uniform(0.3, 0.7, size=(2, 2)), 0.15, [0.5, 0.5])
    b = rng.uniform(0.5, 3.0, size=shape)
    m = 1.0 + rng.uniform(0.0, 1.0, size=shape)
    m[0, :] = 1.0
    D = 64.0
    target = rng.uniform(size=shape)
    target /= target.sum()
    iters = [20, 20]
    en = O.Energy(kind="gen_entropy", coef=b, m_field=m, density_scale=D)

    def fwd(p0_, b_=b):
        e = O.Energy(kind="gen_entropy", coef=b_, m_field=m, density_scale=D)
        q = p0_
        for K in iters:
            q, _ = O.jko_step(q, e, gamma, tau, K)
        return float(((q - target) ** 2).sum())

    loss, gb, gp, _ = loss_and_grads(p0, np.zeros(shape), np.inf, gamma, tau, iters, target, kind="gen_entropy",
                                     coef=b, m=m, density_scale=D)
    assert loss == pytest.approx(fwd(p0), rel=1e-13)
    for c in [(1, 1), (4, 5), (0, 3), (7, 7)]:
        hb = 1e-5 * b[c]
        bp, bm = b.copy(), b.copy()
        bp[c] += hb
        bm[c] -= hb
        fd = (fwd(p0, bp) - fwd(p0, bm)) / (2 * hb)
        assert gb[c] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(loss))
    for c in [(1, 1), (4, 5), (6, 2), (7, 7), (0, 5)]:
        hp = 1e-5 * p0[c]
        pp, pm = p0.copy(), p0.copy()
        pp[c] += hp
        pm[c] -= hp
        fd = (fwd(pp) - fwd(pm)) / (2 * hp)
        assert gp[c] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(loss))


def test_reference_gradient_matches_finite_differences():
    """torch float64 autograd through the unrolled flow == central finite
    differences of the numpy oracle's forward map."""
    shape = (8, 8)
    rng = np.random.default_rng(5)
    gamma, tau = 2e-2, 5e-2
    N = 64
    p0 = gaussian_bumps(shape, rng.uniform(0.3, 0.7, size=(2, 2)), 0.15, [0.5, 0.5])
    w = rng.uniform(0, 1, size=shape)
    kappa = np.full(shape, 1.6 / N)
    kappa[0, :3] = 0.0
    target = rng.uniform(size=shape)
    target /= target.sum()
    iters = [25, 25, 25]
    en = O.Energy(kind="congestion", w=w, kappa=kappa)

    def fwd(p0_, w_):
        e = O.Energy(kind="congestion", w=w_, kappa=kappa)
        q = p0_
        for K in iters:
            q, _ = O.jko_step(q, e, gamma, tau, K)
        return float(((q - target) ** 2).sum())

    loss, gw, gp, pT = loss_and_grads(p0, w, kappa, gamma, tau, iters, target)
    assert loss == pytest.approx(fwd(p0, w), rel=1e-13)
    cells = [(1, 1), (4, 5), (6, 2), (7, 7), (0, 5)]
    for c in cells:
        h = 1e-5
        wp, wm = w.copy(), w.copy()
        wp[c] += h
        wm[c] -= h
        fd = (fwd(p0, wp) - fwd(p0, wm)) / (2 * h)
        assert gw[c] == pytest.approx(fd, rel=1e-5, abs=1e-12 * abs(loss))
        hp = 1e-5 * p0[c]
        pp, pm = p0.copy(), p0.copy()
        pp[c] += hp
        pm[c] -= hp
        fd = (fwd(pp, w) - fwd(pm, w)) / (2 * hp)
        assert gp[c] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(loss))


@pytest.mark.parametrize("kind", ["porous", "entropy", "zero"])
def test_reference_gradient_other_energies_match_finite_differences(kind):
    """autograd through the unrolled flow == central differences of the numpy
    oracle's forward map in p0 for the porous-medium energy (exact Lambert-W
    prox differentiated through its implicit derivative; density units, so
    that the nonlinearity is active), the weighted entropy (per-cell weights)
    and f = 0."""
    shape = (8, 7)
    rng = np.random.default_rng(12)
    gamma, tau = 2e-2, 5e-2
    N = int(np.prod(shape))
    p0 = gaussian_bumps(shape, rng.uniform(0.3, 0.7, size=(2, 2)), 0.15, [0.6, 0.4])
    target = rng.uniform(size=shape)
    target /= target.sum()
    iters = [15, 15]
    coef = m = None
    D = 1.0
    if kind == "porous":
        coef, m, D = rng.uniform(0.5, 2.0, size=shape), 2.0, float(N)
        en = O.Energy(kind="porous", coef=coef, m=m, density_scale=D)
        # the prox is nonlinear here: (m-1) k psi^{m-1} is of order one
        k = en.porous_k(tau / gamma, shape)
        z = ((m - 1.0) * k * O.prox_porous(p0, k, m) ** (m - 1.0)).max()
        assert z > 0.5
    elif kind == "entropy":
        coef = rng.uniform(0.2, 3.0, size=shape)
        en = O.Energy(kind="entropy", coef=coef)
    else:
        en = O.Energy(kind="zero")

    def fwd(p0_):
        q = p0_
        for K in iters:
            q, _ = O.jko_step(q, en, gamma, tau, K)
        return float(((q - target) ** 2).sum())

    loss, _, gp, _ = loss_and_grads(p0, np.zeros(shape), np.inf, gamma, tau, iters, target, kind=kind,
                                    coef=coef, m=m, density_scale=D)
    assert loss == pytest.approx(fwd(p0), rel=1e-12)
    for c in [(1, 1), (4, 5), (6, 2), (7, 6), (0, 3)]:
        hp = 1e-5 * p0[c]
        pp, pm = p0.copy(), p0.copy()
        pp[c] += hp
        pm[c] -= hp
        fd = (fwd(pp) - fwd(pm)) / (2 * hp)
        assert gp[c] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(loss))
