"""FP64 CPU oracle of one entropic JKO step and of the JKO flow.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or links
this module: only the test suite, the smoke check and the CPU-baseline leg of
the benchmark use it.  It is deliberately plain and slow, written in numpy
float64 from the paper's definitions, and shares no code with the HIP library.

Notation follows the paper (Peyre, "Entropic Wasserstein Gradient Flows",
SIAM J. Imaging Sci. 2015):

* grid points x_i on a uniform cell-centred grid of [0,1]^d; cost
  c_ij = |x_i - x_j|^2 (Section 2.1, alpha = 2);
* Gibbs kernel xi = exp(-c / gamma) (Section 3.1, eq. defn-KL-prbm);
* one JKO step q = p_t -> p_{t+1} = argmin_p W_gamma(p, q) + tau f(p)
  (Section 2.2, eq. def-jko-operator), solved by KL Dykstra in its diagonal
  scaling form (Section 3.4, Proposition 3.3) with the stopping test of
  Listing 1 on the violation of the constraint pi^T 1 = q;
* KL proximal maps of f (Section 4.2 Proposition 4.1 congestion,
  Section 4.4 Proposition 4.2 generalised entropies);
* the Wasserstein attraction with congestion of Section 5.2: the M = 2
  scaling of Proposition 5.2 verbatim (``attraction_generic``) and reduced
  (``attraction_step``).

Three forms of the same iteration are kept so that the tests can pin each
against the next:

``dykstra_coupling``  the KL Dykstra iteration on explicit N x N couplings with
                      the two explicit proximal maps of Proposition 3.2
                      (eq. iter-dystra-1/2, eq. formula-prox-explicit);
``dykstra_scaling``   Proposition 3.3 verbatim: scalings a, b and correction
                      factors u, v, half-step counter l;
``jko_step``          the same iteration after the corrections are dropped:
                      u = 1 after odd half-steps and u = 1/a after even ones
                      (and v = 1 after even ones), so the prox argument
                      a * u * (xi b) is xi b itself.  This is the form the
                      HIP path computes; one "iteration" is one odd plus one
                      even half-step.

``jko_step_log`` runs ``jko_step`` with every quantity in log form and the
Gibbs products as exact log-sum-exp sums, for inputs whose scalings leave the
floating-point range.

Energies (``Energy``):

* ``zero``        f = 0, prox = identity;
* ``congestion``  f = iota_[0,kappa](p) + <w, p>, prox min(s e^{-sigma w}, kappa)
                  (Proposition 4.1); kappa may be a field and may be +inf;
* ``binary_congestion``  f = iota_{{0,kappa}^N}(p) + <w, p>, the non-convex
                  functional of Section 4.5 (eq. dfn-congestion-noncvx).  Its
                  KL prox is taken as its definition: per cell the argmin of
                  KL(p|s) + sigma w p over the two candidates p in {0, kappa}
                  (kappa finite), the tie going to kappa;
* ``gen_entropy`` f = sum_i b_i e_{m_i}(D p_i) / D, the generalised entropies
                  of Section 4.4 (eq. defn-gen-entropies) with weights b_i and
                  exponents m_i >= 1 per cell (D = 1: the paper's form).  Per
                  Proposition 4.2 the prox of sigma b e_m is s^{1/(1+sigma b)}
                  for m = 1 and otherwise the root psi of eq. prox-psi
                  (sigma -> sigma b, applied to D s); the oracle takes that
                  root exactly through Lambert W;
* ``entropy``     f = sum c_i p_i (log p_i - 1), prox s^{1/(1 + sigma c)}
                  (Proposition 4.2, m = 1, weight c);
* ``porous``      f = sum c_i (D p_i)^m / ((m-1) D) with density scale D
                  (D = 1: per-cell mass).  Its KL prox psi solves
                  log psi + k psi^{m-1} = log s with k = sigma c m D^{m-1}/(m-1)
                  (the first-order condition, as for Proposition 4.2); the
                  oracle takes the exact root through the Lambert W function:
                  psi = (W((m-1) k s^{m-1}) / ((m-1) k))^{1/(m-1)}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
from scipy.special import lambertw, logsumexp
from scipy.spatial.distance import cdist


# --------------------------------------------------------------------------
# Grid and Gibbs kernel (Section 2.1, Section 3.1, Section 4.1)
# --------------------------------------------------------------------------

def grid_points(n: int) -> np.ndarray:
    """Cell centres (i + 1/2)/n of a uniform grid of [0, 1]."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def all_points(shape) -> np.ndarray:
    """(N, d) array of the cell centres in row-major (last axis fastest) order."""
    mesh = np.meshgrid(*[grid_points(n) for n in shape], indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1)


def gibbs_dense(shape, gamma: float) -> np.ndarray:
    """The full N x N Gibbs kernel xi_ij = exp(-|x_i - x_j|^2 / gamma)
    (Section 3.1) built from the pairwise distances of all grid points."""
    P = all_points(shape)
    return np.exp(-cdist(P, P, "sqeuclidean") / gamma)


def gibbs_rows(shape, gamma: float, flat_index: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(xi x)[I] for selected flat cell indices I, each as the plain sum
    sum_J exp(-|x_I - x_J|^2 / gamma) x_J over all N cells (Section 3.1);
    for spot checks of large grids."""
    P = all_points(shape)
    xv = x.ravel()
    out = np.empty(len(flat_index))
    for r, I in enumerate(np.asarray(flat_index)):
        d2 = ((P - P[I]) ** 2).sum(axis=1)
        out[r] = np.dot(np.exp(-d2 / gamma), xv)
    return out


def gibbs_factor(n: int, gamma: float) -> np.ndarray:
    """One-axis factor K1_ij = exp(-(x_i - x_j)^2 / gamma).  On a uniform grid
    with squared Euclidean cost, xi is the Kronecker product of these factors
    (the separable Gaussian convolution of Section 4.1)."""
    x = grid_points(n)
    return np.exp(-((x[:, None] - x[None, :]) ** 2) / gamma)


def gibbs_apply(x: np.ndarray, gamma: float, mode: str = "separable",
                transpose: bool = False) -> np.ndarray:
    """xi x (or xi^T x) for a field x of the grid's shape."""
    if mode == "dense":
        xi = gibbs_dense(x.shape, gamma)
        if transpose:
            xi = xi.T
        return (xi @ x.ravel()).reshape(x.shape)
    if mode != "separable":
        raise ValueError(mode)
    y = x
    for ax, n in enumerate(x.shape):
        K = gibbs_factor(n, gamma)
        if transpose:
            K = K.T
        y = np.moveaxis(np.tensordot(K, np.moveaxis(y, ax, 0), axes=(1, 0)), 0, ax)
    return y


def log_gibbs_apply(L: np.ndarray, gamma: float) -> np.ndarray:
    """log(xi exp(L)) computed axis by axis with exact log-sum-exp, so that
    neither the kernel entries nor the argument ever leave the float range.
    -inf entries of L stand for exact zeros."""
    y = L
    for ax, n in enumerate(L.shape):
        x = grid_points(n)
        logK = -((x[:, None] - x[None, :]) ** 2) / gamma          # (i, j)
        ym = np.moveaxis(y, ax, -1)                                 # (..., j)
        out = logsumexp(logK[(None,) * (ym.ndim - 1)] + ym[..., None, :], axis=-1)
        y = np.moveaxis(out, -1, ax)
    return y


# --------------------------------------------------------------------------
# Energies and their KL proximal maps (Section 4.2, Section 4.4)
# --------------------------------------------------------------------------

@dataclass
class Energy:
    kind: str = "zero"                     # zero | congestion | binary_congestion | entropy | porous | gen_entropy
    w: Optional[np.ndarray] = None         # congestion potential; None = 0
    kappa: Optional[np.ndarray] = None     # capacity; None = kappa_scalar
    kappa_scalar: float = math.inf
    coef: Optional[np.ndarray] = None      # entropy / porous weight; None = coef_scalar
    coef_scalar: float = 1.0
    m: float = 2.0
    density_scale: float = 1.0
    m_field: Optional[np.ndarray] = None   # gen_entropy exponents per cell; None = m

    def _w(self, shape):
        return np.zeros(shape) if self.w is None else np.asarray(self.w, np.float64)

    def _kappa(self, shape):
        if self.kappa is None:
            return np.full(shape, self.kappa_scalar, dtype=np.float64)
        return np.asarray(self.kappa, np.float64)

    def _coef(self, shape):
        if self.coef is None:
            return np.full(shape, self.coef_scalar, dtype=np.float64)
        return np.asarray(self.coef, np.float64)

    def _m(self, shape):
        if self.m_field is None:
            return np.full(shape, self.m, dtype=np.float64)
        return np.asarray(self.m_field, np.float64)

    def porous_k(self, sigma: float, shape) -> np.ndarray:
        m = self.m
        return sigma * self._coef(shape) * m * self.density_scale ** (m - 1.0) / (m - 1.0)


def prox_congestion(s, sigma, w, kappa):
    """Proposition 4.1: Prox^KL_{sigma f}(s) = min(s e^{-sigma w}, kappa)."""
    return np.minimum(s * np.exp(-sigma * w), kappa)


def kl_cell(p, s):
    """KL(p|s) = p log(p/s) - p + s per cell, with 0 log 0 = 0 and +inf for
    p > 0 = s (Section 3.1, eq. defn-KL-prbm, one term)."""
    p = np.asarray(p, np.float64)
    s = np.asarray(s, np.float64)
    out = np.array(s, dtype=np.float64, copy=True)      # p = 0: the term is s
    pos = p > 0
    with np.errstate(divide="ignore"):
        out[pos] = np.where(s[pos] > 0, p[pos] * np.log(p[pos] / np.where(s[pos] > 0, s[pos], 1.0)) - p[pos] + s[pos],
                            np.inf)
    return out


def prox_binary_congestion(s, sigma, w, kappa):
    """Section 4.5, eq. dfn-congestion-noncvx: KL prox of
    sigma (iota_{{0,kappa}} + <w, .>), written as its definition: per cell
    the candidate p in {0, kappa} of least KL(p|s) + sigma w p; at a tie kappa
    is taken (the prox is two-valued there)."""
    s = np.asarray(s, np.float64)
    shape = s.shape
    w = np.broadcast_to(np.asarray(w, np.float64), shape)
    kappa = np.broadcast_to(np.asarray(kappa, np.float64), shape)
    zero = kl_cell(np.zeros(shape), s)
    full = kl_cell(kappa, s) + sigma * w * kappa
    return np.where(full <= zero, kappa, 0.0)


def prox_entropy(s, sigma, coef):
    """Proposition 4.2, m = 1 with weight c: s^{1/(1 + sigma c)}."""
    return np.power(s, 1.0 / (1.0 + sigma * coef))


def prox_porous(s, k, m):
    """Root psi > 0 of log psi + k psi^{m-1} = log s, exactly, through the
    principal branch of Lambert W; psi = 0 at s = 0 and psi = s where k = 0."""
    s = np.asarray(s, np.float64)
    k = np.broadcast_to(np.asarray(k, np.float64), s.shape)
    out = np.array(s, dtype=np.float64, copy=True)
    pos = (s > 0) & (k > 0)
    z = (m - 1.0) * k[pos] * s[pos] ** (m - 1.0)
    out[pos] = (lambertw(z).real / ((m - 1.0) * k[pos])) ** (1.0 / (m - 1.0))
    return out


def log_prox_gen_entropy(logs, sigma, b, m, D):
    """Proposition 4.2 per cell for sigma b e_m applied to the density D p:
    log psi, psi = D p, is Y = L / (1 + sigma b) for m = 1 (eq. prox-entropy)
    and otherwise the root of eq. prox-psi with sigma -> sigma b:
        Y + sigma b m (e^{(m-1) Y} - 1) / (m - 1) = L,   L = log(D s).
    With c = sigma b m and u = (m-1) Y this is u + c e^u = (m-1) L + c, so
    c e^u = W(c e^{(m-1) L + c}) (Lambert W, principal branch) and
    Y = log(W / c) / (m - 1).  Returns log p = Y - log D (-inf where s = 0)."""
    logs = np.asarray(logs, np.float64)
    shape = logs.shape
    b = np.broadcast_to(np.asarray(b, np.float64), shape)
    m = np.broadcast_to(np.asarray(m, np.float64), shape)
    L = logs + math.log(D)
    out = np.full(shape, -np.inf)
    fin = np.isfinite(logs)
    one = fin & ((m == 1.0) | (b == 0.0))
    out[one] = L[one] / (1.0 + sigma * b[one])          # b = 0: the identity
    gen = fin & ~one
    c = sigma * b[gen] * m[gen]
    eps = m[gen] - 1.0
    W = lambertw_of_log(np.log(c) + eps * L[gen] + c)
    out[gen] = np.log(W / c) / eps
    return out - math.log(D)


def lambertw_of_log(logz: np.ndarray) -> np.ndarray:
    """Principal Lambert W at z = exp(logz), also where exp(logz) overflows:
    there W solves W + log W = logz (Newton from W = logz)."""
    logz = np.asarray(logz, np.float64)
    out = np.zeros_like(logz)
    small = logz < 700.0
    with np.errstate(over="ignore", invalid="ignore"):
        out[small] = lambertw(np.exp(logz[small])).real
    big = ~small
    if big.any():
        L = logz[big]
        Wv = L - np.log(L)
        for _ in range(50):
            Wv = Wv - (Wv + np.log(Wv) - L) / (1.0 + 1.0 / Wv)
        out[big] = Wv
    return out


def prox(s: np.ndarray, sigma: float, en: Energy) -> np.ndarray:
    """Prox^KL_{sigma f}(s) for the energy ``en`` (pointwise)."""
    shape = s.shape
    if en.kind == "zero":
        return s.copy()
    if en.kind == "congestion":
        return prox_congestion(s, sigma, en._w(shape), en._kappa(shape))
    if en.kind == "binary_congestion":
        return prox_binary_congestion(s, sigma, en._w(shape), en._kappa(shape))
    if en.kind == "entropy":
        return prox_entropy(s, sigma, en._coef(shape))
    if en.kind == "porous":
        return prox_porous(s, en.porous_k(sigma, shape), en.m)
    if en.kind == "gen_entropy":
        with np.errstate(divide="ignore"):
            return np.exp(log_prox_gen_entropy(np.log(s), sigma, en._coef(shape), en._m(shape), en.density_scale))
    raise ValueError(en.kind)


def log_prox(logs: np.ndarray, sigma: float, en: Energy) -> np.ndarray:
    """log Prox^KL_{sigma f}(exp(logs)), evaluated without leaving log form."""
    shape = logs.shape
    if en.kind == "zero":
        return logs.copy()
    if en.kind == "congestion":
        with np.errstate(divide="ignore"):
            return np.minimum(logs - sigma * en._w(shape), np.log(en._kappa(shape)))
    if en.kind == "binary_congestion":
        # the same two-candidate argmin with s = e^logs: kappa wins when
        # kappa (log kappa - logs - 1 + sigma w) <= 0, so for kappa > 0 when
        # log kappa - logs + sigma w <= 1 (logs = -inf: never)
        kappa = en._kappa(shape)
        with np.errstate(divide="ignore", invalid="ignore"):
            lk = np.log(kappa)
            take = (kappa > 0) & np.isfinite(logs) & (lk - logs + sigma * en._w(shape) <= 1.0)
        return np.where(take, lk, -np.inf)
    if en.kind == "entropy":
        return logs / (1.0 + sigma * en._coef(shape))
    if en.kind == "porous":
        # y = log psi solves y + k e^{(m-1) y} = logs, i.e.
        # y = logs - W(z) / (m - 1) with z = (m-1) k e^{(m-1) logs}
        k = en.porous_k(sigma, shape)
        m = en.m
        with np.errstate(divide="ignore"):
            logz = np.log((m - 1.0) * k) + (m - 1.0) * logs
        W = lambertw_of_log(logz)
        return np.where(np.isfinite(logs), logs - W / (m - 1.0), -np.inf)
    if en.kind == "gen_entropy":
        return log_prox_gen_entropy(logs, sigma, en._coef(shape), en._m(shape), en.density_scale)
    raise ValueError(en.kind)


def _safe_div(num, den):
    """num / den with the convention 0 / 0 = 0."""
    out = np.zeros_like(num)
    nz = num != 0
    out[nz] = num[nz] / den[nz]
    return out


# --------------------------------------------------------------------------
# The KL Dykstra iteration in its three forms (Section 3.3, Section 3.4)
# --------------------------------------------------------------------------

def dykstra_coupling(q: np.ndarray, en: Energy, gamma: float, tau: float,
                     n_half_steps: int) -> np.ndarray:
    """KL Dykstra on explicit couplings (eq. iter-dystra-1/2) with the two
    proximal maps of Proposition 3.2.  phi_1 = iota_{C_q} (odd half-steps),
    phi_2 = (tau/gamma) f(pi 1) (even half-steps).  Returns p = pi 1 after the
    last half-step.  Tiny grids only (N x N matrices)."""
    shape = q.shape
    sigma = tau / gamma
    qv = q.ravel()
    pi_prev = gibbs_dense(shape, gamma)              # pi^(0) = xi
    ones = np.ones_like(pi_prev)
    z_hist = {-1: ones, 0: ones}                     # z^(-1) = z^(0) = 1
    for l in range(1, n_half_steps + 1):
        arg = pi_prev * z_hist[l - 2]
        if l % 2 == 1:
            col = arg.sum(axis=0)                    # arg^T 1
            pi = arg * (qv / col)[None, :]           # arg diag(q / arg^T 1)
        else:
            row = arg.sum(axis=1)                    # arg 1
            pr = prox(row.reshape(shape), sigma, en).ravel()
            pi = (pr / row)[:, None] * arg           # diag(prox(arg 1)/arg 1) arg
        z_hist[l] = z_hist[l - 2] * pi_prev / pi
        pi_prev = pi
    return pi_prev.sum(axis=1).reshape(shape)


def dykstra_scaling(q: np.ndarray, en: Energy, gamma: float, tau: float,
                    n_half_steps: int, mode: str = "dense"):
    """Proposition 3.3 as stated: pi = diag(a) xi diag(b), z = u v^T, all four
    vectors initialised to 1, odd half-steps by eq. update-formula-1, even ones
    by eq. update-formula-2 with p from eq. defn-pell, and the u, v updates of
    eq. update-formula-3.  Returns (p, a, b, u, v) after the last half-step
    (which should be even, so that p is defined)."""
    sigma = tau / gamma
    one = np.ones_like(q)
    a, b = one.copy(), one.copy()
    u_hist = {-1: one, 0: one}
    v_hist = {-1: one, 0: one}
    p = None
    for l in range(1, n_half_steps + 1):
        a_prev, b_prev = a, b
        if l % 2 == 1:
            a = a_prev * u_hist[l - 2]
            b = q / gibbs_apply(a, gamma, mode, transpose=True)
        else:
            b = b_prev * v_hist[l - 2]
            xb = gibbs_apply(b, gamma, mode)
            p = prox(a_prev * u_hist[l - 2] * xb, sigma, en)
            a = p / xb
        u_hist[l] = u_hist[l - 2] * a_prev / a
        v_hist[l] = v_hist[l - 2] * b_prev / b
    return p, a, b, u_hist[n_half_steps], v_hist[n_half_steps]


def jko_step(q: np.ndarray, en: Energy, gamma: float, tau: float, max_iters: int,
             tol: float = 0.0, check_every: int = 1, mode: str = "separable", op=None,
             observe=None):
    """One JKO step: the reduced scaling iteration (Proposition 3.3 with the
    u, v corrections dropped) and the stopping test of Listing 1.

    Iteration k (k = 1, 2, ...) is one odd half-step (b = q / xi^T a) and one
    even half-step (s = xi b, p = Prox(s), a = p / s).  The violation
    err = || b * xi^T a - q ||_1 after an even half-step reuses t = xi^T a,
    the first product of the next iteration; it is evaluated at iteration k
    when k - 1 is a positive multiple of ``check_every`` and tol > 0.  The step
    stops there if err <= tol and returns the p of iteration k - 1.

    Returns (p, stats) with stats = {iters, marginal_l1, mass, stop}; the
    reported marginal_l1 is the violation of the returned iterate.
    Conventions: 0 / 0 = 0 in both divisions.

    ``op`` (optional) replaces the Gibbs kernel by another symmetric operator
    called as op(x): the heat kernel of Section 4.1 (``HeatKernel``).
    ``observe`` (optional) is called as observe(k, s, p) after the proximal
    half-step of every iteration; it only looks (the tests use it to record
    which cells the congestion clamp caps).
    """
    sigma = tau / gamma

    def K(x, transpose=False):
        return gibbs_apply(x, gamma, mode, transpose=transpose) if op is None else op(x)

    a = np.ones_like(q)
    b = None
    p = None
    err = math.nan
    for k in range(1, max_iters + 1):
        t = K(a, transpose=True)
        if k > 1 and tol > 0 and (k - 1) % check_every == 0:
            err = float(np.abs(b * t - q).sum())
            if err <= tol:
                return p, dict(iters=k - 1, marginal_l1=err, mass=float(p.sum()), stop="tol")
        b = _safe_div(q, t)
        s = K(b)
        p = prox(s, sigma, en)
        if observe is not None:
            observe(k, s, p)
        a = _safe_div(p, s)
    t = K(a, transpose=True)
    err = float(np.abs(b * t - q).sum())
    return p, dict(iters=max_iters, marginal_l1=err, mass=float(p.sum()), stop="cap")


# --------------------------------------------------------------------------
# Wasserstein attraction with congestion (Section 5.1, Section 5.2)
# --------------------------------------------------------------------------

def prox_attraction_psi1(p1, p2, tau, kappa):
    """eq. prox-psi-attraction with h = iota_[0,kappa]: the KL_lambda prox
    (lambda = (1, tau)) of psi_1 = iota_D + h is (p, p) with
    p = Prox^KL_{h/(1+tau)}(p1^{1/(1+tau)} p2^{tau/(1+tau)}), and the KL prox of
    an indicator of [0, kappa] is the clamp (eq. dfn-congestion-prox)."""
    return np.minimum(np.power(p1, 1.0 / (1.0 + tau)) * np.power(p2, tau / (1.0 + tau)), kappa)


def attraction_generic(q, r, kappa, gamma, tau, n_half_steps, first=1, mode="separable"):
    """Proposition 5.2 as stated for M = 2 couplings with xi_1 = xi_2 = xi and
    the functions of Section 5.2: psi_1 = iota_D + h on the left marginals
    pi_m 1, psi_2 = iota_{(q, r)} on the right marginals pi_m^T 1.  All of
    a_m, b_m, u_m, v_m start at 1.  ``first`` names the function of the odd
    half-steps: 1 as printed ([l]_2 = 1 is psi_1), 2 for the other order (the
    marginals first, as Proposition 3.3 orders its two functions).  Returns
    (p, a, b, u, v), p the common left marginal of the last psi_1 half-step.
    Conventions: 0 / 0 = 0."""
    one = np.ones_like(q)
    a = [one.copy(), one.copy()]
    b = [one.copy(), one.copy()]
    u_hist = {-1: [one, one], 0: [one, one]}
    v_hist = {-1: [one, one], 0: [one, one]}
    targets = (q, r)
    p = None
    for l in range(1, n_half_steps + 1):
        which = first if l % 2 == 1 else 3 - first
        at = [a[m] * u_hist[l - 2][m] for m in range(2)]       # a~ = a (l-1) * u (l-2)
        bt = [b[m] * v_hist[l - 2][m] for m in range(2)]       # b~ = b (l-1) * v (l-2)
        a_prev, b_prev = a, b
        if which == 1:
            xb = [gibbs_apply(bt[m], gamma, mode) for m in range(2)]
            pt = [at[m] * xb[m] for m in range(2)]
            p = prox_attraction_psi1(pt[0], pt[1], tau, kappa)
            a = [_safe_div(p, xb[m]) for m in range(2)]
            b = bt
        else:
            xa = [gibbs_apply(at[m], gamma, mode, transpose=True) for m in range(2)]
            b = [_safe_div(targets[m], xa[m]) for m in range(2)]
            a = at
        u_hist[l] = [u_hist[l - 2][m] * _safe_div(a_prev[m], a[m]) for m in range(2)]
        v_hist[l] = [v_hist[l - 2][m] * _safe_div(b_prev[m], b[m]) for m in range(2)]
    return p, a, b, u_hist[n_half_steps], v_hist[n_half_steps]


def attraction_step(q, r, kappa, gamma, tau, max_iters, tol=0.0, check_every=1, mode="separable"):
    """One JKO step of f = W_gamma(r, .) + iota_[0,kappa] (Section 5.2): the
    scaling of Proposition 5.2 with the marginals first and the corrections
    dropped, as ``jko_step`` does for one coupling.  Iteration k:
        t_m = xi^T a_m,  b_1 = q / t_1,  b_2 = r / t_2,  s_m = xi b_m,
        p = min(s_1^{1/(1+tau)} s_2^{tau/(1+tau)}, kappa),  a_m = p / s_m.
    The monitor is the violation of both couplings' right marginals,
    ||b_1 t_1 - q||_1 + ||b_2 t_2 - r||_1, with the stop rule and the
    statistics of ``jko_step``.  The two couplings need marginals of one mass:
    r is taken as a shape and scaled to the mass of q."""
    r = r * (q.sum() / r.sum())
    a = [np.ones_like(q), np.ones_like(q)]
    b = None
    p = None
    targets = (q, r)

    def violation(t):
        return float(sum(np.abs(b[m] * t[m] - targets[m]).sum() for m in range(2)))

    for k in range(1, max_iters + 1):
        t = [gibbs_apply(a[m], gamma, mode, transpose=True) for m in range(2)]
        if k > 1 and tol > 0 and (k - 1) % check_every == 0:
            err = violation(t)
            if err <= tol:
                return p, dict(iters=k - 1, marginal_l1=err, mass=float(p.sum()), stop="tol")
        b = [_safe_div(targets[m], t[m]) for m in range(2)]
        sv = [gibbs_apply(b[m], gamma, mode) for m in range(2)]
        p = prox_attraction_psi1(sv[0], sv[1], tau, kappa)
        a = [_safe_div(p, sv[m]) for m in range(2)]
    t = [gibbs_apply(a[m], gamma, mode, transpose=True) for m in range(2)]
    return p, dict(iters=max_iters, marginal_l1=violation(t), mass=float(p.sum()), stop="cap")


def attraction_step_log(q, r, kappa, gamma, tau, max_iters, tol=0.0, check_every=1):
    """``attraction_step`` with log a_m, log b_m, log t_m, log s_m and the Gibbs
    products as exact log-sum-exp (``log_gibbs_apply``); the proximal step is
    log p = min(log s_1 / (1+tau) + tau log s_2 / (1+tau), log kappa).  Same
    stopping rule and return values; exact zeros are -inf."""
    r = r * (q.sum() / r.sum())
    targets = (q, r)
    with np.errstate(divide="ignore"):
        logt = (np.log(q), np.log(r))
        lk = np.log(np.broadcast_to(np.asarray(kappa, np.float64), q.shape))
    alpha = 1.0 / (1.0 + tau)
    La = [np.zeros_like(q), np.zeros_like(q)]
    Lb = None
    Lp = None

    def violation(Lt):
        return float(sum(np.abs(np.exp(Lb[m] + Lt[m]) - targets[m]).sum() for m in range(2)))

    for k in range(1, max_iters + 1):
        Lt = [log_gibbs_apply(La[m], gamma) for m in range(2)]
        if k > 1 and tol > 0 and (k - 1) % check_every == 0:
            err = violation(Lt)
            if err <= tol:
                p = np.exp(Lp)
                return p, dict(iters=k - 1, marginal_l1=err, mass=float(p.sum()), stop="tol")
        Lb = [logt[m] - Lt[m] for m in range(2)]
        Ls = [log_gibbs_apply(Lb[m], gamma) for m in range(2)]
        Lp = np.minimum(alpha * Ls[0] + (1.0 - alpha) * Ls[1], lk)
        La = [np.where(np.isneginf(Lp), -np.inf, Lp - Ls[m]) for m in range(2)]
    Lt = [log_gibbs_apply(La[m], gamma) for m in range(2)]
    p = np.exp(Lp)
    return p, dict(iters=max_iters, marginal_l1=violation(Lt), mass=float(p.sum()), stop="cap")


def jko_step_log(q: np.ndarray, en: Energy, gamma: float, tau: float, max_iters: int,
                 tol: float = 0.0, check_every: int = 1):
    """``jko_step`` with log a, log b, log t, log s instead of a, b, t, s and the
    Gibbs products as exact log-sum-exp (``log_gibbs_apply``).  Same stopping
    rule and return values; exact zeros are -inf."""
    sigma = tau / gamma
    with np.errstate(divide="ignore"):
        logq = np.log(q)
    La = np.zeros_like(q)
    Lb = None
    Lp = None
    err = math.nan
    for k in range(1, max_iters + 1):
        Lt = log_gibbs_apply(La, gamma)
        if k > 1 and tol > 0 and (k - 1) % check_every == 0:
            err = float(np.abs(np.exp(Lb + Lt) - q).sum())
            if err <= tol:
                p = np.exp(Lp)
                return p, dict(iters=k - 1, marginal_l1=err, mass=float(p.sum()), stop="tol")
        Lb = logq - Lt
        Ls = log_gibbs_apply(Lb, gamma)
        Lp = log_prox(Ls, sigma, en)
        La = np.where(np.isneginf(Lp), -np.inf, Lp - Ls)
    Lt = log_gibbs_apply(La, gamma)
    err = float(np.abs(np.exp(Lb + Lt) - q).sum())
    p = np.exp(Lp)
    return p, dict(iters=max_iters, marginal_l1=err, mass=float(p.sum()), stop="cap",
                   max_abs_log_a=float(np.max(np.abs(La[np.isfinite(La)]), initial=0.0)),
                   max_abs_log_b=float(np.max(np.abs(Lb[np.isfinite(Lb)]), initial=0.0)))


def jko_flow(p0: np.ndarray, en: Energy, gamma: float, tau: float, n_steps: int,
             max_iters: int, tol: float = 0.0, check_every: int = 1,
             mode: str = "separable", log_domain: bool = False):
    """The JKO flow p_{t+1} = Prox^{W_gamma}_{tau f}(p_t) (eq. smooth-jko) with
    fixed gamma and tau, cold-started at every step (Listing 1, step 2).
    Returns (p_T, [p_1, ..., p_T], [stats_1, ...])."""
    q = np.asarray(p0, np.float64)
    traj, stats = [], []
    for _ in range(n_steps):
        if log_domain:
            q, st = jko_step_log(q, en, gamma, tau, max_iters, tol, check_every)
        else:
            q, st = jko_step(q, en, gamma, tau, max_iters, tol, check_every, mode)
        traj.append(q)
        stats.append(st)
    return q, traj, stats
