"""Writes the FP64 reference data of the differentiation workload
(``c4_gradients.npz``): the 256 x 256 crowd-motion flow of 20 JKO steps x 300
iterations (squared distance to the exit as potential w, the obstacle
capacity, loss ||p_T - target||^2 with a Gaussian target near the exit) and
its 32 x 32 instance (the 32 x 32 crowd's geometry and parameters with the
same loss).

For each instance it stores, from the oracle only:
* the loss and the gradients dL/dw and dL/dp0 by float64 autograd through the
  unrolled iteration (``oracle.grad.loss_and_grads``);
* central finite differences of the oracle's forward map at 64 seeded cells:
  w[c] +- 1e-3 (absolute) and p0[c] (1 +- 1e-3) (relative: an absolute 1e-3
  is many times a cell's mass), with a flag per cell telling whether the
  set of cells the congestion clamp caps differs between the two runs at any
  iteration (there the map has a kink inside the difference interval and the
  difference is not a derivative);
* directional central differences along two seeded random directions per
  variable: w + h v (v standard normal on the free cells, h = 1e-3) and
  p0 (1 + h v) (v standard normal on the occupied cells, h = 1e-4), with
  the number of (iteration, cell) pairs whose capped state differs between
  the two runs; the matching directional derivatives of the autograd
  gradients are <dL/dw, v> and <dL/dp0, p0 v>;
* a digest of the float32 inputs, so that the tests can tell when the
  workload recipe has changed since this file was written.

Run from the repository root:  python tests/golden/make_c4_gradients.py
(about 1.6 hours on 8 cores; the 256^2 autograd tape holds ~25 GB).
``--directional-only`` recomputes only the directional differences (a few
minutes) and rewrites them into the existing file.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle.grad import loss_and_grads  # noqa: E402
from workloads import make_workload, gaussian_bumps  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_gradients.npz")
N_STEPS, ITERS, H, N_CELLS = 20, 300, 1e-3, 64
H_DIR_W, H_DIR_P, N_DIRS = 1e-3, 1e-4, 2


def instance(name):
    """(workload, float32-rounded p0, w, kappa as float64, target)."""
    wl = make_workload(name, projected=True)
    ex = wl.extras["exit"]
    target = gaussian_bumps(wl.shape, [ex - np.array([0.1] + [0.0] * (len(wl.shape) - 1))], 0.05, [1.0])
    target[wl.extras["mask"]] = 0.0
    target /= target.sum()
    r = lambda a: np.asarray(a, np.float64).astype(np.float32).astype(np.float64)
    return wl, r(wl.p0), r(wl.w), r(wl.kappa_field()), target


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(np.asarray(a, np.float32)).tobytes())
    return h.hexdigest()


# Rounding error of the oracle's loss relative to its value (a sum after
# 6000 iterations in float64), for the noise floor of a difference quotient.
LOSS_ROUNDING = 1e-14


def fd_cells_valid(data, tag, which, p0):
    """Cells whose central difference is a derivative to within 1e-4 of the
    gradient: the capped set did not change inside the interval, and the
    loss's rounding divided by the step (absolute for w, h p0[c] for p0)
    is below 1e-4 of the stored autograd gradient's magnitude there."""
    cells = data[f"{tag}_cells_{which}"]
    g = np.abs(np.asarray(data[f"{tag}_g{which}"], np.float64).ravel()[cells])
    step = 2 * H if which == "w" else 2 * H * p0.ravel()[cells]
    noise = LOSS_ROUNDING * abs(float(data[f"{tag}_loss"])) / step
    return ~data[f"{tag}_kink_{which}"] & (noise <= 1e-4 * g)


def forward(args):
    """Loss of the oracle's flow and a digest of every iteration's capped set."""
    name, p0, w, kappa, target = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass
    wl = make_workload(name, projected=True)
    en = O.Energy(kind="congestion", w=w, kappa=kappa)
    h = hashlib.sha256()

    def observe(k, s, p):
        h.update(np.packbits(p >= kappa).tobytes())

    q = p0
    for _ in range(N_STEPS):
        q, _ = O.jko_step(q, en, wl.gamma, wl.tau, ITERS, observe=observe)
    return float(((q - target) ** 2).sum()), h.hexdigest()


def forward_masks(args):
    """Loss of the oracle's flow and the capped set of every iteration
    (packed bits, one row per iteration)."""
    name, p0, w, kappa, target = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass
    wl = make_workload(name, projected=True)
    en = O.Energy(kind="congestion", w=w, kappa=kappa)
    masks = []

    def observe(k, s, p):
        masks.append(np.packbits(p >= kappa))

    q = p0
    for _ in range(N_STEPS):
        q, _ = O.jko_step(q, en, wl.gamma, wl.tau, ITERS, observe=observe)
    return float(((q - target) ** 2).sum()), np.stack(masks)


def directional(name, tag):
    """Directional central differences of the oracle's loss (see the module
    docstring); the directions are stored with them."""
    _, p0, w, kappa, target = instance(name)
    rng = np.random.default_rng(7)
    vw = [rng.normal(size=w.shape) * (kappa > 0) for _ in range(N_DIRS)]
    vp = [rng.normal(size=p0.shape) * (p0 > 0) for _ in range(N_DIRS)]
    jobs = []
    for v in vw:
        jobs += [(name, p0, w + sgn * H_DIR_W * v, kappa, target) for sgn in (1.0, -1.0)]
    for v in vp:
        jobs += [(name, p0 * (1.0 + sgn * H_DIR_P * v), w, kappa, target) for sgn in (1.0, -1.0)]
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=min(len(jobs), os.cpu_count())) as ex:
        res = list(ex.map(forward_masks, jobs))
    print(f"{name}: {len(jobs)} directional forwards {time.time() - t0:.0f} s", flush=True)
    fd, flips = [], []
    for i, h in enumerate([H_DIR_W] * N_DIRS + [H_DIR_P] * N_DIRS):
        (lp, mp), (lm, mm) = res[2 * i], res[2 * i + 1]
        fd.append((lp - lm) / (2 * h))
        flips.append(int(np.unpackbits(mp ^ mm).sum()))
    return {f"{tag}_dir_vw": np.stack(vw).astype(np.float32), f"{tag}_dir_vp": np.stack(vp).astype(np.float32),
            f"{tag}_dir_fd_w": np.array(fd[:N_DIRS]), f"{tag}_dir_fd_p": np.array(fd[N_DIRS:]),
            f"{tag}_dir_flips_w": np.array(flips[:N_DIRS]), f"{tag}_dir_flips_p": np.array(flips[N_DIRS:])}


def main():
    if "--directional-only" in sys.argv:
        data = dict(np.load(OUT))
        for name, tag in (("crowd32", "c32"), ("crowd256_fixed", "c256")):
            data.update(directional(name, tag))
        np.savez_compressed(OUT, **data)
        print("wrote", OUT, os.path.getsize(OUT), "bytes")
        return
    data = {}
    for name, tag in (("crowd32", "c32"), ("crowd256_fixed", "c256")):
        wl, p0, w, kappa, target = instance(name)
        t0 = time.time()
        loss, gw, gp, _ = loss_and_grads(p0, w, kappa, wl.gamma, wl.tau, [ITERS] * N_STEPS, target)
        print(f"{name}: autograd {time.time() - t0:.0f} s, loss {loss:.6e}", flush=True)
        rng = np.random.default_rng(1)
        free = np.flatnonzero(kappa.ravel() > 0)
        cw = np.sort(rng.choice(free, size=N_CELLS, replace=False))
        cp = np.sort(rng.choice(np.flatnonzero(p0.ravel() > 0), size=N_CELLS, replace=False))
        jobs = []
        for c in cw:
            for sgn in (1.0, -1.0):
                wv = w.copy().ravel()
                wv[c] += sgn * H
                jobs.append((name, p0, wv.reshape(w.shape), kappa, target))
        for c in cp:
            for sgn in (1.0, -1.0):
                pv = p0.copy().ravel()
                pv[c] *= 1.0 + sgn * H
                jobs.append((name, pv.reshape(p0.shape), w, kappa, target))
        t0 = time.time()
        with ProcessPoolExecutor(max_workers=os.cpu_count()) as ex:
            res = list(ex.map(forward, jobs, chunksize=1))
        print(f"{name}: {len(jobs)} forwards {time.time() - t0:.0f} s", flush=True)
        lw = np.array([r[0] for r in res[:2 * N_CELLS]]).reshape(N_CELLS, 2)
        fw = np.array([r[1] for r in res[:2 * N_CELLS]]).reshape(N_CELLS, 2)
        lp = np.array([r[0] for r in res[2 * N_CELLS:]]).reshape(N_CELLS, 2)
        fp = np.array([r[1] for r in res[2 * N_CELLS:]]).reshape(N_CELLS, 2)
        hp = H * p0.ravel()[cp]
        data.update({
            f"{tag}_loss": loss,
            f"{tag}_gw": gw.astype(np.float64), f"{tag}_gp": gp.astype(np.float64),
            f"{tag}_cells_w": cw, f"{tag}_cells_p": cp,
            f"{tag}_fd_w": (lw[:, 0] - lw[:, 1]) / (2 * H),
            f"{tag}_fd_p": (lp[:, 0] - lp[:, 1]) / (2 * hp),
            f"{tag}_kink_w": fw[:, 0] != fw[:, 1], f"{tag}_kink_p": fp[:, 0] != fp[:, 1],
            f"{tag}_digest": digest(p0, w, kappa, target),
        })
        print(f"{name}: kinks in w {int(data[f'{tag}_kink_w'].sum())}, in p0 {int(data[f'{tag}_kink_p'].sum())}",
              flush=True)
        data.update(directional(name, tag))
    # the 256^2 gradients are stored in float32 (the tests compare at 1e-3)
    for k in ("c256_gw", "c256_gp"):
        data[k] = data[k].astype(np.float32)
    np.savez_compressed(OUT, **data)
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
