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
* a digest of the float32 inputs, so that the tests can tell when the
  workload recipe has changed since this file was written.

Run from the repository root:  python tests/golden/make_c4_gradients.py
(about half an hour on 8 cores; the 256^2 autograd tape holds ~25 GB).
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


def main():
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
    # the 256^2 gradients are stored in float32 (the tests compare at 1e-3)
    for k in ("c256_gw", "c256_gp"):
        data[k] = data[k].astype(np.float32)
    np.savez_compressed(OUT, **data)
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
