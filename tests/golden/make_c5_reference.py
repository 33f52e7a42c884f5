"""Writes ``c5_reference.npz``: the 128^3 crowd flow of the precision
configuration (20 JKO steps x 300 iterations) run by the oracle in float64
(``oracle.jko_step``; absorption on max|log a| > 50 never triggers on this
workload, max|log a| stays near 5, so the plain-domain oracle is the same
iteration), with each step's violation and mass, the final density rounded
to float32, and a digest of the float32 inputs.

Run from the repository root:  python tests/golden/make_c5_reference.py
(about ten minutes on 8 cores).
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from workloads import make_workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_reference.npz")
N_STEPS, ITERS = 20, 300


def inputs():
    """The 128^3 crowd as the device receives it: float32-rounded fields."""
    wl = make_workload("crowd128c")
    r = lambda a: np.asarray(a, np.float64).astype(np.float32).astype(np.float64)
    kap = None if wl.kappa is None else r(wl.kappa)
    en = O.Energy(kind="congestion", w=r(wl.w), kappa=kap, kappa_scalar=float(np.float32(wl.kappa_scalar)))
    return wl, r(wl.p0), en


def digest(wl, p0, en):
    h = hashlib.sha256()
    for a in (p0, en.w) + ((en.kappa,) if en.kappa is not None else ()):
        h.update(np.ascontiguousarray(np.asarray(a, np.float32)).tobytes())
    h.update(np.array([wl.gamma, wl.tau, en.kappa_scalar], np.float64).tobytes())
    return h.hexdigest()


def main():
    wl, p0, en = inputs()
    q = p0
    marg, mass = [], []
    t0 = time.time()
    for t in range(N_STEPS):
        q, st = O.jko_step(q, en, wl.gamma, wl.tau, ITERS)
        marg.append(st["marginal_l1"])
        mass.append(st["mass"])
        print(f"step {t + 1}/{N_STEPS}: {time.time() - t0:.0f} s, marginal {st['marginal_l1']:.6e}, "
              f"mass {st['mass']:.9f}", flush=True)
    np.savez_compressed(OUT, c5_pT=q.astype(np.float32), c5_marginal=np.array(marg), c5_mass=np.array(mass),
                        c5_steps=N_STEPS, c5_iters=ITERS, c5_digest=digest(wl, p0, en))
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
