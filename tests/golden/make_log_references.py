"""Writes ``log_references.npz``: the oracle's exact log-sum-exp step
(``oracle.jko_step_log``, every quantity in log form, FP64) of the literal
256 x 256 crowd (the bump mixture left 26 times above the capacity, where
plain scalings overflow) for 300 iterations, with its violation and mass, and
a digest of the float32 inputs.

Run from the repository root:  python tests/golden/make_log_references.py
(several minutes: the oracle's log-sum-exp products are dense per axis).
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "log_references.npz")
ITERS = 300


def inputs():
    """The literal crowd as the device receives it: float32-rounded fields."""
    wl = make_workload("crowd256", projected=False)
    r = lambda a: np.asarray(a, np.float64).astype(np.float32).astype(np.float64)
    en = O.Energy(kind="congestion", w=r(wl.w), kappa=r(wl.kappa), kappa_scalar=float(np.float32(wl.kappa_scalar)))
    return wl, r(wl.p0), en


def digest(wl, p0, en):
    h = hashlib.sha256()
    for a in (p0, en.w, en.kappa):
        h.update(np.ascontiguousarray(np.asarray(a, np.float32)).tobytes())
    h.update(np.array([wl.gamma, wl.tau], np.float64).tobytes())
    return h.hexdigest()


def main():
    wl, p0, en = inputs()
    t0 = time.time()
    p, st = O.jko_step_log(p0, en, wl.gamma, wl.tau, ITERS)
    print(f"crowd256 literal, {ITERS} log-domain iterations: {time.time() - t0:.0f} s, marginal "
          f"{st['marginal_l1']:.6e}, mass {st['mass']:.9f}", flush=True)
    np.savez_compressed(OUT, crowd256_literal_p=p, crowd256_literal_iters=ITERS,
                        crowd256_literal_marginal=st["marginal_l1"], crowd256_literal_mass=st["mass"],
                        crowd256_literal_digest=digest(wl, p0, en))
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
