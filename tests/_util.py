"""Helpers shared by the GPU tests: move seeded workloads to the device and to
the oracle, and compare densities."""
import numpy as np
import torch

import oracle as O
import paper_1502_06216_amd as jk


def f32(a):
    """float64 array rounded to float32 (the precision the device receives)."""
    return None if a is None else np.asarray(a, np.float64).astype(np.float32)


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(f32(a))).cuda()


def host64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def energies(wl):
    """(device EnergySpec, oracle Energy) for a workload, both seeing the same
    float32-rounded fields."""
    r = lambda a: None if a is None else f32(a).astype(np.float64)
    g = jk.EnergySpec(kind=wl.kind, w=dev(wl.w), kappa=dev(wl.kappa), kappa_scalar=float(np.float32(wl.kappa_scalar)),
                      coef=dev(wl.coef), coef_scalar=wl.coef_scalar, m=wl.m, density_scale=wl.density_scale,
                      m_field=dev(wl.m_field), target=dev(wl.target))
    o = O.Energy(kind=wl.kind, w=r(wl.w), kappa=r(wl.kappa), kappa_scalar=float(np.float32(wl.kappa_scalar)),
                 coef=r(wl.coef), coef_scalar=wl.coef_scalar, m=wl.m, density_scale=wl.density_scale,
                 m_field=r(wl.m_field))
    return g, o


def rel_l1(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.abs(x - ref).sum() / max(np.abs(ref).sum(), 1e-300))


# Per-cell bound beside the rel-L1 one: an error concentrated on a few cells
# (at obstacle edges, say) barely moves the aggregate.
CELL_TOL = {"fp32": 1e-4, "split_bf16": 2e-3}


def cell_err(x, ref, floor=1e-3):
    """Largest per-cell error relative to the cell's reference value; cells
    below `floor` of the field's largest value are measured against that
    floor (their float32 rounding is not a relative quantity)."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), floor * np.abs(ref).max())
    return float((np.abs(x - ref) / scale).max())


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
