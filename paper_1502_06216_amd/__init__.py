"""MI355X-native entropic Wasserstein gradient flows (JKO) -- HIP for gfx950.

The compute path is libjko.so (hand-written HIP kernels behind a C ABI,
``include/jko.h``); this package is its thin Python binding.  See
``paper_1502_06216_amd._native`` for the calls:

* ``gibbs_apply(x, gamma, precision)``   y = xi x
* ``step(p, energy, gamma, tau, ...)``    one JKO step (Listing 1 of the paper)
* ``step_static(...)``                    the same on the library's static workspace
* ``flow(p0, energy, gamma, tau, n_steps, ...)``
* ``backward(checkpoints, iters, dL_dpT, energy, gamma, tau)``
* ``JKOFlowFn`` -- torch.autograd.Function over flow/backward
* ``HeatOperator(shape, gamma, L, mask)`` -- the heat-kernel Gibbs operator
  of Section 4.1 on an obstacle domain: ``apply``, ``step``, ``flow``
"""
from ._native import (  # noqa: F401
    EnergySpec, HeatDomain, HeatOperator, JKOError, JKOFlowFn, backward, time_iteration, flow, gibbs_apply, load, step,
    step_static, workspace_bytes, stats_from_device, STATS_DEV_DOUBLES, ABI_VERSION,
    make_grid, make_params, Grid, EnergyC, Params, Stats, LIB_PATH,
    JKO_OK, JKO_ERR_INVALID, JKO_ERR_WORKSPACE, JKO_ERR_HIP, JKO_ERR_NONFINITE, JKO_ERR_INFEASIBLE,
    OP_GIBBS, OP_STEP, OP_FLOW, OP_BACKWARD,
)
