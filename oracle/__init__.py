"""FP64 CPU oracle of the entropic JKO step (test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The HIP library and its Python binding never do: the
product path has no CPU fallback.
"""
from .jko_oracle import (  # noqa: F401
    Energy, grid_points, all_points, gibbs_dense, gibbs_rows, gibbs_factor, gibbs_apply,
    log_gibbs_apply, prox, log_prox, prox_congestion, prox_binary_congestion, kl_cell, prox_entropy,
    log_prox_gen_entropy,
    prox_porous,
    lambertw_of_log, dykstra_coupling, dykstra_scaling, jko_step, jko_step_log, jko_flow,
    prox_attraction_psi1, attraction_generic, attraction_step, attraction_step_log,
)
from .heat_oracle import HeatKernel, heat_nu, heat_system  # noqa: F401,E402
