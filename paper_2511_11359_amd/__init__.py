"""MI355X (gfx950) implementation of Log-Averaged Mirror Prox (LAMP, arXiv 2511.11359).

The solver lives in liblamp.so (HIP kernels + C ABI, include/lamp.h); this
package only marshals arguments.  ``workloads`` draws seeded synthetic inputs.
"""
from .api import (LampError, LampOT, Problem, State, backward, backward_y, certificate, cost_scale, exp_rate,
                  make_params, solve, solve_batched, step, step_noalloc, sweep_times, transport_cost)

__all__ = ["LampError", "LampOT", "Problem", "State", "backward", "backward_y", "certificate", "cost_scale",
           "exp_rate", "make_params", "solve", "solve_batched", "step", "step_noalloc", "sweep_times",
           "transport_cost"]
