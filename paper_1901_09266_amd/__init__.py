"""MI355X library for the SPGD solve of the per-day DODE NNLS (arXiv 1901.09266).

The computation lives in libdode.so (HIP kernels for gfx950 behind the C ABI of
include/dode.h); this package is its Python binding.
"""
from ._lib import (DodeError, Dar, SpgdParams, STORAGE, EXPORTS, lib, dar_create, dar_info,
                   dar_set_values, dode_apply, dode_loss, dode_loss_noalloc, dode_grad,
                   dode_metrics, spgd_step, spgd_solve, spgd_defaults, make_params, Plan, spgd_plan_create, spgd_run,
                   spgd_plan_load, spgd_plan_store,
                   spgd_plan_timing, spgd_plan_info, spgd_plan_schedule, dode_loss_bwd, Routes, dode_routes_create,
                   dar_from_logits,
                   dar_logits_bwd, dode_dar_from_speeds, dode_path_costs, dar_from_costs,
                   dense_spgd_run, dode_dar_costs_from_speeds, dode_dar_patterns_from_speeds)

__all__ = ["DodeError", "Dar", "SpgdParams", "STORAGE", "EXPORTS", "lib", "dar_create", "dar_info",
           "dar_set_values", "dode_apply", "dode_loss", "dode_loss_noalloc", "dode_grad",
           "dode_metrics", "spgd_step", "spgd_solve", "spgd_defaults", "make_params", "Plan", "spgd_plan_create", "spgd_run",
           "spgd_plan_load", "spgd_plan_store",
           "spgd_plan_timing", "spgd_plan_info", "spgd_plan_schedule", "dode_loss_bwd", "Routes", "dode_routes_create",
           "dar_from_logits",
           "dar_logits_bwd", "dode_dar_from_speeds", "dode_path_costs", "dar_from_costs",
           "dense_spgd_run", "dode_dar_costs_from_speeds", "dode_dar_patterns_from_speeds"]
