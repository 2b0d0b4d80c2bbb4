"""MI355X (gfx950) FDETD field update and laser-envelope exponential propagator (arXiv 2605.12132).

The compute path is the HIP library ``_build/libfdetd.so`` behind the C-ABI of ``include/fdetd.h``;
``binding`` marshals arguments to it.  ``inputs`` holds the seeded synthetic workload generators.
"""
from .binding import (JGEN_BUNCH, JGEN_SAMPLES, ENVELOPE, Jgen, FDETD_E_ARG, FDETD_E_HIP, FDETD_E_NOMEM, FDETD_E_UNSTABLE, FDETD_OK, FP32C, FP64, MAXWELL, PLAN_CURRENT_CORRECTION, PLAN_INCREMENT_FORM, PLAN_MIXED_WIDTHS, PLAN_PER_WIDTH, PLAN_SEPARATE_WN, PLAN_NO_AUTOTUNE,  # noqa: F401
                      PLAN_ONE_STREAM, PLAN_PROFILE, PLAN_SKIP_STABILITY, PLAN_USE_GRAPH, FdetdError, Plan, Problem,
                      envelope_absorber, envelope_gather, envelope_ponderomotive, envelope_step, fdetd_coefficients,
                      fdetd_deposit_current, fdetd_deposit_jz, fdetd_deposit_rho, fdetd_destroy, fdetd_export_state,
                      fdetd_gather, fdetd_gather_supersampled, fdetd_import_state, fdetd_last_error, fdetd_plan, fdetd_query, fdetd_step,
                      fdetd_step_graph, fdetd_step_noalloc,
                      fdetd_taylor_stability_bound)
