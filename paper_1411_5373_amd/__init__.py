"""MI355X-native Fast Dispersion Measure Transform (Zackay & Ofek, arXiv:1411.5373).

The transform runs in libfdmt.so (hand-written HIP for gfx950); this package
only marshals tensors and streams into its C ABI.
"""
from .binding import (EXPORTED, FDMTError, FDMTFunction, Plan, RaggedPlan, boxcar_search, copy_bytes, fdmt,
                      fdmt_adjoint, fdmt_copy_bytes, fdmt_forward_search, fdmt_search_fused,
                      fdmt_search_workspace_bytes, fdmt_tuned_options, fdmt_boxcar_search, fdmt_boxcar_workspace_bytes,
                      fdmt_fft_workspace_bytes, fdmt_forward, fdmt_forward_fft, fdmt_last_error, fdmt_plan, fdmt_plan_destroy, fdmt_plan_info,
                      fdmt_plan_tables, fdmt_ragged_adjoint, fdmt_ragged_destroy,
                      fdmt_ragged_forward, fdmt_ragged_info, fdmt_ragged_plan,
                      fdmt_ragged_run_step, fdmt_ragged_workspace_bytes, fdmt_run_step,
                      fdmt_status_string, fdmt_step_count, fdmt_step_info, fdmt_stream_mix, fdmt_workspace_bytes,
                      library_path, load, stream_mix)
