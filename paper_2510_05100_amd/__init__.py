"""MI355X-native matrix-element reweighting (paper: parameter reweighting
w' = w |M'|^2 / |M|^2 with the per-event |M|^2 as the data-parallel hot path).

The compute path lives in librwgt.so (HIP kernels for gfx950 behind the C ABI
of include/rwgt.h); this package only marshals arguments to it.
"""
from ._abi import (  # noqa: F401
    RWGT_MLP_BF16, RWGT_MLP_FP32, rwgt_mlp_create, rwgt_mlp_destroy, rwgt_mlp_features, rwgt_mlp_forward,
    rwgt_mlp_get_grads, rwgt_mlp_get_params, rwgt_mlp_input_bytes, rwgt_mlp_num_params, rwgt_mlp_set_calibration,
    rwgt_mlp_set_normalisation, rwgt_mlp_set_params, rwgt_mlp_set_stream, rwgt_mlp_set_training, rwgt_mlp_targets,
    rwgt_mlp_train_step, rwgt_sur_eval, RWGT_FEAT_RAW, RWGT_FEAT_PHYS, n_features, rwgt_mlp_set_features,
    rwgt_mlp_set_target_scale, rwgt_mlp_predict, rwgt_mlp_fit_normalisation,
    rwgt_mlp_fit_target_scale, rwgt_mlp_get_normalisation, rwgt_eval_cards, rwgt_mlp_get_adam, rwgt_mlp_fit_grid,
    rwgt_mlp_train, rwgt_mlp_get_progress, rwgt_train_order, rwgt_mlp_calibrate, rwgt_mlp_save, rwgt_mlp_load,
    rwgt_mlp_checkpoint_info, rwgt_set_mixed_guard, rwgt_mixed_guard_count, rwgt_cancellation,
)
from ._abi import (  # noqa: F401
    Segment, make_segments, rwgt_batch_create, rwgt_batch_destroy, rwgt_batch_eval, rwgt_batch_get_schedule,
    rwgt_batch_set_schedule, rwgt_batch_set_stream, rwgt_batch_time, rwgt_batch_tune,
)
from ._abi import (  # noqa: F401
    RWGT_FP64, RWGT_MIXED_BF16, RWGT_MIXED_FP16, RwgtError, load, rwgt_create, rwgt_destroy, rwgt_eval,
    rwgt_flops, rwgt_flops_executed, rwgt_bounds_check, rwgt_kernel_times, rwgt_me2, rwgt_original_params, rwgt_param_layout, rwgt_process_info,
    rwgt_set_profiling, rwgt_set_stream, rwgt_xsec, rwgt_eval_factored, rwgt_eval_alphas, rwgt_nonfinite,
)
from ._abi import (  # noqa: F401
    rwgt_lhe_read, rwgt_lhe_parse, rwgt_lhe_destroy, rwgt_lhe_num_events, rwgt_lhe_event_info, rwgt_lhe_select,
    rwgt_lhe_momenta, rwgt_lhe_info, rwgt_lhe_add_weights, rwgt_lhe_write, rwgt_reweight_card, rwgt_process_layout,
)


class Reweighter:
    """Context manager owning one rwgt context (calls rwgt_create/rwgt_destroy)."""

    def __init__(self, process: str, param_card: str, precision: int = RWGT_FP64):
        self.ctx = rwgt_create(process, param_card, precision)
        self.layout = rwgt_param_layout(self.ctx)

    def eval(self, momenta, weights_in, param_sets, weights_out, stream=None):
        rwgt_set_stream(self.ctx, stream)
        rwgt_eval(self.ctx, momenta, weights_in, param_sets, weights_out)

    def eval_factored(self, momenta, weights_in, param_sets, weights_out, stream=None):
        rwgt_set_stream(self.ctx, stream)
        rwgt_eval_factored(self.ctx, momenta, weights_in, param_sets, weights_out)

    def me2(self, momenta, param_sets, me2_out, stream=None):
        rwgt_set_stream(self.ctx, stream)
        rwgt_me2(self.ctx, momenta, param_sets, me2_out)

    def close(self):
        if self.ctx:
            rwgt_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
