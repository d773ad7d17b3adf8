"""MI355X-native e-ph transition-probability path (HIP library + binding).

The compute lives in libelph.so (csrc/, C ABI in include/elph.h); the
``elph`` module is its ctypes binding.
"""
from . import elph  # noqa: F401
from .elph import (  # noqa: F401
    elph_create, elph_destroy, elph_reset, elph_timing, elph_timing_extra, elph_sizes, elph_tables, elph_interp_g,
    elph_transition_probs, elph_scatt_rates, elph_iterate, elph_ko_enforce, elph_set_delta, elph_set_polar, elph_set_ifc3,
    elph_phph_vertex, elph_phph_rates, elph_phph_inscatter, elph_set_phph, ElphError,
    elph_batch_create, elph_batch_destroy, elph_batch_scatt_rates, elph_batch_tune, elph_batch_set_shape,
    elph_mlp_create, elph_mlp_nparams, elph_mlp_get_params, elph_mlp_set_params, elph_mlp_forward,
    elph_mlp_gradients, elph_mlp_train_step, elph_screen_nin, elph_screen_samples, elph_scatt_rates_screened,
    elph_set_refine, elph_refine_info, elph_refine_estimates, elph_interp_g_noalloc,
    elph_save, elph_load, elph_set_memory_limit, elph_memory_held, elph_set_gemm_chunk,
)
