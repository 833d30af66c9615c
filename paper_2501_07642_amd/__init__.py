"""MI355X (gfx950) rerandomization hot path: Python binding of librr.so.

The functions here have the names of the C ABI (``include/rr.h``) and only marshal
arguments: device buffers are torch tensors on the current HIP device, streams are torch's
current stream, and every step of the computation runs in the library's kernels.  There is
no CPU fallback: if librr.so is missing or cannot be loaded, every call raises.
"""

from . import _lib  # noqa: F401
from ._lib import (  # noqa: F401
    METRIC_DIAGONAL, METRIC_MAHALANOBIS, METRIC_MAX_SMD, MODE_CHI2_QUANTILE, MODE_QUANTILE, MODE_THRESHOLD, PREC_FIXED_I8, PREC_FP32, PREC_GRAM_BF16, PREC_SPLIT_BF16,
    RRError, Problem,
    lib_path, load, rr_balance_keys, rr_balance_keys_noalloc, rr_draw_balance, rr_draw_balance_async, rr_draw_balance_batched,
    rr_diagnose, rr_draw_exact, rr_last_timing, rr_prepare, rr_q_star, rr_rand_test, rr_rand_test_interval,
    rr_realized_rmse, rr_tune_report,
    rr_regenerate, quantile_count,
)
