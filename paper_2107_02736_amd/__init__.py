"""DEANN's query path on AMD Instinct MI355X (gfx950): exact KDE, DEANN with an
exact k-NN, and their adjoints, as hand-written HIP kernels behind a C ABI.

The HIP library must be built (``python -m paper_2107_02736_amd.build``);
there is no CPU fallback.
"""
from ._lib import DeannError, load as load_library  # noqa: F401
from .api import (  # noqa: F401
    kde_exact, deann_query, deann_query_with_grad, deann_query_permuted, deann_query_backward, kde_exact_backward,
    kde_exact_with_grad, kde_hybrid, mean_shift_update, kernel_timing, kernel_times,
    ivf_build, IvfIndex, deann_ivf_query, PermutedIndex, get_options, set_options, default_options, last_stats,
    prepare, Prepared,
)
from .autograd import ExactKDE, DeannKDE, exact_kde, deann_kde, mean_shift, bisect_h  # noqa: F401
