"""MI355X-native Brandes betweenness centrality.

The computation lives in libnkbc.so (hand-written HIP kernels for gfx950
behind the C ABI in include/nk_bc.h); this package is its Python binding.
There is no CPU fallback: calls fail when the library is missing or no GPU
is present.
"""
from ._lib import (  # noqa: F401
    NK_E_BUDGET, NK_E_HIP, NK_E_INTERNAL, NK_E_INVALID_ARG, NK_E_INVALID_GRAPH, NK_E_NO_MEMORY,
    NK_E_SIGMA_OVERFLOW, NK_E_TIMEOUT, NK_OK, NkBatchPlan, NkError, NkServer, load, nk_autotune, nk_bc_exact, nk_bc_exact_batched,
    nk_bc_directed, nk_bc_pair_sample, nk_bc_sources, nk_bc_sources_bisect, nk_bc_sources_noalloc, nk_bc_sources_linear, nk_bc_weighted, nk_closeness, nk_closeness_sampled, nk_edge_bc, nk_get_tuning, nk_last_stats, nk_tuning_lookup, nk_pair_counts, nk_rk_sample_size,
    nk_sample_paths, nk_set_tuning, nk_set_tuning_cache, nk_shutdown, nk_sssp_counts, nk_transpose, nk_validate_graph, nk_vd_bound, nk_version,
)
