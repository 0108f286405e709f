"""homotif: exact and hyperedge-sampled counting of higher-order motifs of
order 3 and 4 on AMD MI355X, behind the C ABI of include/homotif.h."""
from .binding import (  # noqa: F401
    HM_ALLOC_PAPER, HM_ALLOC_PROPORTIONAL, HM_OPT_BITSET_MAX_NODES, HM_OPT_DEDUP_TAG_BITS, HM_OPT_HUB_MIN_DEGREE,
    HM_OPT_ONE_PASS_MAX_EDGES, HM_OPT_SAMPLE_CHUNK_SCALE, count_exact_many, count_nulls, count_sampled, count_sampled_indices,
    hm_null_export, hm_null_tile_sizes,
    HM_NULL_CONFIG, HM_NULL_STUBS, count_nulls_model, hm_motif_profile, hm_null_export_model, hm_profile_quality,
    count_sampled_sizes, hm_stratum_search, count_sampled5, count_sampled5_indices, hm_order5_sizes,
    Model, count_sampled_learned, count_sampled_weighted_indices, hm_contrib, hm_features, hm_mlp_forward,
    hm_mlp_grad, hm_model_train, hm_proposal_probs,
    hm_get_option, hm_sample_draw, hm_sample_sizes, hm_sample_sizes_for, hm_set_option,
    Graph, HMError, LibraryMissing, count_baseline, count_exact, count_exact_noalloc, hm_class_info, hm_graph_create, hm_num_classes,
    hm_pattern_class, hm_profile_enable, hm_profile_read, hm_profile_reset, hm_version, lib,
)
