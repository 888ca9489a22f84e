"""MI355X (gfx950) batched G^2 conditional-independence tests for PC-stable
skeleton learning (Jiang, Wen, Mian, "Fast Parallel Bayesian Network Structure
Learning").

The work runs in libbns.so (HIP kernels behind the C ABI of include/bns.h);
this package only marshals arguments.  See ``_lib`` for the entry points.
"""

from ._lib import (  # noqa: F401
    BNS_CI_INDEPENDENT,
    BNS_CI_RECHECKED,
    BNS_DEPTH0_AUTO,
    BNS_DEPTH0_PAIRS,
    BNS_DEPTH0_TESTS,
    BNS_DEPTH1_AUTO,
    BNS_DEPTH1_GRAM,
    BNS_DEPTH1_TESTS,
    BNS_DF_ADJUSTED,
    BNS_DF_DECLARED,
    BNS_FORM_BATCHED,
    BNS_GROUP_AUTO,
    BNS_GROUP_EDGE,
    BNS_GROUP_TEST,
    BNS_FORM_EDGE,
    BNS_FORM_PLAIN,
    BNS_PREC_FP32_RECHECK,
    BNS_PREC_FP64,
    BNS_STAT_G2,
    BNS_STAT_X2,
    EXPORTS,
    NOALLOC_SCRATCH_BYTES,
    BnsError,
    bns_autotune,
    Dataset,
    Skeleton,
    bns_ci_batch,
    bns_ci_batch_noalloc,
    bns_ci_pairs,
    bns_lds_increment_rate,
    bns_dataset_create,
    bns_dataset_wrap_device,
    bns_options,
    bns_options_default,
    bns_orient,
    bns_pc_skeleton,
    bns_pc_skeleton_batch,
    bns_pc_skeleton_dataset,
    collect,
    free_skeleton,
    load,
    skeleton_batch_handles,
    skeleton_handle,
)
