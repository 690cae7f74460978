"""Prior-predictive sampling on AMD MI355X (gfx950).

A from-scratch GPU implementation of the data-parallel hot path of Warne,
Sisson & Drovandi (arXiv:1902.09046): prior-predictive sampling for ABC
rejection (Alg. 1) and prior-predictive p-values over a hyperparameter grid
(Sec. 4.1), one lane per prior draw (one workgroup per draw for the paper's
toggle-switch model, Sec. 3.2), counter-based Philox streams keyed by (seed,
draw), FP32 simulation with compensated summaries, FP64 tallies and
moments; and the weak-informativity test of Sec. 4.1 (Alg. 2) with one FP64
adaptive SMC evidence sampler (Alg. 3) per workgroup.  The kernels and runtime live in ``libpps.so`` (C ABI in
``include/pps.h``); this package is its thin ctypes binding.
"""
from ._pps import (  # noqa: F401
    PPS_EINVAL, PPS_ENOMEM, PPS_EDEVICE, PPS_EBUSY, PPS_ENOTFOUND, PPS_ETRUNC, PPS_OK, PPS_PENDING,
    PPS_UNIFORM, PPS_NORMAL, PPS_LOGNORMAL, PPS_POINT,
    PPS_LOGISTIC_SDE, PPS_GARCH11, PPS_NORMAL_MEAN, PPS_TOGGLE_SWITCH,
    PPS_EPS_FIXED, PPS_EPS_TOP_FRACTION, PPS_GARCH_NSUMM, PPS_MAX_PARAMS, PPS_TSW_MAX_CELLS,
    CLASS_PATH, CLASS_GARCH, CLASS_GROUP, CLASS_CELLS,
    PPSError, LIB_PATH, lib, make_model, make_sampling,
    pps_version, pps_n_summaries, pps_set_timing, pps_last_kernel_ms, pps_last_finalize_ms, pps_set_block_size, pps_get_block_size,
    pps_set_launch_shape, pps_get_launch_shape, PATH_SHAPES, GARCH_SHAPES, CELL_SHAPES, pps_philox, pps_normals, pps_simulate,
    abc_sample, abc_sample_noalloc, PPS_NOALLOC_MAX_DRAWS, prior_pred_pvalue, pps_summary_tally, simulate, abc,
    PPS_JOB_ABC, PPS_JOB_PVALUE, PPS_POLICY_BATCHED, PPS_POLICY_PLAIN,
    pps_job, pps_job_result, pps_server_config, pps_server_stats,
    make_abc_job, make_pvalue_job, make_server_config, pps_job_arena_bytes, pps_run_batch,
    Server, records, pps_autotune,
    PPS_BIO_MAX_GROUPS, PPS_SMC_MAX_PARTICLES, pps_bioassay, pps_smc_config, make_bioassay,
    make_smc_config, pps_smc_log_evidence, pps_wip_test, pps_bege_loglik, pps_bege_count_ops, BEGE_NPAR,
    PPS_TB, PPS_TB_SUPERCRITICAL, PPS_TB_MAX_POP, PPS_TB_MAX_SAMPLE, CLASS_GILLESPIE, pps_tb_events,
)
