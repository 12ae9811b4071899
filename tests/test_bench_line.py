"""The benchmark's summary line: the last stdout line must be one JSON object
under 4 KB carrying the headline, the roofline, the CPU baseline, the FP64
method and the guard / oracle-recheck figures, however large the full record
of the legs grows."""
import json
import math

import bench


def _full_result():
    """A record shaped like the one bench.main assembles (every leg on),
    with long per-iteration and per-state arrays."""
    leg = {"value": 81.2345678, "ms_per_step": 1256.123456, "certified": 102, "mean_iters": 301.23456,
           "mean_attempts": 1.7}
    app = {"us_per_apply": 42.2123, "alg_bytes": 119425000, "GB/s": 2832.1234, "frac_hbm_peak": 0.354,
           "buffer_sets": 3, "launches_timed": 40, "us_per_call_wall": 45.1}
    traj = {"seconds": 0.91234, "compliance": [3.45 + 1e-3 * i for i in range(40)], "floors": [1e-12] * 40,
            "solve_iters": list(range(40)), "true_eta": [9e-7] * 40}
    return {
        "metric": "certified solves/s at ||f-Ku||/||f||<=1e-6 (mixed precision)", "mixed_form": "bf16x3",
        "selector": "mlp", "orthogonalization": "CGS2, delayed reorthogonalization",
        "value": 101.3456789, "unit": "certified solves/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 1006.98765, "step_ms": {"median": 1006.9, "iqr": [1006.1, 1007.3], "all": [1006.9] * 20},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": bench.DTYPES["bf16x3"],
        "data": "synthetic",
        "config": {"workload": "102 severe random states, 64x32x32 cantilever, guarded floor ladder",
                   "states": 102, "grid": [64, 32, 32], "rungs": [1e-9, 1e-6, 1e-4, 1e-3], "p": 3.0,
                   "probe": "100 its, restart 100", "solve": "FGMRES(30), cap 200, tol 1e-6",
                   "preconditioner": "5-level GMG V-cycle, node-block Jacobi w=0.6 2/2, FP32 vectors"},
        "policy": {"certified": 102, "states": 102, "max_accepted_true_eta": 9.9957e-7, "accepted_above_tolerance": 0,
                   "first_attempt_accepted": 96, "mean_attempts": 1.06,
                   "stats": {"sensitivity": {"k": 40, "n": 45}, "specificity": {"k": 52, "n": 57},
                             "guard_fallbacks": 5, "lowest_admissible_selected": 96}},
        "roofline": {"kernel": "vector_update", "bound": "hbm", "achieved": 5321.123456, "peak": 8000.0,
                     "unit": "GB/s", "frac": 0.66514, "traffic": 1938.0e6, "avg_launch_us": 357.512,
                     "launches": 4123, "alg_bytes_per_launch": 1902.9e6},
        "oracle_recheck": {"checked": 102, "false_acceptances_oracle": 0, "above_tau_oracle": 0,
                           "boundary_ambiguous": 0, "max_eta_oracle": 9.99571e-7, "max_delta": 3.1e-11,
                           "max_abs_gpu_minus_oracle": 1e-15, "max_abs_gpu_minus_oracle_over_delta": 1e-4},
        "apply_K": {"f32": app, "f64": app, "bf16_mfma": app, "bf16x3_mfma": app,
                    "sensitivity_f64": {"us_per_call": 65.0, "GB/s": 4190.0, "frac_hbm_peak": 0.52},
                    "autotuned_zc": {"f32": 17}},
        "kernel_classes": {f"class{i}": {"launches": 100, "total_ms": 1.0, "avg_us": 10.0, "alg_GB/s": 1.0}
                           for i in range(12)},
        "mixed_rule": dict(leg, same_rung=80), "selector_gain": 1.2612345,
        "fp64": dict(leg, selector="rule", same_rung=90), "mixed_over_fp64": 1.62123,
        "fidelity": {"raised": {str(k): {"states": 57} for k in range(3)}},
        "screen": {"states": 102}, "probe_checkpoints": {"checkpoints": 913},
        "adaptive_preconditioner": {"adaptive": {"certified": 67, "seconds_per_solve": 0.197},
                                    "plain_vcycle": {"certified": 57, "seconds_per_solve": 0.054},
                                    "paper_setting": {"adaptive": {"false_acceptances": [[1069, 206, 7.7e-7, 2.5e-3]] * 30}}},
        "small_plain": {"direct_launches": {"value": 196.0, "us_per_iteration": 291.6},
                        "graph_replay": {"value": 207.0, "us_per_iteration": 280.1}},
        "mixed_at_scale": {"mixed": {"iterations": 37, "seconds": 0.06, "true_eta": 9.1e-7},
                           "fp64": {"iterations": 37, "seconds": 0.08, "true_eta": 9.2e-7},
                           "rel_error_vs_fp64": 8.26e-9,
                           "oracle_recheck": {"max_eta_oracle": 9.2e-7, "false_acceptances_oracle": 0}},
        "batch_uneven": {"mixed_batched": {"value": 198.8, "guard_passing": 192},
                         "mixed_batched_graphs": {"value": 199.2}, "mixed_serial": {"value": 16.3},
                         "fp64_batched": {"value": 145.6}, "oracle_recheck": {"false_acceptances_oracle": 0}},
        "trajectory": {k: traj for k in ("guarded", "guarded_reuse", "fixed_1e-12_unguarded", "fixed_1e-3_unguarded")},
        "cpu_baseline": {"value": 0.93, "unit": "certified solves/s", "cores": 16, "kind": "oracle",
                         "sample": "x" * 600},
        "cpu_host": {"cpu_model": "AMD EPYC"},
    }


def test_summary_line_is_short_and_complete():
    full = _full_result()
    assert len(json.dumps(full)) > 8000           # the full record is far longer than the line
    c = bench.compact(full, "bench_full.json")
    line = json.dumps(c)
    assert "\n" not in line and len(line) <= 4096
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "fp64",
              "mixed_over_fp64", "guard", "oracle_recheck", "apply_K_256x128x128"):
        assert k in c, k
    assert c["config"]["workload"].startswith("102 severe")
    assert set(c["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert c["roofline"]["frac"] == round(c["roofline"]["frac"], 4)
    assert set(c["cpu_baseline"]) >= {"value", "unit", "cores", "kind", "sample"}
    assert c["guard"]["accepted_above_tolerance"] == 0
    assert c["oracle_recheck"]["false_acceptances_oracle"] == 0
    assert set(c["apply_K_256x128x128"]) == {"f32", "f64", "bf16_mfma", "bf16x3_mfma", "sensitivity_f64"}
    assert c["dtype"] == "bf16x3-mfma+f32+f64"
    assert math.isclose(c["value"], 101.3, rel_tol=1e-3)


def test_summary_line_without_optional_legs():
    full = {k: v for k, v in _full_result().items()
            if k not in ("apply_K", "fp64", "mixed_rule", "small_plain", "batch_uneven", "mixed_at_scale",
                         "trajectory", "adaptive_preconditioner", "cpu_baseline", "oracle_recheck")}
    c = bench.compact(full)
    assert "fp64" not in c and "cpu_baseline" not in c and "full_record" not in c
    assert len(json.dumps(c)) <= 4096
