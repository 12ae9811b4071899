"""Benchmark: certified solves/s of the guarded SIMP state solve on MI355X.

Workload (one "step" = one pass of the whole hot path): 102 severe random
states on the 64x32x32 cantilever (212,355 DOF each; 50% of 4^3-voxel blobs at
the floor, the rest U[0.01, 1]; seeds 1000-1101), p = 3, solved in one batch by
the guarded policy: 100-iteration probe at rho_0 = 1e-9 (restart 100), the
first rung from the stored learned selector (or the two-feature rule), then
independent FGMRES(30) solves (cap 200) on the ladder
{1e-9, 1e-6, 1e-4, 1e-3} with the recomputed FP64 residual guard
||f - K u|| / ||f|| <= 1e-6 on every rung.  A state is certified when the
policy returns an accepted solve.  The headline runs the mixed form (FP32
V-cycle with the split-BF16 matrix-core fine operator, FP64 Arnoldi / least
squares / guard) with the learned selector; the same mixed form with the
rule, and the plain FP64 form with the rule (the published method), are timed
beside it.  Inputs are resident in HBM before the timed region.

The last line on stdout is one compact JSON object (under 4 KB) with the
headline, the roofline of the dominant kernel, the CPU oracle baseline and
the oracle's recheck of the accepted solutions; every leg's full record goes
to --full-out (default bench_full.json in the working directory).
"""
import argparse
import json
import math
import os
import multiprocessing
import subprocess
import sys
import threading
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HBM bytes per launch of kernel classes on this workload, from rocprofv3
# --pmc FETCH_SIZE and --pmc WRITE_SIZE runs (FETCH_SIZE scaled by 2.000, the
# factor a plain 1 GiB copy needs).  Each entry holds while the source of the
# kernels it measured is unchanged (sha256 prefix of the listed files, or of
# the listed kernel definitions within a file), else the traffic is reported
# as null.
MEASURED_TRAFFIC = {
    "vcycle_fine_op": {"bytes_per_launch": 220.0e6, "sources": {"tg_fine.hip:k_fine_zm": "19467845af83fd66"},
                       "profile": "profiles/policy_severe102_64x32x32_hbm_counters.md"},
    "multidot": {"bytes_per_launch": 1728.5e6, "sources": {"tg_kernels.hip:k_dots2_": "4a3f94abdb36d47c",
                                                           "tg_kernels.hip:k_multidot_": "2ecbcc0448c99c92"},
                 "profile": "profiles/policy_severe102_64x32x32_hbm_counters.md"},
    "vector_update": {"bytes_per_launch": 1920.4e6, "sources": {"tg_kernels.hip:k_update2_": "eb211e836eb4dda9",
                                                                "tg_kernels.hip:k_xupdate_": "0fc098785e738a14"},
                      "profile": "profiles/policy_severe102_64x32x32_hbm_counters.md"},
}


def source_hash(spec):
    """sha256 prefix of a source file under csrc/, or ("file:name") of the
    definition of kernel `name` in it (from its signature to the first line
    that closes it at column 0)."""
    import hashlib
    fname, _, name = spec.partition(":")
    with open(os.path.join(ROOT, "paper_2607_26382_amd", "csrc", fname)) as fh:
        text = fh.read()
    if name:
        i = text.find(" " + name + "(")
        if i < 0:
            return None
        i = text.rfind("\n", 0, i) + 1
        j = text.find("\n}\n", i)
        text = text[i:j + 3]
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def measured_traffic(cls):
    e = MEASURED_TRAFFIC.get(cls)
    if not e:
        return None
    for spec, sha in e["sources"].items():
        if source_hash(spec) != sha:
            return None
    return e["bytes_per_launch"]


GRID = (64, 32, 32)
# arithmetic of the mixed form: the fine V-cycle operator's contraction, the
# FP32 V-cycle vectors, FP64 outer operator / Gram-Schmidt / least squares / guard
DTYPES = {"bf16x3": "bf16x3-mfma+f32+f64", "bf16": "bf16-mfma+f32+f64", "f32": "f32+f64"}
RUNGS = (1e-9, 1e-6, 1e-4, 1e-3)
SEED0 = 1000
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--states", type=int, default=102)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-apply", action="store_true", help="skip the 256x128x128 apply_K bandwidth leg")
    ap.add_argument("--apply-only", action="store_true", help="run only the apply_K bandwidth leg")
    ap.add_argument("--mixed", default="bf16x3", choices=["f32", "bf16", "bf16x3"],
                    help="fine-level contraction of the mixed form (FP32 vector, BF16 or split-BF16 matrix cores)")
    ap.add_argument("--compare-mixed", action="store_true",
                    help="also time the other mixed variants (one step each)")
    ap.add_argument("--selector", default="mlp", choices=["mlp", "rule"],
                    help="first-rung selector of the headline run (stored network or two-feature rule)")
    ap.add_argument("--cgs-passes", type=int, default=2, choices=[1, 2, 3],
                    help="orthogonalization: 1 CGS, 2 CGS2 with delayed reorthogonalization, 3 CGS2 in place")
    ap.add_argument("--no-batch4", action="store_true", help="skip the 192 uneven batched solves")
    ap.add_argument("--no-small", action="store_true", help="skip the 16x8x8 plain-method leg")
    ap.add_argument("--no-scale", action="store_true", help="skip the 256x128x128 mixed-vs-FP64 solve")
    ap.add_argument("--no-rule-leg", action="store_true",
                    help="skip the mixed-precision run with the two-feature rule")
    ap.add_argument("--no-labels", action="store_true",
                    help="skip the reference labels (independent solves at every rung) and the policy statistics")
    ap.add_argument("--no-trajectory", action="store_true",
                    help="skip the optimization-loop runs (guarded, decision reuse, fixed floors)")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the adaptive-preconditioner leg (fine-level correction)")
    ap.add_argument("--adaptive-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--streams", type=int, default=1,
                    help="split the states into this many batches, each on its own stream and host thread")
    ap.add_argument("--stack-states", type=int, default=16,
                    help="states of the full-adaptive-stack policy leg (paper setting, one at a time)")
    ap.add_argument("--no-stack", action="store_true", help="skip the full-adaptive-stack policy leg")
    ap.add_argument("--stack-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--paper-states", type=int, default=102,
                    help="states of the adaptive leg's paper-setting part (p = 4.5, rho_0 = 1e-12, FGMRES(300))")
    ap.add_argument("--trajectory-only", action="store_true", help="run only the optimization-loop leg")
    ap.add_argument("--small-only", action="store_true", help="run only the 16x8x8 plain-method leg")
    ap.add_argument("--no-fixed-legs", action="store_true",
                    help="skip the fixed-first-rung baselines (original floor first; always the top rung)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (calibrates HBM byte counters)")
    ap.add_argument("--no-recheck", action="store_true",
                    help="skip the oracle's recomputation of the accepted solutions' residuals")
    ap.add_argument("--full-out", default="bench_full.json",
                    help="file for the full record of every leg (the stdout line is the compact summary)")
    ap.add_argument("--cpu-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-seed", type=int, default=1000, help=argparse.SUPPRESS)
    return ap.parse_args()


def cpu_baseline_child(seed):
    """Oracle timing sample (runs in a child process with one BLAS thread)."""
    from oracle import fgmres as ofg
    from oracle import ke, mesh
    from oracle import multigrid as omg
    from oracle import operator as op
    from paper_2607_26382_amd import synth

    (nx, ny, nz), rho = synth.severe(seed)
    g = mesh.Grid(nx, ny, nz)
    free = g.free_dofs()
    f = g.edge_load()[free]
    t0 = time.perf_counter()
    H = omg.build_hierarchy(g, op.young(rho, 3.0, RUNGS[0]), ke.ke())
    t1 = time.perf_counter()
    n_it = 20
    ofg.fgmres(lambda v: H[0].K @ v, lambda v: omg.vcycle(H, v), f, 30, n_it, 1e-30)
    t2 = time.perf_counter()
    print(json.dumps({"t_setup": t1 - t0, "t_iter": (t2 - t1) / n_it}), flush=True)


def _get(d, *keys):
    for k in keys:
        if not isinstance(d, dict) or k not in d:
            return None
        d = d[k]
    return d


def _r(x, n=4):
    """Round floats to n significant digits (the summary line stays short)."""
    if isinstance(x, float) and math.isfinite(x):
        return float(f"{x:.{n}g}")
    if isinstance(x, (list, tuple)):
        return [_r(v, n) for v in x]
    if isinstance(x, dict):
        return {k: _r(v, n) for k, v in x.items()}
    return x


def compact(result, full_path=None):
    """The summary line printed last on stdout (kept under 4 KB): headline,
    roofline of the dominant kernel, CPU oracle baseline, the FP64 method,
    apply_K per precision, guard and oracle-recheck figures, and one or two
    numbers per further leg; `full_path` holds the full record."""
    r = result
    c = {k: r.get(k) for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                               "higher_is_better", "scaling", "vs_baseline", "dtype", "data")}
    cfg = r.get("config") or {}
    c["config"] = {k: cfg.get(k) for k in ("workload", "states", "grid", "rungs", "p", "probe", "solve",
                                            "preconditioner", "streams")}
    c["config"]["mixed_form"] = r.get("mixed_form")
    c["config"]["selector"] = r.get("selector")
    rf = r.get("roofline")
    if rf:
        c["roofline"] = {k: rf.get(k) for k in ("kernel", "bound", "achieved", "peak", "unit", "frac", "traffic",
                                                "avg_launch_us", "alg_bytes_per_launch", "launches")}
    cb = r.get("cpu_baseline")
    if cb:
        c["cpu_baseline"] = {k: cb.get(k) for k in ("value", "unit", "cores", "kind")}
        c["cpu_baseline"]["sample"] = (cb.get("sample") or "")[:240]
    c["step_ms"] = {k: _get(r, "step_ms", k) for k in ("median", "iqr")}
    pol = r.get("policy") or {}
    c["guard"] = {"certified": pol.get("certified"), "states": pol.get("states"),
                  "max_accepted_true_eta": pol.get("max_accepted_true_eta"),
                  "accepted_above_tolerance": pol.get("accepted_above_tolerance"),
                  "first_attempt_accepted": pol.get("first_attempt_accepted"),
                  "mean_attempts": pol.get("mean_attempts")}
    orc = r.get("oracle_recheck")
    if orc:
        c["oracle_recheck"] = {k: orc.get(k) for k in ("checked", "false_acceptances_oracle", "above_tau_oracle",
                                                       "boundary_ambiguous", "max_eta_oracle",
                                                       "max_abs_gpu_minus_oracle_over_delta")}
    if "fp64" in r:
        c["fp64"] = {k: r["fp64"].get(k) for k in ("value", "ms_per_step", "certified", "mean_iters")}
        c["mixed_over_fp64"] = r.get("mixed_over_fp64")
    if "mixed_rule" in r:
        c["mixed_rule"] = {k: r["mixed_rule"].get(k) for k in ("value", "ms_per_step", "certified")}
        c["mixed_rule"]["lowest_admissible_selected"] = _get(r, "mixed_rule", "stats", "lowest_admissible_selected")
        c["selector_gain"] = r.get("selector_gain")
    if "mixed_rule_tuned" in r:
        c["mixed_rule_tuned"] = {k: r["mixed_rule_tuned"].get(k) for k in ("value", "ms_per_step", "certified")}
        c["mixed_rule_tuned"]["lowest_admissible_selected"] = _get(r, "mixed_rule_tuned", "stats",
                                                                   "lowest_admissible_selected")
        c["selector_gain_vs_tuned_rule"] = r.get("selector_gain_vs_tuned_rule")
    st = _get(pol, "stats")
    if st:
        c["selector_stats"] = {"sensitivity": _get(st, "sensitivity", "k"), "escalate": _get(st, "sensitivity", "n"),
                               "specificity": _get(st, "specificity", "k"), "preserve": _get(st, "specificity", "n"),
                               "guard_fallbacks": st.get("guard_fallbacks"),
                               "lowest_admissible_selected": st.get("lowest_admissible_selected")}
    ak = r.get("apply_K")
    if ak:
        c["apply_K_256x128x128"] = {}
        for k in ("f32", "f64", "bf16_mfma", "bf16x3_mfma"):
            if isinstance(ak.get(k), dict) and "us_per_apply" in ak[k]:
                c["apply_K_256x128x128"][k] = {"us": ak[k]["us_per_apply"], "GB/s": ak[k]["GB/s"],
                                               "frac": ak[k]["frac_hbm_peak"]}
        se = ak.get("sensitivity_f64")
        if isinstance(se, dict):
            c["apply_K_256x128x128"]["sensitivity_f64"] = {"us": se["us_per_call"], "GB/s": se["GB/s"],
                                                           "frac": se["frac_hbm_peak"]}
    sp_ = r.get("small_plain")
    if sp_:
        c["small_plain_16x8x8"] = {"solves_per_s": _get(sp_, "graph_replay", "value"),
                                   "us_per_iteration": {k: _get(sp_, k, "us_per_iteration") for k in
                                                        ("direct_launches_sync1", "direct_launches", "graph_replay")}}
    bu = r.get("batch_uneven")
    if bu:
        c["batch_uneven_192"] = {"mixed": _get(bu, "mixed_batched", "value"),
                                 "mixed_graphs": _get(bu, "mixed_batched_graphs", "value"),
                                 "mixed_sync1": _get(bu, "mixed_batched_sync1", "value"),
                                 "serial": _get(bu, "mixed_serial", "value"), "fp64": _get(bu, "fp64_batched", "value"),
                                 "guard_passing": _get(bu, "mixed_batched", "guard_passing"),
                                 "oracle_false_acceptances": _get(bu, "oracle_recheck", "false_acceptances_oracle")}
    ms = r.get("mixed_at_scale")
    if ms:
        c["mixed_at_scale_256x128x128"] = {
            "iterations": [_get(ms, "mixed", "iterations"), _get(ms, "fp64", "iterations")],
            "seconds": [_get(ms, "mixed", "seconds"), _get(ms, "fp64", "seconds")],
            "true_eta": [_get(ms, "mixed", "true_eta"), _get(ms, "fp64", "true_eta")],
            "rel_error_vs_fp64": ms.get("rel_error_vs_fp64"),
            "oracle_max_eta": _get(ms, "oracle_recheck", "max_eta_oracle"),
            "oracle_false_acceptances": _get(ms, "oracle_recheck", "false_acceptances_oracle")}
    tr = r.get("trajectory")
    if tr:
        c["trajectory_s"] = {k: _get(tr, k, "seconds") for k in ("guarded", "guarded_reuse")}
    ad = r.get("adaptive_preconditioner")
    if ad:
        c["adaptive"] = {"certified": [_get(ad, "adaptive", "certified"), _get(ad, "plain_vcycle", "certified")],
                         "s_per_solve": [_get(ad, "adaptive", "seconds_per_solve"),
                                         _get(ad, "plain_vcycle", "seconds_per_solve")]}
    sp = r.get("stack_policy")
    if sp:
        c["stack_policy_paper_setting"] = {"states": sp.get("states")}
        for name in ("rule", "always_rho0_then_ladder"):
            v = sp.get(name) or {}
            c["stack_policy_paper_setting"][name] = {
                "certified": v.get("certified"), "false_stops_caught": v.get("false_stops_caught"),
                "accepted_above_tolerance": v.get("accepted_above_tolerance"),
                "oracle_false_acceptances": _get(v, "oracle_recheck", "false_acceptances_oracle"),
                "s_per_state": v.get("seconds_per_state")}
    if full_path:
        c["full_record"] = full_path
    return _r(c)


def recheck_task(item):
    """The oracle's recomputed residual of one GPU solution (runs in a worker
    process): eta = ||f - K u|| / ||f|| over free DOFs with the matrix-free
    FP64 operator of the floor the solution was accepted at, and the rounding
    bound delta of that evaluation."""
    dims, rho, p, floor, f, u = item
    from oracle import ke, mesh
    from oracle import operator as op
    g = mesh.Grid(*dims)
    E = op.young(rho, p, floor)
    Ke = ke.ke()
    return op.relative_residual_full(g, E, Ke, f, u), op.residual_bound_full(g, E, Ke, f, u)


def oracle_recheck(items, gpu_etas, tau=1e-6, workers=None):
    """Recheck accepted GPU solutions with the oracle in a pool of host
    processes.  A false acceptance is an oracle eta above tau by more than
    the evaluation bound delta; |eta - tau| < delta is boundary-ambiguous."""
    if not items:
        return {"checked": 0}
    env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_keep:
        os.environ[k] = "1"
    t0 = time.perf_counter()
    try:
        with ProcessPoolExecutor(workers or cpu_cores(), mp_context=multiprocessing.get_context("spawn")) as ex:
            res = list(ex.map(recheck_task, items))
    finally:
        for k, v in env_keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    eta = np.array([r[0] for r in res])
    dlt = np.array([r[1] for r in res])
    gpu = np.asarray(gpu_etas, dtype=float)
    return {"checked": len(items), "seconds": time.perf_counter() - t0,
            "false_acceptances_oracle": int(np.sum(eta > tau + dlt)),
            "above_tau_oracle": int(np.sum(~(eta <= tau))),
            "boundary_ambiguous": int(np.sum(np.abs(eta - tau) < dlt)),
            "max_eta_oracle": float(np.max(eta)), "max_delta": float(np.max(dlt)),
            "max_abs_gpu_minus_oracle": float(np.max(np.abs(gpu - eta))),
            "max_abs_gpu_minus_oracle_over_delta": float(np.max(np.abs(gpu - eta) / dlt))}


def wilson(k, n, z=1.959963984540054):
    """Wilson score interval for k successes in n trials (95 % by default)."""
    if n == 0:
        return None
    p = k / n
    den = 1.0 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * math.sqrt(p * (1.0 - p) / n + z * z / (4.0 * n * n)) / den
    return [c - h, c + h]


def policy_stats(outs, labels, tau=1e-6, cap=200):
    """Held-out statistics of one policy run against reference labels (the
    lowest rung whose independent solve passes the guard, -1 if none):
    confusion with escalation as the positive class and Wilson intervals,
    guard fallbacks, projected convergences the guard rejected, accepted
    solves above the tolerance (must be 0) and the preserve margin."""
    n = len(outs)
    pred = [o["k0"] > 0 for o in outs]
    ref = [lab != 0 for lab in labels]
    tp = sum(1 for p, r in zip(pred, ref) if p and r)
    tn = sum(1 for p, r in zip(pred, ref) if not p and not r)
    fp = sum(1 for p, r in zip(pred, ref) if p and not r)
    fn = sum(1 for p, r in zip(pred, ref) if not p and r)
    cert = sum(1 for o in outs if o["rung"] >= 0)
    atts = [a for o in outs for a in o["attempts"]]
    kept = [o for o in outs if o["rung"] == 0]
    its = [o["attempts"][-1]["iterations"] for o in kept]
    return {
        "reference": {"escalate": sum(ref), "preserve": n - sum(ref),
                      "none_admissible": sum(1 for lab in labels if lab < 0)},
        "confusion": {"TP": tp, "TN": tn, "FP": fp, "FN": fn},
        "sensitivity": {"k": tp, "n": tp + fn, "wilson95": wilson(tp, tp + fn)},
        "specificity": {"k": tn, "n": tn + fp, "wilson95": wilson(tn, tn + fp)},
        "guard_fallbacks": sum(1 for o in outs if o["k0"] == 0 and o["rung"] != 0),
        "selected_meet_tolerance": {"k": cert, "n": n, "wilson95": wilson(cert, n)},
        "lowest_admissible_selected": sum(1 for o, lab in zip(outs, labels) if o["rung"] == lab),
        "projected_converged_rejected_by_guard": sum(
            1 for a in atts if a["outcome"] == "PROJ_CONVERGED" and not a["true_eta"] <= tau),
        "accepted_above_tolerance": sum(1 for a in atts if a["accepted"] and not a["true_eta"] <= tau),
        "preserve_margin": {"preserved": len(kept), "cap": cap, "max_iterations": max(its, default=None),
                            "at_least_80pct_of_cap": sum(1 for i in its if i >= 0.8 * cap)},
    }


def cpu_cores():
    """Host cores this process may use, capped at the 16 a one-GPU share offers."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_info():
    """CPU model, library versions and BLAS threads of the host that timed
    the CPU baseline."""
    import scipy
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = sorted({d.get("internal_api") for d in threadpool_info()} - {None})
    except Exception:  # threadpoolctl missing or unable to inspect: report nothing
        blas = None
    return {"cpu_model": model, "processes": cpu_cores(), "numpy": np.__version__, "scipy": scipy.__version__,
            "blas": blas, "blas_threads_per_process": 1}


def run_cpu_baseline(setups_per_state, iters_per_state):
    """One oracle process per host core (one BLAS thread each), each timing the
    sample on its own state concurrently; the rate is the sum of the per-process
    state rates."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cores = cpu_cores()
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-only", "--cpu-seed",
                               str(SEED0 + i)], env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                              text=True) for i in range(cores)]
    samples = []
    for pr in procs:
        out, err = pr.communicate(timeout=900)
        if pr.returncode != 0:
            raise RuntimeError("cpu baseline failed: " + err[-2000:])
        samples.append(json.loads(out.strip().splitlines()[-1]))
    rates = [1.0 / (setups_per_state * d["t_setup"] + iters_per_state * d["t_iter"]) for d in samples]
    ts = float(np.median([d["t_setup"] for d in samples]))
    ti = float(np.median([d["t_iter"] for d in samples]))
    return {
        "value": float(sum(rates)), "unit": "certified solves/s", "cores": cores, "kind": "oracle",
        "sample": (f"oracle (assembled CSR, FP64), one process per core on states {SEED0}-{SEED0 + cores - 1} "
                   f"at 64x32x32: each times one hierarchy build (median {ts:.1f} s) and 20 FGMRES(30) "
                   f"iterations (median {ti*1e3:.0f} ms each) concurrently; per-process rates scaled by the "
                   f"GPU run's mean {setups_per_state:.2f} set_density calls and {iters_per_state:.1f} "
                   f"FGMRES iterations per state and summed"),
    }


def apply_leg(tg, torch, dev, reps=40):
    """apply_K HBM bandwidth at 256x128x128 (12.8M DOF) on the strut field.

    Rotates over buffer sets whose total exceeds the 256 MB Infinity Cache so
    every launch streams from HBM.  Algorithmic bytes per apply: read u and
    write y (3 DOF per node each) plus one modulus per element."""
    from paper_2607_26382_amd import synth
    nx, ny, nz = 256, 128, 128
    g = tg.Grid(nx, ny, nz, max_restart=2, device=dev)
    rho = torch.tensor(synth.struts(nx, ny, nz, 3000), device=dev)
    g.set_density(rho, 3.0, 1e-3)
    out = {"autotuned_zc": {}}
    for name, prec, dt, vb in (("f32", tg.F32, torch.float32, 4), ("f64", tg.F64, torch.float64, 8),
                               ("bf16_mfma", tg.BF16MFMA, torch.float32, 4),
                               ("bf16x3_mfma", tg.BF16X3MFMA, torch.float32, 4)):
        # z-tile heights from the autotuner (smoothing sweep timing, per precision)
        zc, _ = g.autotune(prec)
        out["autotuned_zc"][name] = zc[0]
        nsets = max(3, int(np.ceil(600e6 / (2 * g.n_dof * vb))))
        us = [torch.randn(g.n_dof, dtype=dt, device=dev) for _ in range(nsets)]
        ys = [torch.empty_like(us[0]) for _ in range(nsets)]
        try:
            from paper_2607_26382_amd._lib import lib as _l
            import ctypes as C
            st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
            def run(i):
                rc = _l().tg_apply_K(g.handle, C.c_void_p(us[i].data_ptr()), C.c_void_p(ys[i].data_ptr()),
                                     prec, st)
                if rc != 0:
                    raise RuntimeError(_l().tg_last_error().decode())
            for i in range(nsets):
                run(i)
            torch.cuda.synchronize()
            # per-launch HIP events on the launch stream (library kernel timer)
            cls = "apply_f64" if prec == tg.F64 else "vcycle_fine_op"
            tg.kernel_timer_enable(1 << (0 if prec == tg.F64 else 1))
            tg.kernel_timer_reset()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for r in range(reps):
                run(r % nsets)
            e1.record()
            torch.cuda.synchronize()
            kt = tg.kernel_timer_read()[cls]
            tg.kernel_timer_enable(0)
            t_wall = e0.elapsed_time(e1) / reps * 1e-3
            t = kt["avg_us"] * 1e-6
        except RuntimeError as exc:
            out[name] = {"error": str(exc)}
            continue
        alg = 2 * g.n_dof * vb + g.n_elem * vb
        out[name] = {"us_per_apply": t * 1e6, "alg_bytes": alg, "GB/s": alg / t / 1e9,
                     "frac_hbm_peak": alg / t / 1e9 / HBM_PEAK_GBS, "buffer_sets": nsets,
                     "launches_timed": kt["count"], "us_per_call_wall": t_wall * 1e6}
        log(f"apply_K {name}: {t*1e6:.1f} us, {alg / t / 1e9:.0f} GB/s")
        del us, ys
    # compliance sensitivities and f^T u (FP64, one z-march): read u and f
    # (3 DOF per node each) and one density per element, write one
    # sensitivity per element; buffer sets rotate past the Infinity Cache
    from paper_2607_26382_amd._lib import lib as _l
    import ctypes as C
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    nsets = max(3, int(np.ceil(600e6 / (2 * g.n_dof * 8))))
    sets = [(torch.randn(g.n_dof, dtype=torch.float64, device=dev),
             torch.randn(g.n_dof, dtype=torch.float64, device=dev),
             torch.empty(g.n_elem, dtype=torch.float64, device=dev)) for _ in range(nsets)]
    comp = C.c_double()

    def run_s(i):
        u, f, dc = sets[i]
        rc = _l().tg_compliance_sensitivity(g.handle, C.c_void_p(rho.data_ptr()), 3.0, 1e-3,
                                            C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), None,
                                            C.c_void_p(dc.data_ptr()), C.byref(comp), st)
        if rc != 0:
            raise RuntimeError(_l().tg_last_error().decode())
    for i in range(nsets):
        run_s(i)
    tg.kernel_timer_enable(1 << 8)
    tg.kernel_timer_reset()
    for r in range(reps):
        run_s(r % nsets)
    kt = tg.kernel_timer_read()["fidelity"]
    tg.kernel_timer_enable(0)
    t = kt["avg_us"] * 1e-6
    alg = 2 * g.n_dof * 8 + 2 * g.n_elem * 8
    out["sensitivity_f64"] = {"us_per_call": t * 1e6, "alg_bytes": alg, "GB/s": alg / t / 1e9,
                              "frac_hbm_peak": alg / t / 1e9 / HBM_PEAK_GBS, "buffer_sets": nsets,
                              "launches_timed": kt["count"]}
    log(f"compliance sensitivities f64: {t*1e6:.1f} us, {alg / t / 1e9:.0f} GB/s")
    del sets
    out["grid"] = [nx, ny, nz]
    out["n_dof"] = g.n_dof
    del g
    torch.cuda.empty_cache()
    return out


def screen_stats(tg, torch, grids, rhos, labels, rungs, p, prec, tau=1e-6):
    """Sec. 4.2 on the solver's own operator: per state kappa of K(rho_0) from
    the library's Lanczos / LOBPCG, c = kappa rho_0 and the screen
    c eps / tau of Eq. screen, set against the lowest admissible rung of the
    reference labels."""
    eps = float(np.finfo(float).eps)
    rows = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, rho, lab in zip(grids, rhos, labels):
        g.set_density(rho, p, rungs[0])
        r = g.extreme_eigenvalues(prec=prec, max_iters=600, tol=1e-6)
        c = r["kappa"] * rungs[0]
        rows.append(dict(c=c, screen=c * eps / tau, kappa=r["kappa"], conv=r["converged"], lab=lab,
                         iters=r["iters_min"]))
    dt = time.perf_counter() - t0
    scr = np.array([x["screen"] for x in rows])
    lab = [x["lab"] for x in rows]
    adm = [x for x in rows if x["lab"] >= 0]
    # the first rung at or above the screen, and whether it certifies
    first = [next((k for k, fl in enumerate(rungs) if fl >= x["screen"]), None) for x in adm]
    return {
        "floor": rungs[0], "states": len(rows), "lobpcg_converged": int(sum(x["conv"] for x in rows)),
        "seconds": dt, "mean_lobpcg_iters": float(np.mean([x["iters"] for x in rows])),
        "kappa_eps_min": float(min(x["kappa"] for x in rows) * eps),
        "kappa_eps_max": float(max(x["kappa"] for x in rows) * eps),
        "c_min": float(min(x["c"] for x in rows)), "c_median": float(np.median([x["c"] for x in rows])),
        "c_max": float(max(x["c"] for x in rows)),
        "screen_min": float(scr.min()), "screen_max": float(scr.max()),
        "admissible_states": len(adm),
        "certified_below_screen": int(sum(1 for x in adm if rungs[x["lab"]] < x["screen"])),
        "first_rung_above_screen_admissible": int(sum(1 for x, k in zip(adm, first)
                                                      if k is not None and k >= x["lab"])),
        "rungs_skipped_by_screen": int(sum(sum(1 for fl in rungs if fl < x["screen"]) for x in rows)),
        "none_admissible": int(sum(1 for v in lab if v < 0)),
    }


def checkpoint_stats(tg, torch, grids, rhos, fs, rungs, p, prec, every=10, t_high=1e-2, t_plateau=1e-4,
                     t_ratio=0.6):
    """The probe at rho_0 with true-residual checkpoints every `every`
    iterations (Sec. 4.1.1's untested detector variant): the largest ratio of
    recomputed to projected residual, and whether the two-feature rule (Eq.
    trigger) decides differently on recomputed features r50, r100."""
    ratios, flips, both, t0 = [], 0, 0, time.perf_counter()
    rule = lambda a, b: a >= t_high or (b >= t_plateau and b / a >= t_ratio)
    for g, rho, f in zip(grids, rhos, fs):
        g.set_density(rho, p, rungs[0])
        cps, kstop = g.probe_checkpoints(f, iters=100, restart=100, every=every, prec=prec)
        ratios += [tr / pj for _, pj, tr in cps if pj > 0]
        d = {k: (pj, tr) for k, pj, tr in cps}
        if 50 in d and 100 in d:
            both += 1
            flips += rule(d[50][0], d[100][0]) != rule(d[50][1], d[100][1])
    return {"floor": rungs[0], "every": every, "states": len(grids), "checkpoints": len(ratios),
            "seconds": time.perf_counter() - t0,
            "max_true_over_projected": float(max(ratios)) if ratios else None,
            "min_true_over_projected": float(min(ratios)) if ratios else None,
            "median_true_over_projected": float(np.median(ratios)) if ratios else None,
            "states_with_50_and_100": both, "rule_decisions_changed": int(flips)}


def fidelity_stats(grids, rhos, fs, sols, ok, rungs, p, solid_min=0.5):
    """Tab. perturbation on the states whose original floor (rungs[0]) is
    admissible: for every raised rung whose solve is also accepted, the
    absolute relative compliance change and the relative l2 change and Pearson
    correlation of the compliance sensitivities over the solid elements
    (rho >= solid_min), all computed by the library's FP64 kernels."""
    out = {}
    base = {}
    for i, g in enumerate(grids):
        if ok[0][i]:
            base[i] = g.compliance_sensitivity(sols[0][i], f=fs[i], rho=rhos[i], p=p, rho_min=rungs[0])
    for k in range(1, len(rungs)):
        dc, l2, r, decreases = [], [], [], 0
        for i, b in base.items():
            if not ok[k][i]:
                continue
            o = grids[i].compliance_sensitivity(sols[k][i], f=fs[i], rho=rhos[i], p=p, rho_min=rungs[k])
            dc.append(abs(o["compliance"] - b["compliance"]) / abs(b["compliance"]))
            decreases += o["compliance"] < b["compliance"]
            gc = grids[i].gradient_change(rhos[i], b["dc"], o["dc"], solid_min)
            l2.append(gc["rel_l2"])
            r.append(gc["pearson"])
        if dc:
            out[f"{rungs[k]:g}"] = {"states": len(dc), "mean_abs_dC_over_C": float(np.mean(dc)),
                                    "max_abs_dC_over_C": float(np.max(dc)), "compliance_decreases": int(decreases),
                                    "mean_grad_rel_l2": float(np.mean(l2)), "max_grad_rel_l2": float(np.max(l2)),
                                    "min_pearson": float(np.min(r))}
    return {"reference_floor": rungs[0], "reference_admissible_states": len(base), "solid": f"rho >= {solid_min}",
            "raised": out}


def trajectory_leg(tg, torch, dev, mixed_prec):
    """The optimization-loop runs of Sec. 4.1.2 on the 64x32x32 cantilever
    (volume fraction 0.30, filter radius 1.5, continuation p 1.5 -> 3.5,
    beta 1 -> 4, move 0.20 -> 0.15 after outer iteration 15, 40 iterations,
    rungs 1e-12, 1e-3, 1e-2): the guarded policy at every iteration, the
    same with the previous decision reused until the guard rejects it, and
    the unguarded fixed-floor controls 1e-12 and 1e-3.  Every run starts from
    the uniform design; each is timed as a whole (wall clock, synchronized)."""
    g = tg.Grid(64, 32, 32, max_restart=100, device=dev)
    f = torch.tensor(g.edge_load(), device=dev)
    x0 = torch.full((g.n_elem,), 0.30, dtype=torch.float64, device=dev)
    out = {"grid": [64, 32, 32], "volfrac": 0.30, "r_min": 1.5, "outer_iters": 40,
           "stages": [[1, 1.5, 1.0, 0.20], [16, 3.5, 4.0, 0.15]], "rungs": [1e-12, 1e-3, 1e-2],
           "solve": "FGMRES(30), cap 200, split-BF16 V-cycle, FP64 guard"}
    runs = (("guarded", tg.LOOP_GUARDED, None), ("guarded_reuse", tg.LOOP_REUSE, None),
            ("fixed_1e-12_unguarded", tg.LOOP_FIXED, 1e-12), ("fixed_1e-3_unguarded", tg.LOOP_FIXED, 1e-3))
    for name, mode, ff in runs:
        o = tg.topopt_opts(mode=mode, fixed_floor=ff if ff else 1e-3)
        o.policy.solve.prec = mixed_prec
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rec = g.topopt_run(x0, f, o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        acc = [r for r in rec if r["accepted"] == 1]
        switch = next((r["iter"] for r in rec if r["rung"] > 0), None)
        out[name] = {
            "seconds": dt, "outer_iterations": len(rec), "fgmres_iterations": int(sum(r["solve_iters"] for r in rec)),
            "probes": int(sum(r["probed"] for r in rec)), "final_compliance": rec[-1]["compliance"],
            "compliance": [r["compliance"] for r in rec], "floors": [r["floor"] for r in rec],
            "solve_iters": [r["solve_iters"] for r in rec], "true_eta": [r["true_eta"] for r in rec],
            "first_raised_floor_iter": switch,
            "accepted": len(acc), "max_accepted_true_eta": max((r["true_eta"] for r in acc), default=None),
            "solves_at_cap": int(sum(1 for r in rec if mode == tg.LOOP_FIXED and r["solve_iters"] >= 200)),
            "solves_above_tau": int(sum(1 for r in rec if r["true_eta"] > 1e-6)),
        }
        log(f"trajectory {name}: {dt:.1f} s, {len(rec)} outer its, final C {rec[-1]['compliance']:.4g}, "
            f"first raised floor at {switch}")
    out["reuse_speedup"] = out["guarded"]["seconds"] / out["guarded_reuse"]["seconds"]
    del g
    torch.cuda.empty_cache()
    return out


def adaptive_runs(tg, torch, g, rhos, fs, p, floor, opts, inner, tau=1e-6):
    """Solve each state with tg_adaptive_solve; counts and per-state results."""
    its, cert, false_acc, maxit, kept, applied, secs, rows = 0, 0, 0, 0, 0, 0, 0.0, []
    for rho, f in zip(rhos, fs):
        g.set_density(rho, p, floor)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, res, hist, acc = g.adaptive_solve(f, opts, inner)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        eta = g.true_residual(f, u)
        rows.append([res["iterations"], res["outcome"], res["proj_eta"], eta])
        its += res["iterations"]
        cert += eta <= tau
        false_acc += res["outcome"] == "PROJ_CONVERGED" and eta > tau
        maxit += res["outcome"] == "MAXIT"
        kept += sum(acc)
        applied += len(acc)
    n = len(rhos)
    ratio = [row[3] / row[2] for row in rows if row[2] > 0]
    return {"mean_iters": its / n, "certified": int(cert), "proj_converged_guard_rejects": int(false_acc),
            "true_over_projected_at_stop": [min(ratio), max(ratio)] if ratio else None,
            "drifted_twofold": int(sum(1 for r in ratio if r > 2.0)),
            "maxit": int(maxit), "corrections_kept": int(kept), "preconditioner_applications": int(applied),
            "seconds_per_solve": secs / n, "per_state": rows}


def adaptive_leg(tg, torch, dev, rhos, fs, prec, n_states=102, floor=1e-9, n_paper=102):
    """The fine-level adaptive correction of the preconditioner (Tab.
    solver-config), with it (20 inner node-block-Jacobi GMRES steps, kept only
    if they lower the residual) and without it (inner_steps = 0).  Per
    variant: outer iterations, certified solves (FP64 guard <= 1e-6), solves
    whose projected estimate converged while the guard rejects them, kept
    corrections, seconds per solve (synchronized wall clock of the solve).
    workload: the severe states at the original floor, p = 3, FGMRES(30),
    cap 200, V-cycle at `prec`.  paper_setting: the first n_paper states under
    the adaptive stack's own settings (Tab. solver-config: p = 4.5,
    rho_0 = 1e-12, restart = cap = 300, FP64 fine path)."""
    g = tg.Grid(*GRID, max_restart=30, device=dev)
    out = {"states": n_states, "floor": floor, "p": 3.0, "inner_steps": 20,
           "solve": "FGMRES(30), cap 200, FP64 operator and guard"}
    o = tg.solver_opts(restart=30, max_iters=200, prec=prec)
    for name, inner in (("adaptive", 20), ("plain_vcycle", 0)):
        r = adaptive_runs(tg, torch, g, rhos[:n_states], fs[:n_states], 3.0, floor, o, inner)
        out[name] = {k: v for k, v in r.items() if k != "per_state"}
        log(f"adaptive leg {name}: mean its {r['mean_iters']:.1f}, certified {r['certified']}/{n_states}, "
            f"false acceptances caught {r['proj_converged_guard_rejects']}, {r['seconds_per_solve']:.3f} s/solve")
    n_paper = min(n_paper, len(rhos))
    ps = {"states": n_paper, "p": 4.5, "floor": 1e-12, "solve": "FGMRES(300), cap 300, FP64 throughout, CGS2",
          "cgs1": "variants *_cgs1: one Gram-Schmidt sweep per step"}
    for name, inner, passes in (("adaptive", 20, 2), ("plain_vcycle", 0, 2), ("adaptive_cgs1", 20, 1),
                                ("plain_vcycle_cgs1", 0, 1)):
        o = tg.solver_opts(restart=300, max_iters=300, prec=tg.F64, cgs_passes=passes)
        ps[name] = adaptive_runs(tg, torch, g, rhos[:n_paper], fs[:n_paper], 4.5, 1e-12, o, inner)
        r = ps[name]
        log(f"adaptive leg, paper setting, {name}: mean its {r['mean_iters']:.1f}, certified "
            f"{r['certified']}/{n_paper}, false acceptances caught {r['proj_converged_guard_rejects']}, "
            f"MAXIT {r['maxit']}, true/projected at stop {r['true_over_projected_at_stop']} "
            f"({r['drifted_twofold']} above 2), "
            f"{r['seconds_per_solve']:.3f} s/solve")
    # periodic true-residual checkpoints (every 10 iterations) on the states
    # whose one-sweep solve ended with the recomputed residual above twice the
    # estimate: the first checkpoint where that gap appears
    drift = []
    o = tg.solver_opts(restart=300, max_iters=300, prec=tg.F64, cgs_passes=1)
    for i, row in enumerate(ps["adaptive_cgs1"]["per_state"]):
        if not row[3] > 2.0 * row[2]:
            continue
        g.set_density(rhos[i], 4.5, 1e-12)
        _, res, cps = g.adaptive_checkpoints(fs[i], o, 20, every=10)
        first = next((k for k, pj, tr in cps if tr > 2 * pj), None)
        drift.append({"state": SEED0 + i, "stop_iteration": res["iterations"], "first_flagged_checkpoint": first,
                      "true_over_projected": [round(tr / pj, 4) for k, pj, tr in cps if pj > 0]})
        log(f"adaptive leg, checkpoints on state {SEED0 + i}: stop at {res['iterations']}, "
            f"first checkpoint with true > 2 x projected at {first}")
    ps["adaptive_cgs1_checkpoints"] = drift
    # the states whose estimate drifted furthest from the recomputed residual
    # under the fine-level correction with CGS2 (largest recomputed /
    # projected at the stop), for the full-stack policy leg
    rows = ps["adaptive"]["per_state"]
    ps["drift_order"] = sorted(range(len(rows)), key=lambda i: -(rows[i][3] / rows[i][2] if rows[i][2] > 0 else 0.0))
    # per-state rows only where the estimate converged but the guard rejects
    for name in ("adaptive", "plain_vcycle", "adaptive_cgs1", "plain_vcycle_cgs1"):
        rows = ps[name].pop("per_state")
        ps[name]["false_acceptances"] = [[SEED0 + i, row[0], row[2], row[3]] for i, row in enumerate(rows)
                                         if row[1] == "PROJ_CONVERGED" and row[3] > 1e-6]
    out["paper_setting"] = ps
    del g
    torch.cuda.empty_cache()
    return out



PAPER_RUNGS = (1e-12, 1e-3, 1e-2)


def stack_policy_leg(tg, torch, dev, rhos, fs, n_states, recheck=True, tau=1e-6, order=None):
    """Alg. floor_policy with the full adaptive stack (Chebyshev smoothing,
    line-searched and rejectable coarse correction with 10 level-1 GMRES
    steps, fine-level correction) preconditioning the probe and every rung,
    under the paper's settings (Tab. solver-config: p = 4.5, rho_0 = 1e-12,
    ladder {1e-3, 1e-2}, 100-iteration probe, FGMRES(300) with cap 300, FP64
    throughout), one state at a time through tg_stack_select_floor, with the
    two-feature rule (the paper's policy) and with the original floor always
    tried first (the paper's exhaust-the-original-floor baseline).  Per
    variant: certified states, the attempts whose projected estimate
    converged while the recomputed residual is above tau (false stops the
    guard rejects), first and selected rungs, stage iterations, seconds per
    state, and the oracle's recheck of every accepted solution.  `order`
    (state indices) picks the states, by default the first n_states."""
    n = min(n_states, len(rhos))
    pick = list(order[:n]) if order is not None else list(range(n))
    rhos = [rhos[i] for i in pick]
    fs = [fs[i] for i in pick]
    seeds = [SEED0 + i for i in pick]
    g = tg.Grid(*GRID, max_restart=30, device=dev)
    solve = tg.solver_opts(restart=300, max_iters=300, prec=tg.F64)
    out = {"states": n, "seeds": seeds, "p": 4.5, "rungs": list(PAPER_RUNGS), "probe": "100 its, restart 100",
           "solve": "FGMRES(300), cap 300, adaptive stack, FP64 throughout",
           "selection": "first states" if order is None else
           "largest recomputed / projected residual at the stop of the fine-correction paper-setting solve"}
    for name, sel in (("rule", {}), ("always_rho0_then_ladder", dict(selector=tg.SELECT_FIXED, fixed_rung=0))):
        pol = tg.policy(rungs=PAPER_RUNGS, p=4.5, solve=solve, **sel)
        outs, us, secs = [], [], []
        for i in range(n):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, o = g.stack_select_floor(rhos[i], fs[i], pol)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t0)
            outs.append(o)
            us.append(u.cpu().numpy() if o["rung"] >= 0 else None)
            log(f"stack policy ({name}) state {seeds[i]}: k0={o['k0']} rung={o['rung']} r50={o['r50']:.3g} "
                f"r100={o['r100']:.3g} attempts="
                f"{[(a['rung'], a['iterations'], a['outcome'], a['true_eta']) for a in o['attempts']]} "
                f"{secs[-1]:.2f}s")
        false_stops = [[seeds[i], a["rung"], a["iterations"], a["proj_eta"], a["true_eta"]]
                       for i, o in enumerate(outs) for a in o["attempts"]
                       if a["outcome"] == "PROJ_CONVERGED" and not a["true_eta"] <= tau]
        acc = [o for o in outs if o["rung"] >= 0]
        res = {"certified": len(acc),
               "first_rung": {str(r): sum(1 for o in outs if o["k0"] == r) for r in range(len(PAPER_RUNGS))},
               "selected_rungs": {str(r): sum(1 for o in outs if o["rung"] == r)
                                  for r in range(-1, len(PAPER_RUNGS))},
               "false_stops_caught": len(false_stops), "false_stop_rows": false_stops,
               "accepted_above_tolerance": sum(1 for o in outs for a in o["attempts"]
                                               if a["accepted"] and not a["true_eta"] <= tau),
               "max_accepted_true_eta": max((o["attempts"][-1]["true_eta"] for o in acc), default=None),
               "mean_attempts": float(np.mean([len(o["attempts"]) for o in outs])) if outs else None,
               "mean_iters": {k: float(np.mean([o[k] for o in outs])) if outs else None
                              for k in ("iters_probe", "iters_selected", "iters_rejected")},
               "seconds_per_state": float(np.mean(secs)) if secs else None}
        if recheck and acc:
            f_np = fs[0].cpu().numpy()
            items = [(GRID, rhos[i].cpu().numpy(), 4.5, PAPER_RUNGS[o["rung"]], f_np, us[i])
                     for i, o in enumerate(outs) if o["rung"] >= 0]
            res["oracle_recheck"] = oracle_recheck(items, [o["attempts"][-1]["true_eta"] for o in acc])
        log(f"stack policy leg ({name}): certified {res['certified']}/{n}, false stops caught "
            f"{res['false_stops_caught']}, {res['seconds_per_state']:.2f} s/state")
        out[name] = res
        del us
    del g
    torch.cuda.empty_cache()
    return out

B4_GRIDS = ((32, 16, 16), (48, 24, 24), (64, 32, 32), (96, 48, 48))


def batch4_leg(tg, torch, dev, mixed_prec, recheck=True):
    """Batched uneven solves: 48 blob states (seeds 4000-4047, grid
    B4_GRIDS[i % 4], the severe-state generator at that size) x 4 ladder
    floors = 192 independent solves in one batch (FP32 V-cycle, FP64 guard),
    against the same 192 solves one at a time and the FP64 batch.  Rate =
    guard-passing solves / wall time of set_density + solve + guard."""
    from paper_2607_26382_amd import synth
    grids, rhos, floors, fs = [], [], [], []
    loads = {}
    for i in range(48):
        d = B4_GRIDS[i % 4]
        rt = torch.tensor(synth.blobs(*d, 4000 + i, blob=4, floor_frac=0.5), device=dev)
        for r in RUNGS:
            g = tg.Grid(*d, max_restart=30, device=dev)
            if d not in loads:
                loads[d] = torch.tensor(g.edge_load(), device=dev)
            grids.append(g)
            rhos.append(rt)
            floors.append(r)
            fs.append(loads[d])
    batch = tg.Batch(grids)
    log(f"batch of {len(grids)} uneven solves bound")
    batch.set_density(rhos, 3.0, floors)
    zc, _ = batch.autotune(mixed_prec)

    last = {}

    def batched(prec, graphs=False, sync_every=8):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.set_density(rhos, 3.0, floors)
        us, res = batch.solve(fs, tg.solver_opts(prec=prec, graphs=graphs, sync_every=sync_every))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        last["us"], last["res"] = us, res
        ok = sum(1 for r in res if r["true_eta"] <= 1e-6)
        return {"value": ok / dt, "seconds": dt, "guard_passing": ok,
                "mean_iters": float(np.mean([r["iterations"] for r in res]))}

    batched(mixed_prec)   # warm-up
    out = {"solves": len(grids), "grids": [list(d) for d in B4_GRIDS], "autotuned_zc": zc[:2],
           "mixed_batched": batched(mixed_prec)}
    if recheck:
        # the oracle's eta of every guard-passing solution of the mixed batch
        items, etas = [], []
        for q, r in enumerate(last["res"]):
            if r["true_eta"] <= 1e-6:
                g = grids[q]
                items.append(((g.nx, g.ny, g.nz), rhos[q].cpu().numpy(), 3.0, floors[q], fs[q].cpu().numpy(),
                              last["us"][q].cpu().numpy()))
                etas.append(r["true_eta"])
        out["oracle_recheck"] = oracle_recheck(items, etas)
        del items
        log(f"uneven batch oracle recheck: {out['oracle_recheck']['checked']} solutions, "
            f"{out['oracle_recheck']['false_acceptances_oracle']} false acceptances")
    last.clear()
    out["fp64_batched"] = batched(tg.F64)
    # the same batch with every FGMRES step (V-cycle, operator, Gram-Schmidt)
    # replayed from a captured HIP graph; the first pass captures one graph
    # per (active set, step) and is not timed
    t0 = time.perf_counter()
    batched(mixed_prec, graphs=True)
    out["graph_capture_pass_s"] = time.perf_counter() - t0
    out["mixed_batched_graphs"] = batched(mixed_prec, graphs=True)
    out["mixed_batched_sync1"] = batched(mixed_prec, sync_every=1)
    out["tile_heights_per_size"] = {"x".join(map(str, B4_GRIDS[q])): batch.tile_heights(4 * q) for q in range(4)}
    # the same solves one at a time (each grid alone)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok = 0
    for g, r, fl, f in zip(grids, rhos, floors, fs):
        g.set_density(r, 3.0, fl)
        u, res, _ = g.fgmres_solve(f, tg.solver_opts(prec=mixed_prec), want_hist=False)
        ok += int(g.true_residual(f, u) <= 1e-6)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["mixed_serial"] = {"value": ok / dt, "seconds": dt, "guard_passing": ok}
    out["batched_over_serial"] = out["mixed_batched"]["value"] / out["mixed_serial"]["value"]
    out["mixed_over_fp64"] = out["mixed_batched"]["value"] / out["fp64_batched"]["value"]
    log(f"uneven batch: {out['mixed_batched']['value']:.1f} solves/s batched "
        f"({out['mixed_batched_graphs']['value']:.1f} with graph replay), "
        f"{out['mixed_serial']['value']:.1f} serial, {out['fp64_batched']['value']:.1f} FP64 batched")
    del batch, grids
    torch.cuda.empty_cache()
    return out


def scale_leg(tg, torch, dev, mixed_prec, recheck=True):
    """Mixed precision at scale: one solve on 256x128x128 (12.8M DOF), the
    8-strut optimized-like field (seed 3000), p = 3, rho_min = 1e-3,
    FGMRES(30) cap 200, in the mixed form and in FP64; error of the mixed
    solution against the FP64 one, guard values and compliance of both."""
    from paper_2607_26382_amd import synth
    nx, ny, nz = 256, 128, 128
    g = tg.Grid(nx, ny, nz, max_restart=30, device=dev)
    rho = torch.tensor(synth.struts(nx, ny, nz, 3000), device=dev)
    g.set_density(rho, 3.0, 1e-3)
    g.autotune(mixed_prec)
    f = torch.tensor(g.edge_load(), device=dev)
    out = {"grid": [nx, ny, nz], "n_dof": g.n_dof, "rho_min": 1e-3}
    sols = {}
    for name, prec in (("mixed", mixed_prec), ("fp64", tg.F64)):
        o = tg.solver_opts(prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, res, _ = g.fgmres_solve(f, o, want_hist=False)
        eta = g.true_residual(f, u)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sols[name] = u
        out[name] = {"seconds": dt, "iterations": res["iterations"], "outcome": res["outcome"],
                     "true_eta": eta, "certified": bool(eta <= 1e-6),
                     "compliance": float(torch.dot(f, u).item()),
                     "ms_per_iteration": 1e3 * dt / max(res["iterations"], 1)}
    d = sols["mixed"] - sols["fp64"]
    out["rel_error_vs_fp64"] = float((d.norm() / sols["fp64"].norm()).item())
    if recheck:
        # the oracle's eta of both solutions (matrix-free FP64, host processes)
        rho_np, f_np = rho.cpu().numpy(), f.cpu().numpy()
        names = ("mixed", "fp64")
        items = [((nx, ny, nz), rho_np, 3.0, 1e-3, f_np, sols[k].cpu().numpy()) for k in names]
        rc = oracle_recheck(items, [out[k]["true_eta"] for k in names], workers=2)
        out["oracle_recheck"] = rc
        del items
        log(f"256x128x128 oracle recheck: max eta {rc['max_eta_oracle']:.3e}, "
            f"{rc['false_acceptances_oracle']} false acceptances")
    out["compliance_rel_diff"] = abs(out["mixed"]["compliance"] - out["fp64"]["compliance"]) / abs(
        out["fp64"]["compliance"])
    out["mixed_speedup"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    log(f"256x128x128 solve: mixed {out['mixed']['iterations']} its {out['mixed']['seconds']:.2f} s, "
        f"fp64 {out['fp64']['iterations']} its {out['fp64']['seconds']:.2f} s, "
        f"|u_mix - u_64| / |u_64| = {out['rel_error_vs_fp64']:.2e}")
    del g, sols, d
    torch.cuda.empty_cache()
    return out


def small_leg(tg, torch, dev, reps=3):
    """The plain method on the small cantilever: 16x8x8, densities U[0,1)
    (seeds 0-9), rho_min = 1e-3, FP64 throughout, FGMRES(30) cap 200.  A
    launch-latency-bound case: set_density + solve + guard per state, with
    each Arnoldi step launched directly or replayed as a captured graph."""
    from paper_2607_26382_amd import synth
    g = tg.Grid(16, 8, 8, max_restart=30, device=dev)
    f = torch.tensor(g.edge_load(), device=dev)
    rhos = [torch.tensor(synth.uniform(16, 8, 8, sd), device=dev) for sd in range(10)]
    out = {"grid": [16, 8, 8], "states": len(rhos), "dtype": "f64", "levels": g.n_levels}

    def run(graphs, sync_every=8):
        o = tg.solver_opts(prec=tg.F64, graphs=graphs, sync_every=sync_every)
        ok = its = 0
        for r in rhos:   # warm-up (and graph capture)
            g.set_density(r, 3.0, 1e-3)
            g.fgmres_solve(f, o, want_hist=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for r in rhos:
                g.set_density(r, 3.0, 1e-3)
                u, res, _ = g.fgmres_solve(f, o, want_hist=False)
                ok += int(g.true_residual(f, u) <= 1e-6)
                its += res["iterations"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return {"value": ok / dt, "certified": ok, "solves": reps * len(rhos),
                "mean_iters": its / (reps * len(rhos)), "us_per_iteration": 1e6 * dt / its}

    # status read after every Arnoldi step (host round trip per step), then
    # runs of 8 steps per read with device-side gating, launched directly or
    # replayed as captured graphs
    out["direct_launches_sync1"] = run(False, 1)
    out["direct_launches"] = run(False)
    out["graph_replay"] = run(True)
    out["graph_speedup"] = out["graph_replay"]["value"] / out["direct_launches"]["value"]
    log(f"small cantilever: {out['direct_launches_sync1']['us_per_iteration']:.0f} us/iteration with a read per "
        f"step, {out['direct_launches']['us_per_iteration']:.0f} with runs of 8, "
        f"{out['graph_replay']['us_per_iteration']:.0f} with graph replay")
    return out


def main():
    args = parse()
    if args.cpu_only:
        cpu_baseline_child(args.cpu_seed)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent states shard across GPUs with no exchange but a result gather).",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2607_26382_amd import synth
    from paper_2607_26382_amd import topoguard as tg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        # 1 GiB read + 1 GiB written per copy, 4 copies
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 4
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4,
                          "copies": 4, "GB/s": 2 * a.numel() * 4 / dt / 1e9}), flush=True)
        return
    if args.trajectory_only:
        print(json.dumps({"trajectory": trajectory_leg(tg, torch, dev, {"f32": tg.F32, "bf16": tg.BF16MFMA,
                                                                          "bf16x3": tg.BF16X3MFMA}[args.mixed])}),
              flush=True)
        return
    if args.small_only:
        print(json.dumps({"small_plain": small_leg(tg, torch, dev)}), flush=True)
        return
    if args.adaptive_only:
        n_ad = args.states
        rhos = [torch.tensor(synth.severe(SEED0 + i)[1], device=dev) for i in range(n_ad)]
        f0 = torch.tensor(tg.Grid(*GRID, max_restart=1, device=dev).edge_load(), device=dev)
        print(json.dumps({"adaptive_preconditioner": adaptive_leg(
            tg, torch, dev, rhos, [f0] * n_ad, {"f32": tg.F32, "bf16": tg.BF16MFMA, "bf16x3": tg.BF16X3MFMA}[args.mixed],
            n_states=n_ad, n_paper=args.paper_states)}), flush=True)
        return
    if args.stack_only:
        n_st = args.stack_states
        rhos = [torch.tensor(synth.severe(SEED0 + i)[1], device=dev) for i in range(n_st)]
        f0 = torch.tensor(tg.Grid(*GRID, max_restart=1, device=dev).edge_load(), device=dev)
        print(json.dumps({"stack_policy": stack_policy_leg(tg, torch, dev, rhos, [f0] * n_st, n_st,
                                                           recheck=not args.no_recheck)}), flush=True)
        return
    apply_res = None
    if not args.no_apply:
        apply_res = apply_leg(tg, torch, dev)
        if args.apply_only:
            print(json.dumps({"apply_K": apply_res}), flush=True)
            return
    n = args.states
    grids = [tg.Grid(*GRID, max_restart=100, device=dev) for _ in range(n)]
    batch = tg.Batch(grids)
    rhos = [torch.tensor(synth.severe(SEED0 + i)[1], device=dev) for i in range(n)]
    f0 = torch.tensor(grids[0].edge_load(), device=dev)
    fs = [f0.clone() for _ in range(n)]
    torch.cuda.synchronize()
    log(f"{n} grids bound ({sum(g.ws_bytes for g in grids) / 2**30:.1f} GiB workspace)")

    # The states are independent: split them into `streams` contiguous parts,
    # each a batch of its own driven by its own host thread on its own stream
    # (default priority), so one part's bandwidth-bound Krylov sweeps overlap
    # another part's latency- and ALU-bound multigrid kernels.  Every
    # problem's result is the same bits in any batch.
    n_parts = max(1, min(args.streams, n))
    bounds = [(k * n // n_parts, (k + 1) * n // n_parts) for k in range(n_parts)]
    parts = [(tg.Batch(grids[lo:hi]), lo, hi, torch.cuda.Stream(device=dev)) for lo, hi in bounds]
    mlps = [None] * n_parts
    if args.selector == "mlp":
        from paper_2607_26382_amd import selector as sel
        for k in range(n_parts):   # one network per part: its staging buffers are per handle
            mlps[k], model = sel.load_model(device=dev)
        log("stored first-floor selector loaded ({} training states)".format(model["meta"]["train_states"]))
    mlp = mlps[0]

    def policy(prec, use_mlp, k=0):
        solve = tg.solver_opts(restart=30, max_iters=200, prec=prec, cgs_passes=args.cgs_passes)
        if use_mlp:
            return tg.policy(rungs=RUNGS, p=3.0, solve=solve, selector=tg.SELECT_MLP, mlp=mlps[k])
        return tg.policy(rungs=RUNGS, p=3.0, solve=solve)

    def select_all(pols):
        """The policy over every state: one part per thread and stream."""
        if n_parts == 1:
            return batch.select_floor(rhos, fs, pols[0])
        res, err = [None] * n_parts, []

        def work(k):
            b, lo, hi, st = parts[k]
            try:
                with torch.cuda.stream(st):
                    res[k] = b.select_floor(rhos[lo:hi], fs[lo:hi], pols[k])
                st.synchronize()
            except Exception as e:   # re-raised on the calling thread
                err.append(e)
        th = [threading.Thread(target=work, args=(k,)) for k in range(n_parts)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        if err:
            raise err[0]
        return [u for r in res for u in r[0]], [o for r in res for o in r[1]]

    step_times = []   # wall seconds of every timed step of the last run (select_floor syncs)
    last_us = []      # solutions of the last timed step

    def run(prec, steps, warmup, timer_mask, use_mlp, pol=None):
        # (a given policy carries no network, so the parts may share it)
        pols = [pol] * n_parts if pol is not None else [policy(prec, use_mlp, k) for k in range(n_parts)]
        step_times.clear()
        for w in range(warmup):
            t = time.perf_counter()
            select_all(pols)
            log(f"warmup {w} prec={prec} {time.perf_counter() - t:.2f}s")
        tg.kernel_timer_enable(timer_mask)
        tg.kernel_timer_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = None
        us = None
        for st in range(steps):
            t = time.perf_counter()
            us, outs = select_all(pols)
            step_times.append(time.perf_counter() - t)
            log(f"step {st} prec={prec} {time.perf_counter() - t:.2f}s "
                f"certified={sum(1 for o in outs if o['rung'] >= 0)}")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        timers = tg.kernel_timer_read()
        tg.kernel_timer_enable(0)
        last_us[:] = us if us is not None else []
        return dt, outs, timers

    MIXED = {"f32": tg.F32, "bf16": tg.BF16MFMA, "bf16x3": tg.BF16X3MFMA}
    mixed_prec = MIXED[args.mixed]
    # tile heights of the z-march kernels for this batch, from the autotuner
    batch.set_density(rhos, 3.0, [RUNGS[0]] * n)
    zc_mixed, _ = batch.autotune(mixed_prec)
    log(f"autotuned z-tile heights (levels 0, 1): {zc_mixed[:2]}")
    if n_parts > 1:
        for b, lo, hi, _ in parts:
            b.set_density(rhos[lo:hi], 3.0, [RUNGS[0]] * (hi - lo))
            b.autotune(mixed_prec)
    # one untimed pass with every kernel class timed picks the dominant class;
    # the timed steps then carry events around that class only
    use_mlp = args.selector == "mlp"
    _, _, probe_timers = run(mixed_prec, 1, 0, (1 << 8) - 1, use_mlp)
    dom = tg.dominant_kernel(probe_timers)
    dom_mask = 1 << probe_timers[dom]["kind"]
    dt, outs, timers = run(mixed_prec, args.steps, args.warmup, dom_mask, use_mlp)
    steps_s = list(step_times)
    head_us = list(last_us)
    certified = sum(1 for o in outs if o["rung"] >= 0)
    value = certified * args.steps / dt
    result = {
        "metric": "certified solves/s at ||f-Ku||/||f||<=1e-6 (mixed precision)",
        "mixed_form": args.mixed,
        "selector": args.selector,
        "orthogonalization": {1: "CGS", 2: "CGS2, delayed reorthogonalization", 3: "CGS2 in place"}[args.cgs_passes],
        "value": value, "unit": "certified solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
        "step_ms": {"median": 1e3 * float(np.median(steps_s)),
                    "iqr": [1e3 * float(np.percentile(steps_s, 25)), 1e3 * float(np.percentile(steps_s, 75))],
                    "all": [1e3 * t for t in steps_s]},
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPES[args.mixed],
        "data": "synthetic",
        "config": {"workload": "102 severe random states, 64x32x32 cantilever, guarded floor ladder",
                   "states": n, "grid": list(GRID), "rungs": list(RUNGS), "p": 3.0,
                   "probe": "100 its, restart 100", "solve": "FGMRES(30), cap 200, tol 1e-6",
                   "preconditioner": "5-level GMG V-cycle, node-block Jacobi w=0.6 2/2, FP32 vectors",
                   "streams": n_parts},
    }
    acc = [o for o in outs if o["rung"] >= 0]
    result["policy"] = {
        "certified": certified, "states": n,
        "selected_rungs": {str(r): sum(1 for o in outs if o["rung"] == r) for r in range(-1, len(RUNGS))},
        "first_rung": {str(r): sum(1 for o in outs if o["k0"] == r) for r in range(len(RUNGS))},
        "first_attempt_accepted": sum(1 for o in outs if len(o["attempts"]) == 1 and o["rung"] >= 0),
        "max_accepted_true_eta": max((o["attempts"][-1]["true_eta"] for o in acc), default=None),
        "mean_iters_probe": float(np.mean([o["iters_probe"] for o in outs])),
        "mean_iters_selected": float(np.mean([o["iters_selected"] for o in acc])) if acc else None,
        "mean_iters_rejected": float(np.mean([o["iters_rejected"] for o in outs])),
    }
    result["roofline"] = tg.roofline_from_timers(timers, HBM_PEAK_GBS)
    if result["roofline"] is not None:
        result["roofline"]["traffic"] = measured_traffic(result["roofline"]["kernel"])
    result["autotuned_zc"] = zc_mixed[:2]
    if apply_res is not None:
        result["apply_K"] = apply_res
    result["kernel_classes"] = {k: {"launches": v["count"], "total_ms": v["ms"], "avg_us": v["avg_us"],
                                    "alg_GB/s": v["gbs"]}
                                for k, v in probe_timers.items() if v["count"]}
    if args.compare_mixed:
        result["mixed_variants"] = {}
        for name, pr in MIXED.items():
            d, o, _ = run(pr, 1, 0, 0, use_mlp)
            c = sum(1 for x in o if x["rung"] >= 0)
            result["mixed_variants"][name] = {
                "value": c / d, "ms_per_step": 1e3 * d, "certified": c,
                "mean_iters": float(np.mean([x["iters_probe"] + x["iters_selected"] + x["iters_rejected"]
                                             for x in o]))}
    def brief(o, d, steps):
        c = sum(1 for x in o if x["rung"] >= 0)
        return {"value": c * steps / d, "ms_per_step": 1e3 * d / steps, "certified": c,
                "mean_iters": float(np.mean([x["iters_probe"] + x["iters_selected"] + x["iters_rejected"]
                                             for x in o])),
                "mean_attempts": float(np.mean([len(x["attempts"]) for x in o]))}

    result["policy"]["mean_attempts"] = float(np.mean([len(o["attempts"]) for o in outs]))
    result["policy"]["accepted_above_tolerance"] = sum(
        1 for o in outs for a in o["attempts"] if a["accepted"] and not a["true_eta"] <= 1e-6)
    if not args.no_recheck:
        # the oracle recomputes eta of every accepted solution of the last
        # timed step (matrix-free FP64 operator at the accepted floor), untimed
        f_np = f0.cpu().numpy()
        items, etas = [], []
        for i, o in enumerate(outs):
            if o["rung"] >= 0:
                items.append((GRID, rhos[i].cpu().numpy(), 3.0, RUNGS[o["rung"]], f_np, head_us[i].cpu().numpy()))
                etas.append(o["attempts"][-1]["true_eta"])
        result["oracle_recheck"] = oracle_recheck(items, etas)
        log(f"oracle recheck of {len(items)} accepted solutions: "
            f"{result['oracle_recheck'].get('false_acceptances_oracle')} false acceptances, "
            f"{result['oracle_recheck'].get('boundary_ambiguous')} boundary-ambiguous")
    del head_us
    # reference labels (untimed): independent guarded solves at every rung
    labels = None
    if not args.no_labels:
        ok, sols = [], []
        for r in RUNGS:
            batch.set_density(rhos, 3.0, [r] * n)
            us_r, res = batch.solve(fs, tg.solver_opts(restart=30, max_iters=200, prec=mixed_prec,
                                                       cgs_passes=args.cgs_passes))
            ok.append([x["true_eta"] <= 1e-6 for x in res])
            sols.append(us_r)
        labels = [next((k for k in range(len(RUNGS)) if ok[k][i]), -1) for i in range(n)]
        result["policy"]["stats"] = policy_stats(outs, labels)
        # what a raised floor changes where the original one was admissible
        result["fidelity"] = fidelity_stats(grids, rhos, fs, sols, ok, RUNGS, 3.0)
        del sols
        result["screen"] = screen_stats(tg, torch, grids, rhos, labels, RUNGS, 3.0, mixed_prec)
        result["probe_checkpoints"] = checkpoint_stats(tg, torch, grids, rhos, fs, RUNGS, 3.0, mixed_prec)
    if not args.no_adaptive:
        result["adaptive_preconditioner"] = adaptive_leg(tg, torch, dev, rhos, fs, mixed_prec, n_states=n,
                                                         n_paper=args.paper_states)
    if not args.no_stack and args.stack_states > 0:
        order = _get(result, "adaptive_preconditioner", "paper_setting", "drift_order")
        result["stack_policy"] = stack_policy_leg(tg, torch, dev, rhos, fs, args.stack_states,
                                                  recheck=not args.no_recheck, order=order)
    if use_mlp and not args.no_rule_leg:
        d, o, _ = run(mixed_prec, args.steps, 0, 0, False)
        result["mixed_rule"] = brief(o, d, args.steps)
        result["mixed_rule"]["same_rung"] = sum(1 for a, b in zip(outs, o) if a["rung"] == b["rung"])
        if labels is not None:
            result["mixed_rule"]["stats"] = policy_stats(o, labels)
        result["selector_gain"] = value / result["mixed_rule"]["value"]
        # the rule with thresholds re-tuned on the network's training states
        # (the 288-combination search), so the network's gain is not a
        # recalibration of Eq. trigger
        th = model["meta"].get("tuned_rule")
        if th:
            solve = tg.solver_opts(restart=30, max_iters=200, prec=mixed_prec, cgs_passes=args.cgs_passes)
            pol = tg.policy(rungs=RUNGS, p=3.0, solve=solve, t_high=th[0], t_plateau=th[1], t_ratio=th[2])
            d, o, _ = run(mixed_prec, args.steps, 0, 0, False, pol)
            result["mixed_rule_tuned"] = brief(o, d, args.steps)
            result["mixed_rule_tuned"]["thresholds"] = list(th)
            if labels is not None:
                result["mixed_rule_tuned"]["stats"] = policy_stats(o, labels)
            result["selector_gain_vs_tuned_rule"] = value / result["mixed_rule_tuned"]["value"]
    if not args.no_fixed_legs:
        # the two fixed baselines: the original floor first, then the ladder;
        # always the top rung (the conventional floor 1e-3)
        for name, k in (("always_rho0_then_ladder", 0), ("fixed_top_rung", len(RUNGS) - 1)):
            solve = tg.solver_opts(restart=30, max_iters=200, prec=mixed_prec, cgs_passes=args.cgs_passes)
            pol = tg.policy(rungs=RUNGS, p=3.0, solve=solve, selector=tg.SELECT_FIXED, fixed_rung=k)
            d, o, _ = run(mixed_prec, 1, 0, 0, False, pol)
            result[name] = brief(o, d, 1)
            result[name]["preserved"] = sum(1 for x in o if x["rung"] == 0)
            if labels is not None:
                result[name]["lowest_admissible_selected"] = sum(1 for x, lab in zip(o, labels) if x["rung"] == lab)
    if not args.no_fp64:
        # the paper's method as published: every kernel in FP64, two-feature rule
        dt64, outs64, _ = run(tg.F64, args.steps, args.warmup, 0, False)
        cert64 = sum(1 for o in outs64 if o["rung"] >= 0)
        result["fp64"] = brief(outs64, dt64, args.steps)
        result["fp64"]["selector"] = "rule"
        result["fp64"]["same_rung"] = sum(1 for a, b in zip(outs, outs64) if a["rung"] == b["rung"])
        assert cert64 == result["fp64"]["certified"]
        result["mixed_over_fp64"] = value / result["fp64"]["value"]
    if not args.no_small:
        result["small_plain"] = small_leg(tg, torch, dev)
    if not args.no_scale:
        del batch, grids
        torch.cuda.empty_cache()
        result["mixed_at_scale"] = scale_leg(tg, torch, dev, mixed_prec, recheck=not args.no_recheck)
    if not args.no_batch4:
        batch = grids = None
        torch.cuda.empty_cache()
        result["batch_uneven"] = batch4_leg(tg, torch, dev, mixed_prec, recheck=not args.no_recheck)
    if not args.no_trajectory:
        batch = grids = None
        torch.cuda.empty_cache()
        result["trajectory"] = trajectory_leg(tg, torch, dev, mixed_prec)
    if not args.no_cpu:
        setups = float(np.mean([1 + len(o["attempts"]) for o in outs]))
        iters = float(np.mean([o["iters_probe"] + o["iters_selected"] + o["iters_rejected"] for o in outs]))
        result["cpu_baseline"] = run_cpu_baseline(setups, iters)
        result["cpu_host"] = host_info()
    full = None
    try:
        d = os.path.dirname(args.full_out)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(args.full_out, "w") as fh:
            json.dump(result, fh)
        full = args.full_out
    except OSError as exc:
        log(f"full record not written: {exc}")
    # nothing is printed after this line: it is the run's summary
    print(json.dumps(compact(result, full)), flush=True)


if __name__ == "__main__":
    main()
