"""Benchmark of the LM bundle-adjustment step on one MI355X.

One "step" is one ``ba_lm_step``: extraction, linearisation, Schur complement set-up, PCG,
back-substitution, candidate evaluation and accept/scatter, over the whole synthetic
1000-camera scene (10 random walks, 500k points, ~4M observations, 5 % outliers, depth priors
on 50 %). Inputs are resident in HBM before the timed region. The mixed-precision path is the
headline value; the float64 path runs the same steps from the same start for the ratio.

Each precision runs two timed regions of the same steps from the same start: the first
without instrumentation gives the throughput (``value``); the second attaches HIP start/stop
events to every kernel launch and gives the per-kernel durations and the roofline of the
dominant kernel (the event records slow the step itself by ~15 %, so they stay out of the
throughput region). Both regions execute the same launches (the solver is deterministic;
``same_steps`` checks it).

Prints one JSON line. ``--gpus N`` with N > 1 is not supported (single-GPU build).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# the oracle's CPU baseline uses every host core the process may run on (set before NumPy
# loads its BLAS; an environment that already fixes the counts keeps them)
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, str(len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                                  else (os.cpu_count() or 1)))

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BA LM iters/s + Jacobian obs/s, FP32-mixed vs FP64, 1000-cam synthetic scene"
HBM_PEAK_GBS = 8000.0
LINEARIZE_KERNELS = ("lin_point", "cam_assemble", "gp_lin", "gp_cam_assemble")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scene", default="large")
    ap.add_argument("--precision", default="both", choices=["both", "mixed", "fp64"])
    ap.add_argument("--pcg-tol", type=float, default=1e-6)
    ap.add_argument("--pcg-max", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-frac", type=float, default=0.15,
                    help="fraction of points in the oracle's timed sample")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--cpu-full-steps", type=int, default=1,
                    help="oracle LM steps timed on the whole scene, the baseline value (about "
                         "20 s each for the 1000-camera scene on a 16-thread host); 0: the "
                         "rescaled sample only")
    ap.add_argument("--check-every", type=int, default=8,
                    help="PCG iterations enqueued between convergence read-backs")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration)")
    ap.add_argument("--forward-adjoint", type=int, default=0, metavar="ITERS",
                    help="also time a solve of at most ITERS LM iterations (camera 0 fixed) "
                         "and the implicit adjoint of sum |c - c_gt|^2 (mixed precision)")
    ap.add_argument("--adjoint-lambda-d", type=float, default=300.0,
                    help="depth-row weight of the --forward-adjoint problem (the undamped "
                         "adjoint system needs well-weighted priors)")
    ap.add_argument("--adjoint-damping", type=float, default=1e-6,
                    help="Tikhonov damping of the --forward-adjoint system (singular point "
                         "blocks under the robust-corrected metric)")
    ap.add_argument("--adjoint-precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--adjoint-hessian", default="full", choices=["full", "gauss_newton"],
                    help="Hessian of the --forward-adjoint system (the library's default: full)")
    ap.add_argument("--refine-focal", action="store_true",
                    help="refine each camera's focal length too (7-parameter cameras), "
                         "starting from focal lengths off by up to 2%%")
    ap.add_argument("--gp", action="store_true",
                    help="time depth-constrained global positioning steps instead of BA steps "
                         "(true rotations, perturbed centres and points, free scales where the "
                         "depth prior is invalid)")
    ap.add_argument("--gp-huber", type=float, default=0.1)
    ap.add_argument("--solver", default="implicit", choices=["implicit", "explicit"],
                    help="matrix-free Schur PCG, or PCG on the assembled reduced camera system")
    ap.add_argument("--verbose", action="store_true")
    return ap.parse_args()


GP_METRIC = ("GP LM iters/s (depth-constrained global positioning), FP32-mixed vs FP64, "
             "1000-cam synthetic scene")


def gp_start(sc):
    """Global positioning takes the rotations as given: the true ones, with the scene's
    perturbed centres and points."""
    from dataclasses import replace
    cams0 = np.concatenate([sc.cams_gt[:, :4], sc.cams0[:, 4:7]], axis=1)
    return replace(sc, cams0=cams0)


def focal_start(sc):
    """The scene with every camera's focal length scaled by a seeded factor in [0.98, 1.02]."""
    from dataclasses import replace
    rng = np.random.default_rng(77)
    intr = sc.intr.copy()
    intr[:, 0] *= 1.0 + rng.uniform(-0.02, 0.02, size=sc.n_cams)
    return replace(sc, intr=intr)


def run_gpu(sc, precision, steps, warmup, args, torch, timing):
    from paper_2510_13310_amd import BundleAdjuster
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    ba = BundleAdjuster(t(sc.cams0, torch.float64), t(sc.intr, torch.float64),
                        t(sc.points0, torch.float64), precision=precision,
                        huber_px=sc.huber_px, filter_px=sc.filter_px, img_w=sc.img_w,
                        img_h=sc.img_h, pcg_rel_tol=args.pcg_tol, pcg_max_iters=args.pcg_max,
                        pcg_check_every=args.check_every, timing=timing,
                        refine_focal=int(args.refine_focal), gp_huber=args.gp_huber,
                        solver=args.solver)
    ba.set_observations(t(sc.cam_idx, torch.int32), t(sc.pt_idx, torch.int32),
                        t(sc.xy, torch.float32))
    if sc.use_depth:
        ba.set_depth_priors(t(sc.depth, torch.float32), t(sc.depth_valid, torch.uint8),
                            sc.lambda_d)
    step = ba.gp_step if args.gp else ba.lm_step
    min_free = torch.cuda.mem_get_info()[0]
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ba.reset_kernel_stats()
    reps = []
    t0 = time.perf_counter()
    for _ in range(steps):
        reps.append(step())
        if timing:   # device memory in use (hipMemGetInfo), sampled after every step
            min_free = min(min_free, torch.cuda.mem_get_info()[0])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = ba.kernel_stats()
    mem = ba.device_bytes()
    total = torch.cuda.mem_get_info()[1]
    ba.close()
    return dict(seconds=dt, reports=reps, stats=stats, device_bytes=mem,
                device_used_peak=total - min_free)


def forward_adjoint(sc, iters, args, torch):
    """Wall time of a solve (camera 0 fixed, bench PCG settings) and of the implicit adjoint
    of L = sum_i |c_i - c_i^gt|^2 with respect to all observations."""
    from paper_2510_13310_amd import BundleAdjuster, BAError
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    torch.cuda.reset_peak_memory_stats()
    ba = BundleAdjuster(t(sc.cams0, torch.float64), t(sc.intr, torch.float64),
                        t(sc.points0, torch.float64), precision=args.adjoint_precision,
                        huber_px=sc.huber_px, filter_px=sc.filter_px, img_w=sc.img_w,
                        img_h=sc.img_h, pcg_rel_tol=args.pcg_tol, pcg_max_iters=args.pcg_max,
                        max_lm_iters=iters, adjoint_damping=args.adjoint_damping,
                        adjoint_hessian=args.adjoint_hessian, timing=1)
    ba.set_observations(t(sc.cam_idx, torch.int32), t(sc.pt_idx, torch.int32),
                        t(sc.xy, torch.float32))
    ba.set_depth_priors(t(sc.depth, torch.float32), t(sc.depth_valid, torch.uint8),
                        args.adjoint_lambda_d)
    ba.set_fixed_cameras(np.array([0], np.int32))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    srep = ba.solve()
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    cams, pts = ba.get_params()
    g_c = np.zeros_like(cams)
    g_c[:, 4:7] = 2.0 * (cams[:, 4:7] - sc.cams_gt[:, 4:7])
    gxy = torch.empty((sc.n_obs, 2), dtype=torch.float32, device=dev)
    gd = torch.empty(sc.n_obs, dtype=torch.float32, device=dev)
    ba.reset_kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status = "ok"
    try:
        ba.adjoint(t(g_c, torch.float64), t(np.zeros_like(pts), torch.float64), gxy, gd)
    except BAError as e:
        status = str(e)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    st = {k["name"]: k for k in ba.kernel_stats()}
    out = dict(precision=args.adjoint_precision, lambda_d=args.adjoint_lambda_d,
               adjoint_damping=args.adjoint_damping, adjoint_hessian=args.adjoint_hessian,
               fixed_cameras=[0],
               lm_iterations=srep["iterations"], stop_reason=srep["stop_reason"],
               initial_rms_px=round(srep["initial_rms_px"], 6),
               final_rms_px=round(srep["final_rms_px"], 6), solve_s=round(t_solve, 4),
               adjoint_s=round(t_adj, 4), adjoint_status=status,
               adjoint_pcg_iters=int(st["schur_point"]["launches"]) if "schur_point" in st else 0,
               forward_plus_adjoint_s=round(t_solve + t_adj, 4),
               library_device_gb=round(ba.device_bytes() / 1e9, 3),
               torch_peak_gb=round(torch.cuda.max_memory_allocated() / 1e9, 3))
    ba.close()
    return out


def _mean_ms(reps, keep):
    v = [r["ms_total"] for r in reps if keep(r)]
    return round(float(np.mean(v)), 4) if v else None


def summarize(res, n_obs_total):
    """Throughput of one timed region (every step counted, accepted or rejected), with the
    host wall time of the steps split by outcome: a step re-extracts and re-linearises only
    after an accepted one, so accepted and rejected steps cost different amounts."""
    reps = res["reports"]
    K = len(reps)
    its = K / res["seconds"]
    nh = float(np.mean([r["n_obs_active"] for r in reps]))
    return dict(
        lm_iters_per_s=its, ms_per_step=1e3 * res["seconds"] / K, obs_per_s=its * nh,
        n_obs_active=nh, n_obs_total=n_obs_total,
        pcg_iters_mean=float(np.mean([r["pcg_iters"] for r in reps])),
        accepted=int(sum(r["accepted"] for r in reps)),
        relinearized=int(sum(r["relinearized"] for r in reps)),
        ms_step_accepted=_mean_ms(reps, lambda r: r["accepted"]),
        ms_step_rejected=_mean_ms(reps, lambda r: not r["accepted"]),
        ms_step_relinearized=_mean_ms(reps, lambda r: r["relinearized"]),
        ms_step_reused=_mean_ms(reps, lambda r: not r["relinearized"]),
        rms_px_first=reps[0]["rms_px"], rms_px_last=reps[-1]["rms_px"],
        cost_last=reps[-1]["cost_before"], device_gb=res["device_bytes"] / 1e9)


def kernel_summary(res):
    """Per-kernel launches, time and algorithmic GB/s of an instrumented region."""
    reps = res["reports"]
    K = len(reps)
    nh = float(np.mean([r["n_obs_active"] for r in reps]))
    st = {s["name"]: s for s in res["stats"]}
    lin_ms = sum(st[k]["total_ms"] for k in LINEARIZE_KERNELS if k in st)
    lin_launch = max((st[k]["launches"] for k in LINEARIZE_KERNELS if k in st), default=0)
    jac = (nh * lin_launch) / (lin_ms / 1e3) if lin_ms > 0 else None
    kern_ms = sum(s["total_ms"] for s in res["stats"])
    # one PCG iteration = the two matvec passes (or the explicit product) and the update
    pcg_names = ("schur_point", "schur_cam", "schur_spmv", "pcg_update", "gp_schur_point",
                 "gp_schur_cam")
    pcg_ms = sum(st[k]["total_ms"] for k in pcg_names if k in st)
    pcg_n = st["pcg_update"]["launches"] if "pcg_update" in st else 0
    true_res = [r["pcg_true_residual"] for r in reps if r["pcg_true_residual"] >= 0]
    return dict(
        ms_per_step_instrumented=1e3 * res["seconds"] / K, kernel_ms_per_step=kern_ms / K,
        jacobian_obs_per_s=jac,
        us_per_pcg_iter=round(1e3 * pcg_ms / pcg_n, 3) if pcg_n else None,
        pcg_true_residual_mean=float(np.mean(true_res)) if true_res else None,
        pcg_true_residual_max=float(np.max(true_res)) if true_res else None,
        pcg_recursive_residual_mean=float(np.mean([r["pcg_rel_residual"] for r in reps])),
        kernels={s["name"]: dict(launches=s["launches"], ms=round(s["total_ms"], 4),
                                 avg_us=round(1e3 * s["total_ms"] / s["launches"], 2),
                                 gbs=(round(s["total_bytes"] / (s["total_ms"] * 1e6), 1)
                                      if s["total_ms"] > 0 else None))
                 for s in res["stats"] if s["launches"] > 0},
    )


def traffic_file(kernel, scene):
    """The committed counter summary of `kernel` on `scene` (mixed precision)."""
    return os.path.join(ROOT, "profiles", f"{kernel}_{scene}_mixed_traffic.txt")


def measured_traffic(kernel, scene):
    """HBM bytes per launch of `kernel` from its committed counter summary, or None when there
    is none for this kernel and workload, or the library sources changed since."""
    import hashlib
    path = traffic_file(kernel, scene)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, _, v = line.strip().partition(" ")
            kv[k] = v.strip()
    if kv.get("kernel") != kernel or kv.get("workload") != scene:
        return None
    h = hashlib.sha256()
    for f in kv.get("sources", "").split():
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != kv.get("sources_sha256"):
        return None
    return float(kv["traffic_bytes_per_launch"])


def roofline(res, scene):
    """Dominant kernel by total time: algorithmic bytes per launch / mean launch time."""
    stats = [s for s in res["stats"] if s["launches"] > 0]
    dom = max(stats, key=lambda s: s["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    bytes_per_launch = dom["total_bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom["name"], scene)
    out = dict(kernel=dom["name"], bound="hbm", achieved=round(achieved, 1),
               peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
               traffic=traffic, avg_launch_us=round(avg_ms * 1e3, 2),
               bytes_per_launch=int(bytes_per_launch), launches=dom["launches"])
    if traffic is not None:
        out["traffic_gbs"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
    return out


def cpu_baseline_gp(sc, frac, steps, n_obs_full, huber_gp):
    """The FP64 GP oracle on a random fraction of the points (all cameras), per LM step, the
    rate rescaled to the full observation count."""
    from dataclasses import replace
    from oracle.gp import GpOptions, GpState, gp_step
    from oracle.model import Problem
    rng = np.random.default_rng(1234)
    keep = np.sort(rng.choice(sc.n_points, max(1, int(frac * sc.n_points)), replace=False))
    m = np.zeros(sc.n_points, bool)
    m[keep] = True
    ob = m[sc.pt_idx]
    pmap = np.full(sc.n_points, -1)
    pmap[keep] = np.arange(keep.size)
    sub = replace(sc, points_gt=sc.points_gt[keep], points0=sc.points0[keep],
                  cam_idx=sc.cam_idx[ob], pt_idx=pmap[sc.pt_idx[ob]].astype(np.int32),
                  xy=sc.xy[ob], depth=sc.depth[ob], depth_valid=sc.depth_valid[ob],
                  is_outlier=sc.is_outlier[ob])
    opts = GpOptions(huber=huber_gp)
    prob = Problem.from_scene(sub)
    q = sub.cams0[:, :4]
    st = GpState.initial(prob, q, sub.cams0, sub.points0, opts)
    t0 = time.perf_counter()
    nobs = []
    for _ in range(steps):
        st, rep = gp_step(prob, q, st, opts)
        nobs.append(rep.n_obs)
    dt = time.perf_counter() - t0
    its_sample = steps / dt
    cores, model = cpu_info()
    return dict(value=round(its_sample * sub.cam_idx.size / n_obs_full, 5), unit="GP LM iters/s",
                cores=cores, kind="oracle", cpu_model=model,
                sample=(f"{steps} FP64 GP oracle LM steps on {100 * frac:.0f}% of the points "
                        f"({sub.cam_idx.size} of {n_obs_full} observations, all cameras), "
                        f"{dt:.1f} s; rate rescaled by the observation ratio"),
                sample_iters_per_s=round(its_sample, 4),
                obs_per_s=round(its_sample * float(np.mean(nobs)), 1))


def cpu_info():
    """Threads the oracle's BLAS and NumPy may use, and the host CPU model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), model


def cpu_full(sc, steps, refine_focal=False):
    """The FP64 oracle timed on the whole scene for `steps` LM steps (the first from the
    scene's start, like the GPU's first timed step after its own warm-up)."""
    from oracle.lm import Options, State, lm_step
    from oracle.model import Problem
    opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px, refine_focal=refine_focal)
    prob = Problem.from_scene(sc)
    st = State.initial(sc.cams0, sc.points0, opts, focal=sc.intr[:, 0])
    t0 = time.perf_counter()
    nobs = []
    for _ in range(steps):
        st, rep = lm_step(prob, st, opts)
        nobs.append(rep.n_obs)
    dt = time.perf_counter() - t0
    return steps / dt, dt, float(np.mean(nobs))


def cpu_baseline(sc, frac, steps, n_obs_full, refine_focal=False, full_steps=1):
    """The FP64 oracle, untouched: `full_steps` LM steps on the whole scene give the value;
    the rate of `steps` steps on a random fraction of the points (all cameras), rescaled by the
    observation ratio, is reported beside it with its error against the full-scene rate (the
    dense camera Schur complement and its Cholesky do not shrink with the sample)."""
    from dataclasses import replace
    from oracle.lm import Options, State, lm_step
    from oracle.model import Problem
    rng = np.random.default_rng(1234)
    keep = np.sort(rng.choice(sc.n_points, max(1, int(frac * sc.n_points)), replace=False))
    m = np.zeros(sc.n_points, bool)
    m[keep] = True
    ob = m[sc.pt_idx]
    pmap = np.full(sc.n_points, -1)
    pmap[keep] = np.arange(keep.size)
    sub = replace(sc, points_gt=sc.points_gt[keep], points0=sc.points0[keep],
                  cam_idx=sc.cam_idx[ob], pt_idx=pmap[sc.pt_idx[ob]].astype(np.int32),
                  xy=sc.xy[ob], depth=sc.depth[ob], depth_valid=sc.depth_valid[ob],
                  is_outlier=sc.is_outlier[ob])
    opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px, refine_focal=refine_focal)
    prob = Problem.from_scene(sub)
    st = State.initial(sub.cams0, sub.points0, opts, focal=sub.intr[:, 0])
    t0 = time.perf_counter()
    nobs = []
    for _ in range(steps):
        st, rep = lm_step(prob, st, opts)
        nobs.append(rep.n_obs)
    dt = time.perf_counter() - t0
    its_sample = steps / dt
    cores, model = cpu_info()
    scaled = its_sample * sub.n_obs / n_obs_full
    out = dict(value=round(scaled, 5), unit="LM iters/s", cores=cores, kind="oracle",
               cpu_model=model,
               sample=(f"{steps} FP64 oracle LM steps on {100 * frac:.0f}% of the points "
                       f"({sub.n_obs} of {n_obs_full} observations, all cameras), "
                       f"{dt:.1f} s; rate rescaled by the observation ratio"),
               sample_iters_per_s=round(its_sample, 4),
               obs_per_s=round(its_sample * float(np.mean(nobs)), 1))
    if full_steps > 0:
        its_full, dt_full, nobs_full = cpu_full(sc, full_steps, refine_focal)
        out.update(value=round(its_full, 5),
                   sample=(f"{full_steps} FP64 oracle LM step(s) on the whole scene "
                           f"({n_obs_full} observations), {dt_full:.1f} s"),
                   obs_per_s=round(its_full * nobs_full, 1),
                   sampled_value=round(scaled, 5),
                   sampled_desc=(f"{steps} steps on {100 * frac:.0f}% of the points, "
                                 f"{dt:.1f} s, rescaled by the observation ratio"),
                   sampling_error=round(scaled / its_full - 1.0, 4))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU point sharding is design-only).", file=sys.stderr)
        sys.exit(2)
    if args.gp and (args.refine_focal or args.forward_adjoint):
        print("bench.py: --gp times global positioning alone", file=sys.stderr)
        sys.exit(2)
    if args.refine_focal and args.forward_adjoint:
        print("bench.py: the adjoint covers poses and points; --forward-adjoint needs focal "
              "refinement off", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2510_13310_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2510_13310_amd.build import build
        build()
    from scenes import make_scene

    if args.calib_copy:
        n = 1 << 28   # 2^28 float32 = 1 GiB read + 1 GiB written
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    t0 = time.perf_counter()
    sc = make_scene(args.scene)
    if args.refine_focal:
        sc = focal_start(sc)
    if args.gp:
        sc = gp_start(sc)
    workload_key = (args.scene + ("+focal" if args.refine_focal else "") +
                    ("+gp" if args.gp else "") + ("+explicit" if args.solver == "explicit" else ""))
    t_gen = time.perf_counter() - t0
    if args.verbose:
        print(f"scene {args.scene}: C={sc.n_cams} P={sc.n_points} N={sc.n_obs} "
              f"({t_gen:.1f} s)", flush=True)

    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    out = {}
    for p in precs:
        # region 1: the throughput, no instrumentation; region 2: the same steps from the
        # same start with HIP events attached to every launch (kernel durations, roofline)
        res = run_gpu(sc, p, args.steps, args.warmup, args, torch, timing=0)
        ins = run_gpu(sc, p, args.steps, args.warmup, args, torch, timing=1)
        summ = summarize(res, sc.n_obs)
        summ.update(kernel_summary(ins))
        summ["device_used_peak_gb"] = ins["device_used_peak"] / 1e9   # whole process
        summ["same_steps"] = ([r["cost_before"] for r in res["reports"]] ==
                              [r["cost_before"] for r in ins["reports"]])
        out[p] = (ins, summ)
        if args.verbose:
            print(p, json.dumps({k: v for k, v in summ.items() if k != "kernels"}), flush=True)

    head = precs[0]
    ins, summ = out[head]
    line = {
        "metric": GP_METRIC if args.gp else METRIC,
        "value": round(summ["lm_iters_per_s"], 3),
        "unit": "GP LM iters/s" if args.gp else "LM iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(summ["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 mixed" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": (f"{args.scene}: {sc.n_cams} cameras in random walks, "
                                f"{sc.n_points} points, {sc.n_obs} observations, "
                                f"{100 * sc.is_outlier.mean():.0f}% outliers, depth priors on "
                                f"{100 * sc.depth_valid.mean():.0f}%, Huber "
                                f"{sc.huber_px:g} px, {sc.filter_px:g} px filter"
                                + (", focal lengths refined (7-parameter cameras, start "
                                   "off by up to 2%)" if args.refine_focal else "")
                                + (f"; global positioning: true rotations, camera centres, "
                                   f"points and {100 * (1 - sc.depth_valid.mean()):.0f}% free "
                                   f"scales, Huber {args.gp_huber:g} on the ray residual"
                                   if args.gp else "")
                                + ("; explicit reduced camera system (assembled 6x6 blocks)"
                                   if args.solver == "explicit" else "")),
                   "pcg_rel_tol": args.pcg_tol, "pcg_max_iters": args.pcg_max,
                   "pcg_check_every": args.check_every, "solver": args.solver},
        "obs_per_s": round(summ["obs_per_s"], 1),
        "jacobian_obs_per_s": (round(summ["jacobian_obs_per_s"], 1)
                               if summ["jacobian_obs_per_s"] else None),
        "roofline": roofline(ins, workload_key),
    }
    for p in precs:
        s = out[p][1]
        line[p] = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in s.items()
                   if k != "kernels"}
        line[p]["kernels"] = s["kernels"]
    if "fp64" in out and "mixed" in out:
        line["mixed_over_fp64"] = round(out["mixed"][1]["lm_iters_per_s"] /
                                        out["fp64"][1]["lm_iters_per_s"], 3)
        # the same ratio per PCG iteration (PCG kernels only): the speed of the precision
        # itself, apart from the two paths stopping their PCG after different counts
        um, uf = out["mixed"][1]["us_per_pcg_iter"], out["fp64"][1]["us_per_pcg_iter"]
        line["mixed_over_fp64_per_pcg_iter"] = round(uf / um, 3) if um and uf else None
        line["rms_diff_px"] = abs(out["mixed"][1]["rms_px_last"] - out["fp64"][1]["rms_px_last"])
    if args.forward_adjoint > 0:
        line["forward_adjoint"] = forward_adjoint(sc, args.forward_adjoint, args, torch)
    if args.no_cpu:
        line["cpu_baseline"] = None
    elif args.gp:
        line["cpu_baseline"] = cpu_baseline_gp(sc, args.cpu_frac, args.cpu_steps, sc.n_obs,
                                               args.gp_huber)
    else:
        line["cpu_baseline"] = cpu_baseline(sc, args.cpu_frac, args.cpu_steps, sc.n_obs,
                                            args.refine_focal, args.cpu_full_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
