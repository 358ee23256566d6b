#!/usr/bin/env python3
"""Benchmark of the seeded trajectory optimiser on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
upload-free optimisation of every seed of the batch for N_iters L-BFGS
iterations (FK, spheres, ESDF gathers, costs, adjoint, line search, flags,
best seed) plus reading back the best trajectory.  Inputs are resident in
HBM before the timed region.

Default workload (the single-GPU headline configuration): one cluttered
shelf problem, 32 seeds x 32 waypoints, 56 spheres, 200^3 FP32 ESDF at 1 cm,
100 iterations.  Extra fields report the batched-uneven workload (64
problems, one persistent launch vs one launch per problem) and serving.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2410_16727_amd/csrc/dsopt_kernels.hip",
                  "paper_2410_16727_amd/csrc/dsopt_internal.h"]
PMC_SUMMARY = "profiles/k_optimize_pmc_cluttered.json"
COPY_BYTES = 256 << 20


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per optimiser launch from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factors),
    or None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, PMC_SUMMARY)
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None, rec
    return rec.get("traffic_bytes_per_launch"), rec


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def evals_per_seed(res):
    # init + alpha=1 + extra gradient evaluations, cost-only candidates, and
    # the final results pass
    return res["n_evals_grad"] + res["n_evals_cost"] + 1


def run_single(args, dsopt, torch, configs, params):
    key = args.workload
    w = configs.WORKLOADS[key]
    robot = configs.robot(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    S, T, N = prob.S, prob.T, w.iters
    log(f"[bench] workload {key} ({w.name}): S={S} T={T} spheres={robot.n_spheres} "
        f"grid={scene.dims} iters={N}")
    prm = dict(params.DEFAULT, waves_per_seed=args.waves)
    plan = dsopt.Plan(robot, prm, N, 1 << 30)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    seeds = torch.from_numpy(configs.seeds_for(key, 0, prob)).cuda()
    out = torch.zeros_like(seeds)
    spec = {"scene": 0, "q_start": prob.q_start, "goal": prob.goal, "seeds": seeds, "out": out}
    tag = [0]

    def step():
        tag[0] += 1
        plan.optimize([dict(spec, tag=tag[0])])
        traj, res = plan.get_best(tag[0], T)
        plan.release(tag[0])
        return res

    # evaluation counts (deterministic, identical in every step)
    tag[0] += 1
    plan.optimize([dict(spec, tag=tag[0])])
    sres = plan.seed_results(tag[0], S)
    _, best = plan.get_best(tag[0], T)
    plan.release(tag[0])
    n_evals = evals_per_seed(sres)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.kernel_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.kernel_timing(False)
    k_ms, k_n = plan.kernel_timing_read()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # algorithmic bytes: 32 B of cell corners per sphere sample of every
    # evaluation; the bytes the kernel actually gathered (its own per-seed
    # counters x 32 B) are fewer, the coarse-table skip proves the rest zero
    sample_bytes = float(np.sum(n_evals)) * T * robot.n_spheres * 32.0
    gather_bytes = float(np.sum(sres["n_gathers"])) * 32.0
    avg_kernel_s = k_ms / max(k_n, 1) / 1e3
    achieved = sample_bytes / avg_kernel_s / 1e9
    log(f"[bench] {ms_step:.3f} ms/step, kernel {k_ms / max(k_n, 1):.3f} ms/launch, "
        f"evals/seed {np.mean(n_evals):.1f}, gathered {gather_bytes / sample_bytes:.3f} of "
        f"the samples, {achieved:.1f} GB/s, best {best}")
    plan.close()
    return {
        "S": S, "T": T, "N": N, "spheres": robot.n_spheres, "grid": list(scene.dims),
        "ms_per_step": ms_step, "kernel_ms": k_ms / max(k_n, 1),
        "gather_bytes": gather_bytes, "sample_bytes": sample_bytes, "achieved_gbs": achieved,
        "evals_per_seed": float(np.mean(n_evals)), "best": best,
        "scene": scene, "robot": robot, "prob": prob,
    }


def run_batched(args, dsopt, torch, configs, params):
    """64 uneven problems: one persistent launch vs one launch per problem."""
    key = "D"
    w = configs.WORKLOADS[key]
    robot = configs.robot(key)
    t0 = time.perf_counter()
    scenes = configs.scenes(key, threads=host_threads())
    log(f"[bench] batched: built {len(scenes)} grids in {time.perf_counter() - t0:.1f} s")
    probs = configs.problems(key)
    N = w.iters
    cells = sum((s.dims[0] - 1) * (s.dims[1] - 1) * (s.dims[2] - 1) for s in scenes)
    per = lambda T: 64 // (16 if T <= 16 else 32 if T <= 32 else 64)
    state = sum(((p.S + per(p.T) - 1) // per(p.T)) * 40 * 1024 + p.S * p.T * 28 + p.S * 64
                for p in probs)
    arena = cells * 32 + 2 * state + (512 << 20)
    plan = dsopt.Plan(robot, dict(params.DEFAULT, waves_per_seed=args.batched_waves), N, arena)
    for i, sc in enumerate(scenes):
        plan.upload_scene(i, sc.grid, sc.voxel, sc.origin)
        sc.grid = None
    seeds = [torch.from_numpy(configs.seeds_for(key, i, p)).cuda() for i, p in enumerate(probs)]
    specs = [{"scene": p.scene, "q_start": p.q_start, "goal": p.goal, "seeds": seeds[i]}
             for i, p in enumerate(probs)]
    sw = sum(p.S * p.T for p in probs)
    tagc = [1000]

    def batched():
        base = tagc[0]
        tagc[0] += len(specs)
        plan.optimize([dict(s, tag=base + i) for i, s in enumerate(specs)])
        for i in range(len(specs)):
            plan.get_best(base + i, probs[i].T)
        for i in range(len(specs)):
            plan.release(base + i)

    def plain():
        base = tagc[0]
        tagc[0] += len(specs)
        for i, s in enumerate(specs):
            plan.optimize([dict(s, tag=base + i)])
        for i in range(len(specs)):
            plan.get_best(base + i, probs[i].T)
        for i in range(len(specs)):
            plan.release(base + i)

    # evaluation counts of every seed (deterministic): algorithmic gather bytes
    base = tagc[0]
    tagc[0] += len(specs)
    plan.optimize([dict(s, tag=base + i) for i, s in enumerate(specs)])
    gbytes = sbytes = 0.0
    for i, p in enumerate(probs):
        r = plan.seed_results(base + i, p.S)
        gbytes += float(np.sum(r["n_gathers"])) * 32.0
        sbytes += float(np.sum(evals_per_seed(r))) * p.T * robot.n_spheres * 32.0
        plan.release(base + i)
    out = {}
    for name, fn in [("batched", batched), ("plain", plain)]:
        fn()
        torch.cuda.synchronize()
        plan.kernel_timing(True)
        t0 = time.perf_counter()
        reps = max(1, args.batched_steps)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        plan.kernel_timing(False)
        k_ms, k_n = plan.kernel_timing_read()
        out[name] = {"ms_per_batch": dt * 1e3,
                     "seed_waypoint_evals_per_s": sw * N / dt,
                     "problems_per_s": len(probs) / dt,
                     "kernel_ms_per_launch": k_ms / max(k_n, 1),
                     "launches_per_batch": k_n / reps}
        log(f"[bench] batched-uneven {name}: {dt * 1e3:.2f} ms/batch, "
            f"{sw * N / dt:.3e} seed-waypoint evals/s")
    plan.close()
    kb = out["batched"]["kernel_ms_per_launch"] / 1e3
    out["roofline"] = {"bound": "hbm", "kernel": "k_optimize (one persistent launch)",
                       "achieved": sbytes / kb / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": sbytes / kb / 1e9 / HBM_PEAK_GBS,
                       "algorithmic_bytes_per_launch": sbytes,
                       "gathered_bytes_per_launch": gbytes, "gathered_frac": gbytes / sbytes}
    out["speedup_batched_vs_plain"] = out["plain"]["ms_per_batch"] / out["batched"]["ms_per_batch"]
    out["workload"] = (f"batched-uneven: {len(probs)} problems, seeds U{{4..128}}, horizons "
                       f"U{{16..64}}, {sw} seed-waypoints, 128^3 ESDF per problem, {N} iters")
    return out


def run_serving(args, dsopt, torch, configs, params):
    """Poisson arrivals of mixed requests over 16 resident scenes: the
    served (continuous batching, graph-captured blocks) form vs the plain
    serial form (FIFO, one request at a time, one launch each), at the
    workload's rate and at a rate above the plain form's capacity."""
    key = "E"
    w = configs.WORKLOADS[key]
    robot = configs.robot(key)
    t0 = time.perf_counter()
    scenes = configs.scenes(key, threads=host_threads())
    log(f"[bench] serving: built {len(scenes)} grids in {time.perf_counter() - t0:.1f} s")
    pool = configs.problems(key)
    N = w.iters
    cells = sum((s.dims[0] - 1) * (s.dims[1] - 1) * (s.dims[2] - 1) for s in scenes)

    def make_plan(waves, block, drain=0):
        pl = dsopt.Plan(robot, dict(params.DEFAULT, waves_per_seed=waves, serve_drain=drain), N,
                        cells * 32 + (3 << 30), block_iters=block)
        for i, sc in enumerate(scenes):
            pl.upload_scene(i, sc.grid, sc.voxel, sc.origin)
        return pl

    def make_reqs(n, rate):
        reqs = []
        for r, (arr, pi, S, T) in enumerate(configs.serving_trace(n, rate)):
            p = pool[pi]
            sd = torch.from_numpy(configs.seeds_for(key, pi, p, S=S, T=T, stream=r)).cuda()
            reqs.append({"arrival": arr, "S": S, "T": T,
                         "spec": {"scene": p.scene, "q_start": p.q_start, "goal": p.goal,
                                  "seeds": sd}})
        torch.cuda.synchronize()
        return reqs

    def summarize(reqs, lat, done_t, name, warm):
        lat = np.array(lat[warm:])
        span = max(done_t[warm:]) - reqs[warm]["arrival"]
        out = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
               "problems_per_s": float(len(lat) / span), "measured_requests": int(len(lat))}
        log(f"[bench] serving {name}: p50 {out['p50_ms']:.2f} ms p99 {out['p99_ms']:.2f} ms "
            f"{out['problems_per_s']:.1f} problems/s")
        return out

    def served(plan, reqs, warm, name):
        plan.serve_start(max_slots=args.serve_slots, queue_cap=len(reqs) + 1)
        lat = [0.0] * len(reqs)
        done_t = [0.0] * len(reqs)
        pending = {}
        i = 0
        n_done = 0
        start = time.perf_counter()
        while n_done < len(reqs):
            now = time.perf_counter() - start
            while i < len(reqs) and reqs[i]["arrival"] <= now:
                pending[plan.serve_submit(reqs[i]["spec"])] = i
                i += 1
            active = plan.serve_step()
            for t, r in list(pending.items()):
                res = plan.serve_poll(t)
                if res is not None:
                    tt = time.perf_counter() - start
                    lat[r] = (tt - reqs[r]["arrival"]) * 1e3
                    done_t[r] = tt
                    del pending[t]
                    n_done += 1
            if active == 0 and not pending and i < len(reqs):
                time.sleep(max(0.0, reqs[i]["arrival"] - (time.perf_counter() - start)))
        stats = plan.serve_stats()
        plan.serve_stop()
        out = summarize(reqs, lat, done_t, name, warm)
        out["mean_active_slots"] = stats["mean_active_slots"]
        out["graph_replays"] = stats["steps"]
        return out

    def plain(plan, reqs, warm, name):
        lat = [0.0] * len(reqs)
        done_t = [0.0] * len(reqs)
        start = time.perf_counter()
        for r, rq in enumerate(reqs):
            now = time.perf_counter() - start
            if rq["arrival"] > now:
                time.sleep(rq["arrival"] - now)
            plan.optimize([dict(rq["spec"], tag=r + 1)])
            plan.get_best(r + 1, rq["T"])
            plan.release(r + 1)
            tt = time.perf_counter() - start
            lat[r] = (tt - rq["arrival"]) * 1e3
            done_t[r] = tt
        return summarize(reqs, lat, done_t, name, warm)

    sp = make_plan(args.serve_waves, args.serve_block, int(args.serve_drain))
    # plain serial form: on a plan with its own best (latency) team size
    pp = make_plan(args.serve_plain_waves, 10)
    out = {}
    for tag, n, rate in (("rate", args.serve_requests, args.serve_rate),
                         ("saturated", args.serve_sat_requests, args.serve_sat_rate)):
        if n <= 0:
            continue
        reqs = make_reqs(n, rate)
        warm = min(200, n // 10)
        out[tag] = {
            "workload": (f"serving: Poisson {n} requests at {rate:g}/s ({warm} warm-up), "
                         f"seeds U{{8..128}}, horizons U{{32..64}}, 16 resident 200^3 ESDFs, "
                         f"{N} iters, blocks of {args.serve_block} iterations per graph replay, "
                         f"{args.serve_slots} slots{', run to completion when idle' if args.serve_drain else ''}; "
                         f"served form {args.serve_waves} and plain "
                         f"serial form {args.serve_plain_waves} wavefronts per seed"),
            "served": served(sp, reqs, warm, f"served @{rate:g}/s"),
            "plain_serial": plain(pp, reqs, warm, f"plain serial @{rate:g}/s")}
        del reqs
    sp.close()
    pp.close()
    return out


def run_differentiation(args, dsopt, torch, configs, params):
    """Cost + gradient of 256 seeds x 64 waypoints (60 spheres, 200^3) in
    one call, and the same through the autograd function (forward: cost and
    adjoint gradient in one launch, kinematics recomputed; backward: the
    saved gradient scaled by dJ), timed with events on the stream both run
    on."""
    from paper_2410_16727_amd.autograd import trajectory_cost
    key = "C"
    robot = configs.robot(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    cells = (scene.dims[0] - 1) * (scene.dims[1] - 1) * (scene.dims[2] - 1)
    plan = dsopt.Plan(robot, params.DEFAULT, 1, cells * 32 + (1 << 30))
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    X = torch.from_numpy(configs.seeds_for(key, 0, prob)).cuda()
    S, T = X.shape[0], X.shape[1]
    reps = 50

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_cg = timed(lambda: plan.cost_grad(0, prob.q_start, prob.goal, X))

    def fwd_bwd():
        Xr = X.clone().requires_grad_(True)
        trajectory_cost(Xr, plan, 0, prob.q_start, prob.goal).sum().backward()

    ms_ag = timed(fwd_bwd)
    plan.close()
    sample_bytes = float(S * T * robot.n_spheres * 32)
    achieved = sample_bytes / (ms_cg * 1e-3) / 1e9
    log(f"[bench] differentiation: cost+grad {ms_cg:.3f} ms ({S * T / (ms_cg * 1e-3):.3e} "
        f"seed-waypoint evals/s), autograd forward+backward {ms_ag:.3f} ms")
    return {"workload": f"differentiation: {S} seeds x {T} waypoints, {robot.n_spheres} spheres, "
                        f"{scene.dims[0]}^3 ESDF, one cost+gradient call",
            "cost_grad_ms": ms_cg, "seed_waypoint_evals_per_s": S * T / (ms_cg * 1e-3),
            "autograd_fwd_bwd_ms": ms_ag,
            "roofline": {"bound": "hbm", "kernel": "k_cost (cost+gradient)", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_launch": sample_bytes}}


def run_esdf_build(args, dsopt, torch, configs, params, scene):
    """Distance field of the cluttered scene built on the GPU from its
    occupancy grid (exact signed EDT), timed with events."""
    from workloads import gen
    occ = torch.from_numpy(gen.occupancy(scene)).cuda()
    plan = dsopt.Plan(configs.robot("B"), params.DEFAULT, 1, 1 << 30)
    plan.scene_from_occupancy(0, occ, scene.voxel, scene.origin)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.scene_from_occupancy(0, occ, scene.voxel, scene.origin)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    plan.close()
    log(f"[bench] distance field from occupancy {scene.dims}: {ms:.2f} ms")
    return {"grid": list(scene.dims), "ms": ms,
            "what": "signed EDT of the occupancy grid + packing into gather records"}


def cpu_baseline(single, params, configs):
    """The FP64 oracle on the same problem, all host threads, ~10 s."""
    import oracle
    key = "B"
    robot, scene, prob = single["robot"], single["scene"], single["prob"]
    N = single["N"]
    threads = host_threads()
    O = oracle.Oracle(robot, scene, params.as_list(), threads=threads)
    X0 = configs.seeds_for(key, 0, prob).astype(np.float64)
    reps = 0
    t0 = time.perf_counter()
    while True:
        O.optimize(prob.q_start, prob.goal, X0, N)
        reps += 1
        el = time.perf_counter() - t0
        if el > 10.0 or reps >= 200:
            break
    S, T = X0.shape[0], X0.shape[1]
    val = reps * S * T * N / el
    log(f"[bench] cpu oracle: {reps} runs in {el:.1f} s on {threads} threads -> {val:.3e} evals/s")
    return {"value": val, "unit": "seed-waypoint evals/s", "cores": threads, "kind": "oracle",
            "sample": f"cluttered problem ({S} seeds x {T} waypoints x {N} iterations, FP64 "
                      f"oracle, OpenMP over seeds) repeated {reps} times"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="B", choices=["A", "B", "C"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--waves", type=int, default=8,
                    help="wavefronts per seed for the single-problem workload")
    ap.add_argument("--batched-waves", type=int, default=1,
                    help="wavefronts per seed for the batched workload")
    ap.add_argument("--serve-waves", type=int, default=8,
                    help="wavefronts per seed for the served (batched) form")
    ap.add_argument("--serve-plain-waves", type=int, default=8,
                    help="wavefronts per seed for the plain serial form")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy (known traffic) for PMC scaling")
    ap.add_argument("--serve-requests", type=int, default=2200)
    ap.add_argument("--serve-rate", type=float, default=200.0,
                    help="Poisson arrival rate of the serving workload [1/s]")
    ap.add_argument("--serve-sat-requests", type=int, default=1000,
                    help="requests of the saturated serving run (0: skip)")
    ap.add_argument("--serve-sat-rate", type=float, default=2000.0,
                    help="arrival rate of the saturated serving run [1/s]")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-block", type=int, default=25,
                    help="iterations per graph replay in the served form")
    ap.add_argument("--serve-drain", action="store_true",
                    help="served form: run the active requests to completion when none waits")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this path has no multi-GPU form); got "
              f"--gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2410_16727_amd import dsopt
    from workloads import configs, params
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dsopt.load()
    if args.calibrate_copy:
        a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    single = run_single(args, dsopt, torch, configs, params)
    traffic, pmc = measured_traffic()
    S, T, N = single["S"], single["T"], single["N"]
    value = S * T * N / (single["ms_per_step"] / 1e3)
    rec = {
        "metric": "seed-waypoint cost+grad evals/sec, problems/sec; p50/p99 plan latency vs plain",
        "value": value,
        "unit": "seed-waypoint evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": single["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded shelf scene and arm; no dataset)",
        "config": {"workload": f"cluttered: 1 problem, {S} seeds x {T} waypoints, "
                               f"{single['spheres']} spheres, {single['grid'][0]}^3 FP32 ESDF "
                               f"at 1 cm, {N} L-BFGS iters",
                   "seeds": S, "horizon": T, "iters": N, "spheres": single["spheres"],
                   "waves_per_seed": args.waves},
        "problems_per_s": 1e3 / single["ms_per_step"],
        "roofline": {"bound": "hbm", "kernel": "k_optimize",
                     "achieved": single["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": single["achieved_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel_ms": single["kernel_ms"],
                     "algorithmic_bytes_per_launch": single["sample_bytes"],
                     "gathered_bytes_per_launch": single["gather_bytes"],
                     "gathered_frac": single["gather_bytes"] / single["sample_bytes"],
                     "evals_per_seed": single["evals_per_seed"]},
    }
    rec["esdf_from_occupancy"] = run_esdf_build(args, dsopt, torch, configs, params,
                                                single["scene"])
    rec["differentiation"] = run_differentiation(args, dsopt, torch, configs, params)
    if not args.no_batched:
        rec["batched"] = run_batched(args, dsopt, torch, configs, params)
    if not args.no_serving:
        rec["serving"] = run_serving(args, dsopt, torch, configs, params)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(single, params, configs)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
