#!/usr/bin/env python3
"""Benchmark of the seeded trajectory optimiser on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
optimisation of every seed of every problem of the batch for N_iters
L-BFGS iterations (FK, spheres, ESDF gathers, costs, adjoint, line search,
flags, best seed) plus reading back every problem's best trajectory.
Inputs are resident in HBM before the timed region.

Headline workload (the largest single-GPU configuration): the batched-uneven
set -- 64 problems, seeds U{4..128}, horizons U{16..64}, 56 spheres, a 128^3
FP32 ESDF at 1.5 cm per problem, 100 iterations -- as one batched call:
the persistent optimiser runs every seed's initial evaluation, the queues
are ordered, and the persistent optimiser runs the iterations.  Extra fields: the same set as one launch per problem (the plain
form), the cluttered single problem (32 x 32, 200^3, wavefront teams), the
differentiation workload, serving at the workload's rate and a rate sweep
for the largest rate with p99 <= 100 ms, the GPU distance-field build, and
the FP64 oracle on the host cores.

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
# VALU issue ceiling: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 VALU
# instruction per SIMD every 4 cycles (16 lanes per SIMD)
VALU_PEAK_GIPS = 256 * 4 * 2.4e9 / 4 / 1e9
# the same ceiling in lane operations (an FMA is one operation): 64 FP32
# lanes per CU per cycle; x2 for FMA flops and x2 for packed FP32 gives the
# published 157.3 TFLOP/s
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def ops_per_eval(n_spheres, grad):
    """Algorithmic lane operations (FMA = 1) of one seed-waypoint evaluation:
    forward = 7 x 100 (kinematics) + N_s (9 centre + 35 gather/blend/hinge);
    the backward pass adds the forward again plus 30 per sphere (force and
    wrench projection)."""
    fwd = 7 * 100 + n_spheres * (9 + 35)
    return 2 * fwd + 30 * n_spheres if grad else fwd


KERNEL_SOURCES = ["paper_2410_16727_amd/csrc/dsopt_kernels.hip",
                  "paper_2410_16727_amd/csrc/dsopt_internal.h"]
PMC_SUMMARY = "profiles/k_optimize_pmc_batched.json"
COPY_BYTES = 256 << 20


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters():
    """The committed rocprofv3 PMC summary of the batched launch (HBM bytes
    per launch from FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel
    factors, VALU instructions per launch), or None when the kernel source
    changed since the counters were taken."""
    path = os.path.join(ROOT, PMC_SUMMARY)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return rec


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


def hinge_active_fraction(plan, scene, robot, X, eps):
    """Fraction of the sphere samples of trajectories X [S, T, 7] (cuda)
    within the hinge's activation distance of an obstacle: centres from the
    library's kinematics kernel, exact box distances from the scene's boxes
    (a description of the workload, outside any timed region)."""
    from workloads import gen
    c = plan.sphere_centres(X).cpu().numpy().astype(np.float64)
    d = gen.scene_sdf(c, scene) - robot.sphere_radius.astype(np.float64)
    return float(np.mean(d < eps))


def run_single(args, dsopt, torch, configs, params):
    """The cluttered single problem (32 seeds x 32 waypoints, 200^3 shelf
    scene) with wavefront teams: the latency-bound form."""
    key = "B"
    w = configs.WORKLOADS[key]
    robot = configs.robot(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    S, T, N = prob.S, prob.T, w.iters
    log(f"[bench] cluttered: S={S} T={T} spheres={robot.n_spheres} grid={scene.dims} iters={N}")
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
    steps = max(1, args.single_steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.kernel_timing(False)
    k_ms, k_n = plan.kernel_timing_read()
    ms_step = (t1 - t0) * 1e3 / steps
    sample_bytes = float(np.sum(n_evals)) * T * robot.n_spheres * 32.0
    gather_bytes = float(np.sum(sres["n_gathers"])) * 32.0
    avg_kernel_s = k_ms / max(k_n, 1) / 1e3
    active = hinge_active_fraction(plan, scene, robot, seeds, params.DEFAULT["eps"])
    log(f"[bench] cluttered: {ms_step:.3f} ms/step, kernel {k_ms / max(k_n, 1):.3f} ms/launch, "
        f"hinge-active seed samples {active:.3f}, gathered {gather_bytes / sample_bytes:.3f} of "
        f"the samples, best {best}")
    plan.close()
    return {
        "workload": f"cluttered: 1 problem, {S} seeds x {T} waypoints, {robot.n_spheres} spheres, "
                    f"{scene.dims[0]}^3 FP32 ESDF at 1 cm (shelf, 20 boxes), {N} L-BFGS iters, "
                    f"{args.waves} wavefronts per seed",
        "ms_per_step": ms_step, "kernel_ms": k_ms / max(k_n, 1),
        "seed_waypoint_evals_per_s": S * T * N / (ms_step / 1e3),
        "problems_per_s": 1e3 / ms_step,
        "seed_hinge_active_fraction": active,
        "algorithmic_bytes_per_launch": sample_bytes,
        "achieved_algorithmic_gbs": sample_bytes / avg_kernel_s / 1e9,
        "gathered_bytes_per_launch": gather_bytes,
        "gathered_frac_of_samples": gather_bytes / sample_bytes,
        "evals_per_seed": float(np.mean(n_evals)),
        "best_seed": {k: best[k] for k in ("best_seed", "success", "collision_free", "cost",
                                           "min_clearance_m", "pos_err_m", "rot_err_rad",
                                           "max_jerk", "motion_time")},
        "_scene": scene, "_robot": robot, "_prob": prob,
    }


def run_batched(args, dsopt, torch, configs, params):
    """The headline: 64 uneven problems in one batched call per step
    (args.steps timed steps after args.warmup), and the plain form (one
    launch per problem) beside it."""
    key = "D"
    w = configs.WORKLOADS[key]
    robot = configs.robot(key)
    t0 = time.perf_counter()
    scenes = configs.scenes(key, threads=host_threads())
    log(f"[bench] batched: built {len(scenes)} grids in {time.perf_counter() - t0:.1f} s")
    probs = configs.problems(key)
    N = w.iters
    cells = sum((s.dims[0] - 1) * (s.dims[1] - 1) * (s.dims[2] - 1) for s in scenes)
    state = sum(p.S * 40 * 1024 + p.S * p.T * 28 + p.S * 64 for p in probs)
    arena = cells * 32 + max(2, args.batch_depth) * state + (512 << 20)
    plan = dsopt.Plan(robot, dict(params.DEFAULT, waves_per_seed=args.batched_waves), N, arena)
    for i, sc in enumerate(scenes):
        plan.upload_scene(i, sc.grid, sc.voxel, sc.origin)
        sc.grid = None
    seeds = [torch.from_numpy(configs.seeds_for(key, i, p)).cuda() for i, p in enumerate(probs)]
    specs = [{"scene": p.scene, "q_start": p.q_start, "goal": p.goal, "seeds": seeds[i]}
             for i, p in enumerate(probs)]
    sw = sum(p.S * p.T for p in probs)
    tagc = [1000]

    # batched steps are pipelined: a step enqueues its batch, then reads
    # back (best trajectory of every problem) and releases the batch
    # batch_depth - 1 steps older, so the host's table building and
    # read-back run while the GPU works; the timed region ends with the last
    # batch read back.  The batches in flight run on their own streams
    # (default priority), so a batch's launches start on the CUs its
    # predecessor's last tiles leave idle, and a finished batch's small
    # result kernel is not held back behind the next batch's launches.
    pending = []
    streams = [torch.cuda.Stream() for _ in range(max(1, args.batch_streams))]
    stepc = [0]

    def read_back(base):
        for i in range(len(specs)):
            plan.get_best(base + i, probs[i].T)
        for i in range(len(specs)):
            plan.release(base + i)

    def batched():
        base = tagc[0]
        tagc[0] += len(specs)
        st = streams[stepc[0] % len(streams)]
        stepc[0] += 1
        plan.optimize([dict(s, tag=base + i) for i, s in enumerate(specs)], stream=st)
        pending.append(base)
        while len(pending) >= max(1, args.batch_depth):
            read_back(pending.pop(0))

    def drain():
        while pending:
            read_back(pending.pop(0))

    def isolated():
        # one batch at a time on the current stream: the launches' own
        # durations, for the kernel roofline
        base = tagc[0]
        tagc[0] += len(specs)
        plan.optimize([dict(s, tag=base + i) for i, s in enumerate(specs)])
        read_back(base)

    def plain():
        base = tagc[0]
        tagc[0] += len(specs)
        for i, s in enumerate(specs):
            plan.optimize([dict(s, tag=base + i)])
        for i in range(len(specs)):
            plan.get_best(base + i, probs[i].T)
        for i in range(len(specs)):
            plan.release(base + i)

    # evaluation and gather counts of every seed (deterministic)
    base = tagc[0]
    tagc[0] += len(specs)
    plan.optimize([dict(s, tag=base + i) for i, s in enumerate(specs)])
    gbytes = sbytes = sops = 0.0
    n_success = 0
    for i, p in enumerate(probs):
        r = plan.seed_results(base + i, p.S)
        gbytes += float(np.sum(r["n_gathers"])) * 32.0
        sbytes += float(np.sum(evals_per_seed(r))) * p.T * robot.n_spheres * 32.0
        # cost+gradient evaluations, then the cost-only candidates and the
        # result pass
        sops += p.T * (float(np.sum(r["n_evals_grad"])) * ops_per_eval(robot.n_spheres, True) +
                       float(np.sum(r["n_evals_cost"] + 1)) * ops_per_eval(robot.n_spheres, False))
        n_success += int(plan.get_best(base + i, p.T)[1]["success"])
        plan.release(base + i)
    out = {}
    legs = [("isolated", isolated, args.isolated_steps, 1),
            ("batched", batched, args.steps, args.warmup)]
    if args.plain_steps > 0:
        legs.append(("plain", plain, args.plain_steps, 1))
    for name, fn, steps, warm in legs:
        for _ in range(warm):
            fn()
        drain()
        torch.cuda.synchronize()
        plan.kernel_timing(True)
        t0 = time.perf_counter()
        reps = max(1, steps)
        for _ in range(reps):
            fn()
        drain()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        plan.kernel_timing(False)
        k_ms, k_n = plan.kernel_timing_read()
        out[name] = {"ms_per_batch": dt * 1e3,
                     "seed_waypoint_evals_per_s": sw * N / dt,
                     "problems_per_s": len(probs) / dt,
                     "kernel_ms_per_launch": k_ms / max(k_n, 1),
                     "launches_per_batch": k_n / reps, "steps": reps}
        log(f"[bench] batched-uneven {name}: {dt * 1e3:.2f} ms/batch, kernel "
            f"{k_ms / max(k_n, 1):.3f} ms/launch, {sw * N / dt:.3e} seed-waypoint evals/s")
    plan.close()
    out["sw"] = sw
    out["N"] = N
    out["n_problems"] = len(probs)
    out["algorithmic_bytes_per_launch"] = sbytes
    out["algorithmic_ops_per_launch"] = sops
    out["gathered_bytes_per_launch"] = gbytes
    out["problems_successful"] = n_success
    out["workload"] = (f"batched-uneven: {len(probs)} problems, seeds U{{4..128}}, horizons "
                       f"U{{16..64}}, {sw} seed-waypoints, {robot.n_spheres} spheres, a 128^3 FP32 "
                       f"ESDF at 1.5 cm per problem (5-30 random boxes), {N} L-BFGS iters, one "
                       f"batched call per step (persistent launches), steps pipelined: the host "
                       f"enqueues batch k and reads back batch k-{max(1, args.batch_depth - 1)} "
                       f"while the GPU runs, consecutive batches on {max(1, args.batch_streams)} "
                       f"alternating streams")
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
    if args.serve_requests > 0:
        n, rate = args.serve_requests, args.serve_rate
        reqs = make_reqs(n, rate)
        warm = min(200, n // 10)
        out["rate"] = {
            "workload": (f"serving: Poisson {n} requests at {rate:g}/s ({warm} warm-up), "
                         f"seeds U{{8..128}}, horizons U{{32..64}}, 16 resident 200^3 ESDFs, "
                         f"{N} iters, blocks of {args.serve_block} iterations per graph replay, "
                         f"{args.serve_slots} slots{', run to completion when idle' if args.serve_drain else ''}; "
                         f"served form {args.serve_waves} and plain "
                         f"serial form {args.serve_plain_waves} wavefronts per seed"),
            "served": served(sp, reqs, warm, f"served @{rate:g}/s"),
            "plain_serial": plain(pp, reqs, warm, f"plain serial @{rate:g}/s")}
        del reqs
    # the largest sustainable rate: open-loop Poisson arrivals at rising
    # rates until p99 exceeds the latency bound or the completion rate falls
    # below 95 % of the arrival rate
    if args.sweep_requests > 0:
        sweep = {}
        for name, plan, fn, rates in (
                ("served", sp, served, [float(r) for r in args.sweep_rates_served.split(",")]),
                ("plain_serial", pp, plain, [float(r) for r in args.sweep_rates_plain.split(",")])):
            pts = []
            best = 0.0
            for rate in rates:
                reqs = make_reqs(args.sweep_requests, rate)
                warm = args.sweep_requests // 10
                r = fn(plan, reqs, warm, f"{name} sweep @{rate:g}/s")
                del reqs
                ok = r["p99_ms"] <= args.p99_bound_ms and r["problems_per_s"] >= 0.95 * rate
                pts.append({"rate": rate, "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                            "problems_per_s": r["problems_per_s"], "sustained": ok})
                if ok:
                    best = rate
                else:
                    break
            sweep[name] = {"points": pts, "max_sustainable_rate": best}
            log(f"[bench] sweep {name}: max sustainable rate {best:g}/s "
                f"(p99 <= {args.p99_bound_ms:g} ms)")
        sweep["workload"] = (f"open-loop Poisson arrivals, {args.sweep_requests} requests per rate "
                             f"(10 % warm-up), same request mix; a rate is sustained when p99 <= "
                             f"{args.p99_bound_ms:g} ms and the completion rate is >= 95 % of it")
        out["max_rate_sweep"] = sweep
    sp.close()
    pp.close()
    return out


def run_differentiation(args, dsopt, torch, configs, params):
    """Cost + gradient of 256 seeds x 64 waypoints (60 spheres, 200^3) in
    one call, and the same through the autograd function (forward: the cost
    kernel; backward: the adjoint kernel with dJ, kinematics recomputed),
    and in its fused form (one cost+gradient launch in forward, the saved
    gradient scaled by dJ in backward), timed with events on the stream all
    run on."""
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

    def fwd_bwd_fused():
        Xr = X.clone().requires_grad_(True)
        trajectory_cost(Xr, plan, 0, prob.q_start, prob.goal, fused=True).sum().backward()

    ms_ag = timed(fwd_bwd)
    ms_agf = timed(fwd_bwd_fused)
    plan.close()
    sample_bytes = float(S * T * robot.n_spheres * 32)
    achieved = sample_bytes / (ms_cg * 1e-3) / 1e9
    log(f"[bench] differentiation: cost+grad {ms_cg:.3f} ms ({S * T / (ms_cg * 1e-3):.3e} "
        f"seed-waypoint evals/s), autograd forward+backward {ms_ag:.3f} ms (fused {ms_agf:.3f} ms)")
    return {"workload": f"differentiation: {S} seeds x {T} waypoints, {robot.n_spheres} spheres, "
                        f"{scene.dims[0]}^3 ESDF, one cost+gradient call",
            "cost_grad_ms": ms_cg, "seed_waypoint_evals_per_s": S * T / (ms_cg * 1e-3),
            "autograd_fwd_bwd_ms": ms_ag, "autograd_fused_fwd_bwd_ms": ms_agf,
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_rate(key, configs, params, threads, budget_s, max_problems=None, max_seeds=None):
    """The FP64 oracle's free-running optimisation over the workload's
    problems in order (first max_seeds seeds of each), until budget_s of
    wall time is spent (at least one problem): seed-waypoint evals/s and
    what was timed."""
    import oracle
    w = configs.WORKLOADS[key]
    robot = configs.robot(key)
    probs = configs.problems(key)
    if max_problems:
        probs = probs[:max_problems]
    work = 0
    el = 0.0
    done = 0
    cache = {}
    for i, p in enumerate(probs):
        if p.scene not in cache:
            cache = {p.scene: configs.scenes(key, only={p.scene}, threads=threads)[p.scene]}
        O = oracle.Oracle(robot, cache[p.scene], params.as_list(), threads=threads)
        X0 = configs.seeds_for(key, i, p).astype(np.float64)
        if max_seeds:
            X0 = X0[:max_seeds]
        t0 = time.perf_counter()
        O.optimize(p.q_start, p.goal, X0, w.iters)
        el += time.perf_counter() - t0
        work += X0.shape[0] * X0.shape[1] * w.iters
        done += 1
        if el >= budget_s:
            break
    return work / el, f"{done} problem(s){'' if not max_seeds else f' (first {max_seeds} seeds each)'}, {work} seed-waypoint iterations in {el:.1f} s"


def cpu_baseline(args, configs, params):
    """The oracle as it stands on the headline workload (batched-uneven),
    all host threads, a bounded sample (problems in order until ~10 s)."""
    threads = host_threads()
    val, what = cpu_rate("D", configs, params, threads, args.cpu_seconds)
    log(f"[bench] cpu oracle (batched-uneven, {threads} threads): {val:.3e} evals/s, {what}")
    return {"value": val, "unit": "seed-waypoint evals/s", "cores": threads, "kind": "oracle",
            "sample": f"batched-uneven workload: {what}; FP64 oracle, OpenMP over seeds, "
                      f"100 iterations per problem",
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def cpu_detail(args, configs, params):
    """The oracle single-threaded and on all host threads for the tiny,
    cluttered, differentiation and batched-uneven workloads (the last two
    on the first 16 seeds of each problem), each on a short bounded
    sample."""
    threads = host_threads()
    out = {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "threads_all": threads}
    for key, kw in (("A", {}), ("B", {}), ("C", {"max_seeds": 16}), ("D", {"max_seeds": 16})):
        row = {}
        for label, th in (("single_thread", 1), ("all_threads", threads)):
            val, what = cpu_rate(key, configs, params, th, args.cpu_detail_seconds, **kw)
            row[label] = {"seed_waypoint_evals_per_s": val, "sample": what}
        out[configs.WORKLOADS[key].name] = row
        log(f"[bench] cpu oracle {key}: 1 thread {row['single_thread']['seed_waypoint_evals_per_s']:.3e}, "
            f"{threads} threads {row['all_threads']['seed_waypoint_evals_per_s']:.3e} evals/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed steps (batches) of the headline workload")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-detail", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-detail-seconds", type=float, default=1.5)
    ap.add_argument("--waves", type=int, default=8,
                    help="wavefronts per seed for the cluttered single problem")
    ap.add_argument("--batched-waves", type=int, default=1,
                    help="wavefronts per seed for the batched workload")
    ap.add_argument("--batch-streams", type=int, default=3,
                    help="streams the pipelined batched steps alternate between")
    ap.add_argument("--isolated-steps", type=int, default=5,
                    help="batched steps timed one batch at a time (kernel roofline)")
    ap.add_argument("--batch-depth", type=int, default=3,
                    help="batches in flight: a step reads back the batch this many steps back")
    ap.add_argument("--plain-steps", type=int, default=2,
                    help="timed batches of the one-launch-per-problem form")
    ap.add_argument("--single-steps", type=int, default=20)
    ap.add_argument("--serve-waves", type=int, default=8,
                    help="wavefronts per seed for the served (batched) form")
    ap.add_argument("--serve-plain-waves", type=int, default=8,
                    help="wavefronts per seed for the plain serial form")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy (known traffic) for PMC scaling")
    ap.add_argument("--serve-requests", type=int, default=2200)
    ap.add_argument("--serve-rate", type=float, default=200.0,
                    help="Poisson arrival rate of the serving workload [1/s]")
    ap.add_argument("--sweep-requests", type=int, default=600,
                    help="requests per rate of the sustainable-rate sweep (0: skip)")
    ap.add_argument("--sweep-rates-served", default="500,1000,2000,3000,4000,6000,8000")
    ap.add_argument("--sweep-rates-plain", default="200,400,600,800,1000,1200")
    ap.add_argument("--p99-bound-ms", type=float, default=100.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-block", type=int, default=25,
                    help="iterations per graph replay in the served form")
    ap.add_argument("--serve-drain", action="store_true",
                    help="served form: run the active requests to completion when none waits")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this path has no multi-GPU form; the design "
              f"notes describe how it would shard); got --gpus {args.gpus}", file=sys.stderr)
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
    bt = run_batched(args, dsopt, torch, configs, params)
    sw, N = bt["sw"], bt["N"]
    ms = bt["batched"]["ms_per_batch"]
    # the kernel roofline takes the launches' own durations, timed one batch
    # at a time; the pipelined steps overlap consecutive batches
    kms = bt["isolated"]["kernel_ms_per_launch"]
    sbytes = bt["algorithmic_bytes_per_launch"]
    gbytes = bt["gathered_bytes_per_launch"]
    sops = bt["algorithmic_ops_per_launch"]
    achieved_gbs = sbytes / (kms * 1e-3) / 1e9
    achieved_tops = sops / (kms * 1e-3) / 1e12
    pmc = measured_counters()
    # the launch is bound by each wavefront's chain of VALU work and
    # latency (counters: about half the chip's issue slots over the launch,
    # 70 % while waves are resident); the byte view is kept beside it.
    # The headline steps overlap consecutive batches on alternating
    # streams, so the kernel figures come from the isolated leg (one batch
    # at a time, kernel_ms); per_batch divides by the pipelined step, and
    # kernel_ms_overlapped is a launch's duration inside the pipeline.
    roof = {"bound": "alu",
            "kernel": "k_optimize (a batch's initial-evaluation and iteration dispatches, with "
                      "the queue order between them; one wavefront per seed)",
            "achieved": achieved_tops, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved_tops / ALU_PEAK_TOPS,
            "traffic": pmc.get("traffic_bytes_per_launch") if pmc else None,
            "kernel_ms": kms,
            "kernel_ms_overlapped": bt["batched"]["kernel_ms_per_launch"],
            "algorithmic_ops_per_launch": sops,
            "ops_per_unit": {"cost+grad": ops_per_eval(56, True), "cost": ops_per_eval(56, False)},
            "hbm": {"algorithmic_bytes_per_launch": sbytes, "achieved_gbs": achieved_gbs,
                    "peak_gbs": HBM_PEAK_GBS, "frac": achieved_gbs / HBM_PEAK_GBS,
                    "gathered_bytes_per_launch": gbytes, "gathered_frac_of_samples": gbytes / sbytes,
                    "gathered_gbs": gbytes / (kms * 1e-3) / 1e9,
                    "gathered_frac_of_peak": gbytes / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "measured_gbs": (pmc["traffic_bytes_per_launch"] / (kms * 1e-3) / 1e9
                                     if pmc else None)},
            "valu": None,
            "per_batch": {"ms": ms, "achieved": sops / (ms * 1e-3) / 1e12,
                          "frac": sops / (ms * 1e-3) / 1e12 / ALU_PEAK_TOPS,
                          "hbm_achieved_gbs": sbytes / (ms * 1e-3) / 1e9}}
    if pmc and pmc.get("valu_insts_per_launch"):
        vi = pmc["valu_insts_per_launch"]
        roof["valu"] = {"insts_per_launch": vi, "achieved_ginst_s": vi / (kms * 1e-3) / 1e9,
                        "peak_ginst_s": VALU_PEAK_GIPS,
                        "issue_frac": vi / (kms * 1e-3) / 1e9 / VALU_PEAK_GIPS,
                        "lane_ops_per_algorithmic_op": vi * 64 / sops}
    rec = {
        "metric": "seed-waypoint cost+grad evals/sec, problems/sec; p50/p99 plan latency vs plain",
        "value": sw * N / (ms / 1e3),
        "unit": "seed-waypoint evals/s",
        "n_gpus": 1,
        "steps": bt["batched"]["steps"],
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded random-box scenes, synthetic 7-joint arm; no dataset)",
        "config": {"workload": bt["workload"], "problems": bt["n_problems"],
                   "seed_waypoints": sw, "iters": N, "spheres": 56,
                   "waves_per_seed": args.batched_waves},
        "problems_per_s": bt["batched"]["problems_per_s"],
        "roofline": roof,
        "plain_form": (dict(bt["plain"], speedup_batched_vs_plain=bt["plain"]["ms_per_batch"] / ms)
                       if "plain" in bt else None),
        "problems_successful": bt["problems_successful"],
    }
    if not args.no_extras:
        single = None
        if not args.no_single:
            single = run_single(args, dsopt, torch, configs, params)
            rec["esdf_from_occupancy"] = run_esdf_build(args, dsopt, torch, configs, params,
                                                        single["_scene"])
            rec["cluttered"] = {k: v for k, v in single.items() if not k.startswith("_")}
        rec["differentiation"] = run_differentiation(args, dsopt, torch, configs, params)
        if not args.no_serving:
            rec["serving"] = run_serving(args, dsopt, torch, configs, params)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(args, configs, params)
        if not args.no_cpu_detail and not args.no_extras:
            rec["cpu_detail"] = cpu_detail(args, configs, params)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
