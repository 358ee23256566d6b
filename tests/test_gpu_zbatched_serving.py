"""GPU tests of the batched persistent launch, the serving loop and the
autograd function, through the C ABI.

- batched vs plain: every problem's optimised seeds are bitwise identical
  whether it runs alone (one launch) or inside a 64-problem persistent
  launch (per-seed arithmetic and reduction order depend only on T);
- full-size batched workload: per-seed flags/costs of the GPU's final
  trajectories match the FP64 oracle evaluated on them (sampled seeds);
- serving: every request's result is the same alone and in the mix
  (bitwise), over many graph replays with host work between them;
- autograd: gradient of DSCost (backward = the adjoint kernel) equals the
  oracle gradient;
- scenes in use by serving requests cannot be released or replaced."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2410_16727_amd import dsopt  # noqa: E402
from paper_2410_16727_amd.autograd import trajectory_cost  # noqa: E402
from workloads import configs, gen, params  # noqa: E402

from test_gpu_parity import GRAD_RTOL, grad_check  # noqa: E402

P = params.DEFAULT


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def batchD():
    key = "D"
    robot = configs.robot(key)
    scenes = configs.scenes(key)
    probs = configs.problems(key)
    cells = sum((s.dims[0] - 1) * (s.dims[1] - 1) * (s.dims[2] - 1) for s in scenes)
    plan = dsopt.Plan(robot, P, 100, cells * 32 + (2 << 30))
    for i, sc in enumerate(scenes):
        plan.upload_scene(i, sc.grid, sc.voxel, sc.origin)
    seeds = [torch.from_numpy(configs.seeds_for(key, i, p)).cuda() for i, p in enumerate(probs)]
    yield {"robot": robot, "scenes": scenes, "probs": probs, "plan": plan, "seeds": seeds}
    plan.close()


def spec(p, seeds, tag, out=None):
    return {"scene": p.scene, "q_start": p.q_start, "goal": p.goal, "seeds": seeds, "tag": tag,
            "out": out}


def test_team_launch_batched_equals_plain_bitwise():
    """With 4 wavefronts per seed: batched == plain bitwise, and the final
    per-seed costs and flags agree with the FP64 oracle evaluated on the
    final trajectories."""
    key = "D"
    robot = configs.robot(key)
    probs = configs.problems(key)[:6]
    scenes = configs.scenes(key, only=set(p.scene for p in probs))
    pl = dsopt.Plan(robot, dict(P, waves_per_seed=4), 40, 512 << 20)
    for p in probs:
        sc = scenes[p.scene]
        pl.upload_scene(p.scene, sc.grid, sc.voxel, sc.origin)
    seeds = [torch.from_numpy(configs.seeds_for(key, i, p)).cuda() for i, p in enumerate(probs)]
    ob = [torch.zeros_like(sd) for sd in seeds]
    op = [torch.zeros_like(sd) for sd in seeds]
    say("team launch (4 wavefronts per seed): batched vs plain")
    pl.optimize([spec(p, seeds[i], 700 + i, ob[i]) for i, p in enumerate(probs)])
    for i, p in enumerate(probs):
        pl.optimize([spec(p, seeds[i], 800 + i, op[i])])
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        assert torch.equal(ob[i], op[i]), i
        res = pl.seed_results(700 + i, p.S)
        O = oracle.Oracle(robot, scenes[p.scene], params.as_list(), threads=8)
        ref = O.results(p.q_start, p.goal, ob[i].cpu().numpy().astype(np.float64))
        assert (np.abs(res["cost"] - ref["J"]) / ref["J"]).max() < 1e-4, i
        amb = np.abs(ref["clearance"]) < 1e-5
        for f in ["collision_free", "success", "valid"]:
            assert ((res[f] == ref[f].astype(int)) | amb).all(), (i, f)
    pl.close()


def test_batched_equals_plain_bitwise(batchD):
    plan, probs, seeds = batchD["plan"], batchD["probs"], batchD["seeds"]
    idx = list(range(0, 64, 4))       # 16 problems, mixed S and T
    say("batched vs plain", [(probs[i].S, probs[i].T) for i in idx])
    outs_b = [torch.zeros_like(seeds[i]) for i in idx]
    outs_p = [torch.zeros_like(seeds[i]) for i in idx]
    plan.optimize([spec(probs[i], seeds[i], 100 + k, outs_b[k]) for k, i in enumerate(idx)])
    for k, i in enumerate(idx):
        plan.optimize([spec(probs[i], seeds[i], 200 + k, outs_p[k])])
    torch.cuda.synchronize()
    for k, i in enumerate(idx):
        assert torch.equal(outs_b[k], outs_p[k]), (i, probs[i].S, probs[i].T)
        rb = plan.get_best(100 + k, probs[i].T)
        rp = plan.get_best(200 + k, probs[i].T)
        assert np.array_equal(rb[0], rp[0]) and rb[1] == rp[1]
        plan.release(100 + k)
        plan.release(200 + k)


def test_full_batched_workload_flags_vs_oracle(batchD):
    plan, probs, seeds, scenes, robot = (batchD[k] for k in
                                         ["plan", "probs", "seeds", "scenes", "robot"])
    outs = [torch.zeros_like(s) for s in seeds]
    say("full batched workload: 64 problems")
    plan.optimize([spec(p, seeds[i], 300 + i, outs[i]) for i, p in enumerate(probs)])
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    n_checked = 0
    for i, p in enumerate(probs):
        res = plan.seed_results(300 + i, p.S)
        X = outs[i].cpu().numpy().astype(np.float64)
        pick = rng.choice(p.S, size=min(3, p.S), replace=False)
        O = oracle.Oracle(robot, scenes[p.scene], params.as_list(), threads=8)
        ref = O.results(p.q_start, p.goal, X[pick])
        amb = np.abs(ref["clearance"]) < 1e-5
        for f in ["collision_free", "within_limits", "success", "valid"]:
            assert ((res[f][pick] == ref[f].astype(int)) | amb).all(), (i, f)
        rel = np.abs(res["cost"][pick] - ref["J"]) / ref["J"]
        assert rel.max() < 1e-4, (i, rel.max())
        n_checked += len(pick)
        plan.release(300 + i)
    say(f"checked {n_checked} sampled seeds")


def test_full_batch_equals_plain(batchD):
    """The full batch (more tiles than the chip holds at once, spread over
    the per-XCD queues): every sampled seed comes out bitwise as in a
    launch of its problem alone, its counters included."""
    plan, probs, seeds = batchD["plan"], batchD["probs"], batchD["seeds"]
    outs_b = [torch.zeros_like(s) for s in seeds]
    say("full batch vs plain")
    plan.optimize([spec(p, seeds[i], 900 + i, outs_b[i]) for i, p in enumerate(probs)])
    heavy = sorted(range(len(probs)), key=lambda i: -probs[i].S * probs[i].T)[:3]
    for i in sorted(set(heavy + [0, 17, 33, 48, 63])):
        p = probs[i]
        out_p = torch.zeros_like(seeds[i])
        plan.optimize([spec(p, seeds[i], 1000 + i, out_p)])
        torch.cuda.synchronize()
        assert torch.equal(outs_b[i], out_p), (i, p.S, p.T)
        rb, rp = plan.seed_results(900 + i, p.S), plan.seed_results(1000 + i, p.S)
        for k in rb:
            assert np.array_equal(rb[k], rp[k], equal_nan=rb[k].dtype.kind == "f"), (i, k)
        plan.release(1000 + i)
    for i in range(len(probs)):
        plan.release(900 + i)


def test_batches_on_three_streams_equal_one_at_a_time(batchD):
    """Three full batches in flight at once on three streams (each enqueued
    while the previous ones run, as a pipelined caller does): every
    problem's output seeds, best trajectory and seed results are bitwise
    those of the batch run alone."""
    plan, probs, seeds = batchD["plan"], batchD["probs"], batchD["seeds"]
    say("three batches on three streams")
    ref = [torch.zeros_like(s) for s in seeds]
    plan.optimize([spec(p, seeds[i], 1200 + i, ref[i]) for i, p in enumerate(probs)])
    torch.cuda.synchronize()
    outs = [[torch.zeros_like(s) for s in seeds] for _ in range(3)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    torch.cuda.synchronize()   # the outputs' zero fill (default stream) is done
    for b, st in enumerate(streams):
        plan.optimize([spec(p, seeds[i], 1300 + 100 * b + i, outs[b][i])
                       for i, p in enumerate(probs)], stream=st)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        traj0, best0 = plan.get_best(1200 + i, p.T)
        r0 = plan.seed_results(1200 + i, p.S)
        for b in range(3):
            tag = 1300 + 100 * b + i
            assert torch.equal(outs[b][i], ref[i]), (b, i)
            traj, best = plan.get_best(tag, p.T)
            assert np.array_equal(traj, traj0) and best == best0, (b, i)
            r = plan.seed_results(tag, p.S)
            for k in r0:
                assert np.array_equal(r[k], r0[k], equal_nan=r0[k].dtype.kind == "f"), (b, i, k)
    for i in range(len(probs)):
        for tag in (1200 + i, 1300 + i, 1400 + i, 1500 + i):
            plan.release(tag)


@pytest.mark.parametrize("waves,m", [(1, 8), (8, 8), (8, 3), (2, 5)])
def test_serving_matches_alone_bitwise(waves, m):
    """Served in 7-iteration blocks (every request resumes in later
    launches; a team rebuilds its history products from the ring, also with
    a short, often wrapped ring) vs alone in one launch: the same bits."""
    key = "B"
    robot = configs.robot(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    plan = dsopt.Plan(robot, dict(P, waves_per_seed=waves, history=m), 30, 1 << 30,
                      block_iters=7)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    rng = np.random.default_rng(5)
    reqs = []
    for r in range(12):
        S = int(rng.integers(1, 40))
        T = int(rng.choice([4, 9, 16, 17, 32, 40, 64]))
        sd = torch.from_numpy(configs.seeds_for(key, 0, prob, S=S, T=T, stream=r)).cuda()
        reqs.append((S, T, sd))
    say("serving mix", [(S, T) for S, T, _ in reqs])
    # alone
    alone = []
    for r, (S, T, sd) in enumerate(reqs):
        plan.optimize([{"scene": 0, "q_start": prob.q_start, "goal": prob.goal, "seeds": sd,
                        "tag": 500 + r}])
        alone.append(plan.get_best(500 + r, T))
        plan.release(500 + r)
    # in the mix: staggered submissions, eager host work between replays
    plan.serve_start(max_slots=5, queue_cap=64)
    tickets = {}
    pending = list(range(len(reqs)))
    got = {}
    steps = 0
    while len(got) < len(reqs):
        if pending and steps % 2 == 0:
            r = pending.pop(0)
            S, T, sd = reqs[r]
            tickets[r] = plan.serve_submit({"scene": 0, "q_start": prob.q_start,
                                            "goal": prob.goal, "seeds": sd})
        plan.serve_step()
        _ = plan.cost(0, prob.q_start, prob.goal, reqs[0][2])   # eager work in between
        torch.cuda.synchronize()
        for r, t in list(tickets.items()):
            if r in got:
                continue
            res = plan.serve_poll(t, reqs[r][1])
            if res is not None:
                got[r] = res
        steps += 1
        assert steps < 2000
    st = plan.serve_stats()
    say(f"serving: {steps} steps, stats {st}")
    assert st["completed"] == len(reqs)
    assert st["mean_active_slots"] > 1.0       # requests overlapped on the device
    for r in range(len(reqs)):
        assert np.array_equal(got[r][0], alone[r][0]), r
        assert got[r][1] == alone[r][1], (r, got[r][1], alone[r][1])
    plan.serve_stop()
    plan.close()


def test_serving_admission_waits_for_memory():
    key = "A"
    robot = configs.robot(key)
    scene = configs.scenes(key)[0]
    prob = configs.problems(key)[0]
    # an arena with room for the scene and only a few requests' state
    plan = dsopt.Plan(robot, P, 4, 48 << 20, block_iters=2)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    plan.serve_start(max_slots=64, queue_cap=128)
    sd = torch.from_numpy(configs.seeds_for(key, 0, prob, S=128, T=64)).cuda()
    tickets = [plan.serve_submit({"scene": 0, "q_start": prob.q_start, "goal": prob.goal,
                                  "seeds": sd}) for _ in range(12)]
    max_active = 0
    left = set(tickets)
    deadline = time.monotonic() + 120.0
    while left and time.monotonic() < deadline:
        a = plan.serve_step()
        max_active = max(max_active, a)
        for t in list(left):
            if plan.serve_poll(t, 64) is not None:
                left.discard(t)
    done = len(tickets) - len(left)
    say(f"admission by memory: max active {max_active}")
    assert done == len(tickets)
    assert 1 <= max_active < 12           # memory, not slots, limited concurrency
    plan.serve_stop()
    plan.close()


def test_autograd_matches_oracle_gradient():
    key = "C"
    robot = configs.robot(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    plan = dsopt.Plan(robot, P, 1, 512 << 20)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    rng = np.random.default_rng(9)
    X = gen.random_trajectories(rng, 16, 64, prob.q_start)
    Xt = torch.from_numpy(X).cuda().requires_grad_(True)
    w = torch.linspace(0.5, 2.0, 16, device="cuda")
    J = trajectory_cost(Xt, plan, 0, prob.q_start, prob.goal)
    (J * w).sum().backward()
    O = oracle.Oracle(robot, scene, params.as_list(), threads=8)
    ref = O.cost(prob.q_start, prob.goal, X.astype(np.float64), grad=True, absg=True)
    assert np.abs(J.detach().cpu().numpy() - ref["J"]).max() / ref["J"].min() < 1e-4
    # backward launches the adjoint kernel with dJ = w: the same bits as the
    # library's cost+gradient call given the weights
    _, Gw = plan.cost_grad(0, prob.q_start, prob.goal, Xt.detach(), w)
    assert torch.equal(Xt.grad, Gw)
    # the fused form (one cost+gradient launch in forward, the saved gradient
    # scaled in backward) forms the same float32 products
    Xf = Xt.detach().clone().requires_grad_(True)
    Jf = trajectory_cost(Xf, plan, 0, prob.q_start, prob.goal, fused=True)
    (Jf * w).sum().backward()
    assert torch.equal(Xf.grad, Gw)
    # forward alone is the cost-only kernel (its team sum is ordered
    # differently from the cost+gradient kernel's: equal up to rounding)
    assert torch.allclose(Jf.detach(), J.detach(), rtol=1e-6, atol=0)
    G = Xt.grad.cpu().numpy()
    wn = w.cpu().numpy()
    for s in range(16):
        worst, need = grad_check(O, prob, X[s], G[s], ref["G"][s], ref["A"][s], w=wn[s])
        assert worst <= GRAD_RTOL, (s, worst, need)
    # a few plain gradient steps reduce the cost
    with torch.no_grad():
        Y = Xt.detach().clone()
    J0 = trajectory_cost(Y, plan, 0, prob.q_start, prob.goal).sum().item()
    for _ in range(5):
        Y.requires_grad_(True)
        Jy = trajectory_cost(Y, plan, 0, prob.q_start, prob.goal).sum()
        Jy.backward()
        with torch.no_grad():
            Y = Y - 1e-4 * Y.grad / Y.grad.abs().max()
    assert trajectory_cost(Y, plan, 0, prob.q_start, prob.goal).sum().item() < J0
    plan.close()


def test_serving_with_optional_terms_matches_alone():
    """The served loop with the variant kernels (swept sub-samples on):
    every request's result equals its result optimised alone, bitwise."""
    key = "A"
    robot = configs.robot(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    plan = dsopt.Plan(robot, dict(P, waves_per_seed=8, swept_samples=2), 12, 256 << 20,
                      block_iters=5)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    reqs = []
    for r, (S, T) in enumerate([(3, 16), (5, 33), (2, 64), (4, 8)]):
        reqs.append((S, T, torch.from_numpy(configs.seeds_for(key, 0, prob, S=S, T=T,
                                                               stream=r)).cuda()))
    alone = []
    for r, (S, T, sd) in enumerate(reqs):
        plan.optimize([{"scene": 0, "q_start": prob.q_start, "goal": prob.goal, "seeds": sd,
                        "tag": 700 + r}])
        alone.append(plan.get_best(700 + r, T))
        plan.release(700 + r)
    plan.serve_start(max_slots=3, queue_cap=16)
    tickets = {r: plan.serve_submit({"scene": 0, "q_start": prob.q_start, "goal": prob.goal,
                                     "seeds": sd}) for r, (S, T, sd) in enumerate(reqs)}
    got = {}
    deadline = time.monotonic() + 120.0   # replays run asynchronously
    while len(got) < len(reqs) and time.monotonic() < deadline:
        plan.serve_step()
        for r, t in tickets.items():
            if r not in got:
                res = plan.serve_poll(t, reqs[r][1])
                if res is not None:
                    got[r] = res
    assert len(got) == len(reqs)
    for r in range(len(reqs)):
        assert np.array_equal(got[r][0], alone[r][0]), r
        assert got[r][1] == alone[r][1], r
    plan.serve_stop()
    plan.close()


def test_serving_drain_when_idle_matches_alone():
    """serve_drain: with nobody waiting a replay runs the active requests to
    completion; results stay bitwise those of the requests alone, and a
    lone request needs a single replay."""
    key = "A"
    robot = configs.robot(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    plan = dsopt.Plan(robot, dict(P, serve_drain=1), 20, 256 << 20, block_iters=4)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    reqs = [(S, T, torch.from_numpy(configs.seeds_for(key, 0, prob, S=S, T=T, stream=r)).cuda())
            for r, (S, T) in enumerate([(4, 32), (7, 20), (2, 64)])]
    alone = []
    for r, (S, T, sd) in enumerate(reqs):
        plan.optimize([{"scene": 0, "q_start": prob.q_start, "goal": prob.goal, "seeds": sd,
                        "tag": 800 + r}])
        alone.append(plan.get_best(800 + r, T))
        plan.release(800 + r)
    plan.serve_start(max_slots=4, queue_cap=8)
    got = {}
    for r, (S, T, sd) in enumerate(reqs):      # one at a time: one replay each
        t = plan.serve_submit({"scene": 0, "q_start": prob.q_start, "goal": prob.goal,
                               "seeds": sd})
        deadline = time.monotonic() + 60.0
        while r not in got and time.monotonic() < deadline:
            plan.serve_step()
            res = plan.serve_poll(t, T)
            if res is not None:
                got[r] = res
    st = plan.serve_stats()
    assert st["completed"] == len(reqs)
    assert st["steps"] == len(reqs)
    for r in range(len(reqs)):
        assert np.array_equal(got[r][0], alone[r][0]), r
        assert got[r][1] == alone[r][1], r
    plan.serve_stop()
    plan.close()


def test_scene_in_use_by_serving_is_busy():
    """A scene used by a queued or admitted serving request cannot be
    released or replaced (DS_ERR_BUSY); once the request is done it can."""
    key = "A"
    robot = configs.robot(key)
    scene = configs.scenes(key, only={0})[0]
    prob = configs.problems(key)[0]
    plan = dsopt.Plan(robot, P, 20, 256 << 20, block_iters=5)
    plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
    plan.upload_scene(1, scene.grid, scene.voxel, scene.origin)
    sd = torch.from_numpy(configs.seeds_for(key, 0, prob)).cuda()
    plan.serve_start(max_slots=2, queue_cap=4)
    t = plan.serve_submit({"scene": 0, "q_start": prob.q_start, "goal": prob.goal, "seeds": sd})
    for step in range(2):           # queued, then admitted and running
        with pytest.raises(dsopt.DsError) as e:
            plan.release_scene(0)
        assert e.value.code == dsopt.DS_ERR_BUSY
        with pytest.raises(dsopt.DsError) as e:
            plan.upload_scene(0, scene.grid, scene.voxel, scene.origin)
        assert e.value.code == dsopt.DS_ERR_BUSY
        plan.serve_step()
    plan.release_scene(1)           # not used by any request
    res = None
    deadline = time.monotonic() + 60.0   # the replays run asynchronously
    while res is None and time.monotonic() < deadline:
        plan.serve_step()
        res = plan.serve_poll(t, prob.T)
    assert res is not None and res[1]["best_seed"] >= 0
    plan.release_scene(0)
    plan.serve_stop()
    plan.close()
