"""Benchmark of the SGTP planning step on one MI355X.

A step is one closed-loop planning step of the mid-scale race (3 vehicles on a
1.2 km x 12 m synthetic track, N = 40, K = 16384 samples per best response,
5 IBR sweeps): setup, initialisation, 5 Jacobi sweeps and the extra ego response
(19 best responses = 12.45 M sample-steps), then every vehicle applies its first
control through the vehicle model.  Inputs are resident on the GPU before the
timed region.  Prints one JSON line.

Other workloads (--workload): c3 (large field), c4 (256 batched races), c5 (learned
proposal), race (closed-loop race evaluation, full size), race_small (the same at the
paper's scale: kinematic bicycle, K = 128, H = 12).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sample·steps/s per IBR sweep; plan latency p50/p99; learned vs plain cost"
PEAK_FP32_TFLOPS = 157.3  # MI355X published FP32 vector peak

# Hardware counters of the dominant sweep kernel at the mid-scale race (k_sweep in its
# split variant, two waves per sample), medians over the timed eager launches of
# `bench.py --steps 5 --warmup 1 --no-cpu-baseline --no-learned --roofline-steps 2
# --copy-calibration 256` under rocprofv3 --pmc, weighted like the timed launches (6
# all-vehicle sweeps, 1 ego sweep per planning step).  HBM bytes: FETCH_SIZE 460.0 KiB x
# 2.000 + WRITE_SIZE 321.2 KiB x 1.000 per launch, the factors being
# 256 MiB over what the same counter reads for the 256 MiB elementwise copy (131087 KiB
# fetched, 262144 KiB written).  FP32 FLOPs: 64 x (ADD + MUL + TRANS + 2 FMA) wave
# instructions of SQ_INSTS_VALU_*_F32.  They describe the kernel source with this SHA-256
# only; any other source reports null.
SWEEP_COUNTERS = {
    "c2": {"source_sha256": "693eb70a80538a91de084ea1e8c13ffb07b6111bdf2748c5af08dee5ff65c652",
           "hbm_bytes_per_launch": (460.062 * 1.99976 + 321.237) * 1024.0,
           "hw_fp32_flop_per_launch": 1.2483e9, "valu_wave_insts_per_launch": 22.02e6},
}

def _source_sha256() -> str:
    import hashlib
    with open(os.path.join(ROOT, "paper_2607_25388_amd", "csrc", "sgtp.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def flops_per_sample_step(n_opp: int, model: int = 0) -> float:
    """Algorithmic float operations per sample and horizon step (elementary functions count 1).

    noise (Box-Muller pair: log series, sqrt, sin/cos series)      50
    perturbation and clip of (a, delta)                             8
    sin/cos of delta                                                2
    RK4: 4 derivative evaluations of the single-track model x 45,
         stage states 36, update 42, speed clamp 1                259
    Frenet projection: ~3 normal-line tests x 5 + foot 60          75
    tracking, control and control-rate cost                        33
    boundary clearance                                              4
    footprint screening per opponent                                6 n_opp
    tail lateral sum                                                2
    Disc-pair distances beyond the screening are not counted.
    """
    per = 50 + 8 + 2 + 259 + 75 + 33 + 4 + 2 + 6 * n_opp
    if model == 1:
        per -= 4 * (45 - 12)  # kinematic derivative ~12 FLOP
    return float(per)


def cpu_baseline(name: str, seconds: float = 10.0, K_sample: int = 2048):
    """Oracle (float64 C, OpenMP over samples) on this host: planning steps of the same race at a
    reduced K, repeated for about `seconds`; rate in sample-steps/s (linear in K)."""
    import numpy as np
    import oracle
    from paper_2607_25388_amd import inputs

    w = inputs.WORKLOADS[name]
    tr, race, params = inputs.workload_inputs(name)
    orc = oracle.Oracle(tr, params)
    per_step = ((w.L_ibr + 1) * w.n_agents + 1) * K_sample * w.N
    t0 = time.perf_counter()
    done = 0
    x = race.x.copy()
    u_nom = race.u_nom.astype(np.float64)
    s_prev = race.s_abs.copy()
    step = 0
    while True:
        out = orc.plan_step(race, w.L_ibr, K=K_sample, x=x, u_nom=u_nom, s_prev=s_prev, plan_step=step)
        done += per_step
        x = orc.advance(x, out["u_apply"])
        u_nom = out["u_next"]
        s_prev = out["s_abs"]
        step += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        cores = min(cores, int(omp))
    return dict(value=done / el, unit="sample·steps/s", cores=cores, kind="oracle",
                sample=f"{step} closed-loop planning steps of {name} at K={K_sample} per best response "
                       f"({per_step} sample-steps each), {el:.1f} s")


def _latency(plan, steps, warmup=10):
    """p50 / p99 / mean of planning-step latency [ms] (HIP events on the launch stream)."""
    import numpy as np
    import torch
    st = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.run()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(st)
        plan.run()
        b.record(st)
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)), "mean": float(lat.mean())}


def learned_block(planner, n_examples: int, iters: int, eval_races: int = 32, lat_steps: int = 100):
    """Learned proposal against the plain sampler on races of the mid-scale kind with N = 50:
    train the network on the plain planner's own selections (closed loop, 256 races), then on
    held-out races compare the selected best-response cost at K/4 (7/8 of them from the
    proposal, 1/8 about the nominal) with the plain planner at K and at K/4, and time planning steps
    of the held-out batch and of one 3-vehicle race, plain at K against learned at K/4 (the
    network's features, forward pass and tables run inside the captured step)."""
    import numpy as np
    import torch
    import paper_2607_25388_amd.sgtp as sg
    from paper_2607_25388_amd import inputs, learned

    K, N, L = 16384, 50, 5
    K_PROP = 7 * K // 32  # of the K/4 samples, 7/8 from the proposal, 1/8 about the nominal
    t0 = time.perf_counter()
    tr, races, params = inputs.learned_races(256, 5000, N=N)
    planner.upload_track(7, tr)
    rts = [sg.race_from_inputs(r, 7, K, N, params["n_tail"]) for r in races]
    per_step = sum(r.n_agents for r in rts)
    steps = max(1, -(-n_examples // per_step))
    data = learned.collect(planner, params, rts, L, steps)
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    del rts
    mlp = sg.Mlp(4096, seed=1)
    t1 = time.perf_counter()
    losses = learned.train(mlp, data, params, iters, batch=4096, lr=1e-3, log_every=max(1, iters // 4))
    losses += learned.train(mlp, data, params, iters // 2, batch=4096, lr=3e-4, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    n_ex = int(data.X.shape[0])
    del data

    _, hold, _ = inputs.learned_races(eval_races, 1_000_000, N=N)
    rts = [sg.race_from_inputs(r, 7, K, N, params["n_tail"]) for r in hold]
    plan = planner.plan(params, rts, L, sg.plan_options(include_advance=1), trace=False)
    rec = {"K": [], "K4": [], "L4": []}
    for step in range(30):
        plan.run()
        if step % 6 != 5:
            continue
        rec["K"].append(learned.best_response_costs(planner, params, rts, K))
        rec["K4"].append(learned.best_response_costs(planner, params, rts, K // 4))
        rec["L4"].append(learned.best_response_costs(planner, params, rts, K // 4, K_PROP, mlp))
    plan.close()
    cat = {k: (np.concatenate([c for c, f in v]), np.concatenate([f for c, f in v])) for k, v in rec.items()}
    gp, sp = learned.cost_gap(*cat["K4"], *cat["K"])
    gl, sl = learned.cost_gap(*cat["L4"], *cat["K"])

    def timed(batch, Kv, Kp):
        rr = [sg.race_from_inputs(r, 7, Kv, N, params["n_tail"]) for r in batch]
        if Kp:
            learned.ensure_tables(rr, Kp)
        # one workgroup per tile: the dispatcher then picks the latency variants for small grids
        pl = planner.plan(params, rr, L, sg.plan_options(persistent=0, include_advance=1), trace=False)
        if Kp:
            pl.set_proposal(mlp)
        out = _latency(pl, lat_steps)
        pl.close()
        return out

    lat = {"batch": {"races": len(hold), "plain_K": timed(hold, K, 0), "learned_K4": timed(hold, K // 4, K_PROP)},
           "single": {"vehicles": hold[1].n_agents, "plain_K": timed(hold[1:2], K, 0),
                      "learned_K4": timed(hold[1:2], K // 4, K_PROP)}}
    mlp.close()
    return {
        "workload": (f"learned proposal: 256 training races (2-5 vehicles, 1.2 km x 12 m track, N={N}, K={K}, "
                     f"{L} IBR sweeps), {n_ex} selected sequences; {eval_races} held-out races, best responses "
                     f"at 5 closed-loop instants"),
        "train": {"examples": n_ex, "collect_s": t_collect, "adam_iters": iters + iters // 2, "batch": 4096,
                  "train_s": t_train, "loss_first": losses[0], "loss_last": losses[-1]},
        "cost": {"cases": int(len(gl)), "plain_K4_mean_gap": float(gp.mean()), "plain_K4_sum_gap": sp,
                 "learned_K4_mean_gap": float(gl.mean()), "learned_K4_sum_gap": sl,
                 "learned_K4_not_worse_frac": float(np.mean(gl <= 0.0)),
                 "reference": "plain sampler at K, same states and noise stream"},
        "latency_ms": lat,
    }


def _races_for(name, sg, inputs, planner):
    """Device races, parameters, L and per-plan-step sample-steps of a workload."""
    if name == "c4":
        tracks, races, specs, params = inputs.batched_workload(256)
        tid = {20: 10, 40: 11, 50: 12}
        for N, tr in tracks.items():
            planner.upload_track(tid[N], tr)
        rts = [sg.race_from_inputs(rc, tid[sp["N"]], sp["K"], sp["N"], inputs.n_tail_from_fraction(0.3, sp["N"]))
               for rc, sp in zip(races, specs)]
        L = 5
        per_step = sum(((L + 1) * sp["n_agents"] + 1) * sp["K"] * sp["N"] for sp in specs)
        desc = ("c4: 256 seeded races, 2-10 vehicles (uniform), K in {4096, 16384, 65536}, N in {20, 40, 50}, "
                "5 IBR sweeps + init + extra ego per race, 3-disc footprint, one launch per sweep covering every "
                "race, hipGraph planning step, autotuned schedule, closed loop")
        return rts, params, L, per_step, desc, sum(sp["n_agents"] for sp in specs)
    w = inputs.WORKLOADS[name]
    tr, race, params = inputs.workload_inputs(name)
    planner.upload_track(0, tr)
    rt = sg.race_from_inputs(race, 0, w.K, w.N, params["n_tail"])
    L = w.L_ibr
    per_step = ((L + 1) * w.n_agents + 1) * w.K * w.N
    desc = (f"{name}: {w.n_agents} vehicles, {w.track_length:.0f} m x {w.track_width:.0f} m seeded track, "
            f"N={w.N}, K={w.K} per best response, {L} IBR sweeps + init + extra ego, {w.n_disc}-disc footprint, "
            "hipGraph planning step, closed loop")
    return [rt], params, L, per_step, desc, w.n_agents


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--mode", choices=["graph", "eager"], default="graph")
    ap.add_argument("--no-autotune", action="store_true", help="skip the schedule search (default schedule)")
    ap.add_argument("--schedule", default="", metavar="P,B,C,S",
                    help="fixed schedule instead of the search: persistent, blocks per CU, tiles per fetch, "
                         "samples per lane")
    ap.add_argument("--roofline-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal comparison")
    ap.add_argument("--learned-examples", type=int, default=100000,
                    help="training examples of the learned proposal (the c5 workload uses 1e6)")
    ap.add_argument("--learned-iters", type=int, default=4000)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the timed region, one elementwise copy of MIB MiB (reads and writes MIB MiB): "
                         "the reference kernel for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this planner runs on a single device (see the design notes for how "
              "races, vehicles and samples would be spread over several GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2607_25388_amd.sgtp as sg
    from paper_2607_25388_amd import inputs

    name = args.workload
    planner = sg.Planner(max_agents_total=2048, max_races=256)
    if name in ("race", "race_small"):
        # closed-loop race evaluation of the planner variants (Sec. IV-C metrics, Table I)
        from paper_2607_25388_amd import race_eval
        planner.close()
        scale = "full" if name == "race" else "small"
        sc = race_eval.SCALES[scale]
        n_games = 7 * 6 * 3
        rp = sg.Planner(max_agents_total=n_games * 3, max_races=n_games, max_K=sc["K"])
        rp.enable_path_integral()
        res = race_eval.evaluate(rp, race_eval.METHODS, 7, 6, T_max=50.0, scale=scale,
                                 log=lambda m: print(m, file=sys.stderr, flush=True))
        rp.close()
        if scale == "full":
            desc = ("race evaluation: 42 trials (7 seeded 1.2 km x 12 m tracks x 6 starts), 3 vehicles (ego "
                    "rearmost, opponents at 0.9 reference speed), every vehicle plans its own game (dynamic "
                    "single-track model, 3 discs, N=40, K=4096, 5 IBR sweeps), 50 s, all 126 games batched in "
                    "one plan per step")
        else:
            desc = ("race evaluation at the paper's scale: 42 trials (7 seeded 150 m x 2.5 m twisty tracks x 6 "
                    "starts), 3 vehicles queued 2 m apart (ego rearmost, opponents at 0.9 reference speed), "
                    "kinematic bicycle, point footprint (d_col 0.9 m), every vehicle plans its own game (N=12 "
                    "over 1.2 s, K=128, 2 IBR sweeps), 50 s, a collision is contact of 0.58 m x 0.31 m bodies, "
                    "all 126 games batched in one plan per step")
        rec = {"metric": METRIC, "value": res["sgtp"]["wins"], "unit": "win rate", "n_gpus": 1,
               "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": desc}, "race_eval": res}
        print(json.dumps(rec), flush=True)
        return
    if name == "c5":
        rec = {"metric": METRIC, "unit": "relative selected cost", "n_gpus": 1, "higher_is_better": False,
               "vs_baseline": None, "dtype": "f32 planner, bf16 network (f32 accumulation)", "data": "synthetic"}
        lb = learned_block(planner, max(args.learned_examples, 1000000), max(args.learned_iters, 20000),
                           eval_races=64)
        rec.update({"value": lb["cost"]["learned_K4_mean_gap"], "config": {"workload": lb["workload"]},
                    "learned": lb})
        planner.close()
        print(json.dumps(rec), flush=True)
        return
    rts, params, L, per_step, desc, n_total = _races_for(name, sg, inputs, planner)
    stream = torch.cuda.current_stream()
    opts = sg.plan_options(include_advance=1)
    tuned = None
    if args.schedule:
        pp, bb, cc, ss = (int(x) for x in args.schedule.split(","))
        opts = sg.plan_options(persistent=pp, blocks_per_cu=bb, tiles_per_fetch=cc, samples_per_lane=ss,
                               include_advance=1)
    elif not args.no_autotune:
        best, ms = planner.autotune(params, rts, L)
        best.include_advance = 1
        opts = best
        tuned = dict(best.as_dict(), plan_ms=ms)
    if args.mode == "eager":
        opts.use_graph = 0
    plan = planner.plan(params, rts, L, opts, trace=False)

    for i in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        plan.run()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    for r in rts:
        assert np.all(np.isfinite(r.x.cpu().numpy())), "non-finite state"
    info = plan.info()
    plan.close()

    # sweep-kernel duration: the same planning steps launched eagerly with HIP events
    # recorded on the launch stream around every sweep launch
    eager = sg.plan_options(**dict(opts.as_dict(), use_graph=0, include_advance=1))
    eplan = planner.plan(params, rts, L, eager, trace=False)
    planner.sweep_stats(reset=True)
    planner.set_timing(True)
    for i in range(args.roofline_steps):
        eplan.run()
    torch.cuda.synchronize()
    planner.set_timing(False)
    eplan.close()
    sweep_ms, sweep_launches, sweep_ss = planner.sweep_stats(reset=True)
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    value = per_step * args.steps / el
    avg_sweep_ms = sweep_ms / max(1, sweep_launches)
    n_opp = max(r.n_agents for r in rts) - 1 if name != "c4" else 5
    flops = flops_per_sample_step(n_opp, params["model"])
    achieved = flops * (sweep_ss / max(1, sweep_launches)) / (avg_sweep_ms * 1e-3) / 1e12
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "sample·steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "sample_steps_per_plan_step": per_step, "vehicles": n_total,
                   "mode": args.mode, "schedule": opts.as_dict(), "sweep_grid": info},
        "plan_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                            "mean": float(lat.mean())},
        "sweep_kernel": {"launches": sweep_launches, "avg_ms": avg_sweep_ms,
                         "sample_steps_per_launch": sweep_ss / max(1, sweep_launches),
                         "timing": "HIP events on the launch stream, eager replay of the same planning step"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "flops_per_sample_step": flops},
    }
    cnt = SWEEP_COUNTERS.get(name)
    if cnt and cnt["source_sha256"] == _source_sha256():
        rec["roofline"]["traffic"] = cnt["hbm_bytes_per_launch"]
        rec["roofline"]["traffic_unit"] = "bytes per sweep launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)"
        rec["roofline"]["hw_fp32_tflops"] = cnt["hw_fp32_flop_per_launch"] / (avg_sweep_ms * 1e-3) / 1e12
        rec["roofline"]["hbm_gbps"] = cnt["hbm_bytes_per_launch"] / (avg_sweep_ms * 1e-3) / 1e9
    if tuned:
        rec["config"]["autotune"] = tuned
    if not args.no_learned:
        rec["learned"] = learned_block(planner, args.learned_examples, args.learned_iters)
    if not args.no_cpu_baseline and name != "c4":
        rec["cpu_baseline"] = cpu_baseline(name, args.cpu_seconds)
    planner.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
