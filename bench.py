"""Benchmark of the SGTP planning step on one MI355X.

A step is one closed-loop planning step of the batched workload: 256 seeded races with
2-10 vehicles each (uniform), K in {4096, 16384, 65536} samples per best response and
horizons N in {20, 40, 50}, 5 IBR sweeps + initialisation + extra ego response per race
(Alg. 1), every race of the batch in one launch per sweep, the planning step and the
closed-loop advance captured in one hipGraph (about 9.9e9 sample-steps per step).  Inputs
are resident on the GPU before the timed region.  Prints one JSON line, which also holds
the mid-scale race (c2) and the large field (c3) as extra entries, the learned proposal
against the plain sampler at the learned-proposal workload's size, and the CPU oracle
timed on a sample of the same workload.

Other workloads (--workload): c1, c2, c3 alone, c5 (learned proposal only), mlp (the
proposal network's matrix-core timings), race (closed-loop race evaluation, full size),
race_small (the same at the paper's scale: kinematic bicycle, K = 128, H = 12).
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

# Hardware counters of the dominant sweep kernel, means per launch over every launch of
# that kernel in `bench.py --workload W ... --copy-calibration 256` under rocprofv3 --pmc
# (one counter group per run; commands and tables in profiles/sweep_<W>_counters.md):
# c4 k_sweep<0, 3, 9, 0, 1, 0> (one workgroup per tile of 2 x 256 samples), c3 the same
# kernel with one sample per lane and k_sweep_persistent<0, 3, 9> (one record per schedule),
# c2 k_sweep<0, 3, 3, 6, 1, 1> (split variant).  HBM bytes =
# 2.000 x FETCH_SIZE + 1.000 x WRITE_SIZE (KiB), the factors being 256 MiB over what each
# counter reads for the 256 MiB elementwise copy of the same runs (131087.5-131091.5 KiB
# fetched, 262144 KiB written).  FP32 FLOPs = 64 x SQ_INSTS_VALU_FLOPS_FP32, which counts ADD + MUL +
# TRANS + 2 FMA wave instructions (checked on the known-mix kernel of --counter-probe,
# profiles/counter_probe_fp32.md).  They describe the kernel source with this SHA-256 and
# the listed schedule fields only; anything else reports null.
_SRC = "c421a252ca21e8a5f1751fb601b572e87825a5350e304be1ac9bedfc9a12d3ff"
SWEEP_COUNTERS = {
    "c4": [{"source_sha256": _SRC, "hbm_bytes_per_launch": (16584.821 * 1.99977 + 118349.394) * 1024.0,
            "hw_fp32_flop_per_launch": 64 * 14070694659.9, "valu_wave_insts_per_launch": 14309969213.1,
            "schedule": {"persistent": 0, "tiles_per_fetch": 1, "samples_per_lane": 2}}],
    "c3": [{"source_sha256": _SRC, "hbm_bytes_per_launch": (525.500 * 1.99977 + 1799.415) * 1024.0,
            "hw_fp32_flop_per_launch": 64 * 284971384.1, "valu_wave_insts_per_launch": 292403205.4,
            "schedule": {"persistent": 0, "tiles_per_fetch": 1, "samples_per_lane": 1}},
           {"source_sha256": _SRC, "hbm_bytes_per_launch": (6430.919 * 1.99977 + 59507.453) * 1024.0,
            "hw_fp32_flop_per_launch": 64 * 284633401.6, "valu_wave_insts_per_launch": 291140176.1,
            "schedule": {"persistent": 1, "tiles_per_fetch": 1, "samples_per_lane": 1}}],
    "c2": [{"source_sha256": _SRC, "hbm_bytes_per_launch": (376.493 * 1.99977 + 309.205) * 1024.0,
            "hw_fp32_flop_per_launch": 64 * 16737196.9, "valu_wave_insts_per_launch": 19342399.3,
            "schedule": {"samples_per_lane": 1}}],
}


def _source_sha256() -> str:
    import hashlib
    with open(os.path.join(ROOT, "paper_2607_25388_amd", "csrc", "sgtp.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


# Algorithmic FLOP per sample and horizon step, counted by the oracle compiled with an
# operation-counting scalar type (oracle/opcount.cpp; this table is what `python -m
# oracle.opcount` prints, and a CPU test checks that it is current): add, mul, compare/min/max
# 1 each, fma 2, and each elementary operation (div, sqrt, sin, cos, atan, remainder) 1, in
# float64 (rollout, projection, scoring) and float32 (the Box-Muller specification).  The
# footprint term counts every disc pair of every opponent at every step, as the method
# defines it; the kernels skip pairs whose centres are too far apart to matter.  Keys: the
# named workloads (vehicle 0, sweep phase), and "n_opp,N" for the batched workload's races
# (3 discs, dynamic single-track model).
FLOP_PER_SAMPLE_STEP = {
    "c1": 448.5,
    "c2": 580.0,
    "c3": 1027.7,
    "batched (n_opp,N)": {
        "1,20": 515.0,
        "2,20": 576.2,
        "3,20": 641.9,
        "4,20": 705.9,
        "5,20": 769.1,
        "6,20": 832.7,
        "7,20": 897.1,
        "8,20": 961.0,
        "9,20": 1024.3,
        "1,40": 523.1,
        "2,40": 587.6,
        "3,40": 649.6,
        "4,40": 714.7,
        "5,40": 776.9,
        "6,40": 837.6,
        "7,40": 901.5,
        "8,40": 967.3,
        "9,40": 1030.5,
        "1,50": 525.5,
        "2,50": 588.7,
        "3,50": 652.2,
        "4,50": 715.3,
        "5,50": 778.8,
        "6,50": 841.5,
        "7,50": 905.1,
        "8,50": 968.0,
        "9,50": 1031.4
    }
}


def flop_per_sample_step(name: str, n_opp: int = 0, N: int = 0) -> float:
    if name in FLOP_PER_SAMPLE_STEP:
        return FLOP_PER_SAMPLE_STEP[name]
    return FLOP_PER_SAMPLE_STEP["batched (n_opp,N)"][f"{n_opp},{N}"]


def _set_cpu_threads(n):
    """OpenMP threads of the oracle (0 = the runtime's default) through libgomp, which the
    oracle's library loads; returns the number that will run."""
    import ctypes as C
    gomp = C.CDLL("libgomp.so.1")
    if n:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def cpu_baseline(name: str, seconds: float = 10.0, K_sample: int = 2048, threads: int = 0):
    """Oracle (float64 C, OpenMP over samples) on this host: closed-loop planning steps of
    the workload at a reduced K, repeated for about `seconds`; rate in sample-steps/s (the
    work per sample does not depend on K).  For the batched workload (c4) the sample is
    its first 8 races (2-10 vehicles, N 20/40/50), planned one after the other."""
    import numpy as np
    import oracle
    from paper_2607_25388_amd import inputs

    if name == "c4":
        tracks, races, specs, params = inputs.batched_workload(256)
        items = []
        for rc, sp in list(zip(races, specs))[:8]:
            p = dict(params, N=sp["N"], n_tail=inputs.n_tail_from_fraction(0.3, sp["N"]))
            items.append((oracle.Oracle(tracks[sp["N"]], p), rc, 5, sp["N"]))
        what = f"the first 8 races of the batched workload at K={K_sample}"
    else:
        w = inputs.WORKLOADS[name]
        tr, race, params = inputs.workload_inputs(name)
        items = [(oracle.Oracle(tr, params), race, w.L_ibr, w.N)]
        what = f"{name} at K={K_sample}"
    prev = _set_cpu_threads(0)
    cores = _set_cpu_threads(threads)
    state = [dict(x=rc.x.copy(), u=rc.u_nom.astype(np.float64), s=rc.s_abs.copy()) for _, rc, _, _ in items]
    t0 = time.perf_counter()
    done = 0
    step = 0
    while True:
        for (orc, rc, L, N), st in zip(items, state):
            out = orc.plan_step(rc, L, K=K_sample, x=st["x"], u_nom=st["u"], s_prev=st["s"], plan_step=step)
            done += ((L + 1) * rc.n_agents + 1) * K_sample * N
            st["x"] = orc.advance(st["x"], out["u_apply"])
            st["u"] = out["u_next"]
            st["s"] = out["s_abs"]
        step += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    _set_cpu_threads(prev)
    return dict(value=done / el, unit="sample·steps/s", cores=cores, kind="oracle",
                sample=f"{step} closed-loop planning steps of {what} per best response, {done:.3g} sample-steps, "
                       f"{el:.1f} s, {cores} OpenMP threads")


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


PEAK_BF16_TFLOPS = 2500.0  # MI355X published dense BF16 matrix peak
PEAK_HBM_GBPS = 8000.0


def _progress(msg: str):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _events_ms(fn, reps: int) -> float:
    """Mean milliseconds of fn() over reps launches, HIP events on the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def mfma_block(mlp, data, params) -> dict:
    """Matrix-core use of the proposal network: one training step (graph replay of gather,
    gradient and Adam at 4096 rows), its largest products alone, and the forward pass at
    planning and at large batch.  FLOPs are the products' 2 M N K; bytes the BF16 operands
    read once and the float32 result written once."""
    import torch
    import paper_2607_25388_amd.sgtp as sg
    from paper_2607_25388_amd import learned
    out = {}
    tr = learned.Trainer(mlp, data, params, batch=4096, lr=1e-4, seed=99, graph=True)
    ms = _events_ms(tr.step, 50)
    tr.close()
    flop = learned.TRAIN_FLOP_PER_ROW * 4096
    out["train_step"] = {"rows": 4096, "ms": ms, "flop": flop, "tflops": flop / ms / 1e9,
                         "mfma_frac": flop / ms / 1e9 / PEAK_BF16_TFLOPS,
                         "timing": "HIP events over 50 graph replays (index draw + gather + gradient + Adam)"}

    def gemm_case(M, N, K):
        A = torch.randn((M, K), device="cuda").to(torch.bfloat16)
        B = torch.randn((K, N), device="cuda").to(torch.bfloat16)
        C = torch.empty((M, N), device="cuda")
        ms = _events_ms(lambda: sg.gemm_bf16(A, (K, 1), B, (N, 1), M, N, K, out=C), 20)
        fl, by = 2.0 * M * N * K, 2.0 * (M * K + K * N) + 4.0 * M * N
        return {"M": M, "N": N, "K": K, "ms": ms, "tflops": fl / ms / 1e9, "mfma_frac": fl / ms / 1e9 / PEAK_BF16_TFLOPS,
                "hbm_gbps": by / ms / 1e6, "hbm_frac": by / ms / 1e6 / PEAK_HBM_GBPS,
                "roof": "hbm" if fl / by < PEAK_BF16_TFLOPS / PEAK_HBM_GBPS * 1e3 else "mfma"}

    out["gemm"] = [gemm_case(4096, 256, 256), gemm_case(65536, 256, 256), gemm_case(16384, 1024, 1024)]
    fwd = {}
    for rows in (1536, 65536):
        X = torch.randn((rows, 50), device="cuda")
        Y = torch.empty((rows, 200), device="cuda")
        ms = _events_ms(lambda: mlp.forward(X, out=Y), 20)
        fl = rows * 2.0 * (50 * 256 + 256 * 256 + 256 * 200)
        fwd[str(rows)] = {"ms": ms, "tflops": fl / ms / 1e9, "mfma_frac": fl / ms / 1e9 / PEAK_BF16_TFLOPS,
                          "kernel": "fused three-layer" if rows <= 4096 else "tiled products"}
    out["forward"] = fwd
    return out


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
    _progress(f"learned: {int(data.X.shape[0])} training sequences collected in {t_collect:.1f} s")
    del rts
    mlp = sg.Mlp(4096, seed=1)
    t1 = time.perf_counter()
    losses = learned.train(mlp, data, params, iters, batch=4096, lr=1e-3, log_every=max(1, iters // 4))
    losses += learned.train(mlp, data, params, iters // 2, batch=4096, lr=3e-4, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    n_ex = int(data.X.shape[0])
    _progress(f"learned: {iters + iters // 2} Adam steps in {t_train:.1f} s")
    big = sg.Mlp(65536, mlp.get_params())
    mfma = mfma_block(big, data, params)
    big.close()
    _progress("learned: matrix-core timings done")
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
    _progress("learned: held-out best responses done")
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
                  "train_s": t_train, "loss_first": losses[0], "loss_last": losses[-1],
                  "step": "graph replay of gather, gradient and Adam"},
        "mfma_frac": mfma["train_step"]["mfma_frac"],
        "mfma": mfma,
        "cost": {"cases": int(len(gl)), "plain_K4_mean_gap": float(gp.mean()), "plain_K4_sum_gap": sp,
                 "learned_K4_mean_gap": float(gl.mean()), "learned_K4_sum_gap": sl,
                 "learned_K4_not_worse_frac": float(np.mean(gl <= 0.0)),
                 "reference": "plain sampler at K, same states and noise stream"},
        "latency_ms": lat,
    }


def _races_for(name, sg, inputs, planner):
    """Device races, parameters, L, per-plan-step sample-steps and algorithmic FLOP of a workload."""
    if name == "c4":
        tracks, races, specs, params = inputs.batched_workload(256)
        tid = {20: 10, 40: 11, 50: 12}
        for N, tr in tracks.items():
            planner.upload_track(tid[N], tr)
        rts = [sg.race_from_inputs(rc, tid[sp["N"]], sp["K"], sp["N"], inputs.n_tail_from_fraction(0.3, sp["N"]))
               for rc, sp in zip(races, specs)]
        L = 5
        per_step = sum(((L + 1) * sp["n_agents"] + 1) * sp["K"] * sp["N"] for sp in specs)
        flop = sum(((L + 1) * sp["n_agents"] + 1) * sp["K"] * sp["N"] *
                   flop_per_sample_step("c4", sp["n_agents"] - 1, sp["N"]) for sp in specs)
        desc = ("c4: 256 seeded races, 2-10 vehicles (uniform), K in {4096, 16384, 65536}, N in {20, 40, 50}, "
                "5 IBR sweeps + init + extra ego per race, 3-disc footprint, one launch per sweep covering every "
                "race, hipGraph planning step, autotuned schedule, closed loop")
        return rts, params, L, per_step, flop, desc, sum(sp["n_agents"] for sp in specs)
    w = inputs.WORKLOADS[name]
    tr, race, params = inputs.workload_inputs(name)
    planner.upload_track(0, tr)
    rt = sg.race_from_inputs(race, 0, w.K, w.N, params["n_tail"])
    L = w.L_ibr
    per_step = ((L + 1) * w.n_agents + 1) * w.K * w.N
    desc = (f"{name}: {w.n_agents} vehicles, {w.track_length:.0f} m x {w.track_width:.0f} m seeded track, "
            f"N={w.N}, K={w.K} per best response, {L} IBR sweeps + init + extra ego, {w.n_disc}-disc footprint, "
            "hipGraph planning step, closed loop")
    return [rt], params, L, per_step, per_step * flop_per_sample_step(name), desc, w.n_agents


def measure(planner, name: str, steps: int, warmup: int, roofline_steps: int, mode: str = "graph",
            autotune: bool = True, schedule: str = ""):
    """Timed closed-loop planning steps of one workload (graph replays), the sweep kernel's
    launch durations over eager replays of the same steps, and its roofline numbers."""
    import numpy as np
    import torch
    import paper_2607_25388_amd.sgtp as sg
    from paper_2607_25388_amd import inputs

    rts, params, L, per_step, flop_step, desc, n_total = _races_for(name, sg, inputs, planner)
    stream = torch.cuda.current_stream()
    opts = sg.plan_options(include_advance=1)
    tuned = None
    if schedule:
        pp, bb, cc, ss = (int(x) for x in schedule.split(","))
        opts = sg.plan_options(persistent=pp, blocks_per_cu=bb, tiles_per_fetch=cc, samples_per_lane=ss,
                               include_advance=1)
    elif autotune:
        best, ms = planner.autotune(params, rts, L)
        best.include_advance = 1
        opts = best
        tuned = dict(best.as_dict(), plan_ms=ms)
    if mode == "eager":
        opts.use_graph = 0
    plan = planner.plan(params, rts, L, opts, trace=False)
    for _ in range(warmup):
        plan.run()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
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

    # sweep-kernel durations: the same planning steps launched eagerly, HIP events recorded
    # on the launch stream around every sweep launch
    eager = sg.plan_options(**dict(opts.as_dict(), use_graph=0, include_advance=1))
    eplan = planner.plan(params, rts, L, eager, trace=False)
    planner.sweep_stats(reset=True)
    planner.set_timing(True)
    for _ in range(roofline_steps):
        eplan.run()
    torch.cuda.synchronize()
    planner.set_timing(False)
    eplan.close()
    sweep_ms, sweep_launches, sweep_ss = planner.sweep_stats(reset=True)
    status = planner.status()
    if status:
        raise RuntimeError(f"kernel status word {status}: {planner.lib.sgtp_last_error(planner.ctx).decode()}")

    flop_per_ss = flop_step / per_step
    achieved = flop_per_ss * sweep_ss / (sweep_ms * 1e-3) / 1e12
    rec = {
        "value": per_step * steps / el,
        "ms_per_step": el / steps * 1e3,
        "config": {"workload": desc, "sample_steps_per_plan_step": per_step, "vehicles": n_total, "mode": mode,
                   "schedule": opts.as_dict(), "sweep_grid": info},
        "plan_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                            "mean": float(lat.mean())},
        "sweep_kernel": {"launches": sweep_launches, "avg_ms": sweep_ms / max(1, sweep_launches),
                         "sample_steps_per_launch": sweep_ss / max(1, sweep_launches),
                         "timing": "HIP events on the launch stream, eager replay of the same planning steps"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "flop_per_sample_step": flop_per_ss,
                     "flop_count": "oracle op count per sample-step (FLOP_PER_SAMPLE_STEP), weighted by the "
                                   "sample-steps of each race"},
    }
    sched = rec["config"].get("schedule", {})
    cnt = next((c for c in SWEEP_COUNTERS.get(name, []) if c["source_sha256"] == _source_sha256() and
                all(sched.get(k) == v for k, v in c["schedule"].items())), None)
    if cnt:
        avg_s = sweep_ms * 1e-3 / max(1, sweep_launches)
        rec["roofline"]["traffic"] = cnt["hbm_bytes_per_launch"]
        rec["roofline"]["traffic_unit"] = "bytes per sweep launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)"
        rec["roofline"]["hw_fp32_tflops"] = cnt["hw_fp32_flop_per_launch"] / avg_s / 1e12
        rec["roofline"]["hbm_gbps"] = cnt["hbm_bytes_per_launch"] / avg_s / 1e9
        rec["roofline"]["valu_insts_per_sample_step"] = cnt["valu_wave_insts_per_launch"] * 64.0 / (
            sweep_ss / max(1, sweep_launches))
    if tuned:
        rec["config"]["autotune"] = tuned
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--mode", choices=["graph", "eager"], default="graph")
    ap.add_argument("--no-autotune", action="store_true", help="skip the schedule search (default schedule)")
    ap.add_argument("--schedule", default="", metavar="P,B,C,S",
                    help="fixed schedule instead of the search: persistent, blocks per CU, tiles per fetch, "
                         "samples per lane")
    ap.add_argument("--roofline-steps", type=int, default=5)
    ap.add_argument("--no-extra", action="store_true", help="skip the c2 and c3 entries of the default line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal comparison")
    ap.add_argument("--learned-examples", type=int, default=1000000,
                    help="training sequences of the learned proposal (the learned-proposal workload's 1e6)")
    ap.add_argument("--learned-iters", type=int, default=20000)
    ap.add_argument("--counter-probe", default="", metavar="WAVES,ITERS",
                    help="only run the known-mix FP32 kernel (for checking counter formulas under rocprofv3) "
                         "and print the instruction counts it must produce")
    ap.add_argument("--issue-probe", default="", metavar="BLOCKS,ITERS",
                    help="only run the issue-class probe kernels (fma with vector or scalar operands, min, sin, mul, "
                         "xor, cndmask, med3, mad_u64_u32) "
                         "for reading which instructions the SIMDs pair (SQ_ACTIVE_INST_VALU2 under rocprofv3)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the timed region, one elementwise copy of MIB MiB (reads and writes MIB MiB): "
                         "the reference kernel for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this planner runs on a single device (see the design notes for how "
              "races, vehicles and samples would be spread over several GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2607_25388_amd.sgtp as sg

    if args.counter_probe:
        waves, iters = (int(x) for x in args.counter_probe.split(","))
        for _ in range(3):
            sg.counter_probe_fp32(waves, iters)
        torch.cuda.synchronize()
        exp = {"SQ_INSTS_VALU_ADD_F32": waves * (iters + 3), "SQ_INSTS_VALU_MUL_F32": waves * iters,
               "SQ_INSTS_VALU_FMA_F32": waves * iters, "SQ_INSTS_VALU_TRANS_F32": waves * iters,
               "fp32_flop (64 x (ADD + MUL + TRANS + 2 FMA))": 64 * waves * (5 * iters + 3)}
        print(json.dumps({"counter_probe": {"waves": waves, "iters": iters, "launches": 3,
                                            "expected_per_launch": exp}}), flush=True)
        return
    if args.issue_probe:
        # four waves per SIMD at 1024 workgroups; per kind: one warm-up launch, then two timed
        blocks, iters = (int(x) for x in args.issue_probe.split(","))
        kinds = ("fma, vector operands", "fma, one scalar operand", "min", "sin (transcendental)",
                 "mul, literal", "xor", "cndmask, scalar mask", "med3", "mad_u64_u32")
        out = torch.empty(256 * blocks, dtype=torch.float32, device="cuda")
        res = {}
        for kind, label in enumerate(kinds):
            sg.issue_probe(kind, blocks, iters // 10, out)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            for _ in range(2):
                sg.issue_probe(kind, blocks, iters, out)
            ev[1].record()
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / 2
            simds = 1024  # 256 CUs x 4 SIMDs
            insts = 8.0 * iters * blocks * 4 / simds  # per SIMD
            res[label] = {"ms": ms, "ns_per_wave_instruction_per_simd": ms * 1e6 / insts}
        print(json.dumps({"issue_probe": {"blocks": blocks, "iters": iters, "launches_per_kind": 3,
                                          "results": res}}), flush=True)
        return
    name = args.workload
    base = {"metric": METRIC, "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "data": "synthetic"}
    if name in ("race", "race_small"):
        # closed-loop race evaluation of the planner variants (Sec. IV-C metrics, Table I)
        from paper_2607_25388_amd import race_eval
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
        rec = dict(base, value=res["sgtp"]["wins"], unit="win rate", dtype="f32", config={"workload": desc},
                   race_eval=res)
        print(json.dumps(rec), flush=True)
        return
    if name == "mlp":
        # the proposal network's matrix-core timings alone, on seeded synthetic rows
        from paper_2607_25388_amd import learned
        g = torch.Generator(device="cuda")
        g.manual_seed(5)
        M = 200000
        X = torch.randn((M, 50), device="cuda", generator=g)
        U = torch.stack([torch.rand((M, 50), device="cuda", generator=g) * 12.0 - 8.0,
                         torch.rand((M, 50), device="cuda", generator=g) * 0.8 - 0.4], -1).contiguous()
        mlp = sg.Mlp(65536, seed=1)
        mf = mfma_block(mlp, learned.Dataset(X, U, None, None), {"sigma_a": 1.5, "sigma_d": 0.08})
        mlp.close()
        rec = dict(base, value=mf["train_step"]["mfma_frac"], unit="fraction of BF16 matrix peak (training step)",
                   dtype="bf16 operands, f32 accumulation", config={"workload": "proposal network 50-256-256-200, "
                   "training step of 4096 rows, products and forward passes alone"}, mfma=mf)
        print(json.dumps(rec), flush=True)
        return
    planner = sg.Planner(max_agents_total=2048, max_races=256)
    if name == "c5":
        lb = learned_block(planner, max(args.learned_examples, 1000000), max(args.learned_iters, 20000),
                           eval_races=64)
        rec = dict(base, value=lb["cost"]["learned_K4_mean_gap"], unit="relative selected cost",
                   higher_is_better=False, dtype="f32 planner, bf16 network (f32 accumulation)",
                   config={"workload": lb["workload"]}, learned=lb)
        planner.close()
        print(json.dumps(rec), flush=True)
        return

    m = measure(planner, name, args.steps, args.warmup, args.roofline_steps, args.mode, not args.no_autotune,
                args.schedule)
    _progress(f"{name}: {m['value']:.4g} sample-steps/s, {m['ms_per_step']:.3f} ms per step")
    rec = dict(base, value=m["value"], unit="sample·steps/s", steps=args.steps, warmup=args.warmup,
               ms_per_step=m["ms_per_step"], scaling="weak", dtype="f32", config=m["config"],
               plan_latency_ms=m["plan_latency_ms"], sweep_kernel=m["sweep_kernel"], roofline=m["roofline"])
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if name == "c4" and not args.no_extra:
        # the mid-scale race and the large field, each alone on the GPU (latency and throughput cases)
        rec["workloads"] = {}
        for extra, st in (("c3", 100), ("c2", 200)):
            e = measure(planner, extra, st, 5, 5)
            _progress(f"{extra}: {e['value']:.4g} sample-steps/s")
            rec["workloads"][extra] = {k: e[k] for k in ("value", "ms_per_step", "plan_latency_ms", "sweep_kernel",
                                                         "roofline")}
            rec["workloads"][extra]["config"] = e["config"]["workload"]
    if not args.no_learned:
        rec["learned"] = learned_block(planner, args.learned_examples, args.learned_iters)
    if not args.no_cpu_baseline:
        K_cpu = 256 if name in ("c3", "c4") else 2048
        rec["cpu_baseline"] = cpu_baseline(name, args.cpu_seconds, K_cpu)
        _progress(f"cpu baseline: {rec['cpu_baseline']['value']:.4g} sample-steps/s")
        rec["cpu_baseline_1core"] = cpu_baseline(name, args.cpu_seconds, K_cpu, threads=1)
        _progress(f"cpu baseline, 1 thread: {rec['cpu_baseline_1core']['value']:.4g} sample-steps/s")
    rec["context"] = ("the paper reports 0.095 s mean computation time per planning call (K=128, H=12, 3 vehicles, "
                      "L_IBR=2) on an NVIDIA RTX 4060 (Sec. IV-B, Table I): about 1.1-1.6e5 sample-steps/s; a "
                      "different machine and workload, not the target")
    planner.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
