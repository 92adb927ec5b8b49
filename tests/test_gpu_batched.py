"""GPU: batched plans (many uneven races per launch), persistent sweeps, hipGraph replay,
autotuner.  The per-vehicle computation does not depend on the launch schedule, so every
schedule must give the same bits as planning each race on its own."""

import time

import numpy as np
import pytest

from paper_2607_25388_amd import inputs

pytestmark = pytest.mark.gpu

TRACK_ID = {20: 10, 40: 11, 50: 12}


@pytest.fixture(scope="module")
def planner():
    import paper_2607_25388_amd.sgtp as sg
    p = sg.Planner(max_agents_total=256, max_races=64)
    yield p
    p.close()


def _batch(planner, n_races=7, seed=77):
    import paper_2607_25388_amd.sgtp as sg
    tracks, races, specs, params = inputs.batched_workload(n_races, seed, K_override=lambda sp: [300, 777, 1024][
        sp["race"] % 3])
    for N, tr in tracks.items():
        planner.upload_track(TRACK_ID[N], tr)
    rts = [sg.race_from_inputs(rc, TRACK_ID[sp["N"]], sp["K"], sp["N"], inputs.n_tail_from_fraction(0.3, sp["N"]),
                               plan_step=0) for rc, sp in zip(races, specs)]
    return tracks, races, specs, params, rts


def _fresh(rts):
    import copy
    import torch
    out = []
    for r in rts:
        c = copy.copy(r)
        c.x, c.s_abs, c.u_nom = r.x.clone(), r.s_abs.clone(), r.u_nom.clone()
        c.traj = torch.zeros_like(r.traj)
        out.append(c)
    return out


def _eager_reference(planner, params, rts, L, steps):
    """Each race alone, eager sgtp_plan_step, plan_step = 0..steps-1."""
    import torch
    import paper_2607_25388_amd.sgtp as sg
    res = []
    for r in rts:
        tr_all, u_all = [], []
        for s in range(steps):
            r.plan_step = s
            trace = torch.zeros((L + 2) * r.n_agents * sg.CHOICE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
            u = planner.plan_step(params, [r], L, trace=trace)
            torch.cuda.synchronize()
            tr_all.append(sg.choices_to_numpy(trace).reshape(L + 2, r.n_agents))
            u_all.append(u.cpu().numpy())
        res.append(dict(trace=tr_all, u=u_all, traj=r.traj.cpu().numpy(), u_nom=r.u_nom.cpu().numpy()))
    return res


def _plan_run(planner, params, rts, L, steps, options):
    import torch
    plan = planner.plan(params, rts, L, options)
    traces, us = [], []
    for s in range(steps):
        plan.run()
        torch.cuda.synchronize()
        traces.append(plan.choices().copy())
        us.append(plan.u_apply.cpu().numpy().copy())
        # unrelated eager work between replays
        torch.ones(1024, device="cuda").sum().item()
    info = plan.info()
    plan.close()
    return traces, us, info


def _compare(rts, ref, traces, us, L):
    base = 0
    for r, rr in zip(rts, ref):
        n = r.n_agents
        for s in range(len(traces)):
            for ph in range(L + 2):
                for i in range(n):
                    if ph == L + 1 and i != r.ego:
                        continue
                    g = traces[s][ph, base + i]
                    e = rr["trace"][s][ph, i]
                    assert int(g["k"]) == int(e["k"]) and float(g["cost"]) == float(e["cost"]), (s, ph, i)
            np.testing.assert_array_equal(us[s][base:base + n], rr["u"][s])
        np.testing.assert_array_equal(r.traj.cpu().numpy(), rr["traj"])
        np.testing.assert_array_equal(r.u_nom.cpu().numpy(), rr["u_nom"])
        base += n


@pytest.mark.parametrize("opts", [
    dict(persistent=1, tiles_per_fetch=2, use_graph=1),
    dict(persistent=1, tiles_per_fetch=1, blocks_per_cu=1, use_graph=0),
    dict(persistent=1, tiles_per_fetch=4, samples_per_lane=2, use_graph=1),
    dict(persistent=0, samples_per_lane=2, use_graph=1),
])
def test_batched_plan_is_schedule_invariant(planner, opts):
    import paper_2607_25388_amd.sgtp as sg
    tracks, races, specs, params, rts = _batch(planner)
    L, steps = 2, 2
    ref = _eager_reference(planner, params, _fresh(rts), L, steps)
    mine = _fresh(rts)
    traces, us, info = _plan_run(planner, params, mine, L, steps, sg.plan_options(**opts))
    _compare(mine, ref, traces, us, L)


def test_graph_with_closed_loop_advance(planner):
    """Planning step + advance captured in one graph, replayed; equals the eager loop."""
    import torch
    import paper_2607_25388_amd.sgtp as sg
    tracks, races, specs, params, rts = _batch(planner, 4, 91)
    L, steps = 1, 3
    eager = _fresh(rts)
    for s in range(steps):
        for r in eager:
            r.plan_step = s
            u = planner.plan_step(params, [r], L)
            planner.advance(params, [r], u)
    torch.cuda.synchronize()
    mine = _fresh(rts)
    plan = planner.plan(params, mine, L, sg.plan_options(include_advance=1), trace=False)
    for s in range(steps):
        plan.run()
    torch.cuda.synchronize()
    plan.close()
    for a, b in zip(mine, eager):
        np.testing.assert_array_equal(a.x.cpu().numpy(), b.x.cpu().numpy())
        np.testing.assert_array_equal(a.u_nom.cpu().numpy(), b.u_nom.cpu().numpy())


def test_autotune_returns_a_valid_schedule(planner):
    tracks, races, specs, params, rts = _batch(planner, 5, 93)
    before = [r.u_nom.cpu().numpy().copy() for r in rts]
    t0 = time.perf_counter()
    best, ms = planner.autotune(params, rts, 1)
    t_search = time.perf_counter() - t0
    assert ms > 0 and best.use_graph == 1
    assert best.samples_per_lane in (1, 2) and best.tiles_per_fetch in (1, 2, 4)
    for r, b in zip(rts, before):  # state restored
        np.testing.assert_array_equal(r.u_nom.cpu().numpy(), b)
    # the same kind of workload again: the kept schedule, returned without timing
    t0 = time.perf_counter()
    best2, ms2 = planner.autotune(params, rts, 1)
    assert time.perf_counter() - t0 < 0.2 * t_search
    assert (best2.persistent, best2.blocks_per_cu, best2.tiles_per_fetch, best2.samples_per_lane, best2.use_graph) == \
        (best.persistent, best.blocks_per_cu, best.tiles_per_fetch, best.samples_per_lane, best.use_graph)
    assert ms2 == ms
    # after forgetting, the search runs again (and times again)
    planner.autotune_forget()
    best3, ms3 = planner.autotune(params, rts, 1)
    assert ms3 > 0 and best3.use_graph == 1


def _p32(params):
    """The parameter values the C ABI carries (float32), for float64 checks of the advance."""
    return {k: ([float(np.float32(x)) for x in v] if isinstance(v, list) else
                (float(np.float32(v)) if isinstance(v, float) else v)) for k, v in params.items()}


def test_batched_graph_plan_matches_oracle_lockstep(planner):
    """An uneven batch of the batched workload's kind -- 10 races of 2-10 vehicles, horizons
    20/40/50, K in {300, 777, 1024, 2048}, a 3-disc footprint, egos other than vehicle 0 in
    two races of three -- planned in one persistent launch per sweep with the planning step
    and the closed-loop advance captured in a hipGraph.  Over two replays every race is
    replayed by the oracle's Alg. 1 from the state the GPU started that step from,
    adopting the GPU's choices: every choice agrees (or is a near-tie) and the first
    controls, warm starts, trajectories, progress and advanced states match."""
    import torch
    import oracle
    import parity as PY
    import paper_2607_25388_amd.sgtp as sg
    tracks, races, specs, params = inputs.batched_workload(
        10, 77, K_override=lambda sp: [300, 777, 1024, 2048][sp["race"] % 4])
    for rc, sp in zip(races, specs):
        rc.ego = {0: 0, 1: rc.n_agents - 1, 2: rc.n_agents // 2}[sp["race"] % 3]
    assert sorted({rc.n_agents for rc in races}) == [2, 3, 4, 5, 6, 8, 9, 10]
    assert sorted({sp["N"] for sp in specs}) == [20, 40, 50]
    for N, tr in tracks.items():
        planner.upload_track(TRACK_ID[N], tr)
    rts = [sg.race_from_inputs(rc, TRACK_ID[sp["N"]], sp["K"], sp["N"], inputs.n_tail_from_fraction(0.3, sp["N"]),
                               plan_step=0) for rc, sp in zip(races, specs)]
    L = 2
    plan = planner.plan(params, rts, L, sg.plan_options(persistent=1, tiles_per_fetch=2, use_graph=1,
                                                        include_advance=1))
    state = [dict(x=rc.x.copy(), u=np.asarray(rc.u_nom, np.float64), s=rc.s_abs.copy()) for rc in races]
    orcs, orcs32 = {}, {}
    for N, tr in tracks.items():
        p = dict(params, N=N, n_tail=inputs.n_tail_from_fraction(0.3, N))
        orcs[N] = oracle.Oracle(tr, p)
        orcs32[N] = oracle.Oracle(tr, _p32(p))
    exact = total = 0
    for step in range(2):
        plan.run()
        torch.cuda.synchronize()
        gtr_all = plan.choices().copy()
        u_all = plan.u_apply.cpu().numpy().astype(np.float64)
        base = 0
        for r, (rc, sp, rt) in enumerate(zip(races, specs, rts)):
            n, N, K = rc.n_agents, sp["N"], sp["K"]
            label = f"step {step} race {r} (n={n}, N={N}, K={K}, ego={rc.ego})"
            print(label, flush=True)
            gtr = gtr_all[:, base:base + n]
            forced = PY.forced_from_trace(gtr, L, n, rc.ego)
            ref = orcs[N].plan_step(rc, L, K=K, forced=forced, x=state[r]["x"], u_nom=state[r]["u"],
                                    s_prev=state[r]["s"], plan_step=step)
            exact += PY.check_lockstep(gtr, ref, forced, label)
            total += int((forced >= 0).sum())
            np.testing.assert_allclose(u_all[base:base + n], ref["u_apply"], atol=1e-5, err_msg=label)
            u_next = rt.u_nom.cpu().numpy()
            np.testing.assert_allclose(u_next, ref["u_next"], atol=1e-5, err_msg=label)
            traj = rt.traj.cpu().numpy()
            assert np.max(np.abs(traj[:, :, :2] - ref["traj"][:, :, :2])) < PY.TOL_STATE, label
            s_abs = rt.s_abs.cpu().numpy()
            np.testing.assert_allclose(s_abs, ref["s_abs"], atol=1e-6, err_msg=label)
            # closed loop: the advanced state is the oracle's interval from the same controls
            x_next = rt.x.cpu().numpy()
            x_ref = orcs32[N].advance(state[r]["x"], u_all[base:base + n])
            np.testing.assert_allclose(x_next, x_ref, rtol=0, atol=1e-9, err_msg=label)
            state[r] = dict(x=x_next, u=u_next.astype(np.float64), s=s_abs)
            base += n
    plan.close()
    print(f"identical choices {exact} of {total}")
    assert exact >= total // 2


def test_full_batch_in_the_timed_configuration_matches_oracle_on_sampled_races():
    """The 256-race batch at full size (K up to 65536, 1535 vehicles) planned the way the
    benchmark times it -- one workgroup per tile, two samples per lane, the planning step
    and the closed-loop advance captured in a hipGraph -- for one step; four races spread
    over the batch (2 vehicles at K = 65536, 10 vehicles, a 20-step horizon, the last race)
    are replayed by the oracle's Alg. 1 in lockstep: every choice agrees or is a near-tie,
    and the first controls, warm starts, trajectories, progress and advanced states match."""
    import torch
    import oracle
    import parity as PY
    import paper_2607_25388_amd.sgtp as sg
    tracks, races, specs, params = inputs.batched_workload(256)
    p = sg.Planner(max_agents_total=2048, max_races=256)
    try:
        for N, tr in tracks.items():
            p.upload_track(TRACK_ID[N], tr)
        rts = [sg.race_from_inputs(rc, TRACK_ID[sp["N"]], sp["K"], sp["N"], inputs.n_tail_from_fraction(0.3, sp["N"]))
               for rc, sp in zip(races, specs)]
        L = 5
        plan = p.plan(params, rts, L, sg.plan_options(persistent=0, tiles_per_fetch=1, samples_per_lane=2,
                                                      use_graph=1, include_advance=1))
        plan.run()
        torch.cuda.synchronize()
        gtr_all = plan.choices().copy()
        u_all = plan.u_apply.cpu().numpy().astype(np.float64)
        plan.close()
        offs = np.concatenate([[0], np.cumsum([rc.n_agents for rc in races])])
        sample = [102, 58, 74, 255]
        assert specs[102]["K"] == 65536 and specs[58]["n_agents"] == 10 and specs[74]["N"] == 20
        exact = total = 0
        for r in sample:
            rc, sp, rt = races[r], specs[r], rts[r]
            n, N, K = rc.n_agents, sp["N"], sp["K"]
            label = f"race {r} (n={n}, N={N}, K={K})"
            print(label, flush=True)
            base = int(offs[r])
            pr = dict(params, N=N, n_tail=inputs.n_tail_from_fraction(0.3, N))
            gtr = gtr_all[:, base:base + n]
            forced = PY.forced_from_trace(gtr, L, n, rc.ego)
            ref = oracle.Oracle(tracks[N], pr).plan_step(rc, L, K=K, forced=forced, plan_step=0)
            exact += PY.check_lockstep(gtr, ref, forced, label)
            total += int((forced >= 0).sum())
            np.testing.assert_allclose(u_all[base:base + n], ref["u_apply"], atol=1e-5, err_msg=label)
            np.testing.assert_allclose(rt.u_nom.cpu().numpy(), ref["u_next"], atol=1e-5, err_msg=label)
            traj = rt.traj.cpu().numpy()
            assert np.max(np.abs(traj[:, :, :2] - ref["traj"][:, :, :2])) < PY.TOL_STATE, label
            np.testing.assert_allclose(rt.s_abs.cpu().numpy(), ref["s_abs"], atol=1e-6, err_msg=label)
            x_ref = oracle.Oracle(tracks[N], _p32(pr)).advance(rc.x, u_all[base:base + n])
            np.testing.assert_allclose(rt.x.cpu().numpy(), x_ref, rtol=0, atol=1e-9, err_msg=label)
        print(f"identical choices {exact} of {total}")
        assert exact >= total // 2
    finally:
        p.close()
