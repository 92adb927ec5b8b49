"""Closed-loop race evaluation on the GPU: plumbing of the batched per-vehicle games
and the metrics of short trials for every method."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_short_trials_every_method():
    import paper_2607_25388_amd.sgtp as sg
    from paper_2607_25388_amd import inputs, race_eval as RE
    planner = sg.Planner(max_agents_total=64, max_races=16, max_K=1024)
    planner.enable_path_integral()
    params = inputs.default_params(20, 3)
    tracks, trials = RE.make_trials(2, 2, 20)
    for m in RE.METHODS:
        per, ct = RE.run(planner, m, params, tracks, trials, K=512, L_ibr=2, T_max=2.0)
        s = RE.summarize(per, 2.0)
        print(m, s, ct.mean())
        assert s["trials"] == 4 and 0.0 <= s["wins"] <= 1.0 and 0.0 <= s["fpr"] <= 1.0
        assert 0.0 < s["d_mean_s"] <= 2.0 and np.isfinite(s["v_ego_mean"]) and s["v_ego_mean"] > 0.0
        assert np.all(np.isfinite(ct)) and ct.min() > 0.0
    planner.close()


def test_games_share_the_physical_state():
    """After closed-loop steps every game copy of a trial holds the truth state, and
    vehicle e's applied control is the one its own game selected for it."""
    import torch
    import paper_2607_25388_amd.sgtp as sg
    from paper_2607_25388_amd import inputs, race_eval as RE
    planner = sg.Planner(max_agents_total=32, max_races=8, max_K=1024)
    params = inputs.default_params(20, 3)
    tracks, trials = RE.make_trials(1, 2, 20)
    per, ct = RE.run(planner, "sgtp", params, tracks, trials, K=256, L_ibr=1, T_max=0.5)
    assert len(per) == 2 and all(p["duration"] > 0 for p in per)
    planner.close()


def test_small_scale_kinematic_trials():
    """The paper's setup at its own scale (kinematic bicycle, K = 128, H = 12, L = 2,
    point footprint, 2 m queue) runs closed loop for every method."""
    import paper_2607_25388_amd.sgtp as sg
    from paper_2607_25388_amd import race_eval as RE
    sc = RE.SCALES["small"]
    params = sc["params"](sc["N"])
    assert params["model"] == 1 and params["n_disc"] == 1 and params["N"] == 12
    planner = sg.Planner(max_agents_total=32, max_races=8, max_K=sc["K"])
    planner.enable_path_integral()
    tracks, trials = RE.make_trials(1, 2, sc["N"], length=sc["length"], width=sc["width"],
                                    spacing=sc["spacing"], track_seed0=1106, track_kw=sc["track"])
    for m in RE.METHODS:
        per, ct = RE.run(planner, m, params, tracks, trials, K=sc["K"], L_ibr=sc["L"], T_max=3.0,
                         contact=sc["contact"])
        s = RE.summarize(per, 3.0)
        print(m, s, ct.mean())
        assert s["trials"] == 2 and 0.0 <= s["wins"] <= 1.0
        assert 0.0 < s["d_mean_s"] <= 3.0 and np.isfinite(s["v_ego_mean"]) and s["v_ego_mean"] > 0.0
        assert np.all(np.isfinite(ct)) and ct.min() > 0.0
    planner.close()


def test_race_games_match_oracle_lockstep():
    """The closed loop of the race evaluation for two steps: every vehicle plans its own
    game (itself as the ego, its own noise key) on a copy of the shared true state, the
    applied control of each vehicle is its own game's ego control, and the truth advances
    by the float64 interval.  Every game is replayed by the oracle's Alg. 1 in lockstep
    (choices, first controls, warm starts), and the advanced truth is the oracle's interval
    from the applied controls."""
    import copy
    import torch
    import oracle
    import parity as PY
    import paper_2607_25388_amd.sgtp as sg
    from paper_2607_25388_amd import inputs, race_eval as RE
    planner = sg.Planner(max_agents_total=32, max_races=8, max_K=1024)
    params = RE.method_params(inputs.default_params(20, 3), "sgtp")
    p32 = {k: ([float(np.float32(x)) for x in v] if isinstance(v, list) else
               (float(np.float32(v)) if isinstance(v, float) else v)) for k, v in params.items()}
    tracks, trials = RE.make_trials(1, 1, params["N"])
    ti, race = trials[0]
    n, K, L = race.n_agents, 512, 2
    planner.upload_track(0, tracks[ti])
    X = torch.tensor(race.x[None], dtype=torch.float64, device="cuda")
    Xg = X[:, None].repeat(1, n, 1, 1).contiguous()
    games = []
    for e in range(n):
        rt = sg.race_from_inputs(race, 0, K, params["N"], params["n_tail"])
        rt.x = Xg[0, e]
        rt.ego = e
        rt.seed = int(race.seed) * 16 + e
        games.append(rt)
    truth = sg.race_from_inputs(race, 0, K, params["N"], params["n_tail"], with_traj=False)
    truth.x = X[0]
    opts = sg.plan_options()
    opts.include_advance = 0
    plan = planner.plan(params, games, L, opts, trace=True)
    orc, orc32 = oracle.Oracle(tracks[ti], params), oracle.Oracle(tracks[ti], p32)
    state = [dict(u=np.asarray(race.u_nom, np.float64), s=race.s_abs.copy()) for _ in range(n)]
    exact = total = 0
    for step in range(2):
        x_before = X[0].cpu().numpy().copy()
        u_all = plan.run()
        torch.cuda.synchronize()
        gtr_all = plan.choices().copy()
        ua = u_all.cpu().numpy().astype(np.float64)
        for e, g in enumerate(games):
            label = f"step {step} game {e}"
            print(label, flush=True)
            rc = copy.deepcopy(race)
            rc.ego = e
            rc.seed = int(race.seed) * 16 + e
            gtr = gtr_all[:, e * n:(e + 1) * n]
            forced = PY.forced_from_trace(gtr, L, n, e)
            ref = orc.plan_step(rc, L, K=K, forced=forced, x=x_before, u_nom=state[e]["u"], s_prev=state[e]["s"],
                                plan_step=step)
            exact += PY.check_lockstep(gtr, ref, forced, label)
            total += int((forced >= 0).sum())
            np.testing.assert_allclose(ua[e * n:(e + 1) * n], ref["u_apply"], atol=1e-5, err_msg=label)
            u_next = g.u_nom.cpu().numpy()
            np.testing.assert_allclose(u_next, ref["u_next"], atol=1e-5, err_msg=label)
            np.testing.assert_allclose(g.s_abs.cpu().numpy(), ref["s_abs"], atol=1e-6, err_msg=label)
            state[e] = dict(u=u_next.astype(np.float64), s=g.s_abs.cpu().numpy())
        sel = torch.tensor([e * n + e for e in range(n)], device="cuda")
        u = u_all.index_select(0, sel).contiguous()
        planner.advance(params, [truth], u)
        Xg.copy_(X[:, None].expand(-1, n, -1, -1))
        torch.cuda.synchronize()
        x_ref = orc32.advance(x_before, u.cpu().numpy().astype(np.float64))
        np.testing.assert_allclose(X[0].cpu().numpy(), x_ref, rtol=0, atol=1e-9, err_msg=f"step {step} advance")
    plan.close()
    planner.close()
    print(f"identical choices {exact} of {total}")
    assert exact >= total // 2
