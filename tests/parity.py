"""Shared helpers of the GPU parity tests: same seeded inputs to the HIP planner and
to the CPU oracle, then element-by-element comparison under the parity contract:

  - perturbations bit-exact;
  - feasibility flags (b, o, h) bit-exact, except samples within EPS_CONSTRAINT of a
    threshold (oracle values), samples whose segment search hit its limit and
    samples far outside the track, which are compared on h only when both sides
    agree they are far infeasible;
  - final states within 1e-3 (m, rad, m/s, rad/s) after N steps;
  - costs within 1e-4 of the oracle's cost magnitude scale (tracking cost plus the
    absolute game terms), except samples within EPS_CONTEST of the contest
    indicator's threshold, where the cost is discontinuous;
  - the selected index identical, or the oracle cost of the GPU's choice within
    1e-4 of the best when the two best costs are that close.
"""

from __future__ import annotations

import numpy as np

import oracle
from paper_2607_25388_amd import inputs

TOL_STATE = 1e-3
TOL_COST = 1e-4
EPS_CONSTRAINT = 1e-4
EPS_CONTEST = 1e-3
TOL_VIOL = 2 * TOL_STATE  # nu = boundary shortfall + collision shortfall, each within TOL_STATE


def build(planner, track, race, params, K, track_id=0, plan_step=None):
    import paper_2607_25388_amd.sgtp as sg
    planner.upload_track(track_id, track)
    rt = sg.race_from_inputs(race, track_id, K, params["N"], params["n_tail"], plan_step=plan_step)
    return rt


def gpu_rollout(planner, params, rt, agent, phase, want_noise=True):
    import torch
    out = planner.rollout_cost(params, rt, agent, phase, want_noise=want_noise)
    torch.cuda.synchronize()
    import paper_2607_25388_amd.sgtp as sg
    res = {k: (v.cpu().numpy() if k != "choice" and v is not None else v) for k, v in out.items()}
    res["choice"] = sg.choices_to_numpy(out["choice"])[0]
    return res


def compare_samples(g, r, params, width, label=""):
    """Assert the per-sample parity contract; returns a dict of statistics."""
    K = len(r["cost"])
    rflags = r["flags"]
    near = (np.abs(r["rho_bd"] - params["m_bd"]) < EPS_CONSTRAINT) | \
           (np.abs(r["rho_obs"] - params["d_col"]) < EPS_CONSTRAINT)
    far = ((rflags & 8) > 0) | (r["max_abs_d"] > width / 2 + 5.0) | ((rflags & 16) > 0)
    # a search-limit or non-finite flag raised by the GPU alone must fall on a sample the
    # oracle also finds far outside the track (or itself flags): such flags never exempt
    # a sample the oracle tracks normally
    g_only = ((g["flags"] & 24) > 0) & ~far
    assert not g_only.any(), f"{label}: GPU-only limit/non-finite flags at {np.nonzero(g_only)[0][:10]}"
    # samples exempt from the strict checks stay a small minority: the exemption covers
    # clearances within 1e-4 m of a threshold and samples far off the track only
    assert near.sum() <= max(3, K // 500), f"{label}: {int(near.sum())} samples near a threshold"
    strict = ~(near | far)
    gb = g["flags"] & 7
    rb = rflags & 7
    bad_flags = np.nonzero(strict & (gb != rb))[0]
    assert len(bad_flags) == 0, f"{label}: flag mismatch at {bad_flags[:10]} gpu={gb[bad_flags[:10]]} ref={rb[bad_flags[:10]]}"
    # far samples: both must be infeasible
    fb = np.nonzero(far & ~((gb & 4) == (rb & 4)))[0]
    assert len(fb) == 0, f"{label}: far-sample feasibility differs at {fb[:10]}"
    ok = strict & ((rflags & 16) == 0)
    dx = np.abs(g["x_final"] - r["x_final"])
    dx[:, 2] = np.abs(np.remainder(g["x_final"][:, 2] - r["x_final"][:, 2] + np.pi, 2 * np.pi) - np.pi)
    max_dx = dx[ok].max(axis=0) if ok.any() else np.zeros(6)
    assert np.all(max_dx <= TOL_STATE), f"{label}: final state error {max_dx}"
    okc = ok & (r["contest_margin"] > EPS_CONTEST)
    cerr = np.abs(g["cost"].astype(np.float64) - r["cost"]) / np.maximum(r["scale"], 1e-30)
    max_c = cerr[okc].max() if okc.any() else 0.0
    assert max_c <= TOL_COST, f"{label}: cost error {max_c} at {np.argmax(np.where(okc, cerr, 0))}"
    verr = np.abs(g["viol"].astype(np.float64) - r["viol"])
    fin = ok & np.isfinite(r["viol"])
    max_v = verr[fin].max() if fin.any() else 0.0
    # the violation adds two clearance shortfalls, each a distance under the state contract
    assert max_v <= TOL_VIOL, f"{label}: violation error {max_v}"
    print(f"{label}: exempt near={int(near.sum())} far={int(far.sum())} of {K}", flush=True)
    return dict(K=K, strict=int(strict.sum()), near=int(near.sum()), far=int(far.sum()), max_state=max_dx.tolist(),
                max_cost_rel=float(max_c), max_viol=float(max_v), feasible=int(((rb & 4) > 0).sum()))


def check_choice(gchoice, r, params, label=""):
    """Selected index: identical, or a near-tie whose oracle cost is within tolerance."""
    rc = r["choice"]
    kg = int(gchoice["k"])
    kr = int(rc["k"])
    assert int(gchoice["fallback"]) == int(rc["fallback"]), f"{label}: fallback differs"
    if kg == kr:
        return True
    if rc["fallback"]:
        assert abs(r["viol"][kg] - r["viol"][kr]) <= TOL_VIOL, f"{label}: fallback choice {kg} vs {kr}"
        return False
    assert (r["flags"][kg] & 4), f"{label}: GPU chose oracle-infeasible {kg}"
    scale = max(r["scale"][kr], 1e-30)
    assert (r["cost"][kg] - r["cost"][kr]) / scale <= TOL_COST, \
        f"{label}: choice {kg} (cost {r['cost'][kg]}) vs {kr} (cost {r['cost'][kr]})"
    return False


def workload(name, K=None):
    tr, race, params = inputs.workload_inputs(name)
    w = inputs.WORKLOADS[name]
    return tr, race, params, (K or w.K), w


def oracle_for(track, params):
    return oracle.Oracle(track, params)


def check_lockstep(gtr, ref, forced, label=""):
    """One planning step of the GPU against the oracle's replay of it (the oracle adopts
    the GPU's choice in every phase it is forced to).  In every forced phase: the fallback
    flags agree; the GPU's index is the oracle's, or a near-tie (feasible: the oracle's
    cost of the GPU's sample within TOL_COST of the best; fallback: its violation within
    TOL_VIOL of the least); and the cost (violation) the GPU reports for its sample is the
    oracle's for that sample within the contract.  Returns the number of identical indices."""
    exact = 0
    for ph in range(forced.shape[0]):
        for i in range(forced.shape[1]):
            if forced[ph, i] < 0:
                continue
            rc = ref["trace"][ph][i]
            gc = gtr[ph, i]
            where = (label, ph, i)
            assert int(gc["fallback"]) == rc["fallback"], where
            assert rc["k_used"] == int(gc["k"]), where
            if int(gc["k"]) == rc["k"]:
                exact += 1
            elif not rc["fallback"]:
                assert rc["flags_used"] & 4, where
                assert (rc["cost_used"] - rc["cost"]) / rc["scale_used"] <= TOL_COST, (where, rc, gc)
            else:
                assert rc["viol_used"] - rc["viol"] <= TOL_VIOL, (where, rc, gc)
            if not rc["fallback"]:
                assert abs(float(gc["cost"]) - rc["cost_used"]) <= TOL_COST * rc["scale_used"], (where, rc, gc)
            else:
                assert abs(float(gc["viol"]) - rc["viol_used"]) <= TOL_VIOL, (where, rc, gc)
    return exact


def forced_from_trace(gtr, L, n, ego):
    """The GPU's choices as the oracle's forced indices: every vehicle in the sweeps 0..L,
    the ego alone in the extra response."""
    forced = np.full((L + 2, n), -1, np.int32)
    for ph in range(L + 2):
        for i in range(n):
            if ph <= L or i == ego:
                forced[ph, i] = int(gtr[ph, i]["k"])
    return forced
