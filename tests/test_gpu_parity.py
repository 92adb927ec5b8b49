"""GPU parity: the HIP planner (through the C ABI) against the CPU oracle."""

import copy
import math

import numpy as np
import pytest

import parity as PY
from paper_2607_25388_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def planner():
    import paper_2607_25388_amd.sgtp as sg
    p = sg.Planner(max_agents_total=64, max_races=4)
    yield p
    p.close()


def _run(planner, name, agent, phase, K, params_over=None, race_over=None, want_noise=False):
    tr, race, params, _, w = PY.workload(name)
    if params_over:
        params = dict(params, **params_over)
    if race_over:
        race = race_over(copy.deepcopy(race))
    rt = PY.build(planner, tr, race, params, K)
    g = PY.gpu_rollout(planner, params, rt, agent, phase, want_noise=want_noise)
    orc = PY.oracle_for(tr, params)
    r = orc.rollout_cost(race, agent, phase, K, noise=want_noise)
    return tr, race, params, g, r


def test_noise_is_bit_exact(planner):
    tr, race, params, g, r = _run(planner, "c1", 1, 2, 1000, want_noise=True)
    assert g["noise"].shape == r["noise"].shape
    diff = np.nonzero(g["noise"].view(np.uint32) != r["noise"].view(np.uint32))
    assert len(diff[0]) == 0, f"{len(diff[0])} perturbations differ, first at {diff[0][:5]}"


@pytest.mark.parametrize("agent,phase,K", [(0, 0, 1024), (0, 1, 1024), (1, 1, 1024), (1, 3, 1000), (0, 2, 777)])
def test_rollout_cost_c1(planner, agent, phase, K):
    tr, race, params, g, r = _run(planner, "c1", agent, phase, K)
    st = PY.compare_samples(g, r, params, tr.width, f"c1 a{agent} p{phase} K{K}")
    PY.check_choice(g["choice"], r, params, "c1")
    assert int(g["choice"]["n_feasible"]) == int(((r["flags"] & 4) > 0).sum()) or st["near"] > 0
    print(st)


@pytest.mark.parametrize("name,agent,K", [("c2", 0, 2048), ("c2", 2, 1500), ("c3", 0, 1024), ("c3", 7, 700)])
def test_rollout_cost_multi_disc_and_many_agents(planner, name, agent, K):
    tr, race, params, g, r = _run(planner, name, agent, 1, K)
    st = PY.compare_samples(g, r, params, tr.width, f"{name} a{agent}")
    PY.check_choice(g["choice"], r, params, name)
    print(st)


def test_full_size_large_field_sampled(planner):
    """C3 shape at full K = 65536 for one vehicle, every sample compared, and all
    65536 x 50 perturbation pairs bit for bit."""
    tr, race, params, g, r = _run(planner, "c3", 4, 2, 65536, want_noise=True)
    diff = np.count_nonzero(g["noise"].view(np.uint32) != r["noise"].view(np.uint32))
    assert diff == 0, f"{diff} perturbations differ"
    st = PY.compare_samples(g, r, params, tr.width, "c3 full")
    PY.check_choice(g["choice"], r, params, "c3 full")
    print(st)


def test_noise_bit_exact_late_in_the_counter_space(planner):
    """Every field of the Philox counter away from zero: planning step 7, vehicle 9 of
    ten, the extra-response phase 6 (L = 5), a ragged K."""
    def late(rc):
        rc.plan_step = 7
        return rc
    tr, race, params, _, w = PY.workload("c3")
    race = late(copy.deepcopy(race))
    rt = PY.build(planner, tr, race, params, 1999, plan_step=7)
    g = PY.gpu_rollout(planner, params, rt, 9, 6, want_noise=True)
    r = PY.oracle_for(tr, params).rollout_cost(race, 9, 6, 1999, noise=True)
    diff = np.count_nonzero(g["noise"].view(np.uint32) != r["noise"].view(np.uint32))
    assert diff == 0, f"{diff} perturbations differ"
    # the counter fields do select a different stream
    r0 = PY.oracle_for(tr, params).rollout_cost(race, 9, 6, 16, noise=True, plan_step=0)
    assert not np.array_equal(r0["noise"], r["noise"][:16])
    PY.compare_samples(g, r, params, tr.width, "late counter")
    PY.check_choice(g["choice"], r, params, "late counter")


def _field16():
    """Sixteen vehicles (the most one race takes) on the large-field track, staggered grid."""
    tr, _, params, _, w = PY.workload("c3")
    race = inputs.make_race(tr, 16, w.N, 8.0, True, 3016, 2016)
    return tr, race, params


@pytest.mark.parametrize("agent", [0, 9, 15])
def test_sixteen_vehicles_per_sample(planner, agent):
    tr, race, params = _field16()
    rt = PY.build(planner, tr, race, params, 1500)
    g = PY.gpu_rollout(planner, params, rt, agent, 1, want_noise=True)
    r = PY.oracle_for(tr, params).rollout_cost(race, agent, 1, 1500, noise=True)
    assert np.array_equal(g["noise"].view(np.uint32), r["noise"].view(np.uint32))
    PY.compare_samples(g, r, params, tr.width, f"16 vehicles a{agent}")
    PY.check_choice(g["choice"], r, params, f"16 vehicles a{agent}")


def test_sixteen_vehicles_plan_step_lockstep(planner):
    import torch
    import paper_2607_25388_amd.sgtp as sg
    tr, race, params = _field16()
    race.ego = 3
    K, L = 768, 1
    rt = PY.build(planner, tr, race, params, K)
    n = race.n_agents
    trace = torch.zeros((L + 2) * n * sg.CHOICE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    u_apply = planner.plan_step(params, [rt], L, trace=trace).cpu().numpy()
    torch.cuda.synchronize()
    gtr = sg.choices_to_numpy(trace).reshape(L + 2, n)
    forced = PY.forced_from_trace(gtr, L, n, race.ego)
    ref = PY.oracle_for(tr, params).plan_step(race, L, K=K, forced=forced)
    PY.check_lockstep(gtr, ref, forced, "16 vehicles")
    np.testing.assert_allclose(u_apply, ref["u_apply"], atol=1e-5)
    np.testing.assert_allclose(rt.u_nom.cpu().numpy(), ref["u_next"], atol=1e-5)
    assert np.max(np.abs(rt.traj.cpu().numpy()[:, :, :2] - ref["traj"][:, :, :2])) < PY.TOL_STATE


def test_kinematic_model(planner):
    tr, race, params, g, r = _run(planner, "c1", 0, 1, 1024, params_over=dict(model=1))
    PY.compare_samples(g, r, params, tr.width, "kinematic")
    PY.check_choice(g["choice"], r, params, "kinematic")


def test_single_sample_and_single_agent(planner):
    tr, race, params, g, r = _run(planner, "c1", 0, 1, 1)
    PY.compare_samples(g, r, params, tr.width, "K=1")
    assert int(g["choice"]["k"]) == 0

    def solo(rc):
        rc.n_agents = 1
        rc.x = rc.x[:1]
        rc.s_abs = rc.s_abs[:1]
        rc.v_scale = rc.v_scale[:1]
        rc.u_nom = rc.u_nom[:1]
        return rc
    tr, race, params, g, r = _run(planner, "c1", 0, 1, 512, race_over=solo)
    PY.compare_samples(g, r, params, tr.width, "n=1")
    PY.check_choice(g["choice"], r, params, "n=1")


def test_all_infeasible_fallback(planner):
    def stacked(rc):
        rc.x[1] = rc.x[0]
        rc.s_abs[1] = rc.s_abs[0]
        return rc
    tr, race, params, g, r = _run(planner, "c1", 0, 1, 512, race_over=stacked)
    assert r["choice"]["fallback"] == 1
    PY.compare_samples(g, r, params, tr.width, "fallback")
    PY.check_choice(g["choice"], r, params, "fallback")


def test_nan_nominal_is_infeasible(planner):
    def nan(rc):
        rc.u_nom = rc.u_nom.copy()
        rc.u_nom[0, 3, 1] = np.nan
        return rc
    tr, race, params, g, r = _run(planner, "c1", 0, 1, 256, race_over=nan)
    assert np.all(g["flags"] & 16) and np.all(np.isinf(g["viol"]))
    assert int(g["choice"]["k"]) == 0 and int(g["choice"]["fallback"]) == 1


def test_open_straight_track(planner):
    import oracle
    import paper_2607_25388_amd.sgtp as sg
    tr = inputs.make_straight_track(600.0, 10.0, x0=-100.0, y0=20.0, heading=0.3, vref=25.0)
    params = inputs.default_params(20, 3)
    race = inputs.make_race(tr, 3, 20, 10.0, True, 11, 12)
    rt = sg.race_from_inputs(race, 5, 1024, 20, params["n_tail"])
    planner.upload_track(5, tr)
    g = PY.gpu_rollout(planner, params, rt, 1, 1)
    r = oracle.Oracle(tr, params).rollout_cost(race, 1, 1, 1024)
    PY.compare_samples(g, r, params, tr.width, "straight")
    PY.check_choice(g["choice"], r, params, "straight")


def _paper_scale_race():
    """Three 1:10 cars queued 2 m apart on a twisty 150 m x 2.5 m loop with the paper's
    own setup (Sec. IV-B: kinematic bicycle, H = 12 over 1.2 s, point footprint)."""
    from paper_2607_25388_amd import race_eval as RE
    sc = RE.SCALES["small"]
    tr = inputs.make_fourier_track(sc["length"], sc["width"], 1106, **sc["track"])
    race = inputs.make_race(tr, 3, sc["N"], sc["spacing"], False, 60600, 60600)
    return tr, race, sc["params"](sc["N"])


def _plan(planner, name, K, L, params_over=None, ego=0):
    import torch
    import paper_2607_25388_amd.sgtp as sg
    tr, race, params = _paper_scale_race() if name == "paper" else PY.workload(name)[:3]
    if params_over:
        params = dict(params, **params_over)
    race.ego = ego
    rt = PY.build(planner, tr, race, params, K)
    n = race.n_agents
    trace = torch.zeros((L + 2) * n * sg.CHOICE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    u_apply = planner.plan_step(params, [rt], L, trace=trace)
    torch.cuda.synchronize()
    gtr = sg.choices_to_numpy(trace).reshape(L + 2, n)
    return tr, race, params, rt, gtr, u_apply.cpu().numpy()


# prediction perturbation of the robustness experiment at a scale that moves clearances
PERTURB = {"pred_sig_lon": 0.5, "pred_sig_lat": 0.3}


@pytest.mark.parametrize("name,K,L,over,ego", [
    ("c1", 1024, 3, None, 0), ("c2", 1024, 2, None, 0), ("c3", 512, 1, PERTURB, 0), ("c1", 1024, 2, PERTURB, 0),
    # the ego is not vehicle 0: the final phase then writes the ego's first control from
    # its extra response and every other vehicle's from its last sweep
    ("c1", 1024, 2, None, 1), ("c2", 1024, 2, None, 2), ("c3", 512, 2, None, 7),
    # two waves per sample (3 x 11111 samples, ragged last tile)
    ("c2", 11111, 2, None, 0), ("c2", 11111, 1, PERTURB, 1),
    # full sizes, same kernels as the timed planning steps: mid-scale split variant
    # (3 x 16384 samples), large-field throughput variant (10 x 65536 lanes)
    ("c2", 16384, 5, None, 0), ("c3", 65536, 1, None, 0),
    # the paper's own setup: K = 128, L = 2, plain and with the severe prediction
    # perturbation of Table II
    ("paper", 128, 2, None, 0), ("paper", 128, 2, {"pred_sig_lon": 0.08, "pred_sig_lat": 0.04}, 0),
    ("paper", 128, 2, None, 2)])
def test_plan_step_lockstep(planner, name, K, L, over, ego):
    """Alg. 1 on the GPU; the oracle replays it adopting the GPU's choices phase by phase
    and must agree with each choice (or find it a near-tie)."""
    tr, race, params, rt, gtr, u_apply = _plan(planner, name, K, L, over, ego)
    n = race.n_agents
    forced = PY.forced_from_trace(gtr, L, n, race.ego)
    orc = PY.oracle_for(tr, params)
    ref = orc.plan_step(race, L, K=K, forced=forced)
    exact = PY.check_lockstep(gtr, ref, forced, name)
    assert exact >= (L + 1) * n // 2
    np.testing.assert_allclose(u_apply, ref["u_apply"], atol=1e-5)
    np.testing.assert_allclose(rt.u_nom.cpu().numpy(), ref["u_next"], atol=1e-5)
    traj = rt.traj.cpu().numpy()
    assert np.max(np.abs(traj[:, :, :2] - ref["traj"][:, :, :2])) < PY.TOL_STATE
    np.testing.assert_allclose(rt.s_abs.cpu().numpy(), ref["s_abs"], atol=1e-6)


def test_winner_rerollout_is_bit_identical(planner):
    """The selected sample re-rolled by one lane reproduces the sweep lane bit for bit."""
    import torch
    import paper_2607_25388_amd.sgtp as sg
    tr, race, params, _, w = PY.workload("c2")
    K = 2048
    rt = PY.build(planner, tr, race, params, K)
    g = PY.gpu_rollout(planner, params, rt, 1, 1, want_noise=False)
    k = int(g["choice"]["k"])
    out = planner.ibr_sweep(params, [rt], 1)
    torch.cuda.synchronize()
    ch = sg.choices_to_numpy(out)
    assert int(ch[1]["k"]) == k
    assert float(ch[1]["cost"]) == float(g["cost"][k])
    traj = rt.traj.cpu().numpy()
    np.testing.assert_array_equal(traj[1, -1, :6], g["x_final"][k])


def test_ibr_sweep_matches_plan_step_phase(planner):
    """sgtp_ibr_sweep(phase 0) followed by (phase 1) reproduces the first two phases of a plan step."""
    import torch
    import paper_2607_25388_amd.sgtp as sg
    tr, race, params, _, w = PY.workload("c1")
    K, L = 1024, 1
    rt1 = PY.build(planner, tr, race, params, K)
    c0 = sg.choices_to_numpy(planner.ibr_sweep(params, [rt1], 0))
    c1 = sg.choices_to_numpy(planner.ibr_sweep(params, [rt1], 1))
    torch.cuda.synchronize()
    tr_, race_, params_, rt2, gtr, _ = _plan(planner, "c1", K, L)
    assert [int(c["k"]) for c in c0] == [int(c["k"]) for c in gtr[0]]
    assert [int(c["k"]) for c in c1] == [int(c["k"]) for c in gtr[1]]


def test_advance_matches_oracle(planner):
    import torch
    tr, race, params, _, w = PY.workload("c2")
    rt = PY.build(planner, tr, race, params, 64)
    u = torch.tensor([[1.0, 0.02], [-2.0, -0.1], [0.5, 0.3]], dtype=torch.float32, device="cuda")
    planner.advance(params, [rt], u)
    torch.cuda.synchronize()
    # the C ABI carries float32 parameters: give the oracle the same (rounded) values
    p32 = {k: ([float(np.float32(x)) for x in v] if isinstance(v, list) else
               (float(np.float32(v)) if isinstance(v, float) else v)) for k, v in params.items()}
    orc = PY.oracle_for(tr, p32)
    ref = orc.advance(race.x, u.cpu().numpy().astype(np.float64))
    np.testing.assert_allclose(rt.x.cpu().numpy(), ref, rtol=0, atol=1e-11)


def test_argument_errors(planner):
    import paper_2607_25388_amd.sgtp as sg
    tr, race, params, _, w = PY.workload("c1")
    rt = PY.build(planner, tr, race, params, 64)
    with pytest.raises(RuntimeError, match="EINVAL"):
        planner.rollout_cost(dict(params, n_disc=2), rt, 0, 1)
    with pytest.raises(RuntimeError, match="EINVAL"):
        planner.rollout_cost(params, rt, 5, 1)
    bad = copy.copy(rt)
    bad.track_id = 63
    with pytest.raises(RuntimeError, match="ETRACK"):
        planner.rollout_cost(params, bad, 0, 1)
    big = copy.copy(rt)
    big.N = 65
    with pytest.raises(RuntimeError, match="EINVAL|ESHAPE"):
        planner.rollout_cost(params, big, 0, 1)


@pytest.mark.parametrize("name,agent,K,N", [("c1", 0, 2048, None), ("c2", 1, 2048, None), ("c2", 2, 777, None),
                                            ("c1", 1, 1001, 21),
                                            # horizons shorter than the control look-ahead of the
                                            # two-wave variant, and one step longer
                                            ("c1", 0, 300, 1), ("c2", 1, 513, 2), ("c2", 0, 129, 3),
                                            # the longest horizon the library takes
                                            ("c2", 2, 2048, 64)])
def test_small_launch_variants_match_one_lane_variant(planner, name, agent, K, N):
    """Small launches run each sample on two waves (the dynamics on one, perturbation,
    projection and scoring on the other; or, where those rings do not fit in LDS, on a
    pair of lanes); the same samples of a large launch run on one lane.  Both must give
    the same bits for every per-sample output (ragged K and an odd horizon included)."""
    tr, race, params, _, w = PY.workload(name)
    if N is not None:
        race = inputs.make_race(tr, race.x.shape[0], N, 10.0, False, 3000, 2000)
        params = dict(params, N=N, n_tail=inputs.n_tail_from_fraction(0.3, N))
    small = PY.gpu_rollout(planner, params, PY.build(planner, tr, race, params, K), agent, 1, want_noise=True)
    large = PY.gpu_rollout(planner, params, PY.build(planner, tr, race, params, 40000), agent, 1, want_noise=True)
    for nm in ("cost", "viol", "flags", "x_final", "noise"):
        assert np.array_equal(small[nm].view(np.uint8), large[nm][:K].view(np.uint8)), nm
    # the selection over the first K samples: the small launch's choice is its own argmin
    r = PY.oracle_for(tr, params).rollout_cost(race, agent, 1, K)
    PY.check_choice(small["choice"], r, params, f"{name} small-launch variant")


@pytest.mark.parametrize("name,agent,K", [("c2", 0, 2048), ("c3", 3, 1000)])
def test_rollout_cost_with_prediction_perturbation(planner, name, agent, K):
    """Perturbed opponent predictions (robustness experiment): per-sample parity with the
    oracle, and the perturbation does change the clearances seen by the samples."""
    tr, race, params, g, r = _run(planner, name, agent, 1, K, params_over=PERTURB)
    PY.compare_samples(g, r, params, tr.width, f"{name} perturbed")
    PY.check_choice(g["choice"], r, params, f"{name} perturbed")
    _, _, _, g0, r0 = _run(planner, name, agent, 1, K)
    assert not np.array_equal(r["rho_obs"], r0["rho_obs"])
    # where some sample comes within the safety distance, the cost sees the perturbation too
    if np.any(r0["rho_obs"] < params["g_safe"]):
        assert not np.array_equal(g["cost"], g0["cost"])


def test_lds_fallback_when_split_rings_do_not_fit(planner):
    """A raceline with 0.1 m nodes makes the staged window so long (~1300 nodes at N = 40)
    that the two-wave variant's LDS rings no longer fit in the 58 KiB budget: the plan is
    built again without them (here the pair variant) and must still give the one-lane
    bits and the oracle's choice."""
    import paper_2607_25388_amd.sgtp as sg
    budget, rings = 58 * 1024, 4 * 128 * 16 + 4 * 128 * 8 + 32 + 128 * 8 * 4
    tr = inputs.make_fourier_track(300.0, 10.0, 1000, ds=0.1)
    params = inputs.default_params(40, 1)
    race = inputs.make_race(tr, 2, 40, 10.0, False, 3001, 2001)
    plan = planner.plan(params, [PY.build(planner, tr, race, params, 1024)], 1, sg.plan_options(), trace=False)
    info = plan.info()
    plan.close()
    assert info["lds_bytes"] <= budget < info["lds_bytes"] + rings, info
    small = PY.gpu_rollout(planner, params, PY.build(planner, tr, race, params, 1024), 0, 1, want_noise=True)
    large = PY.gpu_rollout(planner, params, PY.build(planner, tr, race, params, 40000), 0, 1, want_noise=True)
    for nm in ("cost", "viol", "flags", "x_final", "noise"):
        assert np.array_equal(small[nm].view(np.uint8), large[nm][:1024].view(np.uint8)), nm
    r = PY.oracle_for(tr, params).rollout_cost(race, 0, 1, 1024)
    PY.check_choice(small["choice"], r, params, "LDS fallback")


def test_bounded_wait_give_up_is_reported_and_never_selected(planner):
    """The two-wave variant's LDS waits always end by construction; their poll bound is a
    guard.  With the bound set from the host to a single poll, waits give up while every
    kernel still ends: the affected samples come out non-finite (never selected), the
    context's status word says so, every other sample keeps the one-lane bits, and with
    the default bound the status stays clear."""
    import paper_2607_25388_amd.sgtp as sg
    tr, race, params, _, w = PY.workload("c2")
    K = 4096  # two-wave variant (small launch, 2 opponents)
    ref = PY.gpu_rollout(planner, params, PY.build(planner, tr, race, params, 40000), 1, 1, want_noise=False)
    assert planner.status() == 0
    planner.set_poll_limit(1)
    try:
        g = PY.gpu_rollout(planner, params, PY.build(planner, tr, race, params, K), 1, 1, want_noise=False)
        st = planner.status()
    finally:
        planner.set_poll_limit(1 << 22)
    gave_up = (g["flags"] & 16) > 0
    print(f"status {st}, samples scored non-finite {int(gave_up.sum())} of {K}", flush=True)
    assert st & sg.SGTP_STATUS_WAIT_GAVE_UP
    assert gave_up.any() and np.all(np.isinf(g["viol"][gave_up]))
    assert not np.any(g["flags"][gave_up] & 7)
    ok = ~gave_up
    for nm in ("cost", "viol", "flags", "x_final"):
        assert np.array_equal(g[nm][ok].view(np.uint8), ref[nm][:K][ok].view(np.uint8)), nm
    k = int(g["choice"]["k"])
    if ok.any() and (ref["flags"][:K][ok] & 4).any():
        assert not gave_up[k]
    # default bound again: a clean run leaves the status clear
    PY.gpu_rollout(planner, params, PY.build(planner, tr, race, params, K), 1, 1, want_noise=False)
    assert planner.status() == 0


def test_gaussian_transform_bit_exact_for_every_radius_and_angle(planner):
    """Every value the sampler's transform can take apart: all 2^23 radius words (angle 0)
    and all 2^24 angle words (one radius) give the oracle's float32 pair bit for bit."""
    import torch
    import paper_2607_25388_amd.sgtp as sg
    tr, race, params, _, w = PY.workload("c1")
    orc = PY.oracle_for(tr, params)
    cases = [(np.arange(1 << 23, dtype=np.uint64) << 9, np.zeros(1 << 23, np.uint64)),
             (np.full(1 << 24, 0x5a5a5a5a, np.uint64) & 0xfffffe00, np.arange(1 << 24, dtype=np.uint64) << 8)]
    for re, ro in cases:
        re32, ro32 = re.astype(np.uint32), ro.astype(np.uint32)
        g = sg.gauss_pairs(torch.as_tensor(re32.view(np.int32)).cuda(), torch.as_tensor(ro32.view(np.int32)).cuda())
        torch.cuda.synchronize()
        gv = g.cpu().numpy()
        r = orc.gauss_pairs(re32, ro32)
        diff = np.count_nonzero(gv.view(np.uint32) != r.view(np.uint32))
        assert diff == 0, f"{diff} of {gv.size} values differ"
