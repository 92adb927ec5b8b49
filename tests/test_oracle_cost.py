"""Pins of the oracle's cost, feasibility checks and selection (Sec. III-A, III-B).

Constructed cases on a straight track where every quantity has a closed form:
ego and opponent moving in parallel at equal constant speed, so that progress
gaps, lateral offsets and the time-aligned distance of eq. (Dmin) are fixed
numbers; stationary vehicles for the disc footprint; brute-force selection over
tiny K; invariants (additivity over opponents, order invariance, w_game = 0).
"""

import math

import numpy as np
import pytest

import oracle
from paper_2607_25388_amd.inputs import default_params, make_straight_track

X0 = -50.0  # track starts here


def straight(width=10.0, vref=20.0):
    return make_straight_track(400.0, width, x0=X0, vref=vref)


def opp_line(x_start, d, v, N, dt, psi=0.0):
    """Opponent prediction along y = d at constant speed (world (x, y, psi, vx, vy, om, s, d))."""
    t = np.arange(N + 1) * dt
    tr = np.zeros((N + 1, 8))
    tr[:, 0] = x_start + v * t * math.cos(psi)
    tr[:, 1] = d + v * t * math.sin(psi)
    tr[:, 2] = psi
    tr[:, 3] = v
    tr[:, 6] = tr[:, 0] - X0
    tr[:, 7] = d
    return tr


def br_inputs(orc, p, x_e, d_e, v, opps, K=4, w_game=None, ubar=None, phase=1):
    N, dt = p["N"], p["dt"]
    x0 = np.array([x_e, d_e, 0.0, v, 0.0, 0.0])
    seg, s0, _, _ = orc.project_global(x0)
    xr = orc.reference(seg, s0, 1.0)
    opp = np.stack([o for o in opps]) if opps else np.zeros((0, N + 1, 8))
    return dict(agent=0, phase=phase, n_opp=len(opps), K=K, seg0=seg, s0=s0,
                w_game=p["w_game"] if w_game is None else w_game, seed=99, plan_step=0,
                x0=x0, xr=xr, ubar=np.zeros((N, 2)) if ubar is None else ubar,
                opp_traj=opp if len(opps) else np.zeros((1, N + 1, 8)),
                opp_s0=np.array([o[0, 6] for o in opps]) if opps else np.zeros(1))


def det_params(N=20, n_disc=1):
    p = default_params(N, n_disc)
    p["sigma_a"] = 0.0
    p["sigma_d"] = 0.0
    return p


def expected_game(p, gap, dd, g):
    """Closed-form c_game for one opponent with constant gap, lateral offset dd and distance g."""
    alpha = 1.0 / (1.0 + abs(gap) / (p["s_contest"] + p["eps_alpha"]))
    gamma = p["w_block"] if (p["s_role"] < gap < p["s_contest"]) else 0.0
    c_contest = -p["w_contest"] if abs(gap) < p["s_contest"] else 0.0
    c_long = -p["w_long"] * alpha * gap
    c_block = -gamma / (1.0 + abs(dd))
    c_safety = p["w_safety"] * max(0.0, p["g_safe"] - g) ** 2
    return c_contest + c_long + c_block + c_safety


@pytest.mark.parametrize("gap,d_e,d_o", [(5.0, 1.0, -1.0), (-20.0, 0.5, 0.5), (0.5, 0.5, -0.5), (9.0, 3.0, -3.0),
                                          (1.0, 0.0, 2.0)])
def test_constructed_cost_parallel_motion(oracle_lib, gap, d_e, d_o):
    p = det_params()
    orc = oracle.Oracle(straight(), p)
    v = 20.0
    xo = 10.0
    opp = opp_line(xo, d_o, v, p["N"], p["dt"])
    br = br_inputs(orc, p, xo + gap, d_e, v, [opp])
    out = orc.best_response(br)
    N = p["N"]
    J = N * p["Q"][1] * d_e ** 2  # only the lateral error is nonzero
    g = math.hypot(gap, d_e - d_o)
    c = J + p["w_game"] * expected_game(p, gap, d_e - d_o, g)
    np.testing.assert_allclose(out["cost"], c, rtol=1e-12, atol=1e-9)
    # feasibility: boundary 5 - |d| vs m_bd, collision g vs d_col
    assert np.all(out["rho_bd"] == pytest.approx(5.0 - abs(d_e), abs=1e-12))
    assert np.all(out["rho_obs"] == pytest.approx(g, abs=1e-12))
    o = g >= p["d_col"]
    b = 5.0 - abs(d_e) >= p["m_bd"]
    assert np.all(((out["flags"] & 2) > 0) == o)
    assert np.all(((out["flags"] & 1) > 0) == b)
    nu = max(0.0, p["m_bd"] - (5.0 - abs(d_e))) + max(0.0, p["d_col"] - g)
    np.testing.assert_allclose(out["viol"], nu, atol=1e-12)


def test_tracking_cost_speed_and_control_terms(oracle_lib):
    """Constant acceleration a on the centreline: e_v and e_x in closed form, R a^2 per step, no S term."""
    p = det_params()
    orc = oracle.Oracle(straight(vref=20.0), p)
    N, dt, a = p["N"], p["dt"], 2.0
    ubar = np.zeros((N, 2))
    ubar[:, 0] = a
    br = br_inputs(orc, p, 0.0, 0.0, 20.0, [], ubar=ubar)
    out = orc.best_response(br)
    t = np.arange(1, N + 1) * dt
    ex = 0.5 * a * t * t
    ev = a * t
    J = np.sum(p["Q"][0] * ex ** 2 + p["Q"][3] * ev ** 2) + N * p["R"][0] * a * a
    np.testing.assert_allclose(out["cost"], J, rtol=1e-10)


def test_control_rate_term(oracle_lib):
    """Alternating steering +-delta: sum_{tau=1}^{H-1} S_d (2 delta)^2 appears in the cost."""
    p = det_params()
    p["Q"] = [0.0, 0.0, 0.0, 0.0]
    orc = oracle.Oracle(straight(), p)
    N, dl = p["N"], 0.01
    ubar = np.zeros((N, 2))
    ubar[:, 1] = dl * (-1.0) ** np.arange(N)
    out = orc.best_response(br_inputs(orc, p, 0.0, 0.0, 20.0, [], ubar=ubar))
    J = N * p["R"][1] * dl * dl + (N - 1) * p["S"][1] * (2 * dl) ** 2
    np.testing.assert_allclose(out["cost"], J, rtol=1e-12)


def test_disc_footprint_distance(oracle_lib):
    """Stationary cars: ego at the origin heading +x, opponent at (3, 2.5) heading +y, discs at -1.5/0/1.5 m."""
    p = det_params(N=5, n_disc=3)
    orc = oracle.Oracle(straight(), p)
    opp = np.zeros((p["N"] + 1, 8))
    opp[:, 0], opp[:, 1], opp[:, 2] = 3.0, 2.5, math.pi / 2
    opp[:, 6] = 3.0 - X0
    br = br_inputs(orc, p, 0.0, 0.0, 0.0, [opp])
    out = orc.best_response(br)
    ego = [(-1.5, 0.0), (0.0, 0.0), (1.5, 0.0)]
    oth = [(3.0, 1.0), (3.0, 2.5), (3.0, 4.0)]
    g = min(math.hypot(a[0] - b[0], a[1] - b[1]) for a in ego for b in oth)
    assert g == pytest.approx(math.hypot(1.5, 1.0))
    np.testing.assert_allclose(out["rho_obs"], g, rtol=1e-12)
    assert np.all((out["flags"] & 2) == 0)  # g < d_col = 2
    np.testing.assert_allclose(out["viol"], p["d_col"] - g, rtol=1e-12)


def test_single_disc_reduces_to_point_distance(oracle_lib):
    """n_disc = 1 at offset 0 is eq. (Dmin): min over tau of the CoG distance."""
    p = det_params(N=10, n_disc=1)
    orc = oracle.Oracle(straight(), p)
    # crossing paths: opponent moves along y at x = 6, ego along x
    N, dt = p["N"], p["dt"]
    opp = np.zeros((N + 1, 8))
    t = np.arange(N + 1) * dt
    opp[:, 0], opp[:, 1], opp[:, 2], opp[:, 3] = 6.0, -3.0 + 8.0 * t, math.pi / 2, 8.0
    opp[:, 6] = 6.0 - X0
    out = orc.best_response(br_inputs(orc, p, 0.0, 0.0, 10.0, [opp]))
    ex = 10.0 * t
    g = np.min(np.hypot(ex[1:] - 6.0, 0.0 - opp[1:, 1]))
    np.testing.assert_allclose(out["rho_obs"], g, rtol=1e-12)


def _random_case(orc, p, K, seed, n_opp=2, d_e=0.0, gap=5.0):
    rng = np.random.default_rng(seed)
    opps = [opp_line(10.0 + 7.0 * j, rng.uniform(-3, 3), 18.0, p["N"], p["dt"]) for j in range(n_opp)]
    ub = np.zeros((p["N"], 2))
    ub[:, 1] = rng.uniform(-0.05, 0.05)
    return br_inputs(orc, p, 10.0 + gap, d_e, 20.0, opps, K=K, ubar=ub)


def test_selection_brute_force(oracle_lib):
    """eq. (selection) and the fallback, against a brute-force argmin over K = 16 samples
    for cases spanning all-feasible, mixed and all-infeasible patterns."""
    p = default_params(20, 3)
    p["sigma_d"] = 0.15  # spread the samples so feasibility patterns vary
    orc = oracle.Oracle(straight(width=9.0), p)
    K = 16
    kinds = set()
    for seed in range(24):
        rng = np.random.default_rng(100 + seed)
        br = _random_case(orc, p, K, seed, d_e=rng.uniform(-3.0, 3.0), gap=rng.uniform(-15.0, 30.0))
        out = orc.best_response(br)
        h = (out["flags"] & 4) > 0
        if h.any():
            idx = np.nonzero(h)[0]
            k = idx[np.argmin(out["cost"][idx])]
            assert out["choice"]["k"] == k and out["choice"]["fallback"] == 0
            kinds.add("all" if h.all() else "mixed")
        else:
            assert out["choice"]["k"] == int(np.argmin(out["viol"])) and out["choice"]["fallback"] == 1
            kinds.add("none")
        assert out["choice"]["n_feasible"] == int(h.sum())
    assert kinds == {"all", "mixed", "none"}


def test_fallback_when_nothing_is_feasible(oracle_lib):
    p = default_params(20, 3)
    orc = oracle.Oracle(straight(), p)
    opp = opp_line(10.0, 0.0, 20.0, p["N"], p["dt"])  # opponent on top of the ego
    out = orc.best_response(br_inputs(orc, p, 10.0, 0.0, 20.0, [opp], K=32))
    assert out["choice"]["fallback"] == 1 and out["choice"]["n_feasible"] == 0
    assert out["choice"]["k"] == int(np.argmin(out["viol"]))
    assert np.all(out["viol"] > 0)


def test_non_finite_samples_are_infeasible(oracle_lib):
    p = default_params(20, 1)
    orc = oracle.Oracle(straight(), p)
    ub = np.full((p["N"], 2), np.nan)
    out = orc.best_response(br_inputs(orc, p, 10.0, 0.0, 20.0, [], K=8, ubar=ub))
    assert np.all(out["flags"] & 16) and np.all(out["viol"] == np.inf)
    assert out["choice"]["k"] == 0 and out["choice"]["fallback"] == 1


def test_single_sample(oracle_lib):
    p = default_params(20, 1)
    orc = oracle.Oracle(straight(), p)
    out = orc.best_response(br_inputs(orc, p, 10.0, 0.0, 20.0, [], K=1))
    assert out["choice"]["k"] == 0


def test_game_cost_is_additive_and_order_invariant(oracle_lib):
    p = default_params(20, 3)
    orc = oracle.Oracle(straight(), p)
    K = 64
    br = _random_case(orc, p, K, 3, n_opp=3, gap=4.0)
    full = orc.best_response(br)["cost"]
    base = orc.best_response(dict(br, w_game=0.0))["cost"]
    parts = 0.0
    for j in range(3):
        one = dict(br, n_opp=1, opp_traj=br["opp_traj"][j:j + 1], opp_s0=br["opp_s0"][j:j + 1])
        parts = parts + (orc.best_response(one)["cost"] - base)
    np.testing.assert_allclose(full - base, parts, rtol=1e-9, atol=1e-7)
    perm = [2, 0, 1]
    shuf = dict(br, opp_traj=br["opp_traj"][perm], opp_s0=br["opp_s0"][perm])
    np.testing.assert_allclose(orc.best_response(shuf)["cost"], full, rtol=1e-12)


def test_zero_game_weight_leaves_tracking_cost(oracle_lib):
    p = default_params(20, 3)
    orc = oracle.Oracle(straight(), p)
    br = _random_case(orc, p, 32, 4)
    out = orc.best_response(dict(br, w_game=0.0))
    np.testing.assert_allclose(out["cost"], out["scale"], rtol=0)
    assert np.all(out["cost"] >= 0)
