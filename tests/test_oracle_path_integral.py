"""Pins of the oracle's path-integral best response (the paper's GA-IBR-MPPI ablation,
Sec. IV-A: the nominal is updated by MPPI importance weighting instead of feasibility
selection).

The adopted sequence is checked against limits with known answers: a vanishing
temperature gives the lowest-score sample, an infinite one the plain mean of the
samples; at a finite temperature a brute-force softmax over the per-sample scores and
controls of tiny K (each sample's controls taken from the plain best response with that
sample forced).
"""

import numpy as np
import pytest

import oracle
from paper_2607_25388_amd.inputs import default_params
from test_oracle_cost import br_inputs, opp_line, straight


@pytest.fixture(scope="module")
def case(oracle_lib):
    p = default_params(20, 1)
    tr = straight()
    N = p["N"]
    ub = np.zeros((N, 2))
    ub[:, 0] = 0.5
    opp = opp_line(14.0, 1.0, 20.0, N, p["dt"])
    return p, tr, ub, opp


def _samples(p, tr, ub, opp, K):
    """Per-sample cost, violation and controls of the plain best response."""
    orc = oracle.Oracle(tr, p)
    br = br_inputs(orc, p, 10.0, 0.0, 20.0, [opp], K=K, ubar=ub)
    out = orc.best_response(br)
    U = np.stack([orc.best_response(br, k_force=k, want_samples=False)["U"] for k in range(K)])
    return br, out["cost"], out["viol"], out["flags"], U


def _pi(p, tr, br, lam, w_viol):
    q = dict(p, update=1, mppi_lambda=lam, mppi_w_viol=w_viol)
    return oracle.Oracle(tr, q).best_response(br, want_samples=False)


@pytest.mark.parametrize("w_viol", [0.0, 100.0])
def test_zero_temperature_adopts_lowest_score(case, w_viol):
    p, tr, ub, opp = case
    br, cost, viol, flags, U = _samples(p, tr, ub, opp, 24)
    S = cost + w_viol * viol
    k = int(np.argmin(S))
    out = _pi(p, tr, br, 1e-12, w_viol)
    assert out["choice"]["k"] == k and out["choice"]["fallback"] == 0
    assert out["choice"]["cost"] == pytest.approx(S[k], rel=1e-15)
    assert out["choice"]["n_feasible"] == int(((flags & 4) > 0).sum())
    np.testing.assert_allclose(out["U"], U[k], rtol=0, atol=1e-15)


def test_infinite_temperature_is_the_sample_mean(case):
    p, tr, ub, opp = case
    br, cost, viol, flags, U = _samples(p, tr, ub, opp, 16)
    out = _pi(p, tr, br, 1e300, 0.0)
    np.testing.assert_allclose(out["U"], U.mean(axis=0), rtol=0, atol=1e-12)


@pytest.mark.parametrize("lam", [1.0, 30.0, 500.0])
def test_softmax_weighting_brute_force(case, lam):
    p, tr, ub, opp = case
    br, cost, viol, flags, U = _samples(p, tr, ub, opp, 16)
    S = cost + 10.0 * viol
    w = np.exp(-(S - S.min()) / lam)
    expect = (w[:, None, None] * U).sum(axis=0) / w.sum()
    out = _pi(p, tr, br, lam, 10.0)
    np.testing.assert_allclose(out["U"], expect, rtol=1e-12, atol=1e-13)
    # a convex combination of clipped sequences stays inside the control box
    assert np.all(out["U"][:, 0] >= p["a_min"]) and np.all(out["U"][:, 0] <= p["a_max"])


def test_plan_step_reduces_to_selection(oracle_lib):
    """With a vanishing temperature and an overwhelming violation weight the lowest score
    is the feasible sample of lowest cost (or the least-violation one), so the
    path-integral planning step reproduces the feasibility-selection step exactly."""
    from paper_2607_25388_amd.inputs import make_fourier_track, make_race
    tr = make_fourier_track(300.0, 10.0, 1000)
    p = default_params(20, 1)
    race = make_race(tr, 3, 20, 10.0, False, 3000, 2000)
    plain = oracle.Oracle(tr, p).plan_step(race, 2, K=128)
    pi = oracle.Oracle(tr, dict(p, update=1, mppi_lambda=1e-12, mppi_w_viol=1e12)).plan_step(race, 2, K=128)
    for a, b in zip(plain["trace"], pi["trace"]):
        assert [c["k"] for c in a] == [c["k"] for c in b]
    for key in ("u_apply", "u_next", "traj", "s_abs"):
        np.testing.assert_array_equal(plain[key], pi[key])
    # warm start: shifted, last entry repeated
    for i in range(3):
        np.testing.assert_array_equal(pi["u_next"][i, -1], pi["u_next"][i, -2])


def test_plan_step_finite_temperature(oracle_lib):
    from paper_2607_25388_amd.inputs import make_fourier_track, make_race
    tr = make_fourier_track(300.0, 10.0, 1000)
    p = dict(default_params(20, 1), update=1, mppi_lambda=50.0, mppi_w_viol=0.0)
    race = make_race(tr, 3, 20, 10.0, False, 3000, 2000)
    out = oracle.Oracle(tr, p).plan_step(race, 2, K=128)
    assert np.all(np.isfinite(out["u_apply"])) and np.all(np.isfinite(out["traj"]))
    assert np.all(out["u_next"][..., 0] >= p["a_min"]) and np.all(out["u_next"][..., 0] <= p["a_max"])
    assert np.all(np.abs(out["u_next"][..., 1]) <= p["d_max"])
    for ph in out["trace"][:3]:
        for c in ph:
            assert c["fallback"] == 0 and np.isfinite(c["cost"])


def test_rejects_nonpositive_temperature(case):
    p, tr, ub, opp = case
    orc = oracle.Oracle(tr, dict(p, update=1, mppi_lambda=0.0))
    br = br_inputs(orc, p, 10.0, 0.0, 20.0, [opp], K=4, ubar=ub)
    with pytest.raises(RuntimeError):
        orc.best_response(br)
