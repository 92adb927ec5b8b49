"""Host-side race metrics (Sec. IV-C) on constructed trajectories with known answers."""

import math

import numpy as np
import pytest

from paper_2607_25388_amd import race_eval as RE
from paper_2607_25388_amd.inputs import default_params

P = default_params(40, 3)
DT = 0.05


def _lineup(T, s0, v, lat):
    """Vehicles on a straight line y = lat[j], x = s = s0[j] + v[j] t."""
    n = len(s0)
    t = np.arange(T) * DT
    s = np.stack([s0[j] + v[j] * t for j in range(n)], axis=1)
    d = np.tile(np.asarray(lat, float), (T, 1))
    X = np.zeros((T, n, 6))
    X[..., 0] = s
    X[..., 1] = d
    X[..., 3] = np.asarray(v)[None, :]
    return s, d, X


def test_footprint_distance_closed_form():
    X = np.zeros((2, 6))
    X[1, 1] = 3.0  # side by side, 3 m apart laterally
    dist = RE.footprint_distance(X, P)
    assert dist[0, 1] == pytest.approx(3.0) and dist[1, 0] == pytest.approx(3.0)
    assert math.isinf(dist[0, 0])
    X[1, 1] = 0.0
    X[1, 0] = 5.0  # in line, 5 m apart: nearest discs 5 - 3 = 2 m
    assert RE.footprint_distance(X, P)[0, 1] == pytest.approx(2.0)


def test_overtake_counts_as_clean_win():
    T = 200
    s, d, X = _lineup(T, [0.0, 10.0, 20.0], [30.0, 20.0, 20.0], [-4.0, 0.0, 4.0])
    m = RE.trial_metrics(s, d, X, np.zeros((T, 2)), np.full(T, 6.0), P, DT)
    assert m["win"] and not m["collided"] and m["fpr"] == 1.0
    assert m["duration"] == pytest.approx(T * DT)
    assert m["mcs"] == 0.0


def test_collision_ends_the_trial():
    T = 100
    s, d, X = _lineup(T, [0.0, 30.0], [30.0, 10.0], [0.0, 0.0])
    # the ego closes 20 m/s on a car 30 m ahead: footprints (5 m long discs chain) meet when
    # the centre gap falls below d_col + 3 m = 5 m -> gap 30 - 20 t < 5 -> t > 1.25 s
    m = RE.trial_metrics(s, d, X, np.zeros((T, 2)), np.full(T, 6.0), P, DT)
    assert m["collided"]
    k_end = int(np.nonzero(30.0 - 20.0 * np.arange(T) * DT < 5.0)[0][0])
    assert m["duration"] == pytest.approx((k_end + 1) * DT)


def test_leaving_the_track_ends_the_trial():
    T = 50
    s, d, X = _lineup(T, [0.0, 50.0], [20.0, 20.0], [0.0, 0.0])
    d[:, 0] = np.linspace(0.0, 8.0, T)  # drifts out of a 6 m half width
    m = RE.trial_metrics(s, d, X, np.zeros((T, 2)), np.full(T, 6.0), P, DT)
    assert m["collided"]
    assert m["duration"] == pytest.approx((int(np.nonzero(d[:, 0] > 6.0)[0][0]) + 1) * DT)


def test_close_interaction_segments_and_smoothness():
    T = 12
    s, d, X = _lineup(T, [0.0, 100.0], [0.0, 0.0], [0.0, 5.0])
    lon, lat = RE.csd_box(P)
    # 3 discs 1.5 m apart and d_col = 2 m: bumper contact at 5 m, box 5.56 m x 1.11 m
    assert lon == pytest.approx(5.0 / 0.9) and lat == pytest.approx(1.0 / 0.9)
    # opponent inside the box at steps 2..4 and 7..8
    for k in (2, 3, 4, 7, 8):
        s[k, 1] = s[k, 0] + 0.5 * lon
        d[k, 1] = d[k, 0] + 0.5 * lat
    u = np.zeros((T, 2))
    u[5:, 0] = 1.0  # one unit step in acceleration
    m = RE.trial_metrics(s, d, X, u, np.full(T, 6.0), P, DT)
    assert m["segments"] == pytest.approx([3 * DT, 2 * DT])
    assert m["mcs"] == pytest.approx(1.0 / (T - 1))


def test_summary():
    trials = [dict(win=True, collided=False, fpr=1.0, duration=50.0, segments=[1.0], v_ego=[10.0], mcs=0.1),
              dict(win=True, collided=True, fpr=0.5, duration=10.0, segments=[], v_ego=[20.0], mcs=0.3),
              dict(win=False, collided=False, fpr=0.0, duration=50.0, segments=[3.0], v_ego=[30.0], mcs=0.2)]
    s = RE.summarize(trials, 50.0)
    assert s["wins"] == pytest.approx(2 / 3) and s["cfw"] == pytest.approx(0.5)
    assert s["fpr"] == pytest.approx(0.5) and s["csd_s"] == pytest.approx(2.0)
    assert s["d_mean_s"] == pytest.approx(110 / 3) and s["d_max_s"] == 50.0
    assert s["d_ratio"] == pytest.approx(110 / 150) and s["v_ego_mean"] == pytest.approx(20.0)
    assert s["ego_collisions"] == 1


def _pair(x, y, psi_e, psi_j):
    X = np.zeros((1, 2, 6))
    X[0, 0, 2] = psi_e
    X[0, 1, 0], X[0, 1, 1], X[0, 1, 2] = x, y, psi_j
    return X


@pytest.mark.parametrize("psi", [0.0, 0.7, -2.1])
def test_body_contact_rectangles(psi):
    """0.58 m x 0.31 m bodies: in line they touch below 0.58 m between centres, side by side
    below 0.31 m, crossed at right angles below 0.29 + 0.155 m; a common rotation of the
    scene changes nothing."""
    Lb, Wb = 0.58, 0.31
    c, s = math.cos(psi), math.sin(psi)

    def hit(x, y, dpsi=0.0):  # offset (x, y) in the ego's frame, relative heading dpsi
        return bool(RE.body_contact(_pair(c * x - s * y, s * x + c * y, psi, psi + dpsi), Lb, Wb)[0, 1])

    assert hit(0.57, 0.0) and not hit(0.59, 0.0) and hit(-0.57, 0.0) and not hit(-0.59, 0.0)
    assert hit(0.0, 0.30) and not hit(0.0, 0.32)
    assert hit(0.44, 0.0, math.pi / 2) and not hit(0.45, 0.0, math.pi / 2)
    assert hit(0.0, 0.44, math.pi / 2) and not hit(0.0, 0.45, math.pi / 2)
    # corner to corner: offset (0.57, 0.30) overlaps, (0.59, 0.30) and (0.57, 0.32) do not
    assert hit(0.57, 0.30) and not hit(0.59, 0.30) and not hit(0.57, 0.32)
    # a 45 degree turn: the rotated body reaches 0.29 cos45 + 0.155 sin45 = 0.3147 m along x
    r = 0.29 * math.cos(math.pi / 4) + 0.155 * math.sin(math.pi / 4)
    assert hit(0.29 + r - 0.005, 0.0, math.pi / 4) and not hit(0.29 + r + 0.005, 0.0, math.pi / 4)
    assert not bool(RE.body_contact(_pair(0.0, 0.0, psi, psi), Lb, Wb)[0, 0])  # never the ego itself


def test_contact_criterion_ends_trials_at_touch_not_at_margin():
    """With the 1:10 cars' point footprint (d_col = 0.9 m), trailing 0.7 m behind is a
    breach of d_col but no contact; closing to 0.5 m is contact."""
    from paper_2607_25388_amd.inputs import small_scale_params
    Ps = small_scale_params()
    T = 50
    s, d, X = _lineup(T, [0.0, 0.7], [5.0, 5.0], [0.0, 0.0])
    m = RE.trial_metrics(s, d, X, np.zeros((T, 2)), np.full(T, 1.25), Ps, 0.1, contact=(0.58, 0.31))
    assert not m["collided"] and m["d_col_breach"] and m["duration"] == pytest.approx(T * 0.1)
    m0 = RE.trial_metrics(s, d, X, np.zeros((T, 2)), np.full(T, 1.25), Ps, 0.1)
    assert m0["collided"] and m0["duration"] == pytest.approx(0.1)
    s, d, X = _lineup(T, [0.0, 0.9], [5.0, 3.0], [0.0, 0.0])  # closes 2 m/s: 0.1 m per record
    m = RE.trial_metrics(s, d, X, np.zeros((T, 2)), np.full(T, 1.25), Ps, 0.1, contact=(0.58, 0.31))
    assert m["collided"] and not m["off_track"]
    assert m["duration"] == pytest.approx(5 * 0.1)  # gap 0.9 - 0.1 k < 0.58 first at k = 4


def test_small_scale_setup_is_the_papers():
    """The paper-scale evaluation uses the constants Sec. IV-B prints: K = 128 samples over
    a 1.2 s horizon of H = 12 steps, sigma = (0.335, 0.025), Q, R, S, w_game = 60,
    s_contest = 8 m, s_role = 1 m, mu_tail = 0.3, g_safe = 1.0 m, L_IBR = 2,
    m_bd = 0.515 m, d_col = 0.9 m, game weights (1, 2, 10, 50), 2 m queue spacing,
    three vehicles; a point footprint (eq. Dmin) and the kinematic bicycle."""
    from paper_2607_25388_amd.inputs import small_scale_params
    sc = RE.SCALES["small"]
    p = sc["params"](sc["N"])
    assert sc["K"] == 128 and sc["N"] == 12 and sc["L"] == 2 and sc["spacing"] == 2.0
    assert p["N"] == 12 and p["dt"] * p["N"] == pytest.approx(1.2)
    assert (p["sigma_a"], p["sigma_d"]) == (0.335, 0.025)
    assert p["Q"] == [60.0, 60.0, 47.75, 39.48] and p["R"] == [8.43, 20.0] and p["S"] == [1.0, 19.26]
    assert (p["w_game"], p["s_contest"], p["s_role"], p["g_safe"]) == (60.0, 8.0, 1.0, 1.0)
    assert (p["w_contest"], p["w_long"], p["w_block"], p["w_safety"]) == (1.0, 2.0, 10.0, 50.0)
    assert (p["m_bd"], p["d_col"]) == (0.515, 0.9)
    assert p["n_tail"] == math.ceil(0.3 * 12)
    assert p["model"] == 1 and p["n_disc"] == 1 and p["disc_off"][0] == 0.0
    assert small_scale_params(12) == p
