"""Pins of the oracle's Frenet projection s(x;G), d(x;G) and reference recursion (Sec. II, III-A).

Straight-track closed form, circle-track polar closed form within the chord
bound, a brute-force foot search on a random track, continuity across nodes,
agreement of the local search with the global one, and the reference
progress recursion with constant v^r.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2607_25388_amd.inputs import default_params, make_circle_track, make_fourier_track, make_straight_track


def test_straight_track_exact(oracle_lib):
    h = 0.4
    tr = make_straight_track(200.0, 10.0, x0=100.0, y0=-50.0, heading=h)
    orc = oracle.Oracle(tr, default_params(20, 1))
    rng = np.random.default_rng(0)
    for _ in range(200):
        s_true = rng.uniform(1.0, 199.0)
        d_true = rng.uniform(-6.0, 6.0)
        p = [100.0 + s_true * math.cos(h) - d_true * math.sin(h), -50.0 + s_true * math.sin(h) + d_true * math.cos(h)]
        seg, s, d, t = orc.project_global(p)
        assert s == pytest.approx(s_true, abs=1e-9)
        assert d == pytest.approx(d_true, abs=1e-9)
        assert seg == int(s_true // 0.5) or abs(s_true / 0.5 - round(s_true / 0.5)) < 1e-9


def test_circle_track_polar_closed_form(oracle_lib):
    R = 40.0
    tr = make_circle_track(R, 10.0, ds=0.5)
    orc = oracle.Oracle(tr, default_params(20, 1))
    dth = 2 * math.pi / tr.n
    sagitta = R * (1 - math.cos(dth / 2))
    rng = np.random.default_rng(1)
    for _ in range(300):
        th = rng.uniform(0, 2 * math.pi)
        r = rng.uniform(R - 5.0, R + 5.0)
        p = [r * math.sin(th), -r * math.cos(th)]  # centre (0,0); track starts at (0,-R) heading +x
        seg, s, d, t = orc.project_global(p)
        assert d == pytest.approx(R - r, abs=sagitta + 1e-9)  # left (inside) positive
        # arc length of the polar angle, within O(R dth^3)
        assert s == pytest.approx(R * th, abs=1e-4 + R * dth ** 3)


def test_foot_matches_brute_force(oracle_lib):
    tr = make_fourier_track(300.0, 10.0, 77)
    orc = oracle.Oracle(tr, default_params(20, 1))
    nd = tr.nodes
    rng = np.random.default_rng(2)
    for _ in range(100):
        i = int(rng.integers(0, tr.n))
        j = (i + 1) % tr.n
        P0, P1 = nd[i, :2], nd[j, :2]
        N0 = np.array([-math.sin(nd[i, 2]), math.cos(nd[i, 2])])
        N1 = np.array([-math.sin(nd[j, 2]), math.cos(nd[j, 2])])
        t_true = rng.uniform(0.02, 0.98)
        d_true = rng.uniform(-5.0, 5.0)
        c = P0 + t_true * (P1 - P0)
        n = N0 + t_true * (N1 - N0)
        p = c + d_true * n / np.linalg.norm(n)
        seg, info = orc.project_walk(p, i)
        assert seg == i
        assert info["t"] == pytest.approx(t_true, abs=1e-9)
        assert info["d"] == pytest.approx(d_true, abs=1e-9)
        # brute force on a fine grid: |p - c(t)| along n(t) is the sign change of cross(p - c, n)
        ts = np.linspace(0, 1, 20001)
        cs = P0[None] + ts[:, None] * (P1 - P0)[None]
        ns = N0[None] + ts[:, None] * (N1 - N0)[None]
        cr = (p[0] - cs[:, 0]) * ns[:, 1] - (p[1] - cs[:, 1]) * ns[:, 0]
        k = np.nonzero(np.sign(cr[:-1]) != np.sign(cr[1:]))[0]
        assert len(k) == 1 and abs(ts[k[0]] - info["t"]) <= 1e-4


def test_continuity_across_nodes(oracle_lib):
    tr = make_fourier_track(300.0, 10.0, 78)
    orc = oracle.Oracle(tr, default_params(20, 1))
    rng = np.random.default_rng(4)
    for _ in range(50):
        i = int(rng.integers(0, tr.n))
        nd = tr.nodes[i]
        d = rng.uniform(-5, 5)
        base = np.array([nd[0] - d * math.sin(nd[2]), nd[1] + d * math.cos(nd[2])])
        tang = np.array([math.cos(nd[2]), math.sin(nd[2])])
        vals = []
        for eps in (-1e-6, 1e-6):
            seg, info = orc.project_walk(base + eps * tang, i)
            vals.append((info["s"], info["d"]))
        assert abs(vals[0][0] - vals[1][0]) < 1e-5
        assert abs(vals[0][1] - vals[1][1]) < 1e-5


def test_walk_agrees_with_global_and_flags_limit(oracle_lib):
    tr = make_fourier_track(300.0, 10.0, 79)
    orc = oracle.Oracle(tr, default_params(20, 1))
    rng = np.random.default_rng(5)
    for _ in range(100):
        i = int(rng.integers(0, tr.n))
        nd = tr.nodes[(i + int(rng.integers(-6, 7))) % tr.n]
        d = rng.uniform(-5, 5)
        p = [nd[0] - d * math.sin(nd[2]) + 0.1, nd[1] + d * math.cos(nd[2])]
        seg_g, s_g, d_g, _ = orc.project_global(p)
        seg_w, info = orc.project_walk(p, i)
        assert not info["limit"]
        assert seg_w % tr.n == seg_g
        s_w = info["s"] - math.floor(seg_w / tr.n) * tr.length
        assert s_w == pytest.approx(s_g, abs=1e-9)
        assert info["d"] == pytest.approx(d_g, abs=1e-9)
    # a point 20 segments away cannot be reached with 16 moves
    nd = tr.nodes[40]
    seg_w, info = orc.project_walk(nd[:2], 20, max_moves=16)
    assert info["limit"] and seg_w == 36


def test_unwrapped_progress_across_the_lap(oracle_lib):
    tr = make_fourier_track(300.0, 10.0, 80)
    orc = oracle.Oracle(tr, default_params(20, 1))
    nd = tr.nodes[2]
    seg, info = orc.project_walk(nd[:2] + 0.01, tr.n - 2)  # start search on the previous lap's tail
    assert seg == tr.n + 2 - (1 if info["t"] > 0.999 else 0) or seg == tr.n + 2
    assert info["s"] == pytest.approx(tr.length + nd[7], abs=0.05)


def test_reference_recursion_constant_speed(oracle_lib):
    tr = make_straight_track(300.0, 10.0, vref=20.0)
    p = default_params(20, 1)
    orc = oracle.Oracle(tr, p)
    lam = 0.9
    s0 = 12.3
    xr = orc.reference(int(s0 // 0.5), s0, lam)
    tau = np.arange(1, 21)
    s_r = s0 + tau * p["dt"] * lam * 20.0
    np.testing.assert_allclose(xr[:, 0], s_r, atol=1e-9)
    np.testing.assert_allclose(xr[:, 1], 0.0, atol=1e-12)
    np.testing.assert_allclose(xr[:, 3], lam * 20.0, atol=1e-12)


def test_reference_recursion_variable_speed_is_euler(oracle_lib):
    """s^r_{t+1} = s^r_t + dt v^r(s^r_t): forward Euler on the speed profile, checked step by step."""
    tr = make_fourier_track(300.0, 10.0, 81)
    p = default_params(20, 1)
    orc = oracle.Oracle(tr, p)
    s0 = 37.25
    xr = orc.reference(int(s0 // 0.5), s0, 1.0)
    nd = tr.nodes
    s_grid = np.concatenate([nd[:, 7], [tr.length]])
    v_grid = np.concatenate([nd[:, 6], [nd[0, 6]]])
    s = s0
    for t in range(20):
        s = s + p["dt"] * np.interp(s % tr.length, s_grid, v_grid)
        assert xr[t, 3] == pytest.approx(np.interp(s % tr.length, s_grid, v_grid), abs=1e-9)
        x_i = np.interp(s % tr.length, s_grid, np.concatenate([nd[:, 0], [nd[0, 0]]]))
        assert xr[t, 0] == pytest.approx(x_i, abs=1e-9)
