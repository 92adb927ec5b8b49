"""Pins of the oracle's vehicle models and integrator (Sec. II, f(x, u)).

Closed forms: constant-steer kinematic arc, straight zero-input and
constant-acceleration motion; RK4 convergence order; mirror symmetry of the
single-track model; steady-state yaw rate of the linear-tyre single-track model
(understeer-gradient formula); the integrator against scipy's DOP853.
"""

import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_2607_25388_amd.inputs import default_params, make_straight_track


def make(model, dt=0.05, N=20, **over):
    p = default_params(N, 1, model=model)
    p["dt"] = dt
    p.update(over)
    return oracle.Oracle(make_straight_track(100.0, 10.0), p), p


def kin_arc(p, x0, delta, t):
    """Closed form of the kinematic bicycle at constant speed and steering."""
    L = p["lf"] + p["lr"]
    beta = math.atan(p["lr"] * math.tan(delta) / L)
    v = x0[3]
    R = p["lr"] / math.sin(beta)
    psi = x0[2] + v * t / R
    x = x0[0] + R * (math.sin(psi + beta) - math.sin(x0[2] + beta))
    y = x0[1] - R * (math.cos(psi + beta) - math.cos(x0[2] + beta))
    return np.array([x, y, psi, v])


def run(orc, x0, u, n):
    x = np.array(x0, float)
    for _ in range(n):
        x = orc.step(x, u)
    return x


@pytest.mark.parametrize("delta", [0.05, -0.2, 0.4])
def test_kinematic_constant_steer_arc(oracle_lib, delta):
    orc, p = make(1)
    x0 = [10.0, -3.0, 0.7, 12.0, 0.0, 0.0]
    n = 40
    x = run(orc, x0, [0.0, delta], n)
    ref = kin_arc(p, x0, delta, n * p["dt"])
    # RK4 global error bound for this arc: C * T * (omega*dt)^4 * R, with omega = v/R
    L = p["lf"] + p["lr"]
    beta = math.atan(p["lr"] * math.tan(delta) / L)
    R = p["lr"] / abs(math.sin(beta))
    om = x0[3] / R
    bound = 2.0 * R * (om * p["dt"]) ** 4 * n + 1e-12
    assert np.max(np.abs(x[:2] - ref[:2])) < bound
    assert abs(x[2] - ref[2]) < 1e-12 + bound / R
    assert x[3] == pytest.approx(ref[3], abs=1e-12)


def test_rk4_fourth_order(oracle_lib):
    errs = []
    for dt in (0.1, 0.05, 0.025):
        orc, p = make(1, dt=dt)
        T = 2.0
        n = int(round(T / dt))
        x0 = [0.0, 0.0, 0.0, 15.0, 0.0, 0.0]
        x = run(orc, x0, [0.0, 0.3], n)
        errs.append(np.linalg.norm(x[:2] - kin_arc(p, x0, 0.3, T)[:2]))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 12.0 < r2 < 20.0, errs


@pytest.mark.parametrize("model", [0, 1])
def test_straight_zero_input_is_exact(oracle_lib, model):
    orc, p = make(model)
    psi = 0.3
    x0 = [5.0, 7.0, psi, 20.0, 0.0, 0.0]
    n = 20
    x = run(orc, x0, [0.0, 0.0], n)
    T = n * p["dt"]
    np.testing.assert_allclose(x, [5.0 + 20.0 * T * math.cos(psi), 7.0 + 20.0 * T * math.sin(psi), psi, 20.0, 0, 0],
                               rtol=0, atol=1e-12)


@pytest.mark.parametrize("model", [0, 1])
def test_constant_acceleration_is_exact(oracle_lib, model):
    orc, p = make(model)
    x0 = [0.0, 0.0, 0.0, 10.0, 0.0, 0.0]
    a = 3.0
    n = 20
    x = run(orc, x0, [a, 0.0], n)
    T = n * p["dt"]
    assert x[0] == pytest.approx(10.0 * T + 0.5 * a * T * T, abs=1e-11)
    assert x[3] == pytest.approx(10.0 + a * T, abs=1e-12)
    assert x[1] == 0.0 and x[2] == 0.0


def test_speed_clamped_at_zero(oracle_lib):
    orc, p = make(0)
    x = run(orc, [0, 0, 0, 1.0, 0, 0], [-8.0, 0.0], 10)
    assert x[3] == 0.0 and x[0] >= 0.0


def test_single_track_mirror_symmetry(oracle_lib):
    orc, p = make(0)
    x0 = np.array([3.0, 1.0, 0.2, 18.0, 0.4, -0.1])
    rng = np.random.default_rng(3)
    xm = x0 * np.array([1, -1, -1, 1, -1, -1])
    xa, xb = x0.copy(), xm.copy()
    for _ in range(30):
        u = np.array([rng.uniform(-8, 4), rng.uniform(-0.4, 0.4)])
        xa = orc.step(xa, u)
        xb = orc.step(xb, u * np.array([1, -1]))
    np.testing.assert_allclose(xb, xa * np.array([1, -1, -1, 1, -1, -1]), rtol=0, atol=1e-12)


def test_single_track_steady_state_yaw_rate(oracle_lib):
    """Linear-tyre limit: omega_ss = v delta / (L + K_us v^2),
    K_us = (m/L)(l_r/C_f - l_f/C_r), C = B C mu F_z (initial slope of the tyre curve)."""
    orc, p = make(0)
    L = p["lf"] + p["lr"]
    Fzf = p["m"] * p["g"] * p["lr"] / L
    Fzr = p["m"] * p["g"] * p["lf"] / L
    Cf = p["B"] * p["C"] * p["mu"] * Fzf
    Cr = p["B"] * p["C"] * p["mu"] * Fzr
    Kus = p["m"] / L * (p["lr"] / Cf - p["lf"] / Cr)
    delta = 0.004
    x = np.array([0.0, 0.0, 0.0, 15.0, 0.0, 0.0])
    for _ in range(400):
        x = orc.step(x, [0.0, delta])
    v = x[3]
    om_ss = v * delta / (L + Kus * v * v)
    assert x[5] == pytest.approx(om_ss, rel=2e-3)


def test_rk4_matches_dop853_under_zero_order_hold(oracle_lib):
    """Same ODE (the oracle's own f) integrated by DOP853 at rtol 1e-12: the RK4 error is
    small against the 1e-3 parity scale and shrinks ~16x when the interval is halved."""
    orc, p = make(0)
    orc2, _ = make(0, dt=p["dt"] / 2)
    rng = np.random.default_rng(5)
    x = np.array([0.0, 0.0, 0.1, 20.0, 0.0, 0.0])
    xh = x.copy()
    xi = x.copy()
    for _ in range(20):
        u = np.array([rng.uniform(-3, 3), rng.uniform(-0.05, 0.05)])
        x = orc.step(x, u)
        xh = orc2.step(orc2.step(xh, u), u)
        sol = solve_ivp(lambda t, y: orc.deriv(y, u), (0, p["dt"]), xi, method="DOP853", rtol=1e-12, atol=1e-12)
        xi = sol.y[:, -1]
        xi[3] = max(xi[3], 0.0)
    e1 = np.max(np.abs(x - xi))
    e2 = np.max(np.abs(xh - xi))
    assert e1 < 2e-4
    assert 10.0 < e1 / e2 < 22.0, (e1, e2)
