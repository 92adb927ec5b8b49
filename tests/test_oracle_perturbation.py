"""Pins of the oracle's opponent-prediction perturbation (robustness experiment,
Sec. IV-F, Table II; reading in the oracle's header comment): each predicted position
moves by sigma_lon z0 along and sigma_lat z1 across the predicted heading, (z0, z1) the
Gaussian pair of a Philox call with a counter of its own."""

import math

import numpy as np
import pytest

import oracle
from paper_2607_25388_amd.inputs import default_params, make_straight_track


def _pred(N, rng):
    tr = np.zeros((N + 1, 8))
    tr[:, 0] = rng.uniform(-100, 100, N + 1)
    tr[:, 1] = rng.uniform(-100, 100, N + 1)
    tr[:, 2] = rng.uniform(-math.pi, math.pi, N + 1)
    tr[:, 3:] = rng.uniform(0, 10, (N + 1, 5))
    return tr


@pytest.fixture(scope="module")
def orcs(oracle_lib):
    track = make_straight_track(100.0, 10.0)
    p = default_params(20, 3)
    return (oracle.Oracle(track, p), oracle.Oracle(track, dict(p, pred_sig_lon=0.3, pred_sig_lat=0.1)), p)


def test_zero_scales_leave_the_prediction(orcs):
    plain, _, p = orcs
    tr = _pred(20, np.random.default_rng(0))
    np.testing.assert_array_equal(plain.perturb_prediction(tr, 7, 3, 0, 1, 2), tr)


@pytest.mark.parametrize("observer,phase,j,step", [(0, 0, 1, 0), (2, 3, 0, 17), (1, 1, 5, 99)])
def test_displacement_is_the_gaussian_pair_in_the_heading_frame(orcs, observer, phase, j, step):
    plain, pert, p = orcs
    seed = 123456789012345
    tr = _pred(20, np.random.default_rng(observer + 10 * j))
    out = pert.perturb_prediction(tr, seed, step, observer, phase, j)
    np.testing.assert_array_equal(out[0], tr[0])
    np.testing.assert_array_equal(out[:, 2:], tr[:, 2:])
    key = (seed & 0xffffffff, seed >> 32)
    for tau in range(1, 21):
        r = plain.philox((0x80000000 | j, tau, observer | (phase << 16), step), key)
        z = plain.gauss_pair(r[0], r[1])
        dx, dy = out[tau, 0] - tr[tau, 0], out[tau, 1] - tr[tau, 1]
        c, s = math.cos(tr[tau, 2]), math.sin(tr[tau, 2])
        assert dx * c + dy * s == pytest.approx(0.3 * float(z[0]), abs=1e-12)
        assert -dx * s + dy * c == pytest.approx(0.1 * float(z[1]), abs=1e-12)


def test_displacement_statistics(orcs):
    _, pert, p = orcs
    tr = np.zeros((51, 8))
    lon, lat = [], []
    for obs in range(4):
        for j in range(50):
            out = pert.perturb_prediction(tr, 42, 0, obs, 1, j)
            lon.extend(out[1:, 0])  # heading 0: along = x, across = y
            lat.extend(out[1:, 1])
    lon, lat = np.array(lon), np.array(lat)
    assert len(lon) == 10000
    assert abs(lon.std() / 0.3 - 1.0) < 0.04 and abs(lat.std() / 0.1 - 1.0) < 0.04
    assert abs(lon.mean()) < 4 * 0.3 / 100 and abs(lat.mean()) < 4 * 0.1 / 100
    assert abs(np.corrcoef(lon, lat)[0, 1]) < 0.04
