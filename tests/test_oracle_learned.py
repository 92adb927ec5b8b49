"""Pins of the oracle's learned-proposal pieces (project extension, not in the paper):
MLP gradients against central finite differences, the Gaussian NLL closed form, the
proposal sampler's reduction to the plain sampler, and the feature definitions."""

import math

import numpy as np
import pytest

import oracle
from oracle.ref import MlpOracle, features
from paper_2607_25388_amd.inputs import default_params, make_circle_track, make_race, make_straight_track


def tiny_mlp(seed=0, d_in=5, d_h=7, N=2):
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, 0.5, (d_in, d_h)); b1 = rng.normal(0, 0.1, d_h)
    W2 = rng.normal(0, 0.5, (d_h, d_h)); b2 = rng.normal(0, 0.1, d_h)
    W3 = rng.normal(0, 0.5, (d_h, 4 * N)); b3 = rng.normal(0, 0.1, 4 * N)
    return MlpOracle(W1, b1, W2, b2, W3, b3), rng


def test_gelu_mlp_forward_closed_form(oracle_lib):
    m, rng = tiny_mlp()
    X = rng.normal(size=(3, 5))
    gelu = lambda x: 0.5 * x * (1 + np.tanh(math.sqrt(2 / math.pi) * (x + 0.044715 * x ** 3)))
    W1, b1, W2, b2, W3, b3 = m.arrs
    ref = gelu(gelu(X @ W1 + b1) @ W2 + b2) @ W3 + b3
    np.testing.assert_allclose(m.forward(X), ref, rtol=1e-13, atol=1e-13)


def test_nll_closed_form_and_sigma_identity(oracle_lib):
    m, rng = tiny_mlp()
    out = np.zeros((1, 8))  # mu = 0, sigma = plain
    U = np.array([[[1.0, 0.05], [-2.0, 0.0]]])
    L, g = m.nll(out, U, 1.5, 0.08)
    exp_L = sum(0.5 * (u / s) ** 2 + math.log(s) for u, s in ((1.0, 1.5), (0.05, 0.08), (-2.0, 1.5), (0.0, 0.08)))
    assert L == pytest.approx(exp_L, rel=1e-14)
    prop = m.proposal(out[0], 2, 1.5, 0.08)
    np.testing.assert_allclose(prop, [[0, 0, 1.5, 0.08], [0, 0, 1.5, 0.08]], rtol=1e-15)
    # residual form: zero outputs give the nominal sequence with the plain scales
    ubar = np.array([[0.5, -0.1], [-1.0, 0.2]])
    prop = m.proposal(out[0], 2, 1.5, 0.08, ubar=ubar)
    np.testing.assert_allclose(prop, [[0.5, -0.1, 1.5, 0.08], [-1.0, 0.2, 1.5, 0.08]], rtol=1e-15)
    # clamps of the log-scale offsets and the mean scales
    o = np.array([1.0, 1.0, -10.0, 10.0])
    prop = m.proposal(o, 1, 1.5, 0.08, ubar=np.array([[0.5, -0.1]]))
    np.testing.assert_allclose(prop, [[4.5, 0.1, 1.5 * math.exp(-4.0), 0.08 * math.e]], rtol=1e-15)


def test_backprop_matches_central_differences(oracle_lib):
    m, rng = tiny_mlp(1)
    B, N = 4, 2
    X = rng.normal(size=(B, 5))
    U = rng.normal(0, 1, (B, N, 2)) * np.array([1.5, 0.08])

    def loss():
        return m.nll(m.forward(X), U, 1.5, 0.08, grad=False)[0]

    out = m.forward(X)
    L, g = m.nll(out, U, 1.5, 0.08)
    grads = m.backward(X, g)
    for arr, gr in zip(m.arrs, grads):
        flat = arr.reshape(-1)
        gflat = gr.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            h = 1e-6
            old = flat[idx]
            flat[idx] = old + h
            lp = loss()
            flat[idx] = old - h
            lm = loss()
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert gflat[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_proposal_equal_to_nominal_reproduces_the_plain_sampler(oracle_lib):
    tr = make_straight_track(400.0, 10.0, x0=-50.0)
    p = default_params(20, 3)
    orc = oracle.Oracle(tr, p)
    race = make_race(tr, 3, 20, 10.0, False, 5, 6)
    race.u_nom = np.random.default_rng(2).normal(0, 0.3, (3, 20, 2)).astype(np.float32) * np.array([1, 0.1], np.float32)
    plain = orc.rollout_cost(race, 1, 1, 256)
    prop = np.zeros((3, 20, 4))
    prop[:, :, :2] = race.u_nom
    prop[:, :, 2] = p["sigma_a"]
    prop[:, :, 3] = p["sigma_d"]
    learned = orc.rollout_cost(race, 1, 1, 256, prop=prop, K_prop=256)
    np.testing.assert_array_equal(plain["cost"], learned["cost"])
    # a different proposal changes exactly the samples k < K_prop
    prop2 = prop.copy()
    prop2[:, :, 0] += 1.0
    mixed = orc.rollout_cost(race, 1, 1, 256, prop=prop2, K_prop=100)
    assert np.all(mixed["cost"][100:] == plain["cost"][100:])
    assert np.all(mixed["cost"][:100] != plain["cost"][:100])


def test_features_on_straight_and_circle_tracks(oracle_lib):
    tr = make_straight_track(400.0, 10.0, x0=0.0, vref=20.0)
    p = default_params(20, 1)
    orc = oracle.Oracle(tr, p)
    race = make_race(tr, 3, 20, 10.0, False, 5, 6)
    race.x[:, 1] = [1.0, -2.0, 0.5]  # lateral offsets
    race.x[:, 3] = [15.0, 16.0, 17.0]
    X = features(orc, race)
    np.testing.assert_allclose(X[:, 0], np.array([1.0, -2.0, 0.5]) / 5.0, atol=1e-12)
    np.testing.assert_allclose(X[:, 1], 0.0, atol=1e-12)
    np.testing.assert_allclose(X[:, 5], (race.x[:, 3] - 20.0) / 10.0, atol=1e-12)
    # ego's nearest opponents: +10 m then +20 m ahead
    np.testing.assert_allclose(X[0, 6:12], [0.5, (-2.0 - 1.0) / 5.0, 0.0, 0.1, 0.0, 1.0], atol=1e-12)
    np.testing.assert_allclose(X[0, 12:18], [1.0, (0.5 - 1.0) / 5.0, 0.0, 0.2, 0.0, 1.0], atol=1e-12)
    np.testing.assert_allclose(X[0, 18:30], 0.0)  # absent opponents
    np.testing.assert_allclose(X[:, 30:], 0.0, atol=1e-12)  # straight: no curvature
    ct = make_circle_track(40.0, 10.0)
    orc2 = oracle.Oracle(ct, p)
    race2 = make_race(ct, 2, 20, 10.0, False, 7, 8)
    X2 = features(orc2, race2)
    np.testing.assert_allclose(X2[:, 30:], 20.0 / 40.0, rtol=1e-12)


def _identity_net(a, c, w, b3):
    """A network whose output is known without evaluating GELU: the tanh-form GELU g
    satisfies g(u) - g(-u) = u (tanh is odd), so with hidden pairs (g(u), g(-u)) the
    next layer recovers u exactly.  Layer 1: u = a . x + c; layer 2 pre-activations
    (u, -u); output_j = w_j (g(u) - g(-u)) + b3_j = w_j u + b3_j.  Shapes d_in = len(a),
    d_h = 2, d_out = len(w) make a transposed weight or a misplaced bias fail."""
    a = np.asarray(a, float)
    W1 = np.stack([a, -a], axis=1)                   # [d_in][2]
    b1 = np.array([c, -c])
    W2 = np.array([[1.0, -1.0], [-1.0, 1.0]])        # pre2 = (h0 - h1, h1 - h0)
    b2 = np.zeros(2)
    w = np.asarray(w, float)
    W3 = np.stack([w, -w], axis=0)                   # [2][d_out]
    return MlpOracle(W1, b1, W2, b2, W3, np.asarray(b3, float))


def test_mlp_forward_wiring_on_a_network_with_a_closed_form(oracle_lib):
    a, c = [0.7, -1.3, 0.25], 0.4
    w = np.linspace(-2.0, 1.5, 8)
    b3 = np.linspace(0.5, -0.5, 8)
    m = _identity_net(a, c, w, b3)
    X = np.array([[0.1, 0.2, 0.3], [-1.0, 0.5, 2.0], [3.0, -2.0, 0.0], [0.0, 0.0, 0.0]])
    u = X @ np.array(a) + c
    out, (pre1, h1, pre2, h2) = m.forward(X, intermediates=True)
    np.testing.assert_allclose(out, u[:, None] * w[None, :] + b3[None, :], rtol=0, atol=1e-12)
    np.testing.assert_allclose(pre1, np.stack([u, -u], 1), rtol=0, atol=1e-14)
    np.testing.assert_allclose(pre2, np.stack([u, -u], 1), rtol=0, atol=1e-13)
    # hidden activations: g(u) + g(-u) = u tanh(c (u + k u^3)) >= 0, and g(u) - g(-u) = u
    np.testing.assert_allclose(h1[:, 0] - h1[:, 1], u, rtol=0, atol=1e-14)
    assert np.all(h1[:, 0] + h1[:, 1] >= 0.0)


def test_mlp_activation_is_the_tanh_form_of_gelu(oracle_lib):
    """The activation read out through the network (output = g(x)) against the exact GELU
    x Phi(x) (scipy's erf): the tanh form of Hendrycks and Gimpel stays within 4.8e-4 of
    it everywhere, while a wrong constant (sqrt(2/pi) -> 0.8, 0.044715 -> 0.04) does not;
    g(0) = 0, g(x) -> x for large x and -> 0 for very negative x."""
    from scipy.special import erf

    # layer 1: (x, -x); layer 2: (g(x) - g(-x), 0) = (x, 0); output g(x) - g(0) = g(x)
    W1 = np.array([[1.0, -1.0]]); b1 = np.zeros(2)
    W2 = np.array([[1.0, 0.0], [-1.0, 0.0]]); b2 = np.zeros(2)
    W3 = np.array([[1.0], [0.0]]); b3 = np.zeros(1)
    m = MlpOracle(W1, b1, W2, b2, W3, b3)
    x = np.linspace(-8.0, 8.0, 4001)
    g = m.forward(x[:, None])[:, 0]
    exact = 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))
    dev = np.abs(g - exact).max()
    assert 4.0e-4 < dev < 4.8e-4, dev
    assert g[2000] == 0.0
    assert g[-1] == pytest.approx(8.0, abs=1e-12)
    assert abs(g[0]) < 1e-12
