"""The element-by-element bounds of the network parity tests, checked on the CPU: a float32
evaluation of the network in the kernels' model (BF16 operands, float32 sums in another
order, float32 GELU) stays inside them against the oracle's BF16-operand mode, and the
oracle without the operand roundings (a plausible mistake in the model) leaves them."""

import numpy as np
import pytest

import mlp_bounds as MB
from oracle.ref import MlpOracle

SHAPES = (("W1", (50, 256)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)), ("W3", (256, 200)), ("b3", (200,)))


def _params(seed, scale3=3.0):
    rng = np.random.default_rng(seed)
    P = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            P[name] = (rng.standard_normal(shp) * np.sqrt(2.0 / shp[0]) * (0.1 * scale3 if name == "W3" else 1.0))
        else:
            P[name] = 0.1 * rng.standard_normal(shp)
        P[name] = P[name].astype(np.float32).astype(np.float64)
    return P


def _f32(a):
    return np.asarray(a, np.float32)


def _bf(a):
    return MB.bf16(a).astype(np.float32)


def _gelu32(x):
    x = _f32(x)
    c, a = np.float32(0.7978845608), np.float32(0.044715)
    return np.float32(0.5) * x * (np.float32(1.0) + np.tanh(c * (x + a * x * x * x)))


def _gelu_grad32(x):
    x = _f32(x)
    c, a = np.float32(0.7978845608), np.float32(0.044715)
    t = np.tanh(c * (x + a * x * x * x))
    return np.float32(0.5) * (np.float32(1.0) + t) + np.float32(0.5) * x * (np.float32(1.0) - t * t) * c * \
        (np.float32(1.0) + np.float32(3.0) * a * x * x)


def _emulate(P, X, U, sig_a, sig_d):
    """Float32 evaluation in the kernels' arithmetic model (sums in numpy's order)."""
    W = {k: (_bf(v) if k.startswith("W") else _f32(v)) for k, v in P.items()}
    xb = _bf(X)
    pre1 = xb @ W["W1"] + W["b1"]
    h1 = _bf(_gelu32(pre1))
    pre2 = h1 @ W["W2"] + W["b2"]
    h2 = _bf(_gelu32(pre2))
    out = h2 @ W["W3"] + W["b3"]
    B, N = U.shape[0], U.shape[1]
    D = np.zeros_like(out)
    terms = []
    for c, (scale, sig) in enumerate(((np.float32(4.0), sig_a), (np.float32(0.2), sig_d))):
        cm = 4 * np.arange(N) + c
        mu = scale * out[:, cm]
        raw = out[:, cm + 2]
        ls = np.log(np.float32(sig)) + np.clip(raw, np.float32(-4.0), np.float32(1.0))
        inv = np.exp(np.float32(-2.0) * ls)
        res = _f32(U[:, :, c]) - mu
        terms.append(np.float32(0.5) * res * res * inv + ls)
        D[:, cm] = _bf(-scale * res * inv / np.float32(B))
        D[:, cm + 2] = _bf(np.where((raw > -4.0) & (raw < 1.0), (np.float32(1.0) - res * res * inv) / np.float32(B),
                                    np.float32(0.0)))
    loss = np.float32(np.sum(np.concatenate([t.ravel() for t in terms]), dtype=np.float32) / np.float32(B))
    g = {"W3": h2.T @ D, "b3": D.sum(0, dtype=np.float32)}
    D2 = _bf((D @ W["W3"].T) * _gelu_grad32(pre2))
    g["W2"], g["b2"] = h1.T @ D2, D2.sum(0, dtype=np.float32)
    D1 = _bf((D2 @ W["W2"].T) * _gelu_grad32(pre1))
    g["W1"], g["b1"] = xb.T @ D1, D1.sum(0, dtype=np.float32)
    f = lambda a: np.asarray(a, np.float64)
    return dict(h1=f(h1), h2=f(h2), out=f(out), d3=f(D), d2=f(D2), d1=f(D1), loss=float(loss),
                grads={k: f(v) for k, v in g.items()})


def _case(seed, B, N):
    P = _params(seed)
    rng = np.random.default_rng(seed + 10)
    X = rng.standard_normal((B, 50)).astype(np.float32)
    U = np.stack([rng.uniform(-8, 4, (B, N)), rng.uniform(-0.4, 0.4, (B, N))], -1).astype(np.float32)
    return P, X.astype(np.float64), U.astype(np.float64), float(np.float32(1.5)), float(np.float32(0.08))


@pytest.mark.parametrize("B,N,seed", [(200, 50, 1), (600, 40, 2)])
def test_float32_evaluation_passes_the_lockstep_comparison(oracle_lib, B, N, seed):
    P, X, U, sa, sd = _case(seed, B, N)
    side = _emulate(P, X, U, sa, sd)
    orc = MlpOracle(*[P[n] for n, _ in SHAPES], bf16=True)
    st = MB.lockstep(orc, P, X, U, sa, sd, side)
    print(st)
    # the rounding decisions agree almost everywhere; the gradient bounds are a small
    # fraction of the values
    for k, n in st["values"].items():
        assert st[k + "_equal"] >= 0.99 * n, (k, st[k + "_equal"], n)
    for nm in MB.NAMES:
        assert st[nm + "_median_rel_bound"] < 1e-3, (nm, st[nm + "_median_rel_bound"])


def test_oracle_without_operand_rounding_fails_the_comparison(oracle_lib):
    """An oracle that skipped the BF16 operand roundings (a plausible modelling mistake)
    fails the comparison: the check separates the kernels' arithmetic from a float64
    network."""
    P, X, U, sa, sd = _case(5, 128, 50)
    side = _emulate(P, X, U, sa, sd)
    orc = MlpOracle(*[P[n] for n, _ in SHAPES], bf16=False)
    with pytest.raises(AssertionError):
        MB.lockstep(orc, P, X, U, sa, sd, side)


@pytest.mark.parametrize("what", ["h2", "d1"])
def test_a_wrong_rounding_fails_the_comparison(oracle_lib, what):
    """One BF16 value moved by one step where the oracle leaves no doubt is caught."""
    P, X, U, sa, sd = _case(6, 64, 30)
    side = _emulate(P, X, U, sa, sd)
    orc = MlpOracle(*[P[n] for n, _ in SHAPES], bf16=True)
    a = side[what]
    i = np.unravel_index(np.argmax(np.abs(a)), a.shape)
    a[i] += 2.0 ** (np.floor(np.log2(abs(a[i]))) - 7) * np.sign(a[i])  # the next BF16 value outwards
    assert MB.bf16(a[i]) == a[i]
    with pytest.raises(AssertionError):
        MB.lockstep(orc, P, X, U, sa, sd, side)
