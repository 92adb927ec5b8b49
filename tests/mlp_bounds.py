"""Element-by-element lockstep comparison of an implementation of the proposal network in
the kernels' arithmetic (BF16 operands, float32 accumulation, float32 GELU) with the
oracle's network in its BF16-operand mode (same operand roundings, float64 arithmetic).

Rounding a hidden activation or a gradient to BF16 is a quantisation decision: where the
two sides' values straddle a BF16 rounding boundary, both roundings are correct results
of the arithmetic.  So the comparison runs in lockstep, layer by layer, as the planner's
parity tests do with near-tied choices:

  1. every BF16 value of the implementation must be a rounding of some value within the
     derived bound of the oracle's value before rounding: it lies in
     [bf16(v - d), bf16(v + d)] (BF16 rounding through float32, both to nearest, is
     monotone), which for all but values next to a rounding boundary means it equals the
     oracle's own rounding bf16(v);
  2. the oracle then continues from the implementation's BF16 values (it adopts them),
     so every later layer sees the same operands on both sides;
  3. with equal operands, every float32 output differs from the oracle's only by float32
     accumulation: a float32 sum of n terms in any order and grouping is within
     gamma(n) = n u / (1 - n u), u = 2^-24, times the sum of the absolute terms, of the
     exact sum (products of two BF16 values are exact in float32).

The GELU and its derivative are evaluated in float32 with tanhf; their errors are bounded
by a few units of 2^-24 in the absolute size of the terms (eps_gelu, eps_gelu_grad), and
they are Lipschitz with constants 1.129 and 0.798 (maxima of |GELU'| and |GELU''| of the
tanh form on the real line).  No bound is fitted to data.
"""

from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
GELU_C = 0.7978845608028654
GELU_LIP = 1.13
GELU_GRAD_LIP = 0.80
A_SCALE, D_SCALE, LS_MIN, LS_MAX = 4.0, 0.2, -4.0, 1.0
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def gam(n):
    return n * U32 / (1.0 - n * U32)


def bf16(a):
    """Round to float32 (nearest even), then to bfloat16 (nearest even); as float64."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = np.where(finite, (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000, u).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    t = np.tanh(GELU_C * (x + 0.044715 * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * 0.044715 * x * x)


def eps_gelu(x):
    # 0.5 x (1 + t): tanhf within a few ulp, i.e. a few units of 2^-24 absolute near
    # |t| = 1; its argument within 3 ulp; 1 + t and two products rounded
    return U32 * (16.0 * np.abs(x) + 1e-30)


def eps_gelu_grad(x):
    # 0.5 (1 + t) + 0.5 x (1 - t^2) c (1 + 3 a x^2): 1 - t^2 carries an absolute error of
    # a few units of 2^-24 however small it is, times the polynomial in x
    ax = np.abs(x)
    return U32 * (8.0 + 8.0 * ax * (1.0 + 0.134 * ax * ax))


def check_rounding(name, got, v, d):
    """Step 1: got (BF16 values of the implementation) within [bf16(v - d), bf16(v + d)].
    Returns the number of values equal to the oracle's own rounding."""
    d = d * 1.0001 + 1e-12 * np.abs(v)
    lo, hi = bf16(v - d), bf16(v + d)
    bad = np.nonzero(~((got >= lo) & (got <= hi)))
    assert len(bad[0]) == 0, (f"{name}: {len(bad[0])} values are no rounding within the bound, first at "
                              f"{tuple(int(b[0]) for b in bad)}: got {got[bad][0]} oracle {v[bad][0]} bound {d[bad][0]}")
    return int((got == bf16(v)).sum())


def check_close(name, got, ref, bound):
    bound = bound * 1.0001 + 1e-12 * np.abs(ref)
    bad = np.nonzero(np.abs(got - ref) > bound)
    assert len(bad[0]) == 0, (f"{name}: {len(bad[0])} elements outside the bound, worst ratio "
                              f"{np.max(np.abs(got - ref) / np.maximum(bound, 1e-300))}")
    return float(np.max(np.abs(got - ref) / np.maximum(bound, 1e-300)))


def nll_interval(out, E3, U, sig_a, sig_d, dout):
    """For the output gradient of the Gaussian negative log-likelihood: an interval [lo, hi]
    [B][200] holding the implementation's value before rounding to BF16, given the
    oracle's outputs `out` (the implementation's within E3) and float64 gradient `dout`;
    and a bound on the loss difference.  sig_a, sig_d: the float32 plain scales."""
    B, N = U.shape[0], U.shape[1]
    lo, hi = dout.copy(), dout.copy()
    lerr = labs = 0.0
    for c, (scale, sig) in enumerate(((A_SCALE, sig_a), (D_SCALE, sig_d))):
        cm = 4 * np.arange(N) + c
        cl_ = cm + 2
        o_mu, o_raw = out[:, cm], out[:, cl_]
        e_mu, e_raw = scale * E3[:, cm], E3[:, cl_]
        lsp = np.log(sig)
        ls = lsp + np.clip(o_raw, LS_MIN, LS_MAX)
        inv = np.exp(-2.0 * ls)
        near_clip = (np.abs(o_raw - LS_MIN) <= e_raw) | (np.abs(o_raw - LS_MAX) <= e_raw)
        inside = (o_raw > LS_MIN) & (o_raw < LS_MAX)
        e_ls = np.where(inside | near_clip, e_raw, 0.0) + 4.0 * U32 * (np.abs(lsp) + np.abs(ls) + 1.0)
        rel_inv = 2.0 * e_ls * 1.0001 + 4.0 * U32
        mu = scale * o_mu
        res = U[:, :, c] - mu
        e_res = e_mu * 1.0001 + 2.0 * U32 * (np.abs(U[:, :, c]) + np.abs(mu))
        d_mu = scale * inv / B * (e_res + np.abs(res) * rel_inv + 6.0 * U32 * np.abs(res)) * 1.0001
        lo[:, cm], hi[:, cm] = dout[:, cm] - d_mu, dout[:, cm] + d_mu
        q = res * res * inv
        dq = inv * (2.0 * np.abs(res) * e_res + e_res ** 2) * (1.0 + rel_inv) + q * (rel_inv + 6.0 * U32)
        d_ls = (dq + 2.0 * U32 * (1.0 + q)) / B * 1.0001
        v = dout[:, cl_]
        l_, h_ = v - d_ls, v + d_ls
        # next to a clip bound the indicator itself may differ: 0 or the unclipped value
        full = (1.0 - q) / B
        lo[:, cl_] = np.where(near_clip, np.minimum(np.minimum(l_, 0.0), full - d_ls), l_)
        hi[:, cl_] = np.where(near_clip, np.maximum(np.maximum(h_, 0.0), full + d_ls), h_)
        contrib = 0.5 * q + ls
        lerr += np.sum(np.abs(res) * inv * e_res + 0.5 * dq + np.where(inside | near_clip, e_raw, 0.0) +
                       8.0 * U32 * (np.abs(contrib) + np.abs(lsp) + 1.0)) / B
        labs += np.sum(np.abs(contrib)) / B
    # float32 reduction of the B x N x 2 terms: wave sums, then one atomic add per wave
    lerr += gam(2 * B + 16) * labs
    return lo, hi, lerr


def lockstep(orc, P, X, U, sig_a, sig_d, side):
    """Compare `side` -- dict with h1, h2, out [B][>=200], d3 [B][>=200], d2, d1 (float64
    arrays of the implementation's values), loss and grads {name: array} -- with the
    oracle `orc` (an MlpOracle in BF16-operand mode with parameters P) on features X and
    targets U.  Raises AssertionError on any violation; returns statistics."""
    B, N = U.shape[0], U.shape[1]
    Wb = {k: (bf16(P[k]) if k.startswith("W") else np.asarray(P[k], np.float64)) for k in NAMES}
    aW = {k: np.abs(Wb[k]) for k in ("W1", "W2", "W3")}
    xb = bf16(X)
    h1, h2 = side["h1"], side["h2"]
    st = {}
    fw = orc.lockstep(X, h1=h1, h2=h2)
    E1 = gam(xb.shape[1] + 2) * (np.abs(xb) @ aW["W1"] + np.abs(Wb["b1"]))
    st["h1_equal"] = check_rounding("h1", h1, gelu(fw["pre1"]), GELU_LIP * E1 + eps_gelu(fw["pre1"]))
    E2 = gam(h1.shape[1] + 2) * (np.abs(h1) @ aW["W2"] + np.abs(Wb["b2"]))
    st["h2_equal"] = check_rounding("h2", h2, gelu(fw["pre2"]), GELU_LIP * E2 + eps_gelu(fw["pre2"]))
    E3 = gam(h2.shape[1] + 2) * (np.abs(h2) @ aW["W3"] + np.abs(Wb["b3"]))
    out = fw["out"]
    st["out_ratio"] = check_close("out", side["out"][:, :out.shape[1]], out, E3)
    L, dout = orc.nll(out, U, sig_a, sig_d)
    lo, hi, lerr = nll_interval(out, E3, U, sig_a, sig_d, dout)
    d3 = side["d3"][:, :out.shape[1]]
    bad = np.nonzero(~((d3 >= bf16(lo)) & (d3 <= bf16(hi))))
    assert len(bad[0]) == 0, f"d3: {len(bad[0])} values are no rounding within the bound"
    assert np.all(d3[:, 4 * N:] == 0.0)
    st["d3_equal"] = int((d3 == bf16(dout)).sum())
    assert abs(float(side["loss"]) - L) <= lerr * 1.0001, (float(side["loss"]), L, lerr)
    st["loss_ratio"] = abs(float(side["loss"]) - L) / lerr
    d2, d1 = side["d2"], side["d1"]
    bw = orc.lockstep(X, h1=h1, h2=h2, d_out=d3, d2=d2, d1=d1)
    dh2 = d3 @ Wb["W3"].T
    e_dh2 = gam(258) * (np.abs(d3) @ aW["W3"].T)
    gg2 = gelu_grad(bw["pre2"])
    st["d2_equal"] = check_rounding("d2", d2, bw["d2_pre"], np.abs(gg2) * e_dh2 + (np.abs(dh2) + e_dh2) * (
        GELU_GRAD_LIP * E2 + eps_gelu_grad(bw["pre2"])) + 2.0 * U32 * np.abs(bw["d2_pre"]))
    dh1 = d2 @ Wb["W2"].T
    e_dh1 = gam(258) * (np.abs(d2) @ aW["W2"].T)
    gg1 = gelu_grad(bw["pre1"])
    st["d1_equal"] = check_rounding("d1", d1, bw["d1_pre"], np.abs(gg1) * e_dh1 + (np.abs(dh1) + e_dh1) * (
        GELU_GRAD_LIP * E1 + eps_gelu_grad(bw["pre1"])) + 2.0 * U32 * np.abs(bw["d1_pre"]))
    # weight and bias gradients: sums over the batch (split into at most 64 partial sums)
    gB = gam(B + 66)
    bound = {"W3": gB * (np.abs(h2).T @ np.abs(d3)), "b3": gB * np.abs(d3).sum(0),
             "W2": gB * (np.abs(h1).T @ np.abs(d2)), "b2": gB * np.abs(d2).sum(0),
             "W1": gB * (np.abs(xb).T @ np.abs(d1)), "b1": gB * np.abs(d1).sum(0)}
    for nm, g in zip(NAMES, bw["grads"]):
        st[nm + "_ratio"] = check_close(nm, side["grads"][nm], g, bound[nm])
        rel = bound[nm] / np.maximum(np.abs(g), 1e-30)
        st[nm + "_median_rel_bound"] = float(np.median(rel))
    st["values"] = {k: int(side[k].shape[0] * side[k].shape[1]) for k in ("h1", "h2", "d2", "d1")}
    return st
