"""Pins of the oracle's MLP (16-64-64-1, ReLU, sigmoid, mean BCE) by central
finite differences, of its Adam step by the update written out, and of its
BF16 inference by cases where BF16 rounding is exact or known by hand."""
import numpy as np

import oracle
import synth


def _params(seed=0):
    r = synth.rng(seed)
    n = oracle.mlp_nparams()
    p = r.standard_normal(n) * 0.3
    return p


def test_gradient_central_differences():
    P = _params(1)
    X = synth.small_float(31, 40, 16)
    y = (synth.rng(2).random(40) < 0.5).astype(np.float32)
    loss, g, _ = oracle.mlp_fwd_bwd(P, X, y)
    r = synth.rng(3)
    idx = r.choice(P.shape[0], size=200, replace=False)
    h = 1e-6
    for i in idx:
        a = P.copy(); a[i] += h
        b = P.copy(); b[i] -= h
        fd = (oracle.mlp_fwd_bwd(a, X, y, want_grad=False)[0] -
              oracle.mlp_fwd_bwd(b, X, y, want_grad=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8


def test_forward_matches_numpy():
    P = _params(4)
    X = synth.small_float(32, 10, 16)
    W1 = P[:1024].reshape(64, 16); b1 = P[1024:1088]
    W2 = P[1088:5184].reshape(64, 64); b2 = P[5184:5248]
    w3 = P[5248:5312]; b3 = P[5312]
    h1 = np.maximum(X.astype(np.float64) @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    z = h2 @ w3 + b3
    _, _, logits = oracle.mlp_fwd_bwd(P, X)
    assert np.allclose(logits, z, rtol=1e-12, atol=1e-12)


def test_adam_step():
    P = _params(5)
    g = _params(6)
    m = np.zeros_like(P); v = np.zeros_like(P)
    p1 = P.copy()
    oracle.adam_step(p1, g, m, v, 1, lr=0.01)
    # first step: m = (1-b1) g, v = (1-b2) g^2, bias corrected -> g / (|g| + eps')
    expect = P - 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p1, expect, rtol=1e-9, atol=1e-12)




def test_bf16_inference_equals_plain_when_every_value_is_bf16_exact():
    # small integers everywhere: inputs and first-layer outputs are integers
    # below 256, which BF16 holds exactly, so rounding changes nothing
    r = synth.rng(7)
    P = np.zeros(oracle.mlp_nparams())
    P[0:1024] = r.integers(-2, 3, 1024)
    P[1024:1088] = r.integers(0, 4, 64)
    P[1088:5184] = r.integers(-1, 2, 4096)
    P[5184:5248] = r.integers(0, 3, 64)
    P[5248:5312] = r.integers(-2, 3, 64)
    P[5312] = 1.0
    X = r.integers(0, 4, (50, 16)).astype(np.float32)
    _, _, plain = oracle.mlp_fwd_bwd(P, X)
    assert np.abs(P[0:1024]).sum(axis=None) > 0 and np.abs(plain).max() > 0
    w = oracle.bf16_encode(P.astype(np.float32))
    assert (oracle.bf16_decode(w) == P).all()
    assert (oracle.mlp_logits_bf16(w, X).astype(np.float64) == plain).all()


def test_bf16_inference_rounds_hidden_values_to_nearest_even():
    # one path: x0 + x1 -> h1[0] -> h2[0] -> z; 128 and 129 are exact in BF16,
    # their sum 257 is not: it lies halfway between 256 and 258 and rounds to
    # the even significand (256); 259 lies halfway between 258 and 260 -> 260
    P = np.zeros(oracle.mlp_nparams())
    P[0] = 1.0          # W1[0][0]
    P[1] = 1.0          # W1[0][1]
    P[1088] = 1.0       # W2[0][0]
    P[5248] = 1.0       # w3[0]
    X = np.zeros((3, 16), np.float32)
    X[0, :2] = (128, 129)
    X[1, :2] = (128, 131)
    X[2, :2] = (257, 0)  # the input itself is rounded first: 257 -> 256
    z = oracle.mlp_logits_bf16(oracle.bf16_encode(P.astype(np.float32)), X)
    assert z.tolist() == [256.0, 260.0, 256.0]
    _, _, plain = oracle.mlp_fwd_bwd(P, X)
    assert plain.tolist() == [257.0, 259.0, 257.0]


def _fp64_bf16(v):
    """Round FP64 values to the nearest BF16 value, ties to even (exact arithmetic)."""
    v = np.asarray(v, np.float64)
    out = np.zeros_like(v)
    nz = v != 0
    e = np.floor(np.log2(np.abs(v[nz])))
    ulp = 2.0 ** (e - 7)               # BF16 keeps 8 significant bits
    q = v[nz] / ulp
    fl = np.floor(q)
    frac = q - fl
    up = (frac > 0.5) | ((frac == 0.5) & (np.mod(fl, 2) == 1))
    out[nz] = (fl + up) * ulp
    return out


def _near_midpoint(v, bound):
    """True where a BF16 rounding of v could change under a perturbation of `bound`."""
    v = np.asarray(v, np.float64)
    return (_fp64_bf16(v - bound) != _fp64_bf16(v + bound))


def test_bf16_inference_within_fp32_error_bound_of_exact():
    # The FP32 definition (fused multiply-adds in index order, halving tree)
    # against exact (FP64) evaluation of the same BF16 network. Rows where an
    # FP32 rounding error could move a hidden value across a BF16 rounding
    # midpoint are left out (and must be rare); on the others the FP32 logit is
    # within the accumulated rounding bound of the exact one.
    r = synth.rng(21)
    P = r.standard_normal(oracle.mlp_nparams()) * 0.3
    w = oracle.bf16_encode(P.astype(np.float32))
    Pb = oracle.bf16_decode(w).astype(np.float64)
    W1 = Pb[0:1024].reshape(64, 16); b1 = Pb[1024:1088]
    W2 = Pb[1088:5184].reshape(64, 64); b2 = Pb[5184:5248]
    w3 = Pb[5248:5312]; b3 = Pb[5312]
    X = synth.small_float(22, 2000, 16)
    z32 = oracle.mlp_logits_bf16(w, X).astype(np.float64)
    u = 2.0 ** -24
    xb = oracle.bf16_decode(oracle.bf16_encode(X)).astype(np.float64)
    a1 = xb @ W1.T + b1
    m1 = 18 * u * (np.abs(xb) @ np.abs(W1).T + np.abs(b1))   # 16 fused adds + slack
    h1 = np.maximum(a1, 0.0)
    amb = (_near_midpoint(h1, m1) & (a1 > m1)).any(axis=1) | ((np.abs(a1) <= m1).any(axis=1))
    h1b = _fp64_bf16(h1)
    a2 = h1b @ W2.T + b2
    m2 = 66 * u * (np.abs(h1b) @ np.abs(W2).T + np.abs(b2))
    amb |= (np.abs(a2) <= m2).any(axis=1)
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    # hidden values carry the FP32 error of layer 2 (m2); products and the tree add 8u
    bound = m2 @ np.abs(w3) * 1.01 + 8 * u * (np.abs(h2) @ np.abs(w3) + abs(b3))
    ok = ~amb
    assert ok.mean() > 0.7
    assert (np.abs(z32 - z)[ok] <= bound[ok]).all()
    # a dropped term or a transposed weight matrix is far outside the bound
    assert np.abs(z32 - z)[ok].max() < 1e-3
