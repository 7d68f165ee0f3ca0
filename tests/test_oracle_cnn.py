"""Pins of the oracle network: gradients against central differences of the
oracle's own loss, the forward pass against a direct dense convolution of a
single impulse, and the features' definitions on a stencil matrix."""
import numpy as np
import pytest

import oracle
from paper_1902_00095_amd import synth


def _theta(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(oracle.CNN_NPARAM) * scale


def test_gradient_matches_central_differences():
    g = synth.Grid(4, 3, 3, 1, 1, 1)
    n = g.n
    rng = np.random.default_rng(1)
    f = rng.standard_normal((8, n))
    y = rng.standard_normal(n)
    th = _theta()
    loss, grad = oracle.cnn_backward(g, th, f, y)
    h = 1e-6
    idx = list(range(0, 3456, 97)) + list(range(3456, 3472)) + list(range(3472, 3904, 13)) + [3904]
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (oracle.cnn_backward(g, tp, f, y)[0] - oracle.cnn_backward(g, tm, f, y)[0]) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-7 * max(1.0, abs(grad[k])), (k, fd, grad[k])


def test_forward_impulse_response():
    """A single unit impulse in channel c at an interior cell with ReLU kept
    active (b1 large) gives out = b2 + sum_o W2[o] (*) (W1[o][c] (*) delta):
    a dense 5x5x5 correlation computed here from the weights by explicit
    index arithmetic."""
    g = synth.Grid(7, 7, 7, 1, 1, 1)
    n = g.n
    th = _theta(3)
    p = oracle.cnn_unpack(th)
    p["b1"][:] = 50.0          # keep every pre-activation positive
    th = np.concatenate([p["W1"], p["b1"], p["W2"], p["b2"]])
    c = 5
    f = np.zeros((8, n))
    ci = 3 + 7 * (3 + 7 * 3)
    f[c, ci] = 1.0
    out, h = oracle.cnn_forward(g, th, f)
    W1 = p["W1"].reshape(16, 8, 3, 3, 3)
    W2 = p["W2"].reshape(16, 3, 3, 3)
    ref = np.full((7, 7, 7), p["b2"][0] + np.einsum("o,oijk->", p["b1"], W2 * 0 + 1) * 0)
    # constant part: b2 + sum_o b1_o * sum of W2[o] taps that stay inside the grid
    ref = np.zeros((7, 7, 7))
    for z in range(7):
        for yv in range(7):
            for x in range(7):
                s = p["b2"][0]
                for o in range(16):
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                zz, yy, xx = z + dz, yv + dy, x + dx
                                if not (0 <= zz < 7 and 0 <= yy < 7 and 0 <= xx < 7):
                                    continue
                                a = p["b1"][o]
                                ez, ey, ex = 3 - zz, 3 - yy, 3 - xx   # impulse offset from (zz,yy,xx)
                                if max(abs(ez), abs(ey), abs(ex)) <= 1:
                                    a += W1[o, c, ez + 1, ey + 1, ex + 1]
                                s += W2[o, dz + 1, dy + 1, dx + 1] * a
                ref[z, yv, x] = s
    np.testing.assert_allclose(out.reshape(7, 7, 7), ref, rtol=1e-12, atol=1e-12)


def test_features_definition():
    p = synth.make_problem("W2", grid=synth.Grid(5, 4, 3, 1, 1, 1))
    J = oracle.jacobian(p)
    r = np.random.default_rng(2).standard_normal(J.n)
    f, s = oracle.cnn_features(p.grid, J.rowptr, J.col, J.S, r)
    A = J.block("S").toarray()
    D = np.abs(A).sum(axis=1)
    z = r / D
    assert abs(s - np.sqrt(np.mean(z * z))) <= 1e-14 * s
    np.testing.assert_allclose(f[0], z / s, rtol=1e-14)
    np.testing.assert_allclose(f[7], np.diag(A) / D, rtol=1e-14)
    i = 1 + 5 * (1 + 4 * 1)          # interior cell
    for q, off in enumerate((-1, 1, -5, 5, -20, 20)):
        assert f[1 + q, i] == A[i, i + off] / A[i, i]
    assert f[1, 0] == 0.0 and f[5, 0] == 0.0          # no -x / -z neighbour at cell 0
