"""Pins of the warm-start network oracle (oracle/mlp.py) against facts that do
not come from the oracle itself: published generator outputs, bf16 rounding
of chosen values, finite differences, permutation invariance, a pure-Python
loop evaluation on a tiny case, and Adam's closed-form first step."""
import numpy as np
import pytest

from oracle import mlp


def test_splitmix64_published_sequence():
    # the first two outputs of SplitMix64 started from state 0 (the counter
    # after k steps is k * 0x9E3779B97F4A7C15)
    out = mlp.splitmix64(np.array([0, 0x9E3779B97F4A7C15], dtype=np.uint64))
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4


def test_init_params_range_and_layout():
    p = mlp.init_params(7)
    assert p.dtype == np.float32 and p.shape == (mlp.N_PARAMS,)
    P = mlp.unflatten(p)
    for li, (fi, fo) in enumerate(mlp.LAYERS):
        W, b = P[f"W{li + 1}"], P[f"b{li + 1}"]
        a = np.sqrt(6.0 / fi)
        assert W.shape == (fi, fo) and np.all(np.abs(W) <= a) and np.all(b == 0)
        # uniform draw: mean ~ 0, variance ~ a^2 / 3
        assert abs(W.mean()) < 0.1 * a and abs(W.var() / (a * a / 3) - 1) < 0.2
    assert not np.array_equal(p, mlp.init_params(8))


def test_bf16_rounding_values():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, -2.5, 3.0e38])
    got = mlp.bf16(x)
    # 1+2^-8 is the midpoint of 1 and 1+2^-7: ties to the even mantissa (1);
    # 1+3*2^-8 is the midpoint of 1+2^-7 and 1+2^-6: even is 1+2^-6
    assert list(got[:5]) == [1.0, 1.0, 1 + 2 ** -6, 1.0, -2.5]
    assert abs(got[5] - 3.0e38) / 3.0e38 < 2 ** -8


def _loop_forward(P, X):
    """Pure-Python loops for one pair (tiny N): the network written out."""
    def dense(v, W, b, relu):
        out = []
        for j in range(W.shape[1]):
            s = b[j]
            for i in range(W.shape[0]):
                s += v[i] * W[i, j]
            out.append(max(s, 0.0) if relu else s)
        return out
    rows = []
    for r in range(X.shape[0]):
        h = dense(X[r], P["W1"], P["b1"], True)
        h = dense(h, P["W2"], P["b2"], True)
        h = dense(h, P["W3"], P["b3"], True)
        rows.append(h)
    g = [max(rows[r][c] for r in range(len(rows))) for c in range(256)]
    z = dense(g, P["W4"], P["b4"], True)
    return np.array(dense(z, P["W5"], P["b5"], False))


def test_forward_matches_loops():
    rng = np.random.default_rng(0)
    p = mlp.init_params(3).astype(np.float64)
    p += rng.normal(0, 0.05, p.shape)   # non-zero biases too
    X = rng.normal(0, 1, (1, 3, 6))
    y, _ = mlp.forward(p, X)
    assert np.allclose(y[0], _loop_forward(mlp.unflatten(p), X[0]), rtol=1e-12, atol=1e-12)


def test_forward_permutation_invariant():
    rng = np.random.default_rng(1)
    p = mlp.init_params(4)
    X = rng.normal(0, 1, (2, 64, 6))
    y, _ = mlp.forward(p, X)
    y2, _ = mlp.forward(p, X[:, rng.permutation(64)])
    assert np.allclose(y, y2, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_finite_differences(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(10 + seed).astype(np.float64)
    p += rng.normal(0, 0.02, p.shape)
    X = rng.normal(0, 1, (2, 12, 6))
    ystar = rng.normal(0, 0.1, (2, 6))
    y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, mlp.loss_grad(y, ystar))
    # every bias and a sample of weights of every layer
    pick = []
    for name, off, shape in mlp.LAYOUT:
        n = int(np.prod(shape))
        pick += list(off + rng.choice(n, size=min(n, 12), replace=False))
    h = 1e-6
    for j in pick:
        e = np.zeros_like(p)
        e[j] = h
        fd = (mlp.loss(mlp.forward(p + e, X)[0], ystar) - mlp.loss(mlp.forward(p - e, X)[0], ystar)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), (j, fd, g[j])


def test_backward_only_argmax_rows_carry_gradient():
    # rows that are never a channel's maximum do not influence the output
    rng = np.random.default_rng(5)
    p = mlp.init_params(6)
    X = rng.normal(0, 1, (1, 40, 6))
    y, cache = mlp.forward(p, X)
    used = np.unique(cache["arg"][0])
    X2 = X.copy()
    others = np.setdiff1d(np.arange(40), used)
    X2[0, others] *= 0.5   # shrink unused rows: maxima are unchanged if they stay below
    y2, cache2 = mlp.forward(p, X2)
    if np.array_equal(np.unique(cache2["arg"][0]), used):
        assert np.allclose(y, y2, atol=1e-12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    p0 = rng.normal(0, 1, 50)
    g = rng.normal(0, 1, 50)
    p1, m, v = mlp.adam_step(p0, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    # bias correction makes the first moments exactly g and g^2
    assert np.allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_label_unpack_round_trip():
    rng = np.random.default_rng(3)
    w = rng.normal(0, 0.05, 3)
    T = np.eye(4)
    T[:3, :3] = mlp.rotvec_to_matrix(w)
    T[:3, 3] = rng.normal(0, 0.05, 3)
    c = rng.normal(0, 2, 3)
    y = mlp.label(T, c)
    assert np.allclose(y[:3], w, atol=1e-12)
    assert np.allclose(mlp.unpack(y, c), T, atol=1e-12)
    # in centred coordinates the pose maps (x - c) to (R x + t - c)
    x = rng.normal(0, 1, 3)
    Rc = mlp.rotvec_to_matrix(y[:3])
    assert np.allclose(Rc @ (x - c) + y[3:], T[:3, :3] @ x + T[:3, 3] - c, atol=1e-12)


def test_pack_rows():
    rng = np.random.default_rng(4)
    src, tgt = rng.normal(0, 1, (100, 3)), rng.normal(0, 1, (90, 3))
    si, ti = rng.permutation(100)[:16], rng.permutation(90)[:16]
    X, c = mlp.pack(src, tgt, si, ti)
    assert np.allclose(c, tgt[ti].mean(axis=0))
    assert np.allclose(X[:, :3], (src[si] - c) * mlp.SCALE) and np.allclose(X[:, 3:], (tgt[ti] - c) * mlp.SCALE)
