"""Oracle: the learned warm start of the tracker (test infrastructure only).

This part is NOT from the paper.  The paper's tracker starts every G-ICP
registration from the previous pose (Sec. 3 describes the registration, not
its initialisation); the learned warm start is an extension of this project:
a point-set network that regresses the relative pose of a frame pair from
the two clouds, used as the initial pose, with the constant-velocity
prediction as the fallback.  Everything below is therefore the project's own
definition, written plainly:

Network (PointNet-style shared MLP, ReLU after every layer but the last):
    per row r of X (N rows, 6 channels = [source point r ; target point r]):
        H1 = relu(X W1 + b1)      6 -> 64
        H2 = relu(H1 W2 + b2)    64 -> 128
        H3 = relu(H2 W3 + b3)   128 -> 256
    g   = max over rows of H3                        (256)
    z   = relu(g W4 + b4)                          256 -> 128
    y   = z W5 + b5                                128 -> 6
The output y = [omega; t] is the relative pose in the centred frame:
R = exp([omega]x), translation t in metres (see `pack` / `unpack`).

Loss: L = (1/B) sum_b 1/2 |y_b - y*_b|^2 over a batch of B pairs.
Optimiser: Adam (Kingma & Ba, 2015, Algorithm 1) with bias correction.
Parameter draw: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014; the
finaliser constants of Vigna's reference implementation) as a
counter-based generator; weight j of the flat parameter vector (layout in
LAYOUT) is a * (2u - 1), u = (splitmix64(seed * 2^32 + j) >> 11) * 2^-53,
a = sqrt(6 / fan_in); biases start at 0.

Storage precision of the GPU path (bf16 inputs and shared weights, bf16
hidden activations between the shared layers, FP32 accumulation) can be
emulated with ``bf16=True``: the same roundings are applied to the same
values and all arithmetic stays FP64, so the GPU and the oracle differ only
by accumulation order.
"""
from __future__ import annotations

import numpy as np

N_POINTS = 4096
LAYERS = [(6, 64), (64, 128), (128, 256), (256, 128), (128, 6)]


def _layout():
    out, off = [], 0
    for li, (fi, fo) in enumerate(LAYERS):
        out.append((f"W{li + 1}", off, (fi, fo)))
        off += fi * fo
        out.append((f"b{li + 1}", off, (fo,)))
        off += fo
    return out, off


LAYOUT, N_PARAMS = _layout()


# ---------------------------------------------------------------------------
# counter-based parameter draw
# ---------------------------------------------------------------------------
def splitmix64(x):
    """SplitMix64 output function of the 64-bit counter x (uint64 array)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def init_params(seed: int) -> np.ndarray:
    """Flat FP32 parameter vector in LAYOUT order."""
    p = np.zeros(N_PARAMS, np.float64)
    for name, off, shape in LAYOUT:
        if name[0] != "W":
            continue
        n = int(np.prod(shape))
        j = np.arange(off, off + n, dtype=np.uint64)
        u = (splitmix64((np.uint64(seed) << np.uint64(32)) + j) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        a = np.sqrt(6.0 / shape[0])
        p[off:off + n] = a * (2.0 * u - 1.0)
    return p.astype(np.float32)


def unflatten(p) -> dict:
    p = np.asarray(p, np.float64)
    return {name: p[off:off + int(np.prod(shape))].reshape(shape) for name, off, shape in LAYOUT}


def flatten(d: dict) -> np.ndarray:
    out = np.zeros(N_PARAMS, np.float64)
    for name, off, shape in LAYOUT:
        out[off:off + int(np.prod(shape))] = np.asarray(d[name], np.float64).reshape(-1)
    return out


# ---------------------------------------------------------------------------
# bf16 storage rounding (round to nearest, ties to even, from FP32)
# ---------------------------------------------------------------------------
def bf16(x):
    b = np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32).astype(np.uint64)
    b = (b + np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _id(x):
    return np.asarray(x, np.float64)


# ---------------------------------------------------------------------------
# input packing and output decoding
# ---------------------------------------------------------------------------
SCALE = 0.5   # centred coordinates are multiplied by this before rounding


def pack(src, tgt, src_idx, tgt_idx):
    """Rows [ (src[src_idx[r]] - c) * SCALE ; (tgt[tgt_idx[r]] - c) * SCALE ]
    with c the mean of the chosen target points (FP64), and c itself."""
    s = np.asarray(src, np.float64)[np.asarray(src_idx)]
    t = np.asarray(tgt, np.float64)[np.asarray(tgt_idx)]
    c = t.mean(axis=0)
    return np.hstack([(s - c) * SCALE, (t - c) * SCALE]), c


def rotvec_to_matrix(w):
    w = np.asarray(w, np.float64)
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K


def matrix_to_rotvec(R):
    R = np.asarray(R, np.float64)
    c = np.clip((np.trace(R) - 1) / 2, -1.0, 1.0)
    th = np.arccos(c)
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-9:
        return 0.5 * v
    return th / (2 * np.sin(th)) * v


def label(T, c):
    """Target output for relative pose T (source -> target) and centre c:
    in centred coordinates the pose is [R, t + (R - I) c]."""
    T = np.asarray(T, np.float64)
    R, t = T[:3, :3], T[:3, 3]
    return np.concatenate([matrix_to_rotvec(R), t + (R - np.eye(3)) @ c])


def unpack(y, c):
    """Relative pose (4x4) from a network output y and the centre c."""
    R = rotvec_to_matrix(y[:3])
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = np.asarray(y[3:], np.float64) - (R - np.eye(3)) @ c
    return T


# ---------------------------------------------------------------------------
# forward / backward / loss / Adam
# ---------------------------------------------------------------------------
def forward(params, X, bf16_storage: bool = False):
    """X: [B, N, 6].  Returns y [B, 6] and the cache for `backward`."""
    P = unflatten(params)
    r = bf16 if bf16_storage else _id
    X = r(X)
    W1, W2, W3 = r(P["W1"]), r(P["W2"]), r(P["W3"])
    A1 = X @ W1 + P["b1"]
    H1 = np.maximum(A1, 0.0)
    A2 = r(H1) @ W2 + P["b2"]
    H2 = np.maximum(A2, 0.0)
    A3 = r(H2) @ W3 + P["b3"]
    H3 = np.maximum(A3, 0.0)
    # max over rows; the lowest row index among equal maxima
    arg = np.argmax(H3, axis=1)                       # [B, 256]
    g = np.take_along_axis(H3, arg[:, None, :], axis=1)[:, 0, :]
    A4 = g @ P["W4"] + P["b4"]
    z = np.maximum(A4, 0.0)
    y = z @ P["W5"] + P["b5"]
    cache = dict(X=X, A1=A1, H1=r(H1), A2=A2, H2=r(H2), A3=A3, arg=arg, g=g, A4=A4, z=z, W1=W1, W2=W2, W3=W3)
    return y, cache


def loss(y, ystar):
    d = np.asarray(y, np.float64) - np.asarray(ystar, np.float64)
    return 0.5 * float(np.sum(d * d)) / d.shape[0]


def loss_grad(y, ystar):
    d = np.asarray(y, np.float64) - np.asarray(ystar, np.float64)
    return d / d.shape[0]


def backward(params, cache, dy):
    """Gradient of sum_b dy_b . y_b with respect to the flat parameters."""
    P = unflatten(params)
    dy = np.asarray(dy, np.float64)
    G = {}
    G["W5"] = np.einsum("bi,bj->ij", cache["z"], dy)
    G["b5"] = dy.sum(axis=0)
    dA4 = (dy @ P["W5"].T) * (cache["A4"] > 0)
    G["W4"] = np.einsum("bi,bj->ij", cache["g"], dA4)
    G["b4"] = dA4.sum(axis=0)
    dg = dA4 @ P["W4"].T                              # [B, 256]
    B, N = cache["A3"].shape[:2]
    dH3 = np.zeros((B, N, 256))
    bi = np.arange(B)[:, None]
    ci = np.arange(256)[None, :]
    dH3[bi, cache["arg"], ci] = dg
    dA3 = dH3 * (cache["A3"] > 0)
    G["W3"] = np.einsum("bni,bnj->ij", cache["H2"], dA3)
    G["b3"] = dA3.sum(axis=(0, 1))
    dA2 = (dA3 @ cache["W3"].T) * (cache["A2"] > 0)
    G["W2"] = np.einsum("bni,bnj->ij", cache["H1"], dA2)
    G["b2"] = dA2.sum(axis=(0, 1))
    dA1 = (dA2 @ cache["W2"].T) * (cache["A1"] > 0)
    G["W1"] = np.einsum("bni,bnj->ij", cache["X"], dA1)
    G["b1"] = dA1.sum(axis=(0, 1))
    return flatten(G)


ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_step(params, grad, m, v, t, lr=1e-3, b1=ADAM_B1, b2=ADAM_B2, eps=ADAM_EPS):
    """One Adam update (step count t >= 1).  Returns (params, m, v)."""
    g = np.asarray(grad, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
