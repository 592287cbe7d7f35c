"""FP64 oracle of the learned edge proposal: edge features, the 32-64-64-1 MLP
with BF16 operands, softmax cross-entropy per view, and the backward pass.

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module. It shares no code with the HIP path.

The thesis learns nothing for edge sampling; it lists what a good edge pdf
should follow (Ch. 5, Importance Sampling the Edges: the edge's length, its
distance and orientation, the radiance difference across it, how much of it is
visible) and builds its hierarchy from exactly these geometric terms. The
network below sees those quantities per (edge, view) and is trained to put
probability where the method's own boundary samples were large; the renderer
mixes its output with the plain edge pdf so every edge the plain sampler can
draw keeps a positive probability (unbiasedness of importance sampling).

Arithmetic mirrored from the kernels:
  * inputs and the three weight matrices are rounded to bfloat16 (round to
    nearest even); biases, hidden activations, logits and all gradients are
    real numbers here. The kernels keep activations and gradients in FP32 and
    feed them to the BF16 matrix cores as a sum of three BF16 terms (exact to
    about 2^-24), accumulating in FP32, so GPU and oracle differ by rounding
    only;
  * the one discrete decision, ReLU at zero, can differ where a pre-activation
    lies within FP32 accumulation error of 0. Such rows are flagged.

Parameter vector theta (float32, 6337 entries), row-major:
  W1 [32][64] | b1 [64] | W2 [64][64] | b2 [64] | W3 [64] | b3 [1]
"""
from __future__ import annotations

import math

import numpy as np

NF = 32            # input features (29 used, zero-padded)
H = 64             # hidden width
OFF_W1, OFF_B1 = 0, 32 * 64
OFF_W2, OFF_B2 = OFF_B1 + 64, OFF_B1 + 64 + 64 * 64
OFF_W3, OFF_B3 = OFF_B2 + 64, OFF_B2 + 64 + 64
N_PARAMS = OFF_B3 + 1
U32 = 2.0 ** -24
NDC_CLAMP = 8.0


def unpack(theta):
    t = np.asarray(theta, np.float64)
    assert t.shape == (N_PARAMS,)
    return (t[OFF_W1:OFF_B1].reshape(32, 64), t[OFF_B1:OFF_W2], t[OFF_W2:OFF_B2].reshape(64, 64),
            t[OFF_B2:OFF_W3], t[OFF_W3:OFF_B3], t[OFF_B3])


def bf16(x):
    """Round to the nearest bfloat16 (8 significant bits), ties to even."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)                  # x = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)


# ---------------------------------------------------------------------------
# features of one (edge, view)
# ---------------------------------------------------------------------------
def camera_frame(cam):
    c = np.asarray(cam.position, np.float64)
    f = np.asarray(cam.look_at, np.float64) - c
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(cam.up, np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return c, r, u, f


def edge_features(scene, cam, edges):
    """[E][32] features for the edges (rows va, vb, f0, f1) seen from cam.

    0-5   endpoints in the camera frame (right, up, forward)
    6-11  unit face normals in the camera frame (zeros for a missing face)
    12-17 endpoints in world space
    18-21 albedo and emission of both faces (zeros for a missing face)
    22    1 for a boundary edge
    23    cosine between the two face normals (0 for a boundary edge)
    24-27 normalised screen coordinates of both endpoints, x / (z tan(fov/2) aspect)
          and y / (z tan(fov/2)), depth clamped to the near plane, clamped to +-8
    28    edge length
    29-31 zero
    """
    P = scene.vertices.astype(np.float64)
    I = scene.indices.astype(np.int64)
    c, r, u, f = camera_frame(cam)
    R = np.stack([r, u, f])
    th = math.tan(math.radians(cam.fov_y_deg) / 2.0)
    asp = cam.width / cam.height
    E = len(edges)
    X = np.zeros((E, NF))
    va, vb, f0, f1 = (edges[:, k].astype(np.int64) for k in range(4))
    A, B = P[va], P[vb]
    qa, qb = (A - c) @ R.T, (B - c) @ R.T
    X[:, 0:3], X[:, 3:6] = qa, qb

    def face_normal(fi):
        p0, p1, p2 = P[I[fi, 0]], P[I[fi, 1]], P[I[fi, 2]]
        n = np.cross(p1 - p0, p2 - p0)
        return n / np.linalg.norm(n, axis=1, keepdims=True)

    has1 = f1 >= 0
    n0 = face_normal(f0)
    n1 = np.zeros((E, 3))
    if has1.any():
        n1[has1] = face_normal(f1[has1])
    X[:, 6:9], X[:, 9:12] = n0 @ R.T, n1 @ R.T
    X[:, 12:15], X[:, 15:18] = A, B
    alb = scene.albedo.astype(np.float64)
    emi = scene.emission.astype(np.float64)
    X[:, 18] = alb[f0]
    X[:, 19] = np.where(has1, alb[np.maximum(f1, 0)], 0.0)
    X[:, 20] = emi[f0]
    X[:, 21] = np.where(has1, emi[np.maximum(f1, 0)], 0.0)
    X[:, 22] = (~has1).astype(np.float64)
    X[:, 23] = np.where(has1, (n0 * n1).sum(1), 0.0)
    near = float(cam.near_clip)
    for j, q in ((24, qa), (26, qb)):
        z = np.maximum(q[:, 2], near)
        X[:, j] = np.clip(q[:, 0] / (z * th * asp), -NDC_CLAMP, NDC_CLAMP)
        X[:, j + 1] = np.clip(q[:, 1] / (z * th), -NDC_CLAMP, NDC_CLAMP)
    X[:, 28] = np.linalg.norm(B - A, axis=1)
    return X


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def forward(theta, X, rounding=True):
    """Logits z[N], their absolute-value mass, `flag[N]` (rows with a ReLU
    decision within FP32 accumulation error of zero) and the intermediate
    values. rounding=False: no BF16 rounding of inputs and weights."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    rd = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    Xb, W1b, W2b, W3b = rd(X), rd(W1), rd(W2), rd(W3)
    a1 = Xb @ W1b + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2b + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3b + b3
    m1 = np.abs(Xb) @ np.abs(W1b) + np.abs(b1)
    m2 = np.abs(h1) @ np.abs(W2b) + np.abs(b2)
    mz = np.abs(h2) @ np.abs(W3b) + abs(b3)
    # FP32 error bounds of the kernels' pre-activations: K exact BF16 products
    # (three split terms per FP32 operand in layer 2) summed in FP32, plus the bias
    flag = (np.abs(a1) <= 2 * 34 * U32 * m1).any(1) | (np.abs(a2) <= 2 * 200 * U32 * m2).any(1)
    cache = dict(Xb=Xb, W1b=W1b, W2b=W2b, W3b=W3b, a1=a1, h1=h1, a2=a2, h2=h2, m1=m1, m2=m2)
    return z, mz, flag, cache


def softmax_xent(z, target, offsets):
    """Per view v (rows offsets[v]..offsets[v+1]): p = softmax(z), loss =
    -sum t log p with t = target normalised to sum 1 (views whose target sums
    to 0 are skipped), dz = (p - t) / (number of views used). Returns p, the
    mean loss and dz."""
    z = np.asarray(z, np.float64)
    target = np.asarray(target, np.float64)
    nv = len(offsets) - 1
    p = np.zeros_like(z)
    dz = np.zeros_like(z)
    used = [v for v in range(nv) if offsets[v + 1] > offsets[v] and target[offsets[v]:offsets[v + 1]].sum() > 0]
    losses = []
    for v in range(nv):
        lo, hi = offsets[v], offsets[v + 1]
        if hi <= lo:
            continue
        e = np.exp(z[lo:hi] - z[lo:hi].max())
        p[lo:hi] = e / e.sum()
        if v in used:
            t = target[lo:hi] / target[lo:hi].sum()
            losses.append(-(t * np.log(np.maximum(p[lo:hi], 1e-300))).sum())
            dz[lo:hi] = (p[lo:hi] - t) / len(used)
    return p, (float(np.mean(losses)) if losses else 0.0), dz


def backward(theta, cache, dz):
    """Gradient of sum(dz * z) w.r.t. theta (the BF16 rounding of weights and
    inputs passes gradients through unchanged) and its absolute-value mass per
    entry (the scale of the kernels' FP32 rounding error)."""
    Xb, W2b, W3b = cache["Xb"], cache["W2b"], cache["W3b"]
    a1, h1, a2, h2 = cache["a1"], cache["h1"], cache["a2"], cache["h2"]
    dz = np.asarray(dz, np.float64)
    g = np.zeros(N_PARAMS)
    mass = np.zeros(N_PARAMS)
    g[OFF_W3:OFF_B3] = h2.T @ dz
    mass[OFF_W3:OFF_B3] = np.abs(h2).T @ np.abs(dz)
    g[OFF_B3] = dz.sum()
    mass[OFF_B3] = np.abs(dz).sum()
    g2 = (dz[:, None] * W3b[None, :]) * (a2 > 0)
    g[OFF_B2:OFF_W3] = g2.sum(0)
    mass[OFF_B2:OFF_W3] = np.abs(g2).sum(0)
    g[OFF_W2:OFF_B2] = (h1.T @ g2).ravel()
    mass[OFF_W2:OFF_B2] = (np.abs(h1).T @ np.abs(g2)).ravel()
    mg1 = (np.abs(g2) @ np.abs(W2b).T) * (a1 > 0)
    g1 = (g2 @ W2b.T) * (a1 > 0)
    g[OFF_B1:OFF_W2] = g1.sum(0)
    mass[OFF_B1:OFF_W2] = mg1.sum(0)
    g[OFF_W1:OFF_B1] = (Xb.T @ g1).ravel()
    mass[OFF_W1:OFF_B1] = (np.abs(Xb).T @ mg1).ravel()
    return g, mass
