"""FP64 reference of the cost model and its features -- TEST INFRASTRUCTURE ONLY.

Same layout as the library's model (a flat float array of 8713 entries):
W1[64][4], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[64], b4,
mean[4], std[4].  Forward: a0 = (x - mean) / std, h1 = relu(W1 a0 + b1),
h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3), y = W4 . h3 + b4.  Loss: mean of
(y - t)^2.  Backward: reverse-mode differentiation of that loss.  Adam:
Kingma and Ba, "Adam: A Method for Stochastic Optimization", ICLR 2015
(bias-corrected first and second moments).

Features of a first-level subtree of root v (plain definitions): log(1 +
degree), log(1 + core number), log(1 + sum of neighbour degrees), and the edge
density of P = the later neighbours of v: edges inside P over C(|P|, 2) (0 if
|P| < 2) when C(|P|, 2) <= 256, else the fraction of adjacent pairs among 256
pairs of P drawn from SplitMix64 (see sampled_pair).
"""
from __future__ import annotations

import numpy as np

IN, H = 4, 64
oW1 = 0
ob1 = oW1 + H * IN
oW2 = ob1 + H
ob2 = oW2 + H * H
oW3 = ob2 + H
ob3 = oW3 + H * H
oW4 = ob3 + H
ob4 = oW4 + H
oMean = ob4 + 1
oStd = oMean + IN
N_PARAMS = oStd + IN
N_TRAINABLE = oMean


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    return dict(
        W1=t[oW1:ob1].reshape(H, IN), b1=t[ob1:oW2], W2=t[oW2:ob2].reshape(H, H), b2=t[ob2:oW3],
        W3=t[oW3:ob3].reshape(H, H), b3=t[ob3:oW4], W4=t[oW4:ob4], b4=t[ob4], mean=t[oMean:oStd],
        std=t[oStd:N_PARAMS])


def forward(theta, X):
    """Outputs y (n,) and the intermediate values needed by backward."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a0 = (X - p["mean"]) / p["std"]
    z1 = a0 @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0)
    z3 = h2 @ p["W3"].T + p["b3"]
    h3 = np.maximum(z3, 0)
    y = h3 @ p["W4"] + p["b4"]
    return y, dict(a0=a0, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3)


def loss(theta, X, t):
    y, _ = forward(theta, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def loss_grad(theta, X, t):
    """(loss, gradient over all 8713 entries; zero for mean/std)."""
    p = unpack(theta)
    y, c = forward(theta, X)
    n = y.shape[0]
    r = y - np.asarray(t, dtype=np.float64)
    dy = 2.0 * r / n
    g = np.zeros(N_PARAMS)
    g[oW4:ob4] = c["h3"].T @ dy
    g[ob4] = dy.sum()
    dz3 = np.outer(dy, p["W4"]) * (c["z3"] > 0)
    g[oW3:ob3] = (dz3.T @ c["h2"]).ravel()
    g[ob3:oW4] = dz3.sum(0)
    dz2 = (dz3 @ p["W3"]) * (c["z2"] > 0)
    g[oW2:ob2] = (dz2.T @ c["h1"]).ravel()
    g[ob2:oW3] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (c["z1"] > 0)
    g[oW1:ob1] = (dz1.T @ c["a0"]).ravel()
    g[ob1:oW2] = dz1.sum(0)
    return float(np.mean(r ** 2)), g


class Adam:
    def __init__(self, lr=3e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = np.zeros(N_TRAINABLE)
        self.v = np.zeros(N_TRAINABLE)
        self.t = 0

    def step(self, theta, grad):
        self.t += 1
        g = grad[:N_TRAINABLE]
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        out = np.array(theta, dtype=np.float64)
        out[:N_TRAINABLE] -= self.lr * mh / (np.sqrt(vh) + self.eps)
        return out


def fit_norm(theta, X):
    out = np.array(theta, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    sd = X.std(0)
    out[oMean:oStd] = X.mean(0)
    out[oStd:N_PARAMS] = np.where(sd > 1e-6, sd, 1.0)
    return out


DENSITY_PAIRS = 256
_GAMMA = 0x9E3779B97F4A7C15
_MASK = (1 << 64) - 1


def splitmix64(c: int, seed: int = 0) -> int:
    """Output number c (from 0) of SplitMix64 with the given seed (Steele, Lea
    and Flood, OOPSLA 2014): the finaliser applied to seed + (c + 1) * gamma."""
    z = (seed + (c + 1) * _GAMMA) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def sampled_pair(v: int, t: int, k: int):
    """Pair t (0 <= t < DENSITY_PAIRS) of positions in a k-element P of root v
    (input id): x = output t of SplitMix64 seeded with the vertex key of v
    (output v of SplitMix64 seeded with 0); a = (low 32 bits of x) mod k;
    b = (high 32 bits) mod (k - 1), moved past a.  Returns (i, j), i < j."""
    x = splitmix64(t, seed=splitmix64(v))
    a = (x & 0xFFFFFFFF) % k
    b = (x >> 32) % (k - 1)
    if b >= a:
        b += 1
    return min(a, b), max(a, b)


def features(g, roots, order):
    """Features of the given roots (input ids) under the given vertex order."""
    n = g.n
    pos = np.empty(n, dtype=np.int64)
    pos[np.asarray(order, dtype=np.int64)] = np.arange(n)
    deg = g.degrees()
    import oracle

    core, _, _ = oracle.sync_peel(g)
    out = np.zeros((len(roots), 4))
    for i, v in enumerate(roots):
        nb = g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].astype(np.int64)
        P = nb[pos[nb] > pos[v]]
        k = len(P)
        if k < 2:
            density = 0.0
        elif k * (k - 1) // 2 <= DENSITY_PAIRS:
            Pset = set(P.tolist())
            e = 0
            for u in P:
                for w in g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]:
                    if int(w) in Pset and pos[w] > pos[u]:
                        e += 1
            density = e / (k * (k - 1) / 2)
        else:
            Ps = P[np.argsort(pos[P], kind="stable")]  # P in the order's sequence
            hits = 0
            for t in range(DENSITY_PAIRS):
                a, b = sampled_pair(int(v), t, k)
                u, w = int(Ps[a]), int(Ps[b])
                row = g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]
                hits += int(np.any(row == w))
            density = hits / DENSITY_PAIRS
        out[i] = [np.log1p(deg[v]), np.log1p(core[v]), np.log1p(deg[nb].sum()), density]
    return out


# ------------------------------------------------------------ rounding-aware references
# Error bounds follow the classical forward analysis of sums of products
# (Higham, "Accuracy and Stability of Numerical Algorithms", 2nd ed., Sec. 3.1
# and 3.5): a quantity formed through at most k floating-point roundings of
# unit roundoff u differs from its exact value by at most gamma_k times the
# same expression evaluated with the absolute value of every operand, where
# gamma_k = k u / (1 - k u).

U32 = 2.0 ** -24  # unit roundoff of FP32


def gamma(k, u=U32):
    return k * u / (1.0 - k * u)


def bf16_round(x):
    """FP32 values rounded to bfloat16 (round to nearest, ties to even), as
    float64.  The input is first converted to FP32 (round to nearest)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, X):
    """Forward pass with BF16 weights, biases and activations (rounded after
    every ReLU, and the normalised input after its FP32 arithmetic) and FP32
    sums, as an FP64 reference value y plus a radius r such that every FP32
    evaluation of the same network with any summation order lies in
    [y - r, y + r].

    Interval propagation: a layer's pre-activation lies within gamma_k times
    its absolute sum (k = number of terms) plus the propagated deviation of its
    inputs; ReLU and round-to-nearest are monotone, so the deviation of a
    rounded activation is bounded by rounding the interval's end points.  An
    activation whose interval does not reach a BF16 rounding boundary is
    exact."""
    p = unpack(theta)
    W = [bf16_round(p["W1"]), bf16_round(p["W2"]), bf16_round(p["W3"])]
    B = [bf16_round(p["b1"]), bf16_round(p["b2"]), bf16_round(p["b3"])]
    W4, b4 = bf16_round(p["W4"]), float(bf16_round(p["b4"]))
    X32 = np.asarray(X, dtype=np.float32)
    mean = np.asarray(p["mean"], dtype=np.float32)
    sd = np.asarray(p["std"], dtype=np.float32)
    h = bf16_round((X32 - mean) / sd)  # FP32 subtraction and division, then BF16
    dh = np.zeros_like(h)
    for li, (Wl, bl) in enumerate(zip(W, B)):
        # the 64-input layers may accumulate on matrix units whose internal
        # rounding is not specified: their bound takes twice the roundings
        k = (Wl.shape[1] + 1) * (2 if li else 1)
        z = h @ Wl.T + bl
        mag = (np.abs(h) + dh) @ np.abs(Wl).T + np.abs(bl)
        rad = gamma(k) * mag + dh @ np.abs(Wl).T
        hr = bf16_round(np.maximum(z, 0.0))
        lo = bf16_round(np.maximum(z - rad, 0.0))
        hi = bf16_round(np.maximum(z + rad, 0.0))
        dh = np.maximum(hi - hr, hr - lo)
        h = hr
    y = h @ W4 + b4
    mag = (np.abs(h) + dh) @ np.abs(W4) + abs(b4)
    rad = gamma(W4.shape[0] + 1) * mag + dh @ np.abs(W4)
    return y, rad


def loss_grad_bound(theta, X, t, k_rounds):
    """Magnitudes for an element-wise bound on an FP32 evaluation of
    loss_grad: (A_grad, A_loss, margin).  A_grad is the gradient evaluated with
    absolute values throughout (|W|, absolute forward sums, and |dL/dy|
    replaced by 2 (|y - t| + |y|_abs) / n, which covers the forward error
    that enters y - t; t must be representable in FP32).  An FP32
    evaluation whose longest chain of roundings per entry is k_rounds differs
    from the exact gradient by at most gamma(k_rounds) * A_grad, provided it
    takes the same ReLU decisions.  margin[s] is the
    smallest |z| / (gamma(k_rounds) * |z|_abs) over the pre-activations of
    sample s: where it exceeds 1 no rounding can flip that sample's decisions."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = X.shape[0]
    y, c = forward(theta, X)
    # |x - mean| / std rounds relative to (|x| + |mean|) / std
    a0 = (np.abs(X) + np.abs(p["mean"])) / np.abs(p["std"])
    aW1, aW2, aW3, aW4 = (np.abs(p[k]) for k in ("W1", "W2", "W3", "W4"))
    m1 = np.abs(a0) @ aW1.T + np.abs(p["b1"])
    m2 = (m1 * (c["z1"] > 0)) @ aW2.T + np.abs(p["b2"])
    m3 = (m2 * (c["z2"] > 0)) @ aW3.T + np.abs(p["b3"])
    ya = (m3 * (c["z3"] > 0)) @ aW4 + abs(p["b4"])
    g = gamma(k_rounds)
    margin = np.full(n, np.inf)
    for z, m in ((c["z1"], m1), (c["z2"], m2), (c["z3"], m3)):
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(m > 0, np.abs(z) / (g * m), np.inf)
        margin = np.minimum(margin, r.min(axis=1))
    dya = 2.0 * (ya + np.abs(y - t)) / n
    h1a, h2a, h3a = m1 * (c["z1"] > 0), m2 * (c["z2"] > 0), m3 * (c["z3"] > 0)
    A = np.zeros(N_PARAMS)
    A[oW4:ob4] = h3a.T @ dya
    A[ob4] = dya.sum()
    d3 = np.outer(dya, aW4) * (c["z3"] > 0)
    A[oW3:ob3] = (d3.T @ h2a).ravel()
    A[ob3:oW4] = d3.sum(0)
    d2 = (d3 @ aW3) * (c["z2"] > 0)
    A[oW2:ob2] = (d2.T @ h1a).ravel()
    A[ob2:oW3] = d2.sum(0)
    d1 = (d2 @ aW2) * (c["z1"] > 0)
    A[oW1:ob1] = (d1.T @ np.abs(a0)).ravel()
    A[ob1:oW2] = d1.sum(0)
    A_loss = float(np.mean((ya + np.abs(y - t)) ** 2))
    return A, A_loss, margin
