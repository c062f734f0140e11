"""FP64 reference for the learned per-query nprobe model — TEST INFRASTRUCTURE ONLY.

The learned nprobe is not part of the paper (its related-work section only
mentions machine-learned routing for ANN search); the features, buckets and
network below are project definitions, so their parity is unpinned beyond
calculus: gradients are checked by finite differences, the softmax/cross-entropy
by closed forms, and the feature layout by its definition.

Network: x[96] -> h = ReLU(x W1 + b1)[128] -> z = h W2 + b2 [32] -> softmax.
Loss: mean cross-entropy of integer labels.
"""
from __future__ import annotations

import math

import numpy as np

from . import rabitq_oracle as O

N_IN, N_HID, N_OUT = 96, 128, 32
N_NEAR = 64      # centroid distances used as features
N_STATS = 8      # nearest lists whose quantiser statistics are used


def split_params(w):
    """Flat FP32/FP64 vector in the order W1[96x128], b1[128], W2[128x32], b2[32]."""
    w = np.asarray(w, dtype=np.float64)
    o = 0
    W1 = w[o:o + N_IN * N_HID].reshape(N_IN, N_HID); o += N_IN * N_HID
    b1 = w[o:o + N_HID]; o += N_HID
    W2 = w[o:o + N_HID * N_OUT].reshape(N_HID, N_OUT); o += N_HID * N_OUT
    b2 = w[o:o + N_OUT]; o += N_OUT
    assert o == len(w)
    return W1, b1, W2, b2


def join_params(W1, b1, W2, b2):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2)])


def forward(x, w):
    W1, b1, W2, b2 = split_params(w)
    x = np.asarray(x, dtype=np.float64)
    a = x @ W1 + b1
    h = np.maximum(a, 0.0)
    z = h @ W2 + b2
    return a, h, z


def softmax(z):
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(z - z.max(-1, keepdims=True))
    return e / e.sum(-1, keepdims=True)


def loss_and_grad(x, y, w):
    """Mean cross-entropy and its gradient with respect to the flat parameters."""
    W1, b1, W2, b2 = split_params(w)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.int64)
    n = len(y)
    a, h, z = forward(x, w)
    p = softmax(z)
    loss = float(-np.mean(np.log(p[np.arange(n), y])))
    dz = p.copy()
    dz[np.arange(n), y] -= 1.0
    dz /= n
    dW2 = h.T @ dz
    db2 = dz.sum(0)
    dh = dz @ W2.T
    da = dh * (a > 0)
    dW1 = x.T @ da
    db1 = da.sum(0)
    return loss, join_params(dW1, db1, dW2, db2)


# ------------------------------------------------------------------ buckets and policy

def bucket_table():
    """b_0 = 4, b_j = max(b_{j-1} + 1, round(4 * 2^(7j/31))), so b_31 = 512."""
    b = [4]
    for j in range(1, N_OUT):
        b.append(max(b[-1] + 1, int(round(4 * 2 ** (7 * j / 31)))))
    return np.array(b, dtype=np.int64)


def label_of(min_nprobe):
    """Smallest bucket whose nprobe covers `min_nprobe` (clamped to the last bucket)."""
    b = bucket_table()
    j = np.searchsorted(b, np.asarray(min_nprobe), side="left")
    return np.minimum(j, N_OUT - 1)


def policy(logits, threshold):
    """nprobe of the smallest bucket whose cumulative softmax reaches `threshold`."""
    p = softmax(logits)
    c = np.cumsum(p, -1)
    j = np.argmax(c >= threshold - 1e-12, axis=-1)
    return bucket_table()[j]


# ------------------------------------------------------------------ features

def expected_sq_fraction(qq) -> float:
    """E[S_q] / (15 * code length) of a quantised pair: E[q_u,i] = (q'_i - v_l)/Delta
    (Theorem 3.3), Delta = (v_r - v_l)/15; 0 when b = 0 or v_r = v_l."""
    if qq.b == 0.0 or qq.vr <= qq.vl:
        return 0.0
    qp = np.asarray(qq.qprime, np.float64)
    return float(np.mean((qp - qq.vl) / (qq.vr - qq.vl)))


def features(index: "O.OracleIndex", q_raw, qid: int, seed: int):
    """96 features of one query:
    [0]      log d_(1), the squared distance to the nearest centroid
    [1..63]  log(d_(j)/d_(1)) for the 2nd..64th nearest centroids
    [64..95] for each of the 8 nearest lists: ||q_r - c_k||/||q_r - c_1||, v_l, v_r,
             E[sum q_u] / (15 * code length) = the mean of (q'_i - v_l) / (v_r - v_l)
             over the code length (Sec. 3.3.1 quantiser of that pair; the
             randomized rounding is unbiased, Theorem 3.3, so no draw is needed)
    Missing centroids (fewer than 64 lists) repeat the last available value.
    """
    c = index.centroids
    d = ((c - np.asarray(q_raw, np.float64)[None, :]) ** 2).sum(1)
    order = np.lexsort((np.arange(len(d)), d))
    near = d[order[:N_NEAR]]
    if len(near) < N_NEAR:
        near = np.concatenate([near, np.full(N_NEAR - len(near), near[-1])])
    tiny = 1e-30
    f = np.zeros(N_IN)
    f[0] = math.log(max(near[0], tiny))
    f[1:N_NEAR] = np.log(np.maximum(near[1:], tiny)) - math.log(max(near[0], tiny))
    b1 = None
    for r in range(N_STATS):
        lid = int(order[min(r, len(order) - 1)])
        u = O.rounding_uniforms_fast(seed, qid, lid, index.dp)
        qq = O.quantize_query(q_raw, c[lid], index.p, u)
        if b1 is None:
            b1 = max(qq.b, tiny)
        base = N_NEAR + 4 * r
        f[base + 0] = qq.b / b1
        f[base + 1] = qq.vl
        f[base + 2] = qq.vr
        f[base + 3] = expected_sq_fraction(qq)
    return f
