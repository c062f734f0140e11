"""Pins for the FP64 learned-nprobe reference: calculus and closed forms."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M
from oracle import rabitq_oracle as O


def _params(seed=0, scale=0.2):
    rng = np.random.default_rng(seed)
    n = M.N_IN * M.N_HID + M.N_HID + M.N_HID * M.N_OUT + M.N_OUT
    return rng.normal(0, scale, n)


def test_gradient_matches_central_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(0, 1, (7, M.N_IN))
    y = rng.integers(0, M.N_OUT, 7)
    w = _params(2)
    loss, g = M.loss_and_grad(x, y, w)
    idx = rng.choice(len(w), 60, replace=False)
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (M.loss_and_grad(x, y, wp)[0] - M.loss_and_grad(x, y, wm)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-9)


def test_softmax_and_cross_entropy_closed_forms():
    z = np.zeros((3, M.N_OUT))
    np.testing.assert_allclose(M.softmax(z).sum(-1), 1.0)
    w = np.zeros(M.N_IN * M.N_HID + M.N_HID + M.N_HID * M.N_OUT + M.N_OUT)
    loss, g = M.loss_and_grad(np.ones((4, M.N_IN)), np.array([0, 5, 9, 31]), w)
    assert loss == pytest.approx(math.log(M.N_OUT))
    # with zero weights the only non-zero gradient is that of b2: mean(p - onehot)
    W1, b1, W2, b2 = M.split_params(g)
    assert np.all(W1 == 0) and np.all(b1 == 0) and np.all(W2 == 0)
    assert b2.sum() == pytest.approx(0.0, abs=1e-12)


def test_bucket_table_and_policy():
    b = M.bucket_table()
    assert len(b) == 32 and b[0] == 4 and b[-1] == 512 and np.all(np.diff(b) > 0)
    assert list(M.label_of([1, 4, 5, 512, 2000])) == [0, 0, 1, 31, 31]
    z = np.full((1, 32), -50.0)
    z[0, 7] = 50.0
    assert M.policy(z, 0.9)[0] == b[7]
    assert M.policy(np.zeros((1, 32)), 1.0)[0] == 512


def test_feature_layout():
    rng = np.random.default_rng(3)
    data = rng.normal(0, 1, (400, 64))
    cent = data[rng.choice(400, 70, replace=False)] + 0.1
    assign = np.argmin(((data[:, None] - cent[None]) ** 2).sum(-1), 1)
    idx = O.build_index(data, cent, assign, rng.normal(0, 1, (64, 64)))
    q = rng.normal(0, 1, 64)
    f = M.features(idx, q, 0, 11)
    d = np.sort(((cent - q) ** 2).sum(1))
    assert f[0] == pytest.approx(math.log(d[0]))
    np.testing.assert_allclose(f[1:64], np.log(d[1:64] / d[0]), rtol=1e-12)
    assert np.all(np.diff(f[1:64]) >= 0)
    assert f[64] == pytest.approx(1.0)
    assert np.all(f[64::4][:8] >= 1.0 - 1e-12)
    assert np.all(f[65::4][:8] < 0) and np.all(f[66::4][:8] > 0)
    assert np.all((f[67::4][:8] >= 0) & (f[67::4][:8] <= 1))


def test_expected_sq_feature_is_the_mean_of_the_randomized_rounding():
    """The S_q feature is E[S_q] / (15 D): averaged over many independent
    roundings (Sec. 3.3.1 with u_i uniform), the drawn S_q / (15 D) converges to
    it (unbiasedness, Theorem 3.3). 4000 draws: the sample mean's standard error
    is below sqrt(D) / 2 / (15 D) / sqrt(4000)."""
    rng = np.random.default_rng(21)
    dim = 64
    data = rng.normal(0, 1, (300, dim))
    cent = data[rng.choice(300, 10, replace=False)] + 0.05
    assign = np.argmin(((data[:, None] - cent[None]) ** 2).sum(-1), 1)
    idx = O.build_index(data, cent, assign, rng.normal(0, 1, (dim, dim)))
    q = rng.normal(0, 1, dim)
    for lid in range(3):
        qq0 = O.quantize_query(q, cent[lid], idx.p, np.zeros(idx.dp))
        want = M.expected_sq_fraction(qq0)
        draws = 4000
        tot = 0.0
        for _ in range(draws):
            qq = O.quantize_query(q, cent[lid], idx.p, rng.random(idx.dp))
            tot += qq.sq / (15.0 * idx.dp)
        se = math.sqrt(idx.dp) / 2 / (15.0 * idx.dp) / math.sqrt(draws)
        assert abs(tot / draws - want) <= 5 * se, (lid, tot / draws, want)
