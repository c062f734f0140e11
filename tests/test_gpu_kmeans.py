"""rbq_kmeans (the IVF clustering run before Algorithm 1) against the plain
definition of Lloyd's algorithm in FP64: one round from given centroids moves
every centroid to the mean of the rows nearest to it, and the final
assignment is the nearest centroid; the result is bit-identical run to run and
for host or device inputs. (k-means is not part of RaBitQ: parity unpinned
beyond this definition.)"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[{msg}]", flush=True)
    sys.stdout.flush()


def _d2(x, c):
    x = x.astype(np.float64)
    c = c.astype(np.float64)
    return (x * x).sum(1)[:, None] + (c * c).sum(1)[None, :] - 2.0 * x @ c.T


def test_one_lloyd_round_matches_definition():
    from paper_2405_12497_amd import rabitq as R
    _say("k-means one round")
    data, _ = synth.sift_like(20000, 1, seed_data=401, seed_query=402)
    c0 = data[np.random.default_rng(403).choice(len(data), 64, replace=False)].copy()
    cent, asg = R.rbq_kmeans(data, 64, iters=1, init=c0)
    d0 = _d2(data, c0)
    near = np.argmin(d0, 1)
    srt = np.sort(d0, 1)
    clear = (srt[:, 1] - srt[:, 0]) > 1e-4 * srt[:, 1]      # rows without a near-tie
    for l in range(64):
        members = near == l
        if not members.any():
            np.testing.assert_array_equal(cent[l], c0[l])   # empty lists keep their centroid
            continue
        if not np.all(clear[members]):
            continue
        np.testing.assert_allclose(cent[l], data[members].astype(np.float64).mean(0), rtol=1e-5, atol=1e-4)
    d1 = _d2(data, cent)
    best = np.argmin(d1, 1)
    s1 = np.sort(d1, 1)
    ok = (asg == best) | ((s1[:, 1] - s1[:, 0]) <= 1e-4 * s1[:, 1])
    assert ok.all(), f"{(~ok).sum()} rows not at their nearest centroid"


def test_kmeans_deterministic_and_host_device_equal():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("k-means determinism")
    data, _ = synth.embedding_like(30000, 1, dim=128, seed_data=411, seed_query=412)
    c1, a1 = R.rbq_kmeans(data, 100, iters=6, sample=12000, seed=9)
    c2, a2 = R.rbq_kmeans(data, 100, iters=6, sample=12000, seed=9)
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_array_equal(a1, a2)
    c3, a3 = R.rbq_kmeans(torch.from_numpy(data).cuda(), 100, iters=6, sample=12000, seed=9)
    np.testing.assert_array_equal(c3.cpu().numpy(), c1)
    np.testing.assert_array_equal(a3.cpu().numpy(), a1)
    # every list is used and the objective fell from the seeded start
    assert len(np.unique(a1)) == 100
    c0, _ = R.rbq_kmeans(data, 100, iters=0, sample=12000, seed=9)
    obj0 = np.min(_d2(data, c0), 1).mean()
    obj = np.min(_d2(data, c1), 1).mean()
    print(f"k-means objective {obj0:.5f} -> {obj:.5f}")
    assert obj < 0.95 * obj0
    with pytest.raises(R.RbqError):
        R.rbq_kmeans(data[:50], 100, iters=1)
