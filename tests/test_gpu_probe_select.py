"""Probe selection (Sec. 4, IVF) checked bit-exactly on the GPU's own FP32
centroid distances: the lists returned are the nprobe smallest entries of the
query's distance row, nearest first, equal distances in list-id order (a
stable sort of the row), and the distances returned are the row's entries.
Cases cover list counts that are not a multiple of 16 or 64, selections
larger than the number of list groups, the grouped selection (nprobe <= 64
on batches whose centroid product uses 128-wide tiles, so the group minima
exist: ceil(nq / 128) * ceil(nlist / 128) >= 1024), the full-row wave
selection (nprobe > 64, and a small batch), 16,384 lists, exact ties from
duplicated centroids and queries placed on centroids. Batches of at most 16
queries with nprobe above 256 take the rank selection, and batches of at
most 8 queries the few-row distance kernel, whose distances are also checked
against FP64."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NPROBES = (1, 5, 16, 33, 64, 65, 100, 256)
CASES = [
    # dim, nlist, nq, duplicated centroids
    (32, 37, 131072, False),
    (48, 100, 131072, True),
    (64, 257, 45000, False),
    (64, 1000, 16384, True),
    (64, 1000, 300, True),
    (128, 4096, 4200, False),
    (64, 5000, 3300, True),
    (32, 16384, 1100, False),
]


def _say(msg):
    print(f"[{msg}]", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dim,nlist,nq,dup", CASES, ids=[f"n{c[1]}q{c[2]}" + ("dup" if c[3] else "") for c in CASES])
def test_probe_selection_exact_on_gpu_distances(dim, nlist, nq, dup):
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say(f"probe selection dim={dim} nlist={nlist} nq={nq} dup={dup}")
    rng = np.random.default_rng(nlist + dim)
    cent = (rng.standard_normal((nlist, dim)) * 2).astype(np.float32)
    if dup:
        lo, hi = nlist // 5, nlist // 2
        cent[lo:hi] = cent[lo - 1]
    n = 2 * nlist + 64
    data = (cent[rng.integers(0, nlist, n)] + rng.standard_normal((n, dim))).astype(np.float32)
    assign = np.empty(n, dtype=np.int32)
    step = max(16, (1 << 24) // (nlist * dim))
    for s in range(0, n, step):
        d = ((data[s:s + step, None, :] - cent[None]) ** 2).sum(-1)
        assign[s:s + step] = np.argmin(d, 1)
    q = (cent[rng.integers(0, nlist, nq)] + rng.standard_normal((nq, dim))).astype(np.float32)
    q[::7] = cent[rng.integers(0, nlist, len(q[::7]))]   # on a centroid: distance 0
    idx = R.Index(dim, nlist, seed=5)
    try:
        idx.build(data, cent, assign)   # generated rotation
        qt = torch.from_numpy(q).to("cuda")
        D = R.rbq_debug_centroid_dists(idx.h, qt, nlist).cpu().numpy()
        assert np.all(D >= 0) and np.all(np.isfinite(D))
        order = np.argsort(D, axis=1, kind="stable")
        for nprobe in NPROBES:
            if nprobe > nlist:
                continue
            lists, d = R.rbq_debug_probe(idx.h, qt, nprobe)
            lists, d = lists.cpu().numpy(), d.cpu().numpy()
            want = order[:, :nprobe]
            np.testing.assert_array_equal(lists, want, err_msg=f"nprobe={nprobe}")
            np.testing.assert_array_equal(d, np.take_along_axis(D, want, 1), err_msg=f"nprobe={nprobe}")
    finally:
        idx.close()


FEW_CASES = [
    # dim, nlist, nq, duplicated centroids
    (32, 300, 1, True),
    (48, 1000, 3, True),
    (128, 4096, 8, False),
    (64, 2500, 16, True),
    (96, 16384, 1, False),
    (200, 5000, 5, False),
]


@pytest.mark.parametrize("dim,nlist,nq,dup", FEW_CASES, ids=[f"n{c[1]}q{c[2]}" + ("dup" if c[3] else "") for c in FEW_CASES])
def test_few_query_probe_selection_exact(dim, nlist, nq, dup):
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say(f"few-query probe selection dim={dim} nlist={nlist} nq={nq} dup={dup}")
    rng = np.random.default_rng(7 * nlist + dim)
    cent = (rng.standard_normal((nlist, dim)) * 2).astype(np.float32)
    if dup:
        lo, hi = nlist // 5, nlist // 2
        cent[lo:hi] = cent[lo - 1]
    n = 2 * nlist + 64
    data = (cent[rng.integers(0, nlist, n)] + rng.standard_normal((n, dim))).astype(np.float32)
    assign = rng.integers(0, nlist, n).astype(np.int32)
    q = (cent[rng.integers(0, nlist, nq)] + rng.standard_normal((nq, dim))).astype(np.float32)
    q[::3] = cent[rng.integers(0, nlist, len(q[::3]))]   # on a centroid: distance 0
    idx = R.Index(dim, nlist, seed=9)
    try:
        idx.build(data, cent, assign)
        qt = torch.from_numpy(q).to("cuda")
        D = R.rbq_debug_centroid_dists(idx.h, qt, nlist).cpu().numpy()
        # FP32 sums of dim products: within 1e-5 of the scale |q|^2 + |c|^2
        q64, c64 = q.astype(np.float64), cent.astype(np.float64)
        exact = ((q64[:, None, :] - c64[None]) ** 2).sum(-1)
        scale = (q64 ** 2).sum(1)[:, None] + (c64 ** 2).sum(1)[None]
        assert np.all(np.abs(D - exact) <= 1e-5 * scale + 1e-6)
        order = np.argsort(D, axis=1, kind="stable")
        for nprobe in (1, 64, 256, 257, 1000, 2048, 2049, nlist):
            if nprobe > nlist:
                continue
            lists, d = R.rbq_debug_probe(idx.h, qt, nprobe)
            lists, d = lists.cpu().numpy(), d.cpu().numpy()
            want = order[:, :nprobe]
            np.testing.assert_array_equal(lists, want, err_msg=f"nprobe={nprobe}")
            np.testing.assert_array_equal(d, np.take_along_axis(D, want, 1), err_msg=f"nprobe={nprobe}")
    finally:
        idx.close()


BF16X3_CASES = [
    # dim, nlist, nq, duplicated centroids (the first two take the group minima)
    (128, 4096, 4200, False),
    (32, 16384, 1100, False),
    (64, 1000, 300, True),
    (100, 2000, 700, False),
]


@pytest.mark.parametrize("dim,nlist,nq,dup", BF16X3_CASES,
                         ids=[f"n{c[1]}q{c[2]}d{c[0]}" + ("dup" if c[3] else "") for c in BF16X3_CASES])
def test_probe_selection_bf16x3_distances(dim, nlist, nq, dup):
    """BF16X3 indexes score centroids with split-BF16 products (hi*hi + hi*lo
    + lo*hi): the distances stay within 1e-5 of the scale |q|^2 + |c|^2 of
    their FP64 values, and the selection is exact on them (including the
    group minima of large batches)."""
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say(f"bf16x3 centroid distances dim={dim} nlist={nlist} nq={nq} dup={dup}")
    rng = np.random.default_rng(3 * nlist + dim)
    cent = (rng.standard_normal((nlist, dim)) * 2).astype(np.float32)
    if dup:
        lo, hi = nlist // 5, nlist // 2
        cent[lo:hi] = cent[lo - 1]
    n = 2 * nlist + 64
    data = (cent[rng.integers(0, nlist, n)] + rng.standard_normal((n, dim))).astype(np.float32)
    assign = rng.integers(0, nlist, n).astype(np.int32)
    q = (cent[rng.integers(0, nlist, nq)] + rng.standard_normal((nq, dim))).astype(np.float32)
    q[::7] = cent[rng.integers(0, nlist, len(q[::7]))]   # on a centroid: distance 0
    idx = R.Index(dim, nlist, seed=11, rot_precision=R.RBQ_ROT_BF16X3)
    try:
        idx.build(data, cent, assign)
        qt = torch.from_numpy(q).to("cuda")
        D = R.rbq_debug_centroid_dists(idx.h, qt, nlist).cpu().numpy()
        assert np.all(D >= 0) and np.all(np.isfinite(D))
        rows = rng.choice(nq, min(nq, 256), replace=False)
        q64, c64 = q[rows].astype(np.float64), cent.astype(np.float64)
        exact = ((q64[:, None, :] - c64[None]) ** 2).sum(-1)
        scale = (q64 ** 2).sum(1)[:, None] + (c64 ** 2).sum(1)[None]
        err = np.abs(D[rows] - exact) / scale
        print(f"max error / scale {err.max():.3g}")
        assert err.max() <= 1e-5
        order = np.argsort(D, axis=1, kind="stable")
        for nprobe in (1, 16, 64, 65, 256):
            if nprobe > nlist:
                continue
            lists, d = R.rbq_debug_probe(idx.h, qt, nprobe)
            lists, d = lists.cpu().numpy(), d.cpu().numpy()
            want = order[:, :nprobe]
            np.testing.assert_array_equal(lists, want, err_msg=f"nprobe={nprobe}")
            np.testing.assert_array_equal(d, np.take_along_axis(D, want, 1), err_msg=f"nprobe={nprobe}")
    finally:
        idx.close()
