"""Searches replayed from captured HIP graphs (use_graph = 1) against the same
searches launched directly: every replay, interleaved with other eager work
and synchronisations, must return identical ids, distances and counters."""
import sys

import numpy as np
import pytest

from gpu_common import Built, make_case

pytestmark = pytest.mark.gpu
_B = {}


def _say(msg):
    print(f"[{msg}]", flush=True)
    sys.stdout.flush()


def _built():
    if "ivf128" not in _B:
        _B["ivf128"] = Built(make_case("ivf128"))
    return _B["ivf128"]


def _batch(b, nq, seed):
    import torch
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, len(b.case.queries), nq)
    q = b.case.queries[rows] + rng.normal(0, 0.5, (nq, b.case.dim)).astype(np.float32)
    return torch.from_numpy(q.astype(np.float32)).to(b.dev)


def _same(a, g):
    np.testing.assert_array_equal(a[0].cpu().numpy(), g[0].cpu().numpy())
    np.testing.assert_array_equal(a[1].cpu().numpy(), g[1].cpu().numpy())
    assert a[2] == g[2]


@pytest.mark.parametrize("kernel", ["popcnt", "mfma"])
def test_graph_replays_match_eager(kernel):
    import torch
    _say(f"graph replays, {kernel}")
    b = _built()
    R = b.R
    kern = R.RBQ_SCAN_POPCNT if kernel == "popcnt" else R.RBQ_SCAN_MFMA
    sizes = (1, 5, 17, 40, 33)            # 17 -> 18 rows, 40 -> 40, 33 -> 36: padded captures
    batches = {n: _batch(b, n, 100 + n) for n in sizes}
    eager = {n: b.idx.search(batches[n], 10, 8, scan_kernel=kern, stats=True) for n in sizes}
    for rep in range(3):
        if rep == 1:
            captured = b.idx.info()["graph_captures"]
        for n in sizes:
            g = b.idx.search(batches[n], 10, 8, scan_kernel=kern, stats=True, use_graph=True)
            _same(eager[n], g)
            # eager work of another shape between replays
            other = sizes[(sizes.index(n) + 1) % len(sizes)]
            e2 = b.idx.search(batches[other], 10, 8, scan_kernel=kern, stats=True)
            _same(eager[other], e2)
            torch.cuda.synchronize()
    # later rounds replay: no shape is captured again
    assert b.idx.info()["graph_captures"] == captured


def test_graph_with_per_query_nprobe_and_qid_base():
    import torch
    _say("graph replays, per-query nprobe")
    b = _built()
    q = _batch(b, 21, 7)
    npq = torch.from_numpy(np.random.default_rng(8).integers(1, 9, 21).astype(np.int32)).to(b.dev)
    e = b.idx.search(q, 10, 8, nprobe_per_query=npq, qid_base=1000, stats=True)
    for rep in range(3):
        g = b.idx.search(q, 10, 8, nprobe_per_query=npq, qid_base=1000, stats=True, use_graph=True)
        _same(e, g)
        b.idx.search(q[:3].contiguous(), 5, 2)
        torch.cuda.synchronize()
    # a different qid_base is a different shape: captured anew, still equal to eager
    e2 = b.idx.search(q, 10, 8, nprobe_per_query=npq, qid_base=5, stats=True)
    g2 = b.idx.search(q, 10, 8, nprobe_per_query=npq, qid_base=5, stats=True, use_graph=True)
    _same(e2, g2)


def test_graph_learned_nprobe_and_model_change():
    import torch
    R = _built().R
    _say("graph replays, learned nprobe")
    b = _built()
    q = _batch(b, 12, 9)
    for j in (3, 9):
        w = np.zeros(R.MLP_NPARAM, np.float32)
        w[-32 + j] = 40.0                     # all softmax mass on bucket j
        R.rbq_nprobe_model_set(b.idx.h, w, 0.9)
        e = b.idx.search(q, 10, 16, use_learned_nprobe=True, stats=True)
        for rep in range(2):
            g = b.idx.search(q, 10, 16, use_learned_nprobe=True, stats=True, use_graph=True)
            _same(e, g)
            torch.cuda.synchronize()
    R.rbq_nprobe_model_set(b.idx.h, None, 0.9)
    e = b.idx.search(q, 10, 16, use_learned_nprobe=True, stats=True)
    g = b.idx.search(q, 10, 16, use_learned_nprobe=True, stats=True, use_graph=True)
    _same(e, g)


def test_graph_after_workspace_growth():
    """A larger eager batch reallocates the workspace; the next replay of a
    smaller shape must be recaptured, not replay stale addresses."""
    import torch
    _say("graph after workspace growth")
    b = _built()
    small, big = _batch(b, 9, 11), _batch(b, 700, 12)
    e = b.idx.search(small, 10, 8, stats=True)
    _same(e, b.idx.search(small, 10, 8, stats=True, use_graph=True))
    b.idx.search(big, 10, 40)
    torch.cuda.synchronize()
    _same(e, b.idx.search(small, 10, 8, stats=True, use_graph=True))
