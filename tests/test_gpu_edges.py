"""Edge cases and error paths of the HIP path, through the C ABI."""
import ctypes as C
import sys

import numpy as np
import pytest

from oracle import rabitq_oracle as O

from gpu_common import sqdist64

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[{msg}]", flush=True)
    sys.stdout.flush()


def _dev():
    import torch
    return torch.device("cuda:0")


def _index(data, cent, assign, seed=7, rot=0, code_bits=0, eps0=1.9):
    from paper_2405_12497_amd import rabitq as R
    dp = code_bits or O.code_length(data.shape[1])
    gauss = np.random.default_rng(seed).standard_normal((dp, dp))
    idx = R.Index(data.shape[1], cent.shape[0], code_bits=code_bits, rot_precision=rot, seed=seed,
                  eps0=eps0)
    idx.build(data, cent, assign, gauss)
    return idx


def test_fewer_vectors_than_k_pads_output():
    import torch
    _say("fewer vectors than k")
    rng = np.random.default_rng(1)
    data = rng.standard_normal((5, 64)).astype(np.float32)
    idx = _index(data, data.mean(0, keepdims=True), np.zeros(5, np.int32))
    q = torch.from_numpy(rng.standard_normal((3, 64)).astype(np.float32)).to(_dev())
    ids, d, st = idx.search(q, 10, 1, stats=True)
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    for qi in range(3):
        want, wd = O.exact_topk(data, q[qi].cpu().numpy(), 5)
        np.testing.assert_array_equal(ids[qi, :5], want)
        assert np.all(ids[qi, 5:] == -1) and np.all(np.isinf(d[qi, 5:]))
        np.testing.assert_allclose(d[qi, :5], wd, rtol=1e-5)


def test_degenerate_points_and_duplicates():
    """A vector at its centroid (||o_r - c|| = 0), a query at a centroid
    (||q_r - c|| = 0) and duplicated vectors (ties ordered by id)."""
    import torch
    _say("degenerate points")
    rng = np.random.default_rng(2)
    cent = rng.standard_normal((2, 128)).astype(np.float32) * 3
    data = np.concatenate([cent[0:1], cent[1:2], cent[0] + rng.standard_normal((300, 128)),
                           cent[1] + rng.standard_normal((300, 128))]).astype(np.float32)
    data = np.concatenate([data, data[10:20]])          # duplicates of ids 10..19 as 602..611
    assign = np.argmin(((data[:, None, :] - cent[None]) ** 2).sum(-1), 1).astype(np.int32)
    idx = _index(data, cent, assign)
    qs = np.stack([cent[0], cent[1], data[15], data[400]]).astype(np.float32)
    ids, d, _ = idx.search(torch.from_numpy(qs).to(_dev()), 10, 2)
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    for qi, q in enumerate(qs):
        want, wd = O.exact_topk(data, q, 10)
        np.testing.assert_array_equal(ids[qi], want)
    # the duplicate pair (15, 607) comes back in id order at distance 0
    assert ids[2, 0] == 15 and ids[2, 1] == 607 and d[2, 0] == 0 and d[2, 1] == 0


def test_empty_lists_and_full_probe():
    import torch
    _say("empty lists")
    rng = np.random.default_rng(3)
    data = rng.standard_normal((700, 64)).astype(np.float32)
    cent = np.concatenate([rng.standard_normal((4, 64)), rng.standard_normal((4, 64)) + 50]).astype(np.float32)
    assign = np.argmin(((data[:, None, :] - cent[None, :4]) ** 2).sum(-1), 1).astype(np.int32)
    # eps0 = 4 makes a bound failure among the true neighbours practically impossible,
    # so the probed-everything result must equal the exact top-k
    idx = _index(data, cent, assign, eps0=4.0)
    sizes = idx.list_sizes()
    assert np.all(sizes[4:] == 0)
    q = rng.standard_normal((6, 64)).astype(np.float32)
    ids, d, st = idx.search(torch.from_numpy(q).to(_dev()), 7, 8, stats=True)
    ids = ids.cpu().numpy()
    for qi in range(6):
        want, _ = O.exact_topk(data, q[qi], 7)
        np.testing.assert_array_equal(ids[qi], want)
    assert st["codes_scanned"] == 6 * 700


def test_zero_queries_is_a_noop():
    import torch
    _say("nq = 0")
    rng = np.random.default_rng(4)
    data = rng.standard_normal((100, 64)).astype(np.float32)
    idx = _index(data, data.mean(0, keepdims=True), np.zeros(100, np.int32))
    q = torch.empty((0, 64), dtype=torch.float32, device=_dev())
    ids, d, st = idx.search(q, 5, 1, stats=True)
    assert ids.shape == (0, 5) and st["queries"] == 0


def test_argument_errors():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("argument errors")
    rng = np.random.default_rng(5)
    data = rng.standard_normal((200, 64)).astype(np.float32)
    cent = data[:4].copy()
    idx = _index(data, cent, (np.arange(200) % 4).astype(np.int32))
    q = torch.from_numpy(data[:2]).to(_dev())
    for k, nprobe in ((0, 1), (257, 1), (5, 0), (5, 5)):
        with pytest.raises(R.RbqError) as e:
            idx.search(q, k, nprobe)
        assert e.value.status == R.RBQ_EINVAL
    # NULL buffers are rejected
    o = R.RbqSearchOpts(5, 1, 0, 0, None, 0, 0, 0)
    out_i = torch.empty((2, 5), dtype=torch.int64, device=_dev())
    out_d = torch.empty((2, 5), dtype=torch.float32, device=_dev())
    st = R.lib().rbq_search(idx.h, None, 2, C.byref(o),
                            C.c_void_p(out_i.data_ptr()), C.c_void_p(out_d.data_ptr()), None, None)
    assert st == R.RBQ_EINVAL
    # build rejects out-of-range assignments and leaves nothing half-built
    bad = np.zeros(200, np.int32)
    bad[7] = 9
    with pytest.raises(R.RbqError):
        R.rbq_index_build(idx.h, data, cent, bad)


def test_allocation_failure_reports_enomem_and_recovers():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("allocation failure")
    rng = np.random.default_rng(6)
    data = rng.standard_normal((300, 64)).astype(np.float32)
    idx = _index(data, data.mean(0, keepdims=True), np.zeros(300, np.int32))
    q = torch.from_numpy(rng.standard_normal((40, 64)).astype(np.float32)).to(_dev())
    R.rbq_debug_fail_alloc_after(1)          # the workspace allocation of the next search fails
    with pytest.raises(R.RbqError) as e:
        idx.search(q, 5, 1)
    assert e.value.status == R.RBQ_ENOMEM
    R.rbq_debug_fail_alloc_after(0)
    ids, _, _ = idx.search(q, 5, 1)
    want = np.stack([O.exact_topk(data, x, 5)[0] for x in q.cpu().numpy()])
    assert (ids.cpu().numpy() == want).mean() > 0.95


def test_save_load_roundtrip(tmp_path):
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("save/load")
    rng = np.random.default_rng(7)
    data = rng.standard_normal((1500, 96)).astype(np.float32)
    cent = data[rng.choice(1500, 8, replace=False)]
    assign = np.argmin(((data[:, None, :] - cent[None]) ** 2).sum(-1), 1).astype(np.int32)
    idx = _index(data, cent, assign, rot=R.RBQ_ROT_BF16X3)
    q = torch.from_numpy(rng.standard_normal((9, 96)).astype(np.float32)).to(_dev())
    a1, d1, _ = idx.search(q, 10, 3)
    path = str(tmp_path / "i.rbq")
    idx.save(path)
    idx2 = R.Index.load(path)
    a2, d2, _ = idx2.search(q, 10, 3)
    np.testing.assert_array_equal(a1.cpu().numpy(), a2.cpu().numpy())
    np.testing.assert_array_equal(d1.cpu().numpy(), d2.cpu().numpy())
    c1 = R.rbq_debug_export_codes(idx.h, 1500, 2)
    c2 = R.rbq_debug_export_codes(idx2.h, 1500, 2)
    for x, y in zip(c1, c2):
        np.testing.assert_array_equal(x, y)
    # flip one payload byte: checksum mismatch
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0xFF
    open(path, "wb").write(bytes(raw))
    with pytest.raises(R.RbqError) as e:
        R.Index.load(path)
    assert e.value.status == R.RBQ_EFORMAT


def test_generated_rotation_when_none_given():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("generated rotation")
    rng = np.random.default_rng(8)
    data = rng.standard_normal((800, 128)).astype(np.float32)
    idx = R.Index(128, 1, seed=99)
    idx.build(data, data.mean(0, keepdims=True), np.zeros(800, np.int32))
    q = torch.from_numpy(data[:4] + 0.01).to(_dev())
    ids, d, _ = idx.search(q, 3, 1)
    assert list(ids.cpu().numpy()[:, 0]) == [0, 1, 2, 3]
    np.testing.assert_allclose(d.cpu().numpy()[:, 0], sqdist64(data[:4], data[:4] + 0.01), rtol=1e-3)


def test_sub_batches_equal_one_batch():
    """A batch whose candidate segments exceed the budget is searched in
    sub-batches (query ids, per-query nprobe and outputs offset per
    sub-batch): same ids, distances and counters as one batch."""
    import torch
    from paper_2405_12497_amd import rabitq as R
    from gpu_common import Built, make_case
    _say("sub-batches")
    b = Built(make_case("ivf128"))
    rng = np.random.default_rng(13)
    qs = (b.case.queries[rng.integers(0, len(b.case.queries), 37)] +
          rng.normal(0, 1, (37, b.case.dim))).astype(np.float32)
    q = torch.from_numpy(qs).to(_dev())
    npq = torch.from_numpy(rng.integers(1, 9, 37).astype(np.int32)).to(_dev())
    one = b.idx.search(q, 10, 8, nprobe_per_query=npq, qid_base=100, stats=True)
    row = int(b.idx.list_sizes()[np.argsort(-b.idx.list_sizes())[:8]].sum()) * 8
    try:
        R.rbq_debug_seg_budget(row * 5)          # 5 queries per sub-batch
        split = b.idx.search(q, 10, 8, nprobe_per_query=npq, qid_base=100, stats=True)
    finally:
        R.rbq_debug_seg_budget(0)
    np.testing.assert_array_equal(one[0].cpu().numpy(), split[0].cpu().numpy())
    np.testing.assert_array_equal(one[1].cpu().numpy(), split[1].cpu().numpy())
    assert one[2] == split[2]


def test_profile_levels():
    """Stage timing (RBQ_PROFILE_STAGES) bounds every stage; the scan level
    (RBQ_PROFILE_SCAN) only the main scan and the rerank; both count the same
    codes per scan phase, profiling leaves the results unchanged, and other
    levels are rejected."""
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("profile levels")
    rng = np.random.default_rng(11)
    cent = (rng.standard_normal((64, 64)) * 3).astype(np.float32)
    data = (cent[rng.integers(0, 64, 6000)] + rng.standard_normal((6000, 64))).astype(np.float32)
    assign = np.argmin(((data[:, None, :] - cent[None]) ** 2).sum(-1), 1).astype(np.int32)
    idx = _index(data, cent, assign)
    q = torch.from_numpy(data[:300] + 0.1).to(_dev())
    ids0, d0, _ = idx.search(q, 10, 8)
    got = {}
    for level in (R.RBQ_PROFILE_STAGES, R.RBQ_PROFILE_SCAN):
        R.rbq_profile_enable(idx.h, level)
        ids, d, _ = idx.search(q, 10, 8)
        ids, d, _ = idx.search(q, 10, 8)
        p = R.rbq_profile_read(idx.h)
        R.rbq_profile_enable(idx.h, False)
        assert torch.equal(ids, ids0) and torch.equal(d, d0)
        assert p["searches"] == 2
        assert p["ms_scan1"] > 0 and p["ms_finalize"] > 0
        got[level] = p
    st, sc = got[R.RBQ_PROFILE_STAGES], got[R.RBQ_PROFILE_SCAN]
    assert all(st[kk] > 0 for kk in ("ms_front", "ms_prep", "ms_scan0", "ms_tau"))
    assert all(sc[kk] == 0 for kk in ("ms_front", "ms_prep", "ms_scan0", "ms_tau"))
    assert st["codes_scan0"] == sc["codes_scan0"] > 0
    assert st["codes_scan1"] == sc["codes_scan1"] > 0
    with pytest.raises(R.RbqError):
        R.rbq_profile_enable(idx.h, 3)
    idx.close()
