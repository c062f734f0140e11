"""rbq_autotune: per batch-size bucket it picks the chunk length, the scan
kernel and the rerank waves by timing whole searches; afterwards searches use
those choices and still return the exact top-k of the probed lists wherever
the error bound holds (Sec. 4)."""
import sys

import numpy as np
import pytest

from oracle import rabitq_oracle as O
import synth

from gpu_common import oracle_estimates_on, tie_equivalent, unpack_codes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[{msg}]", flush=True)
    sys.stdout.flush()


def test_autotune_table_and_results():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("autotune")
    data, qs = synth.sift_like(30000, 600, seed_data=501, seed_query=502)
    cent, assign = synth.kmeans(data, 96, iters=4, seed=503)
    idx = R.Index(128, 96, seed=504)
    idx.build(data, cent, assign, synth.gaussian_matrix(128, 505))
    assert R.rbq_autotune_get(idx.h) == []
    q = torch.from_numpy(qs).cuda()
    k, nprobe = 10, 8
    before, _, _ = idx.search(q, k, nprobe)
    R.rbq_autotune(idx.h, qs, k, nprobe)            # host queries
    table = R.rbq_autotune_get(idx.h)
    print("tuned:", table)
    assert [t["max_nq"] for t in table][:-1] == sorted(t["max_nq"] for t in table[:-1])
    assert len(table) == 5                           # 1, 8, 64, 512 and the 600-query sample
    for t in table:
        assert t["chunk"] in (256, 512, 1024, 2048)
        assert t["scan_kernel"] in (R.RBQ_SCAN_POPCNT, R.RBQ_SCAN_MFMA)
        assert 0 <= t["rerank_waves"] <= 64 and t["ms"] > 0
    R.rbq_autotune(idx.h, q[:100].contiguous(), k, nprobe)   # device queries
    assert len(R.rbq_autotune_get(idx.h)) == 4
    # searches after tuning: the exact top-k of the probed lists unless a bound failed
    codes, norm, ipo = R.rbq_debug_export_codes(idx.h, len(data), 2)
    bits = unpack_codes(codes, 128)
    lists, _ = R.rbq_debug_probe(idx.h, q, nprobe)
    lists = lists.cpu().numpy()
    for sub in (q[:1], q[:7], q[:64], q):
        ids, _, _ = idx.search(sub.contiguous(), k, nprobe)
        ids = ids.cpu().numpy()
        for qi in range(len(ids)):
            cand = np.flatnonzero(np.isin(assign, lists[qi]))
            t_ids, t_d = O.exact_topk(data, qs[qi], k, cand)
            if tie_equivalent(ids[qi], t_ids, qs[qi], data):
                continue
            qu, scal = R.rbq_debug_quantize(idx.h, q[qi:qi + 1].contiguous(),
                                            torch.from_numpy(lists[qi:qi + 1]).cuda(), 128, qid_base=qi)
            qu, scal = qu.cpu().numpy().astype(np.int64), scal.cpu().numpy()
            fail = False
            for oid, dv in zip(t_ids, t_d):
                r = int(np.flatnonzero(lists[qi] == assign[oid])[0])
                lbv = oracle_estimates_on(bits[oid:oid + 1], norm[oid:oid + 1], ipo[oid:oid + 1], qu[r],
                                          scal[r, 0], scal[r, 1], scal[r, 2], 128)[4][0]
                fail |= lbv > dv * (1 + 1e-6)
            assert fail, f"query {qi}: differs from the exact top-k without a bound failure"
    after, _, _ = idx.search(q, k, nprobe)
    same = (after.cpu().numpy() == before.cpu().numpy()).all(1).mean()
    print(f"queries with the same result before and after tuning: {same:.3f}")
    assert same >= 0.95
    idx.close()
