"""Parity at the real shapes of the batched and the single-query workloads,
on sampled queries the FP64 oracle checks one by one:
  - GIST-like 1M x 960 with 4096 lists of Zipf(1.1)-skewed sizes (the largest
    above 100,000 codes), one batch of 256 queries, top-100, with the int8-MFMA
    and the popcount scan: bit-exact integer <x_b, q_u> on the largest list and
    the exact top-100 of the probed lists for sampled queries;
  - embedding-like 1M x 768 with 16,384 lists, 1, 3 and 16 queries probing every list (the
    rank selection, the block-per-query plan, the 64-wave rerank and its block
    merge): the exact top-10 of the whole data set.
A query may differ from the exact top-k only where a true neighbour's lower
bound, recomputed by the oracle on the GPU path's own quantised query,
exceeds its distance."""
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


def test_gist_zipf_batch_of_256_top100():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("GIST-like 1M x 960, Zipf lists: generating")
    data, qs, means = synth.gist_like(1_000_000, 256, seed_data=1003, seed_query=2003)
    x = torch.from_numpy(data).cuda()
    cent, assign = R.rbq_kmeans(x, 4096, iters=10, seed=5003, init=means)
    assign = assign.cpu().numpy()
    sizes = np.bincount(assign, minlength=4096)
    print(f"largest lists {np.sort(sizes)[-3:]}, median {np.median(sizes)}")
    assert sizes.max() >= 100_000
    _say("building")
    idx = R.Index(960, 4096, rot_precision=R.RBQ_ROT_BF16X3, seed=4003)
    idx.build(x, cent, torch.from_numpy(assign).cuda(), synth.gaussian_matrix(960, 3003))
    codes, norm, ipo = R.rbq_debug_export_codes(idx.h, len(data), 15)
    q = torch.from_numpy(qs).cuda()
    oidx_p = O.orthogonal_from_gaussian(synth.gaussian_matrix(960, 3003))
    # bit-exact scan on the largest list, both kernels
    big = int(np.argmax(sizes))
    ids_big = R.rbq_debug_list_ids(idx.h, big, int(sizes[big]))
    bits_big = unpack_codes(codes[ids_big], 960)
    u = O.rounding_uniforms_fast(4003, 0, big, 960)
    oq = O.quantize_query(qs[0], cent[big].cpu().numpy(), oidx_p, u)
    oip = O.ip_naive(bits_big, oq.qu)
    opc = O.popcount_code(bits_big)
    for kern in (R.RBQ_SCAN_POPCNT, R.RBQ_SCAN_MFMA):
        _say(f"largest list ({sizes[big]} codes), kernel {kern}")
        ip, pc, _, _, _ = R.rbq_debug_scan(idx.h, big, torch.from_numpy(oq.qu.astype(np.uint8)).cuda(),
                                           np.float32(oq.b), np.float32(oq.vl), np.float32(oq.delta),
                                           int(sizes[big]), kernel=kern)
        np.testing.assert_array_equal(ip.cpu().numpy(), oip)
        np.testing.assert_array_equal(pc.cpu().numpy(), opc)
    del bits_big
    # one batch of 256 queries, top-100
    k, nprobe = 100, 16
    lists, _ = R.rbq_debug_probe(idx.h, q, nprobe)
    lists = lists.cpu().numpy()
    rng = np.random.default_rng(7)
    sample = rng.choice(256, 8, replace=False)
    order = np.argsort(assign, kind="stable")
    bounds = np.searchsorted(assign[order], np.arange(4097))
    bits_cache = {}
    for kern in (R.RBQ_SCAN_MFMA, R.RBQ_SCAN_POPCNT):
        _say(f"batch of 256, top-100, kernel {kern}")
        ids, d, st = idx.search(q, k, nprobe, scan_kernel=kern, stats=True)
        ids, d = ids.cpu().numpy(), d.cpu().numpy()
        print(f"kernel {kern}: stats {st}")
        bad = 0
        for qi in sample:
            cand = np.concatenate([order[bounds[l]:bounds[l + 1]] for l in lists[qi]])
            t_ids, t_d = O.exact_topk(data, qs[qi], k, cand)
            if tie_equivalent(ids[qi], t_ids, qs[qi], data):
                continue
            need = [i for i in t_ids if i not in bits_cache]
            if need:
                b = unpack_codes(codes[need], 960)
                for j, i in enumerate(need):
                    bits_cache[i] = b[j]
            sub_bits = {i: bits_cache[i] for i in t_ids}
            fail = False
            lids = np.unique(assign[t_ids]).astype(np.int32)
            qu, scal = R.rbq_debug_quantize(idx.h, q[qi:qi + 1].contiguous(),
                                            torch.from_numpy(lids[None, :]).cuda(), 960, qid_base=int(qi))
            qu, scal = qu.cpu().numpy().astype(np.int64), scal.cpu().numpy()
            for oid, dv in zip(t_ids, t_d):
                r = int(np.flatnonzero(lids == assign[oid])[0])
                lbv = oracle_estimates_on(sub_bits[oid][None, :], norm[oid:oid + 1], ipo[oid:oid + 1], qu[r],
                                          scal[r, 0], scal[r, 1], scal[r, 2], 960)[4][0]
                fail |= lbv > dv * (1 + 1e-6)
            assert fail, f"query {qi}: differs from the exact top-100 of its probed lists without a bound failure"
            bad += 1
        print(f"kernel {kern}: {bad} of {len(sample)} sampled queries differ, all with bound failures")
    idx.close()


def test_embedding_16384_lists_every_list_probed():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("embedding-like 1M x 768, 16,384 lists: generating")
    n, nlist = 1_000_000, 16384
    x, q = synth.embedding_like_gpu(n, 16, "cuda", seed_data=1004, seed_query=2404)
    cent, assign = R.rbq_kmeans(x, nlist, iters=6, sample=400_000, seed=5004)
    idx = R.Index(768, nlist, rot_precision=R.RBQ_ROT_BF16X3, seed=4004)
    idx.build(x, cent, assign, synth.gaussian_matrix(768, 3004))
    assign = assign.cpu().numpy()
    data = x.cpu().numpy()
    qs = q.cpu().numpy()
    codes, norm, ipo = R.rbq_debug_export_codes(idx.h, n, 12)
    exact = {qi: O.exact_topk(data, qs[qi], 10) for qi in range(3)}   # sampled: the first three queries
    for nq in (1, 3, 16):
        _say(f"{nq} queries probing all {nlist} lists")
        ids, d, st = idx.search(q[:nq].contiguous(), 10, nlist, stats=True)
        ids = ids.cpu().numpy()
        assert st["pairs"] == nq * nlist and st["codes_scanned"] == nq * n
        for qi in range(min(nq, 3)):
            t_ids, t_d = exact[qi]
            if tie_equivalent(ids[qi], t_ids, qs[qi], data):
                continue
            bits = unpack_codes(codes[t_ids], 768)
            fail = False
            lids = np.unique(assign[t_ids]).astype(np.int32)
            qu, scal = R.rbq_debug_quantize(idx.h, q[qi:qi + 1].contiguous(),
                                            torch.from_numpy(lids[None, :]).cuda(), 768, qid_base=qi)
            qu, scal = qu.cpu().numpy().astype(np.int64), scal.cpu().numpy()
            for j, (oid, dv) in enumerate(zip(t_ids, t_d)):
                r = int(np.flatnonzero(lids == assign[oid])[0])
                lbv = oracle_estimates_on(bits[j:j + 1], norm[oid:oid + 1], ipo[oid:oid + 1], qu[r],
                                          scal[r, 0], scal[r, 1], scal[r, 2], 768)[4][0]
                fail |= lbv > dv * (1 + 1e-6)
            assert fail, f"{nq} queries, query {qi}: differs from the exact top-10 without a bound failure"
    idx.close()
