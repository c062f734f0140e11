"""Learned per-query nprobe on the GPU against the FP64 reference (oracle/mlp_oracle.py).

Tolerances: forward logits within 1e-2 relative (BF16 operands, FP32
accumulation, hidden activations rounded to BF16 on the GPU only); gradients
within 2e-2 relative norm per parameter block, both against FP64 evaluated on
the same BF16-rounded weights and inputs.
"""
import sys

import numpy as np
import pytest

from oracle import mlp_oracle as M
from oracle import rabitq_oracle as O

from gpu_common import Built, make_case

pytestmark = pytest.mark.gpu
_B = {}


def _say(msg):
    print(f"[{msg}]", flush=True)
    sys.stdout.flush()


def _built(name):
    if name not in _B:
        _B[name] = Built(make_case(name))
    return _B[name]


def bf16_round(x):
    """Round-to-nearest-even to BF16, returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _params(seed, scale=0.15):
    return np.random.default_rng(seed).normal(0, scale, M.N_IN * M.N_HID + M.N_HID + M.N_HID * M.N_OUT + M.N_OUT)


def test_features_match_reference():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("features")
    b = _built("ivf128")
    c = b.case
    f = R.rbq_nprobe_features(b.idx.h, b.q, qid_base=0).cpu().numpy().astype(np.float64)
    for qi, q in enumerate(c.queries):
        want = M.features(b.oidx, q, qi, c.seed)
        np.testing.assert_allclose(f[qi, :64], want[:64], atol=2e-4, rtol=1e-5)
        np.testing.assert_allclose(f[qi, 64::4], want[64::4], rtol=1e-5)       # b ratios
        np.testing.assert_allclose(f[qi, 65::4], want[65::4], rtol=1e-4, atol=1e-6)   # v_l
        np.testing.assert_allclose(f[qi, 66::4], want[66::4], rtol=1e-4, atol=1e-6)   # v_r
        # expected S_q fraction: a mean of dp terms, FP32 on the GPU
        np.testing.assert_allclose(f[qi, 67::4], want[67::4], rtol=1e-4, atol=1e-5)


def test_forward_logits_match_reference():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("forward")
    b = _built("ivf128")
    w = _params(1).astype(np.float32)
    R.rbq_nprobe_model_set(b.idx.h, w, 0.9)
    x = np.random.default_rng(2).normal(0, 1, (300, 96)).astype(np.float32)
    _, logits = R.rbq_nprobe_predict(b.idx.h, torch.from_numpy(x).cuda(), want_logits=True)
    got = logits.cpu().numpy().astype(np.float64)
    W1, b1, W2, b2 = M.split_params(w)
    wr = M.join_params(bf16_round(W1), b1.astype(np.float32), bf16_round(W2), b2.astype(np.float32))
    _, h, want = M.forward(bf16_round(x), wr)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"forward relative error {err:.2e}")
    assert err < 1e-2
    # per logit: the GPU rounds the hidden activations to BF16 (relative 2^-9)
    # before the second product, so each logit may differ by 1e-2 of the size
    # of its terms, sum_j |h_j W2_jk| + |b2_k| (FP32 accumulation adds far less)
    W2r = M.split_params(wr)[2]
    scale = np.abs(h) @ np.abs(W2r) + np.abs(M.split_params(wr)[3])[None, :]
    bad = np.abs(got - want) > 1e-2 * scale
    print(f"per-logit max |err| / term size {np.max(np.abs(got - want) / scale):.2e}")
    assert not bad.any(), f"{bad.sum()} logits outside 1e-2 of their term size"
    R.rbq_nprobe_model_set(b.idx.h, None, 0.9)


def test_fused_inference_equals_separate_forward():
    """The search's fused features + MLP + policy launch picks, per query, the
    nprobe that rbq_nprobe_predict picks from rbq_nprobe_features (same BF16
    operands, same MFMA order), and the search equals a per-query-nprobe search."""
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("fused inference")
    b = _built("ivf128")
    c = b.case
    w = _params(11, 0.2).astype(np.float32)
    for thr in (0.3, 0.7, 0.95):
        R.rbq_nprobe_model_set(b.idx.h, w, thr)
        feats = R.rbq_nprobe_features(b.idx.h, b.q, qid_base=0)
        npq, _ = R.rbq_nprobe_predict(b.idx.h, feats)
        cap = 40
        npq = torch.clamp(npq, max=cap)
        ids, d, st = b.idx.search(b.q, 10, cap, use_learned_nprobe=True, stats=True)
        ids2, d2, st2 = b.idx.search(b.q, 10, cap, nprobe_per_query=npq, stats=True)
        assert st["pairs"] == st2["pairs"] == int(npq.sum().item())
        assert st["nonfinite_fallbacks"] == 0
        np.testing.assert_array_equal(ids.cpu().numpy(), ids2.cpu().numpy())
        np.testing.assert_array_equal(d.cpu().numpy(), d2.cpu().numpy())
    R.rbq_nprobe_model_set(b.idx.h, None, 0.9)


def test_nonfinite_logits_fall_back_to_fixed_nprobe():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("non-finite fallback")
    b = _built("ivf128")
    c = b.case
    # finite weights whose products overflow FP32: every logit is +-inf or NaN
    w = np.full(M.N_IN * M.N_HID + M.N_HID + M.N_HID * M.N_OUT + M.N_OUT, 3e38, np.float32)
    R.rbq_nprobe_model_set(b.idx.h, w, 0.9)
    ids, d, st = b.idx.search(b.q, 10, 8, use_learned_nprobe=True, stats=True)
    assert st["nonfinite_fallbacks"] == len(c.queries)
    assert st["pairs"] == 8 * len(c.queries)
    ids2, _, _ = b.idx.search(b.q, 10, 8)
    np.testing.assert_array_equal(ids.cpu().numpy(), ids2.cpu().numpy())
    feats = R.rbq_nprobe_features(b.idx.h, b.q)
    npq, _ = R.rbq_nprobe_predict(b.idx.h, feats)
    assert np.all(npq.cpu().numpy() == 64)            # min(nlist, 512) for this index
    R.rbq_nprobe_model_set(b.idx.h, None, 0.9)


def _gt_gpu(x, q, k):
    """Exact top-k ids by squared L2 (FP32 shortlist of 4k, FP64 recheck)."""
    import torch
    xn = (x.double() ** 2).sum(1).float()
    d = xn[None, :] - 2.0 * (q @ x.T)
    cand = torch.topk(d, 4 * k, dim=1, largest=False).indices
    ex = ((x[cand].double() - q[:, None, :].double()) ** 2).sum(-1)
    o = torch.argsort(ex, dim=1, stable=True)[:, :k]
    return torch.gather(cand, 1, o), torch.gather(ex, 1, o)


def _recall(ids, gt_d, x, q, k):
    import torch
    rows = x[ids.clamp(min=0)]
    d = ((rows.double() - q[:, None, :].double()) ** 2).sum(-1)
    hit = (ids >= 0) & (d <= gt_d[:, k - 1:k] * (1 + 1e-6))
    return hit.double().mean().item()


def test_learned_nprobe_beats_fixed_at_equal_recall():
    """Train on labels from the method's own probe order (rbq_nprobe_labels on
    exact neighbours), calibrate the policy threshold and the fixed nprobe on
    validation queries to recall@10 >= 0.95, and compare on test queries: the
    learned search scans fewer codes at no lower recall."""
    import torch
    import synth
    from paper_2405_12497_amd import rabitq as R
    _say("learned vs fixed")
    k, dim, nlist = 10, 128, 512
    data, qs = synth.embedding_like(120_000, 60_000, dim=dim, seed_data=301, seed_query=302)
    cent, assign = synth.kmeans(data, nlist, iters=6, seed=303)
    idx = R.Index(dim, nlist, seed=304)
    idx.build(data, cent, assign, synth.gaussian_matrix(dim, 305))
    x = torch.from_numpy(data).cuda()
    q = torch.from_numpy(qs).cuda()
    tr, va, te = q[:40_000], q[40_000:50_000], q[50_000:]
    gt_i, gt_d = zip(*[_gt_gpu(x, q[s:s + 2000], k) for s in range(0, len(q), 2000)])
    gt_i, gt_d = torch.cat(gt_i), torch.cat(gt_d)
    labels, need = R.rbq_nprobe_labels(idx.h, tr, gt_i[:40_000].contiguous())
    feats = R.rbq_nprobe_features(idx.h, tr, qid_base=0)
    losses = R.rbq_nprobe_model_train(idx.h, feats, labels, epochs=8, batch=1024, lr=2e-3, seed=3)
    print(f"losses {np.round(losses, 3)}; mean need {need.float().mean().item():.1f}")
    w, _ = R.rbq_nprobe_model_get(idx.h)
    gva, gte = gt_d[40_000:50_000], gt_d[50_000:]
    cap = 512

    def learned(qq, thr):
        R.rbq_nprobe_model_set(idx.h, w, thr)
        ids, _, st = idx.search(qq, k, cap, use_learned_nprobe=True, stats=True)
        return ids, st

    lo, hi = 0.2, 0.9995
    for _ in range(14):
        mid = 0.5 * (lo + hi)
        ids, _ = learned(va, mid)
        if _recall(ids, gva, x, va, k) >= 0.95:
            hi = mid
        else:
            lo = mid
    plo, phi = 1, cap
    while plo < phi:
        mid = (plo + phi) // 2
        ids, _, _ = idx.search(va, k, mid)
        if _recall(ids, gva, x, va, k) >= 0.95:
            phi = mid
        else:
            plo = mid + 1
    ids_l, st_l = learned(te, hi)
    rc_l = _recall(ids_l, gte, x, te, k)
    R.rbq_nprobe_model_set(idx.h, None, 0.9)
    ids_f, _, st_f = idx.search(te, k, phi, stats=True)
    rc_f = _recall(ids_f, gte, x, te, k)
    cl, cf = st_l["codes_scanned"] / len(te), st_f["codes_scanned"] / len(te)
    print(f"learned: threshold {hi:.4f} recall {rc_l:.4f} codes/query {cl:.0f} mean nprobe "
          f"{st_l['pairs'] / len(te):.1f}; fixed: nprobe {phi} recall {rc_f:.4f} codes/query {cf:.0f}")
    assert rc_l >= rc_f - 0.004
    assert cl < cf
    idx.close()


def test_gradients_match_reference():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("gradients")
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1, (1000, 96)).astype(np.float32)
    y = rng.integers(0, 32, 1000).astype(np.int32)
    w = _params(4).astype(np.float32)
    loss, g = R.rbq_mlp_loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(),
                                  torch.from_numpy(w).cuda())
    g = g.cpu().numpy().astype(np.float64)
    W1, b1, W2, b2 = M.split_params(w)
    wr = M.join_params(bf16_round(W1), b1.astype(np.float32), bf16_round(W2), b2.astype(np.float32))
    oloss, og = M.loss_and_grad(bf16_round(x), y, wr)
    assert loss == pytest.approx(oloss, rel=1e-2)
    for name, gg, oo in zip(("W1", "b1", "W2", "b2"), M.split_params(g), M.split_params(og)):
        rel = np.linalg.norm(gg - oo) / np.linalg.norm(oo)
        print(f"grad {name}: relative norm error {rel:.2e}")
        assert rel < 2e-2, name


def test_training_fits_a_teacher():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("training")
    b = _built("ivf128")
    rng = np.random.default_rng(5)
    x = rng.normal(0, 1, (20000, 96)).astype(np.float32)
    teacher = _params(6, 0.3)
    y = np.argmax(M.forward(x, teacher)[2], 1).astype(np.int32)
    losses = R.rbq_nprobe_model_train(b.idx.h, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(),
                                      epochs=6, batch=1024, lr=3e-3, seed=7)
    print(f"training losses {losses}")
    assert losses[-1] < 0.5 * losses[0]
    w, thr = R.rbq_nprobe_model_get(b.idx.h)
    acc = np.mean(np.argmax(M.forward(x[:4000], w.astype(np.float64))[2], 1) == y[:4000])
    print(f"teacher accuracy {acc:.3f}")
    assert acc > 0.5
    R.rbq_nprobe_model_set(b.idx.h, None, 0.9)


def test_policy_buckets_and_learned_search():
    import torch
    from paper_2405_12497_amd import rabitq as R
    _say("policy and learned search")
    b = _built("ivf128")
    c = b.case
    table = M.bucket_table()
    for j in (0, 1, 3, 31):
        w = np.zeros(M.N_IN * M.N_HID + M.N_HID + M.N_HID * M.N_OUT + M.N_OUT, np.float32)
        w[-32 + j] = 40.0             # b2[j]: the softmax puts all mass on bucket j
        R.rbq_nprobe_model_set(b.idx.h, w, 0.9)
        feats = R.rbq_nprobe_features(b.idx.h, b.q)
        npq, _ = R.rbq_nprobe_predict(b.idx.h, feats)
        want = min(int(table[j]), 64)
        assert np.all(npq.cpu().numpy() == want)
        cap = 16
        ids, d, st = b.idx.search(b.q, 10, cap, use_learned_nprobe=True, stats=True)
        eff = min(want, cap)
        ids2, d2, st2 = b.idx.search(b.q, 10, eff, stats=True)
        assert st["pairs"] == len(c.queries) * eff
        np.testing.assert_array_equal(ids.cpu().numpy(), ids2.cpu().numpy())
    # no model: the fixed nprobe is used
    R.rbq_nprobe_model_set(b.idx.h, None, 0.9)
    ids, _, st = b.idx.search(b.q, 10, 8, use_learned_nprobe=True, stats=True)
    assert st["pairs"] == len(c.queries) * 8
