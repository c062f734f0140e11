"""ctypes binding of include/rabitq.h: the same function names, argument
marshalling only. Device buffers are torch tensors on the GPU (PyTorch serves
as allocator and stream provider); every computation runs in librabitq.so.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librabitq.so")

RBQ_OK, RBQ_EINVAL, RBQ_ENOMEM, RBQ_EDEVICE, RBQ_ESTATE, RBQ_EFORMAT, RBQ_EUNSUPPORTED = range(7)
RBQ_ROT_FP32, RBQ_ROT_BF16X3 = 0, 1
RBQ_SCAN_AUTO, RBQ_SCAN_POPCNT, RBQ_SCAN_MFMA, RBQ_SCAN_MFMA_FP4 = 0, 1, 2, 3
RBQ_PROFILE_STAGES, RBQ_PROFILE_SCAN = 1, 2
MLP_IN, MLP_HIDDEN, MLP_OUT = 96, 128, 32
MAX_K, MAX_NPROBE, MAX_NLIST = 256, 16384, 24576
MLP_NPARAM = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_OUT + MLP_OUT


RBQ_METRIC_L2, RBQ_METRIC_IP, RBQ_METRIC_COSINE = 0, 1, 2


class RbqParams(C.Structure):
    _fields_ = [("dim", C.c_int32), ("code_bits", C.c_int32), ("nlist", C.c_int32),
                ("bq", C.c_int32), ("eps0", C.c_float), ("rot_precision", C.c_int32),
                ("seed", C.c_uint64), ("metric", C.c_int32)]


class RbqSearchOpts(C.Structure):
    _fields_ = [("k", C.c_int32), ("nprobe", C.c_int32), ("scan_kernel", C.c_int32),
                ("use_learned_nprobe", C.c_int32), ("nprobe_per_query", C.c_void_p),
                ("qid_base", C.c_int64), ("use_graph", C.c_int32), ("rerank_waves", C.c_int32)]


class RbqSearchStats(C.Structure):
    _fields_ = [("queries", C.c_int64), ("pairs", C.c_int64), ("codes_scanned", C.c_int64),
                ("reranked", C.c_int64), ("candidates", C.c_int64),
                ("reranked_bootstrap", C.c_int64), ("nonfinite_fallbacks", C.c_int64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class RbqIndexInfo(C.Structure):
    _fields_ = [("dim", C.c_int32), ("code_bits", C.c_int32), ("nlist", C.c_int32),
                ("rot_precision", C.c_int32), ("n", C.c_int64), ("device_bytes", C.c_int64),
                ("graph_captures", C.c_int64), ("graphs_cached", C.c_int64)]


class RbqProfile(C.Structure):
    _fields_ = [("searches", C.c_int64), ("ms_front", C.c_double), ("ms_prep", C.c_double),
                ("ms_scan0", C.c_double), ("ms_tau", C.c_double), ("ms_scan1", C.c_double),
                ("ms_finalize", C.c_double), ("codes_scan0", C.c_int64), ("codes_scan1", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class RbqTrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("seed", C.c_uint64)]


class RbqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rabitq status {status}: {msg}")
        self.status = status


_P = C.c_void_p
_SIGS = {
    "rbq_last_error": (C.c_char_p, []),
    "rbq_params_default": (C.c_int, [C.POINTER(RbqParams), C.c_int32, C.c_int32]),
    "rbq_index_create": (C.c_int, [C.POINTER(RbqParams), C.POINTER(_P)]),
    "rbq_index_build": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P, _P]),
    "rbq_index_build_rotation": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P, _P]),
    "rbq_search": (C.c_int, [_P, _P, C.c_int64, C.POINTER(RbqSearchOpts), _P, _P,
                             C.POINTER(RbqSearchStats), _P]),
    "rbq_index_set_eps0": (C.c_int, [_P, C.c_float]),
    "rbq_kmeans": (C.c_int, [_P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_uint64, _P, _P, _P,
                             _P]),
    "rbq_search_noalloc": (C.c_int, [_P, _P, C.c_int64, C.POINTER(RbqSearchOpts), _P, _P, _P]),
    "rbq_index_info_get": (C.c_int, [_P, C.POINTER(RbqIndexInfo)]),
    "rbq_index_list_sizes": (C.c_int, [_P, _P]),
    "rbq_index_save": (C.c_int, [_P, C.c_char_p]),
    "rbq_index_load": (C.c_int, [C.c_char_p, C.POINTER(_P)]),
    "rbq_index_destroy": (C.c_int, [_P]),
    "rbq_autotune": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.c_int32, _P]),
    "rbq_autotune_get": (C.c_int, [_P, C.c_int32, _P, _P]),
    "rbq_profile_enable": (C.c_int, [_P, C.c_int32]),
    "rbq_profile_read": (C.c_int, [_P, C.POINTER(RbqProfile)]),
    "rbq_nprobe_features": (C.c_int, [_P, _P, C.c_int64, C.c_int64, _P, _P]),
    "rbq_nprobe_model_train": (C.c_int, [_P, _P, _P, C.c_int64, C.POINTER(RbqTrainCfg), _P, _P]),
    "rbq_nprobe_model_set": (C.c_int, [_P, _P, C.c_float]),
    "rbq_nprobe_model_get": (C.c_int, [_P, _P, _P]),
    "rbq_nprobe_predict": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P]),
    "rbq_mlp_loss_grad": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P, _P]),
    "rbq_nprobe_bucket_table": (C.c_int, [_P]),
    "rbq_nprobe_labels": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int32, _P, _P, _P]),
    "rbq_debug_export_codes": (C.c_int, [_P, _P, _P, _P]),
    "rbq_debug_rotate": (C.c_int, [_P, _P, C.c_int64, _P, _P]),
    "rbq_debug_centroid_dists": (C.c_int, [_P, _P, C.c_int64, _P, _P]),
    "rbq_debug_probe": (C.c_int, [_P, _P, C.c_int64, C.c_int32, _P, _P, _P]),
    "rbq_debug_quantize": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int32, C.c_int64, _P, _P, _P]),
    "rbq_debug_scan": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int32, _P, _P, _P, _P, _P, _P]),
    "rbq_debug_list_ids": (C.c_int, [_P, C.c_int32, _P]),
    "rbq_debug_fail_alloc_after": (C.c_int, [C.c_int32]),
    "rbq_debug_seg_budget": (C.c_int, [C.c_int64]),
}

_lib = None


def lib():
    """The loaded librabitq.so. Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with python -m paper_2405_12497_amd.build")
        # torch ships its own HIP runtime under the same soname as the system's.
        # Loading torch first makes the library bind to that runtime; loaded the
        # other way round, the process would hold two HIP runtimes, and the one
        # initialised second finds no device.
        import torch  # noqa: F401
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def exported_symbols():
    return list(_SIGS)


def rbq_last_error() -> str:
    return lib().rbq_last_error().decode()


def _check(st):
    if st != RBQ_OK:
        raise RbqError(st, rbq_last_error())


# ----------------------------------------------------------------- marshalling helpers

def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _dev(t, dtype=None):
    """Pointer of a contiguous GPU tensor (or None)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    """A HIP stream handle: an int, a torch.cuda.Stream, or None (torch's current stream)."""
    if stream is not None:
        return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ----------------------------------------------------------------- API (same names as the C ABI)

def rbq_params_default(dim: int, nlist: int) -> RbqParams:
    p = RbqParams()
    _check(lib().rbq_params_default(C.byref(p), dim, nlist))
    return p


def rbq_index_create(params: RbqParams):
    h = C.c_void_p()
    _check(lib().rbq_index_create(C.byref(params), C.byref(h)))
    return h


def _any(a, np_dtype):
    """(keep-alive object, pointer) of a numpy array (host) or a contiguous GPU tensor."""
    if hasattr(a, "is_cuda") and a.is_cuda:
        import torch
        want = {np.float32: torch.float32, np.int32: torch.int32, np.float64: torch.float64,
                np.int64: torch.int64}[np_dtype]
        return a, _dev(a, want)
    return _host(a, np_dtype)


def rbq_index_build(idx, data, centroids, assign, gauss=None, stream=None):
    """data, centroids, assign, gauss: numpy arrays (host) or GPU tensors, independently."""
    d, dp = _any(data, np.float32)
    c, cp = _any(centroids, np.float32)
    a, ap = _any(assign, np.int32)
    gp = None
    if gauss is not None:
        g, gp = _any(gauss, np.float64)
    _check(lib().rbq_index_build(idx, dp, d.shape[0], cp, ap, gp, _stream(stream)))


def rbq_index_build_rotation(idx, data, centroids, assign, P, stream=None):
    """As rbq_index_build with a caller-supplied orthogonal P [code_bits x code_bits] float64."""
    d, dp = _any(data, np.float32)
    c, cp = _any(centroids, np.float32)
    a, ap = _any(assign, np.int32)
    p, pp = _any(P, np.float64)
    _check(lib().rbq_index_build_rotation(idx, dp, d.shape[0], cp, ap, pp, _stream(stream)))


def rbq_search(idx, queries, k, nprobe, scan_kernel=RBQ_SCAN_AUTO, use_learned_nprobe=False,
               nprobe_per_query=None, qid_base=0, stats=False, out_ids=None, out_dists=None,
               stream=None, use_graph=False, rerank_waves=0):
    """queries: float32 GPU tensor [nq, dim] (outputs are GPU tensors), or a numpy
    array (host pointers through the C ABI; outputs are numpy arrays).
    Returns (ids int64 [nq,k], dists float32 [nq,k], stats|None)."""
    if not hasattr(queries, "is_cuda"):
        q, qp = _host(queries, np.float32)
        nq = q.shape[0]
        ids = np.empty((nq, k), np.int64)
        ds = np.empty((nq, k), np.float32)
        npq = None
        if nprobe_per_query is not None:
            npq, _ = _host(nprobe_per_query, np.int32)
        o = RbqSearchOpts(k, nprobe, scan_kernel, int(bool(use_learned_nprobe)),
                          None if npq is None else npq.ctypes.data, qid_base, int(bool(use_graph)),
                          int(rerank_waves))
        st = RbqSearchStats()
        _check(lib().rbq_search(idx, qp, nq, C.byref(o), ids.ctypes.data_as(C.c_void_p),
                                ds.ctypes.data_as(C.c_void_p), C.byref(st) if stats else None,
                                _stream(stream)))
        return ids, ds, (st.as_dict() if stats else None)
    import torch
    nq = queries.shape[0]
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int64, device=queries.device)
    if out_dists is None:
        out_dists = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    o = RbqSearchOpts(k, nprobe, scan_kernel, int(bool(use_learned_nprobe)),
                      _dev(nprobe_per_query, torch.int32), qid_base, int(bool(use_graph)), int(rerank_waves))
    st = RbqSearchStats()
    _check(lib().rbq_search(idx, _dev(queries, torch.float32), nq, C.byref(o),
                            _dev(out_ids, torch.int64), _dev(out_dists, torch.float32),
                            C.byref(st) if stats else None, _stream(stream)))
    return out_ids, out_dists, (st.as_dict() if stats else None)


def rbq_kmeans(data, nlist, iters=10, sample=0, seed=0, init=None, stream=None):
    """data: numpy [n, dim] or a GPU tensor. Returns (centroids, assign) as numpy
    arrays for numpy data, GPU tensors for GPU data."""
    n, dim = data.shape
    d, dp = _any(data, np.float32)
    ip = None
    if init is not None:
        i_, ip = _any(init, np.float32)
    if hasattr(data, "is_cuda") and data.is_cuda:
        import torch
        cent = torch.empty((nlist, dim), dtype=torch.float32, device=data.device)
        asg = torch.empty(n, dtype=torch.int32, device=data.device)
        cp, ap = _dev(cent, torch.float32), _dev(asg, torch.int32)
    else:
        cent = np.empty((nlist, dim), np.float32)
        asg = np.empty(n, np.int32)
        cp, ap = cent.ctypes.data_as(C.c_void_p), asg.ctypes.data_as(C.c_void_p)
    _check(lib().rbq_kmeans(dp, n, dim, nlist, iters, sample, seed, ip, cp, ap, _stream(stream)))
    return cent, asg


def rbq_index_set_eps0(idx, eps0):
    _check(lib().rbq_index_set_eps0(idx, float(eps0)))


NOALLOC_SCRATCH_BYTES = 128 << 20


def rbq_search_noalloc(idx, queries, k, nprobe, scan_kernel=RBQ_SCAN_AUTO, use_learned_nprobe=False,
                       nprobe_per_query=None, qid_base=0, out_ids=None, out_dists=None, stream=None,
                       rerank_waves=0):
    """rbq_search_noalloc on GPU tensors; out_ids/out_dists (GPU, caller-owned) are
    allocated here by torch when not given. Returns (ids, dists)."""
    import torch
    nq = queries.shape[0]
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int64, device=queries.device)
    if out_dists is None:
        out_dists = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    o = RbqSearchOpts(k, nprobe, scan_kernel, int(bool(use_learned_nprobe)),
                      _dev(nprobe_per_query, torch.int32), qid_base, 0, int(rerank_waves))
    _check(lib().rbq_search_noalloc(idx, _dev(queries, torch.float32), nq, C.byref(o),
                                    _dev(out_ids, torch.int64), _dev(out_dists, torch.float32),
                                    _stream(stream)))
    return out_ids, out_dists


def rbq_index_info_get(idx) -> dict:
    i = RbqIndexInfo()
    _check(lib().rbq_index_info_get(idx, C.byref(i)))
    return {f: int(getattr(i, f)) for f, _ in i._fields_}


def rbq_index_list_sizes(idx, nlist) -> np.ndarray:
    out = np.zeros(nlist, dtype=np.int64)
    _check(lib().rbq_index_list_sizes(idx, out.ctypes.data_as(C.c_void_p)))
    return out


def rbq_index_save(idx, path: str):
    _check(lib().rbq_index_save(idx, path.encode()))


def rbq_index_load(path: str):
    h = C.c_void_p()
    _check(lib().rbq_index_load(path.encode(), C.byref(h)))
    return h


def rbq_index_destroy(idx):
    _check(lib().rbq_index_destroy(idx))


class RbqTuneEntry(C.Structure):
    _fields_ = [("max_nq", C.c_int64), ("chunk", C.c_int32), ("scan_kernel", C.c_int32),
                ("rerank_waves", C.c_int32), ("ms", C.c_float), ("mfma_row_groups", C.c_int32)]


def rbq_autotune(idx, queries, k, nprobe, stream=None):
    """queries: numpy (host) or a GPU tensor [nq, dim]."""
    q, qp = _any(queries, np.float32)
    _check(lib().rbq_autotune(idx, qp, q.shape[0], k, nprobe, _stream(stream)))


def rbq_autotune_get(idx):
    n = C.c_int32()
    _check(lib().rbq_autotune_get(idx, 0, None, C.byref(n)))
    arr = (RbqTuneEntry * max(1, n.value))()
    _check(lib().rbq_autotune_get(idx, n.value, arr, C.byref(n)))
    return [{f: getattr(arr[i], f) for f, _ in RbqTuneEntry._fields_} for i in range(n.value)]


def rbq_profile_enable(idx, on=True):
    """on: False/0 off, True/RBQ_PROFILE_STAGES all stages, RBQ_PROFILE_SCAN main scan and rerank only."""
    _check(lib().rbq_profile_enable(idx, int(on)))


def rbq_profile_read(idx) -> dict:
    p = RbqProfile()
    _check(lib().rbq_profile_read(idx, C.byref(p)))
    return p.as_dict()


def rbq_nprobe_features(idx, queries, qid_base=0, feats=None, stream=None):
    import torch
    nq = queries.shape[0]
    if feats is None:
        feats = torch.empty((nq, MLP_IN), dtype=torch.float32, device=queries.device)
    _check(lib().rbq_nprobe_features(idx, _dev(queries, torch.float32), nq, qid_base,
                                     _dev(feats, torch.float32), _stream(stream)))
    return feats


def rbq_nprobe_model_train(idx, feats, labels, epochs=5, batch=4096, lr=1e-3, beta1=0.9,
                           beta2=0.999, eps=1e-8, seed=0, stream=None):
    import torch
    cfg = RbqTrainCfg(epochs, batch, lr, beta1, beta2, eps, seed)
    losses = np.zeros(epochs, dtype=np.float32)
    _check(lib().rbq_nprobe_model_train(idx, _dev(feats, torch.float32), _dev(labels, torch.int32),
                                        feats.shape[0], C.byref(cfg),
                                        losses.ctypes.data_as(C.c_void_p), _stream(stream)))
    return losses


def rbq_nprobe_model_set(idx, weights, threshold):
    if weights is None:
        _check(lib().rbq_nprobe_model_set(idx, None, threshold))
        return
    w, wp = _host(weights, np.float32)
    if w.size != MLP_NPARAM:
        raise ValueError(f"expected {MLP_NPARAM} weights")
    _check(lib().rbq_nprobe_model_set(idx, wp, threshold))


def rbq_nprobe_model_get(idx):
    w = np.zeros(MLP_NPARAM, dtype=np.float32)
    t = np.zeros(1, dtype=np.float32)
    _check(lib().rbq_nprobe_model_get(idx, w.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p)))
    return w, float(t[0])


def rbq_nprobe_predict(idx, feats, want_logits=False, stream=None):
    import torch
    nq = feats.shape[0]
    npq = torch.empty(nq, dtype=torch.int32, device=feats.device)
    logits = torch.empty((nq, MLP_OUT), dtype=torch.float32, device=feats.device) if want_logits else None
    _check(lib().rbq_nprobe_predict(idx, _dev(feats, torch.float32), nq, _dev(npq, torch.int32),
                                    _dev(logits, torch.float32), _stream(stream)))
    return npq, logits


def rbq_mlp_loss_grad(x, labels, weights, stream=None):
    import torch
    grads = torch.empty_like(weights)
    loss = np.zeros(1, dtype=np.float32)
    _check(lib().rbq_mlp_loss_grad(_dev(x, torch.float32), _dev(labels, torch.int32), x.shape[0],
                                   _dev(weights, torch.float32), _dev(grads, torch.float32),
                                   loss.ctypes.data_as(C.c_void_p), _stream(stream)))
    return float(loss[0]), grads


def rbq_nprobe_bucket_table():
    out = np.zeros(MLP_OUT, dtype=np.int32)
    _check(lib().rbq_nprobe_bucket_table(out.ctypes.data_as(C.c_void_p)))
    return out


def rbq_nprobe_labels(idx, queries, nn_ids, stream=None):
    """queries GPU float32 [nq, dim], nn_ids GPU int64 [nq, k] -> (labels int32 [nq], need int32 [nq])."""
    import torch
    nq, k = nn_ids.shape
    labels = torch.empty(nq, dtype=torch.int32, device=queries.device)
    need = torch.empty(nq, dtype=torch.int32, device=queries.device)
    _check(lib().rbq_nprobe_labels(idx, _dev(queries, torch.float32), nq, _dev(nn_ids, torch.int64), k,
                                   _dev(labels, torch.int32), _dev(need, torch.int32), _stream(stream)))
    return labels, need


def rbq_debug_export_codes(idx, n, words):
    codes = np.zeros((n, words), dtype=np.uint64)
    norm = np.zeros(n, dtype=np.float32)
    ipo = np.zeros(n, dtype=np.float32)
    _check(lib().rbq_debug_export_codes(idx, codes.ctypes.data_as(C.c_void_p),
                                        norm.ctypes.data_as(C.c_void_p), ipo.ctypes.data_as(C.c_void_p)))
    return codes, norm, ipo


def rbq_debug_rotate(idx, queries, code_bits, stream=None):
    import torch
    out = torch.empty((queries.shape[0], code_bits), dtype=torch.float32, device=queries.device)
    _check(lib().rbq_debug_rotate(idx, _dev(queries, torch.float32), queries.shape[0],
                                  _dev(out, torch.float32), _stream(stream)))
    return out


def rbq_debug_centroid_dists(idx, queries, nlist, stream=None):
    import torch
    nq = queries.shape[0]
    dists = torch.empty((nq, nlist), dtype=torch.float32, device=queries.device)
    _check(lib().rbq_debug_centroid_dists(idx, _dev(queries, torch.float32), nq, _dev(dists, torch.float32),
                                          _stream(stream)))
    return dists


def rbq_debug_probe(idx, queries, nprobe, stream=None):
    import torch
    nq = queries.shape[0]
    lists = torch.empty((nq, nprobe), dtype=torch.int32, device=queries.device)
    dists = torch.empty((nq, nprobe), dtype=torch.float32, device=queries.device)
    _check(lib().rbq_debug_probe(idx, _dev(queries, torch.float32), nq, nprobe,
                                 _dev(lists, torch.int32), _dev(dists, torch.float32), _stream(stream)))
    return lists, dists


def rbq_debug_quantize(idx, queries, lists, code_bits, qid_base=0, stream=None):
    import torch
    nq, nprobe = lists.shape
    qu = torch.empty((nq * nprobe, code_bits), dtype=torch.uint8, device=queries.device)
    scal = torch.empty((nq * nprobe, 4), dtype=torch.float32, device=queries.device)
    _check(lib().rbq_debug_quantize(idx, _dev(queries, torch.float32), nq, _dev(lists, torch.int32),
                                    nprobe, qid_base, _dev(qu, torch.uint8), _dev(scal, torch.float32),
                                    _stream(stream)))
    return qu, scal


def rbq_debug_scan(idx, list_id, qu, b, vl, delta, n, kernel=RBQ_SCAN_POPCNT, stream=None, pair_term=0.0):
    import torch
    dev = qu.device
    ip = torch.empty(n, dtype=torch.int32, device=dev)
    pc = torch.empty(n, dtype=torch.int32, device=dev)
    est = torch.empty(n, dtype=torch.float32, device=dev)
    dist = torch.empty(n, dtype=torch.float32, device=dev)
    lb = torch.empty(n, dtype=torch.float32, device=dev)
    scal = np.array([b, vl, delta, pair_term], dtype=np.float32)
    _check(lib().rbq_debug_scan(idx, list_id, _dev(qu, torch.uint8), scal.ctypes.data_as(C.c_void_p),
                                kernel, _dev(ip), _dev(pc), _dev(est), _dev(dist), _dev(lb),
                                _stream(stream)))
    return ip, pc, est, dist, lb


def rbq_debug_list_ids(idx, list_id, size):
    out = np.zeros(size, dtype=np.int64)
    _check(lib().rbq_debug_list_ids(idx, list_id, out.ctypes.data_as(C.c_void_p)))
    return out


def rbq_debug_seg_budget(nbytes: int):
    _check(lib().rbq_debug_seg_budget(int(nbytes)))


def rbq_debug_fail_alloc_after(n: int):
    _check(lib().rbq_debug_fail_alloc_after(n))


# ----------------------------------------------------------------- convenience wrapper

class Index:
    """Owns an rbq_index handle."""

    def __init__(self, dim, nlist, code_bits=0, eps0=1.9, rot_precision=RBQ_ROT_FP32, seed=0,
                 handle=None, bq=4, metric=RBQ_METRIC_L2):
        if handle is not None:
            self.h = handle
        else:
            p = rbq_params_default(dim, nlist)
            p.code_bits = code_bits
            p.bq = bq
            p.metric = metric
            p.eps0 = eps0
            p.rot_precision = rot_precision
            p.seed = seed
            self.h = rbq_index_create(p)
        info = rbq_index_info_get(self.h)
        self.dim, self.code_bits, self.nlist = info["dim"], info["code_bits"], info["nlist"]

    @classmethod
    def load(cls, path):
        return cls(0, 0, handle=rbq_index_load(path))

    def build(self, data, centroids, assign, gauss=None):
        rbq_index_build(self.h, data, centroids, assign, gauss)
        return self

    def build_rotation(self, data, centroids, assign, P):
        rbq_index_build_rotation(self.h, data, centroids, assign, P)
        return self

    def search(self, queries, k, nprobe, **kw):
        return rbq_search(self.h, queries, k, nprobe, **kw)

    def info(self):
        return rbq_index_info_get(self.h)

    def list_sizes(self):
        return rbq_index_list_sizes(self.h, self.nlist)

    def save(self, path):
        rbq_index_save(self.h, path)

    def close(self):
        if self.h:
            rbq_index_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
