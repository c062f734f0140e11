"""Shared helpers for the GPU parity tests: small seeded workloads, a GPU index
built through the C ABI, and the FP64 oracle evaluated on the same inputs."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from oracle import rabitq_oracle as O
import synth


@dataclass
class Case:
    name: str
    data: np.ndarray
    queries: np.ndarray
    cent: np.ndarray
    assign: np.ndarray
    gauss: np.ndarray
    k: int
    nprobe: int
    rot: int
    seed: int
    code_bits: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def dim(self):
        return self.data.shape[1]

    @property
    def dp(self):
        return self.gauss.shape[0]


def make_case(name: str) -> Case:
    from paper_2405_12497_amd import rabitq as R
    if name == "flat128":
        data, qs = synth.mixture_flat(3000, 16, seed_data=101, seed_query=102)
        cent = data.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
        assign = np.zeros(len(data), np.int32)
        return Case(name, data, qs, cent, assign, synth.gaussian_matrix(128, 103), 10, 1,
                    R.RBQ_ROT_FP32, 4101)
    if name == "ivf128":
        data, qs = synth.sift_like(20000, 24, seed_data=111, seed_query=112)
        cent, assign = synth.kmeans(data, 64, iters=5, seed=113)
        return Case(name, data, qs, cent, assign, synth.gaussian_matrix(128, 114), 10, 8,
                    R.RBQ_ROT_FP32, 4102)
    if name == "pad100":
        data, qs = synth.mixture_flat(2500, 12, dim=100, seed_data=121, seed_query=122)
        cent, assign = synth.kmeans(data, 4, iters=5, seed=123)
        return Case(name, data, qs, cent, assign, synth.gaussian_matrix(128, 124), 10, 2,
                    R.RBQ_ROT_FP32, 4103)
    if name == "ivf960z":
        data, qs, means = synth.gist_like(8000, 8, ncomp=48, seed_data=131, seed_query=132)
        cent, assign = synth.kmeans(data, 48, iters=4, init=means)
        return Case(name, data, qs, cent, assign, synth.gaussian_matrix(960, 133), 100, 6,
                    R.RBQ_ROT_BF16X3, 4104)
    if name == "ivf768":
        data, qs = synth.embedding_like(6000, 10, seed_data=141, seed_query=142)
        cent, assign = synth.kmeans(data, 32, iters=4, seed=143)
        return Case(name, data, qs, cent, assign, synth.gaussian_matrix(768, 144), 10, 4,
                    R.RBQ_ROT_BF16X3, 4105)
    if name == "many2500":
        # many small lists and nprobe above 2048 (the large probe selection)
        data, qs = synth.mixture_flat(12000, 12, dim=64, seed_data=151, seed_query=152)
        rng = np.random.default_rng(153)
        cent = data[rng.choice(len(data), 3000, replace=False)].copy()
        x, c = data.astype(np.float64), cent.astype(np.float64)
        d = (x * x).sum(1)[:, None] + (c * c).sum(1)[None, :] - 2.0 * (x @ c.T)
        assign = np.argmin(d, 1).astype(np.int32)
        return Case(name, data, qs, cent, assign, synth.gaussian_matrix(64, 154), 10, 2500,
                    R.RBQ_ROT_FP32, 4106)
    if name == "ivf192":
        # W = 3 words per code (the quarter-wave quantisation's odd width)
        data, qs = synth.mixture_flat(5000, 12, dim=192, seed_data=161, seed_query=162)
        cent, assign = synth.kmeans(data, 24, iters=4, seed=163)
        return Case(name, data, qs, cent, assign, synth.gaussian_matrix(192, 164), 10, 5,
                    R.RBQ_ROT_FP32, 4107)
    if name == "ivf256":
        # W = 4 words per code, split-BF16 rotation
        data, qs = synth.mixture_flat(5000, 12, dim=256, seed_data=171, seed_query=172)
        cent, assign = synth.kmeans(data, 24, iters=4, seed=173)
        return Case(name, data, qs, cent, assign, synth.gaussian_matrix(256, 174), 10, 5,
                    R.RBQ_ROT_BF16X3, 4108)
    if name == "ivf512":
        # W = 8 words per code: the two-pairs-per-wave quantisation and the runtime-width scan
        data, qs = synth.mixture_flat(4000, 10, dim=512, seed_data=181, seed_query=182)
        cent, assign = synth.kmeans(data, 16, iters=4, seed=183)
        return Case(name, data, qs, cent, assign, synth.gaussian_matrix(512, 184), 10, 4,
                    R.RBQ_ROT_BF16X3, 4109)
    if name == "cb2048":
        # code length 2048 for D = 160 (W = 32, padded far beyond D; planes in LDS)
        data, qs = synth.mixture_flat(2500, 8, dim=160, seed_data=191, seed_query=192)
        cent, assign = synth.kmeans(data, 8, iters=4, seed=193)
        return Case(name, data, qs, cent, assign, synth.gaussian_matrix(2048, 194), 10, 3,
                    R.RBQ_ROT_FP32, 4110, code_bits=2048)
    raise KeyError(name)


class Built:
    """GPU index + oracle index for a Case."""

    def __init__(self, case: Case):
        import torch
        from paper_2405_12497_amd import rabitq as R
        self.R = R
        self.case = case
        self.dev = torch.device("cuda:0")
        self.idx = R.Index(case.dim, case.cent.shape[0], code_bits=case.code_bits,
                           rot_precision=case.rot, seed=case.seed)
        self.idx.build(case.data, case.cent, case.assign, case.gauss)
        self.oidx = O.build_index(case.data, case.cent, case.assign, case.gauss)
        self.W = case.dp // 64
        codes, self.norm, self.ipo = R.rbq_debug_export_codes(self.idx.h, len(case.data), self.W)
        self.bits = unpack_codes(codes, case.dp)
        self.q = torch.from_numpy(np.ascontiguousarray(case.queries)).to(self.dev)

    def probe(self, nprobe=None):
        lists, d = self.R.rbq_debug_probe(self.idx.h, self.q, nprobe or self.case.nprobe)
        return lists.cpu().numpy(), d.cpu().numpy()

    def search(self, k=None, nprobe=None, **kw):
        ids, d, st = self.idx.search(self.q, k or self.case.k, nprobe or self.case.nprobe, **kw)
        return ids.cpu().numpy(), d.cpu().numpy(), st


def unpack_codes(codes: np.ndarray, dp: int) -> np.ndarray:
    """uint64 words (bit i%64 of word i/64 = coordinate i) -> [n, dp] uint8 bits."""
    b = np.unpackbits(codes.view(np.uint8), axis=1, bitorder="little")
    return b[:, :dp].astype(np.uint8)


def oracle_estimates_on(bits, norm, ipo, qu, b, vl, delta, dp, eps0=O.EPS0):
    """The oracle's Sec. 3.3.2 / Theorem 3.2 / Eq. (2) arithmetic in FP64 on
    given codes, factors and quantised query."""
    ip = O.ip_naive(bits, qu)
    pc = O.popcount_code(bits)
    if b == 0.0:
        xq = np.zeros(len(bits))
    else:
        xq = O.xbar_dot_qbar(ip, pc, float(vl), float(delta), int(np.sum(qu)), dp)
    est, dist, lb = O.estimate(xq, np.asarray(ipo, np.float64), np.asarray(norm, np.float64),
                               float(b), dp, eps0)
    return ip, pc, est, dist, lb


def near_integer(x, tol):
    f = x - np.floor(x)
    return np.minimum(f, 1.0 - f) <= tol


def rel_ok(got, want, scale, tol):
    return np.abs(np.asarray(got, np.float64) - np.asarray(want, np.float64)) <= tol * np.maximum(scale, 1e-30)


def sqdist64(a, b):
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return (d * d).sum(-1)


def tie_equivalent(got_ids, want_ids, q, data, rel=1e-6):
    """True when the two id lists differ only by exact-distance near-ties."""
    if np.array_equal(got_ids, want_ids):
        return True
    gd = np.sort(sqdist64(data[got_ids[got_ids >= 0]], q))
    wd = np.sort(sqdist64(data[want_ids[want_ids >= 0]], q))
    if len(gd) != len(wd):
        return False
    return bool(np.all(np.abs(gd - wd) <= rel * np.maximum(wd, 1e-12)))


def mean_rel_error(est, true):
    m = true > 0
    return float(np.mean(np.abs(est[m] - true[m]) / true[m])), float(np.max(np.abs(est[m] - true[m]) / true[m]))
