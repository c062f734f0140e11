"""Seeded synthetic workloads shared by the tests, the bench and the oracle timing.

This module only draws random inputs (data vectors, queries, the Gaussian matrix
that the rotation is orthonormalised from) and runs the k-means clustering that
an IVF index takes as input. It contains none of RaBitQ's own arithmetic: no
rotation, no quantisation, no estimator. Both the FP64 oracle and the HIP
library consume exactly the arrays produced here.

The paper evaluates on public datasets (SIFT, GIST, DEEP, ...; experiments
section, "Dataset Statistics" table) that are not available here. The
generators below stand in for them with the same shapes and the value
structure described for each workload.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Workload",
    "code_bits_for",
    "gaussian_matrix",
    "mixture_flat",
    "sift_like",
    "gist_like",
    "embedding_like",
    "embedding_like_gpu",
    "kmeans",
    "kmeans_gpu",
    "workload",
    "query_batch_sizes",
]


def code_bits_for(dim: int) -> int:
    """Smallest multiple of 64 that is >= dim (default code length)."""
    return 64 * ((dim + 63) // 64)


def gaussian_matrix(dim_pad: int, seed: int) -> np.ndarray:
    """Standard Gaussian [dim_pad x dim_pad] float64 matrix; the random draw behind P."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((dim_pad, dim_pad))


def mixture_flat(n: int, nq: int, dim: int = 128, ncomp: int = 32,
                 seed_data: int = 1001, seed_query: int = 2001):
    """Mixture of isotropic Gaussians: means ~ N(0, 4 I), per-component std 1.

    Component means are shared by data and queries (drawn from seed_data); the
    queries use their own seed so they are not database points.
    """
    rng = np.random.default_rng(seed_data)
    means = rng.normal(0.0, 2.0, size=(ncomp, dim))
    comp = rng.integers(0, ncomp, size=n)
    data = means[comp] + rng.standard_normal((n, dim))
    rq = np.random.default_rng(seed_query)
    qcomp = rq.integers(0, ncomp, size=nq)
    queries = means[qcomp] + rq.standard_normal((nq, dim))
    return data.astype(np.float32), queries.astype(np.float32)


def _sift_params(dim, ncomp, rng):
    scale = np.exp(rng.normal(0.0, 1.0, size=dim)) * 20.0          # heavy-tailed per-dim scale
    means = np.abs(rng.normal(0.0, 1.0, size=(ncomp, dim)) * (2.0 * scale)) + 10.0
    return scale, means


def sift_like(n: int, nq: int, dim: int = 128, ncomp: int = 64,
              seed_data: int = 1002, seed_query: int = 2002, chunk: int = 1 << 18):
    """Non-negative integer-valued (0..255) vectors with heavy-tailed per-dim spread."""
    rng = np.random.default_rng(seed_data)
    scale, means = _sift_params(dim, ncomp, rng)

    def draw(r, m):
        out = np.empty((m, dim), dtype=np.float32)
        for s in range(0, m, chunk):
            e = min(m, s + chunk)
            comp = r.integers(0, ncomp, size=e - s)
            x = means[comp] + scale * r.standard_normal((e - s, dim))
            out[s:e] = np.clip(np.round(x), 0.0, 255.0)
        return out

    data = draw(rng, n)
    queries = draw(np.random.default_rng(seed_query), nq)
    return data, queries


def zipf_weights(ncomp: int, s: float = 1.1) -> np.ndarray:
    w = np.arange(1, ncomp + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def gist_like(n: int, nq: int, dim: int = 960, ncomp: int = 4096,
              seed_data: int = 1003, seed_query: int = 2003, chunk: int = 1 << 16):
    """Values in [0, 1] with a decaying per-dimension spread and Zipf(1.1) component sizes.

    Returns (data, queries, component_means); the means seed the k-means.
    """
    rng = np.random.default_rng(seed_data)
    sigma = 0.25 * (np.arange(1, dim + 1, dtype=np.float64) ** -0.5)
    means = rng.uniform(0.1, 0.6, size=(ncomp, dim))
    w = zipf_weights(ncomp)

    def draw(r, m):
        out = np.empty((m, dim), dtype=np.float32)
        for s in range(0, m, chunk):
            e = min(m, s + chunk)
            comp = r.choice(ncomp, size=e - s, p=w)
            x = means[comp] + sigma * r.standard_normal((e - s, dim))
            out[s:e] = np.clip(x, 0.0, 1.0)
        return out

    data = draw(rng, n)
    queries = draw(np.random.default_rng(seed_query), nq)
    return data, queries, means.astype(np.float32)


def embedding_like(n: int, nq: int, dim: int = 768, seed_data: int = 1004,
                   seed_query: int = 2004, exponent: float = 1.0, chunk: int = 1 << 16):
    """Unit-norm vectors from an anisotropic Gaussian with power-law eigenvalues."""
    rng = np.random.default_rng(seed_data)
    lam = np.arange(1, dim + 1, dtype=np.float64) ** (-exponent)
    qm, r = np.linalg.qr(rng.standard_normal((dim, dim)))
    u = qm * np.sign(np.diag(r))
    basis = (u * np.sqrt(lam)[None, :]).T.astype(np.float32)   # rows: sqrt(lam_i) * u_i

    def draw(r_, m):
        out = np.empty((m, dim), dtype=np.float32)
        for s in range(0, m, chunk):
            e = min(m, s + chunk)
            z = r_.standard_normal((e - s, dim)).astype(np.float32)
            x = z @ basis
            x /= np.linalg.norm(x, axis=1, keepdims=True)
            out[s:e] = x
        return out

    data = draw(rng, n)
    queries = draw(np.random.default_rng(seed_query), nq)
    return data, queries


def embedding_like_gpu(n: int, nq: int, device, dim: int = 768, seed_data: int = 1004,
                       seed_query: int = 2004, exponent: float = 1.0, chunk: int = 1 << 18):
    """The distribution of `embedding_like` drawn on the GPU (for tens of
    millions of vectors): the same seeded basis, Gaussian coefficients from a
    seeded torch generator on `device`. Returns float32 tensors on `device`.
    (Not the same numbers as `embedding_like` for equal seeds.)"""
    import torch
    rng = np.random.default_rng(seed_data)
    lam = np.arange(1, dim + 1, dtype=np.float64) ** (-exponent)
    qm, r = np.linalg.qr(rng.standard_normal((dim, dim)))
    u = qm * np.sign(np.diag(r))
    basis = torch.from_numpy((u * np.sqrt(lam)[None, :]).T.astype(np.float32)).to(device)

    def draw(seed, m):
        g = torch.Generator(device=device)
        g.manual_seed(seed)
        out = torch.empty((m, dim), dtype=torch.float32, device=device)
        for s in range(0, m, chunk):
            e = min(m, s + chunk)
            z = torch.randn((e - s, dim), generator=g, device=device, dtype=torch.float32)
            x = z @ basis
            out[s:e] = x / torch.linalg.vector_norm(x, dim=1, keepdim=True)
        return out

    return draw(seed_data, n), draw(seed_query, nq)


def embedding_queries_gpu(nq: int, device, seed_query: int, dim: int = 768, seed_data: int = 1004,
                          exponent: float = 1.0, chunk: int = 1 << 18):
    """Queries from the distribution of `embedding_like_gpu(..., seed_data)` with
    their own seed, without drawing the data again."""
    return embedding_like_gpu(0, nq, device, dim=dim, seed_data=seed_data, seed_query=seed_query,
                              exponent=exponent, chunk=chunk)[1]


def kmeans_gpu(x, nlist: int, iters: int = 10, seed: int = 7, sample: int | None = None,
               chunk: int = 8192, init: np.ndarray | None = None):
    """Lloyd k-means of a float32 GPU tensor x [n, dim]: seeded init from a
    seeded sample of `sample` rows (all rows when None), `iters` rounds of
    FP64 nearest-centroid assignment + mean update on the sample, then a final
    FP64 assignment of every row. `init` (nlist x dim) replaces the seeded
    initial centroids. Empty clusters keep their centroid.
    Returns (centroids float32 numpy, assign int32 numpy)."""
    import torch
    n, dim = x.shape
    rng = np.random.default_rng(seed)
    xs = x
    if sample is not None and sample < n:
        xs = x[torch.from_numpy(np.sort(rng.choice(n, size=sample, replace=False))).to(x.device)]
    if init is not None:
        cent = torch.as_tensor(np.asarray(init, dtype=np.float64), device=x.device).clone()
    else:
        cent = xs[torch.from_numpy(rng.choice(xs.shape[0], size=nlist, replace=False)).to(x.device)].double()

    def assign(rows):
        cn = (cent * cent).sum(1)
        lab = torch.empty(rows.shape[0], dtype=torch.int64, device=x.device)
        for s0 in range(0, rows.shape[0], chunk):
            d = cn[None, :] - 2.0 * (rows[s0:s0 + chunk].double() @ cent.T)
            lab[s0:s0 + chunk] = torch.argmin(d, dim=1)
        return lab

    for _ in range(iters):
        lab = assign(xs)
        sums = torch.zeros((nlist, dim), dtype=torch.float64, device=x.device)
        for s0 in range(0, xs.shape[0], 1 << 16):
            sums.index_add_(0, lab[s0:s0 + (1 << 16)], xs[s0:s0 + (1 << 16)].double())
        cnt = torch.bincount(lab, minlength=nlist).double()
        nz = cnt > 0
        cent[nz] = sums[nz] / cnt[nz, None]
    lab = assign(x)
    return cent.float().cpu().numpy(), lab.to(torch.int32).cpu().numpy()


def query_batch_sizes(total: int, seed: int = 2104, lo: int = 1, hi: int = 1024):
    """Batch sizes ~ uniform{lo..hi} (seeded) that add up to `total`."""
    rng = np.random.default_rng(seed)
    sizes = []
    left = total
    while left > 0:
        b = int(min(left, rng.integers(lo, hi + 1)))
        sizes.append(b)
        left -= b
    return sizes


# ---------------------------------------------------------------- k-means (IVF input)

def _assign_numpy(x, cent, chunk=1 << 15):
    cn = (cent.astype(np.float64) ** 2).sum(1)
    out = np.empty(x.shape[0], dtype=np.int64)
    c32 = cent.astype(np.float32)
    for s in range(0, x.shape[0], chunk):
        xs = x[s:s + chunk].astype(np.float32)
        d = cn[None, :] - 2.0 * (xs @ c32.T).astype(np.float64)
        out[s:s + chunk] = np.argmin(d, axis=1)
    return out


def _assign_torch(x, cent, device, chunk=1 << 16):
    """Nearest-centroid assignment on a GPU in float64, so repeated runs agree."""
    import torch
    c = torch.as_tensor(cent, dtype=torch.float64, device=device)
    cn = (c * c).sum(1)
    out = np.empty(x.shape[0], dtype=np.int64)
    for s in range(0, x.shape[0], chunk):
        xs = torch.as_tensor(x[s:s + chunk], dtype=torch.float64, device=device)
        d = cn[None, :] - 2.0 * (xs @ c.T)
        out[s:s + chunk] = torch.argmin(d, dim=1).cpu().numpy()
    return out


def kmeans(x: np.ndarray, nlist: int, iters: int = 10, seed: int = 7,
           init: np.ndarray | None = None, device=None):
    """Plain Lloyd k-means: seeded init (distinct sample points unless `init`),
    `iters` rounds of assign + mean update, a final assignment.
    Empty clusters keep their previous centroid. Returns (centroids f32, assign i32).
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, dim = x.shape
    if nlist == 1:
        return x.astype(np.float64).mean(0, keepdims=True).astype(np.float32), np.zeros(n, np.int32)
    rng = np.random.default_rng(seed)
    if init is None:
        cent = x[rng.choice(n, size=nlist, replace=False)].astype(np.float64)
    else:
        cent = np.array(init, dtype=np.float64, copy=True)
    assign_fn = (lambda a, c: _assign_torch(a, c, device)) if device is not None else _assign_numpy
    for _ in range(iters):
        lab = assign_fn(x, cent)
        sums = np.zeros((nlist, dim), dtype=np.float64)
        _cluster_sums(sums, lab, x)
        cnt = np.bincount(lab, minlength=nlist).astype(np.float64)
        nz = cnt > 0
        cent[nz] = sums[nz] / cnt[nz, None]
    lab = assign_fn(x, cent)
    return cent.astype(np.float32), lab.astype(np.int32)


def _cluster_sums(sums, lab, x):
    order = np.argsort(lab, kind="stable")
    sl = lab[order]
    bounds = np.flatnonzero(np.diff(sl)) + 1
    starts = np.concatenate([[0], bounds])
    ends = np.concatenate([bounds, [len(sl)]])
    for s, e in zip(starts, ends):
        sums[sl[s]] = x[order[s:e]].astype(np.float64).sum(0)


# ---------------------------------------------------------------- named workloads

@dataclass
class Workload:
    name: str
    data: np.ndarray          # [n, D] float32
    queries: np.ndarray       # [nq, D] float32
    centroids: np.ndarray     # [nlist, D] float32
    assign: np.ndarray        # [n] int32
    gauss: np.ndarray         # [Dp, Dp] float64, the draw the rotation is built from
    seed: int                 # randomised-rounding seed
    k: int
    nprobe: int

    @property
    def dim(self):
        return self.data.shape[1]

    @property
    def dim_pad(self):
        return self.gauss.shape[0]


def workload(cfg: int, n: int | None = None, nq: int | None = None, nlist: int | None = None,
             kmeans_iters: int = 10, device=None) -> Workload:
    """The five workloads, optionally scaled down (n, nq, nlist) for tests.

    Seeds: data 1000+cfg, queries 2000+cfg, Gaussian for P 3000+cfg, rounding 4000+cfg.
    """
    if cfg == 1:
        n = n or 10_000
        nq = nq or 100
        data, queries = mixture_flat(n, nq, seed_data=1001, seed_query=2001)
        cent = data.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
        assign = np.zeros(n, np.int32)
        k, nprobe = 10, 1
    elif cfg == 2:
        n = n or 1_000_000
        nq = nq or 10_000
        nlist = nlist or 4096
        data, queries = sift_like(n, nq)
        cent, assign = kmeans(data, nlist, iters=kmeans_iters, seed=5002, device=device)
        k, nprobe = 10, 64
    elif cfg == 3:
        n = n or 1_000_000
        nq = nq or 10_000
        nlist = nlist or 4096
        data, queries, means = gist_like(n, nq, ncomp=nlist)
        cent, assign = kmeans(data, nlist, iters=kmeans_iters, init=means, device=device)
        k, nprobe = 100, 64
    elif cfg == 4:
        n = n or 10_000_000
        nq = nq or 100_000
        nlist = nlist or 16_384
        data, queries = embedding_like(n, nq)
        cent, assign = kmeans(data, nlist, iters=kmeans_iters, seed=5004, device=device)
        k, nprobe = 10, 64
    else:
        raise ValueError(f"unknown workload {cfg}")
    dp = code_bits_for(data.shape[1])
    return Workload(f"cfg{cfg}", data, queries, cent, assign,
                    gaussian_matrix(dp, 3000 + cfg), 4000 + cfg, k, nprobe)


def zipf_sizes_report(assign: np.ndarray, nlist: int):
    sizes = np.bincount(assign, minlength=nlist)
    srt = np.sort(sizes)[::-1]
    return {"max": int(srt[0]), "median": float(np.median(sizes)),
            "top10_frac": float(srt[:10].sum() / max(1, sizes.sum())),
            "empty": int((sizes == 0).sum())}
