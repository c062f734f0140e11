"""FP64 CPU oracle for RaBitQ (Gao & Long, SIGMOD 2024) — TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of
`bench.py` may import this module. The HIP library never calls it, and it
shares no code, header, table or constant generator with the HIP library.

Everything is computed in float64 with NumPy, step by step in the paper's order
and notation:

  index phase  (Algorithm 1; Sec. 3.1.1 normalisation, Sec. 3.1.2 codebook,
                Sec. 3.1.3 quantisation codes, Appendix B for <o_bar, o>)
  query phase  (Algorithm 2; Sec. 3.3.1 randomised uniform scalar quantisation,
                Sec. 3.3.2 the inner-product decomposition and its bitwise and
                LUT forms, Theorem 3.2 estimator and confidence interval,
                Eq. (2) distance from inner product)
  IVF search   (Sec. 4: probe the nearest centroids, rerank by the error bound)

Where the paper leaves a choice open, the reading taken is stated at the
function that makes it. Functions whose result no independent pin checks say
"parity unpinned" in their docstring.
"""
from __future__ import annotations

import math

import numpy as np

# ----------------------------------------------------------------------------
# Parameters (Sec. 5.1, parameter setting): eps0 = 1.9, B_q = 4, code length is
# the smallest multiple of 64 not below D.
EPS0 = 1.9
BQ = 4


def code_length(dim: int) -> int:
    """Default code length: smallest multiple of 64 >= D (Sec. 5.1, parameter setting)."""
    return 64 * ((dim + 63) // 64)


# ----------------------------------------------------------------------------
# Sec. 3.1.2 + Appendix B: a Haar-random orthogonal P from a Gaussian matrix.

def orthogonal_from_gaussian(gauss: np.ndarray) -> np.ndarray:
    """Orthonormalise the rows of a standard Gaussian matrix (Appendix B builds P
    row by row with Gram-Schmidt). Gram-Schmidt on the rows of G equals the Q
    factor of G^T = Q R with diag(R) > 0, so P = Q^T; the result is Haar
    distributed. Works on a single matrix or a stack [..., D, D].
    """
    g = np.asarray(gauss, dtype=np.float64)
    gt = np.swapaxes(g, -1, -2)
    q, r = np.linalg.qr(gt)
    d = np.sign(np.diagonal(r, axis1=-2, axis2=-1))
    d = np.where(d == 0, 1.0, d)
    q = q * d[..., None, :]
    return np.swapaxes(q, -1, -2)


def inverse_rotate(p: np.ndarray, v: np.ndarray) -> np.ndarray:
    """P^{-1} v = P^T v for an orthogonal P (Sec. 3.1.3), applied to the rows of v.

    With v zero-padded to the code length Dp. Row form: (P^T v)^T = v^T P.
    """
    return np.asarray(v, dtype=np.float64) @ p


def pad(v: np.ndarray, dp: int) -> np.ndarray:
    """Append zeros up to the code length (Sec. 5.1: padding the raw vectors with 0s)."""
    v = np.atleast_2d(np.asarray(v, dtype=np.float64))
    out = np.zeros((v.shape[0], dp))
    out[:, :v.shape[1]] = v
    return out


# ----------------------------------------------------------------------------
# Index phase (Algorithm 1).

class OracleIndex:
    """Index-phase outputs for vectors grouped in IVF lists.

    Attributes (one row per data vector, in the caller's order):
      bits   [N, Dp] uint8  quantisation code x_b (Sec. 3.1.3)
      ipo    [N]     <o_bar, o> = <x_bar, P^{-1} o> (Algorithm 1, last step)
      norm   [N]     ||o_r - c|| (Algorithm 1, last step)
      z      [N, Dp] P^{-1} o, kept for tests
    """

    def __init__(self, data, centroids, assign, p):
        self.data = np.asarray(data, dtype=np.float64)
        self.centroids = np.asarray(centroids, dtype=np.float64)
        self.assign = np.asarray(assign, dtype=np.int64)
        self.p = np.asarray(p, dtype=np.float64)
        self.dp = self.p.shape[0]
        n, dim = self.data.shape
        assert self.dp >= dim
        resid = self.data - self.centroids[self.assign]           # o_r - c (Sec. 3.1.1)
        self.norm = np.sqrt((resid * resid).sum(1))
        safe = np.where(self.norm > 0, self.norm, 1.0)
        o = pad(resid / safe[:, None], self.dp)                    # unit vector o, zero padded
        self.z = inverse_rotate(self.p, o)                         # P^{-1} o
        # Sec. 3.1.3: the nearest codebook vector has the signs of P^{-1} o.
        # Reading: a zero coordinate gets bit 0 (either sign is an argmax).
        self.bits = (self.z > 0).astype(np.uint8)
        xbar = (2.0 * self.bits - 1.0) / math.sqrt(self.dp)
        self.ipo = (xbar * self.z).sum(1)                          # <o_bar, o> = <x_bar, P^{-1} o>
        # Reading for o_r == c: o is undefined; the estimate is multiplied by
        # ||o_r - c|| = 0 in Eq. (2), so any code works; <o_bar, o> := 1.
        zero = self.norm == 0
        self.bits[zero] = 0
        self.ipo[zero] = 1.0
        self.lists = [np.flatnonzero(self.assign == k) for k in range(self.centroids.shape[0])]


def build_index(data, centroids, assign, gauss) -> OracleIndex:
    """Algorithm 1 with P orthonormalised from the given Gaussian draw."""
    return OracleIndex(data, centroids, assign, orthogonal_from_gaussian(gauss))


# ----------------------------------------------------------------------------
# Randomised rounding source. Reading: the paper draws u_i ~ U[0, 1] without
# naming a generator; the theory needs the u_i independent. Both sides use a
# counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) keyed by
# (seed, query id, list id, draw), one 64-bit output per two coordinates:
#     j   = (i // 128) * 64 + i % 64                         (i and i + 64 share a draw)
#     key = seed XOR (qid * 2^40 + list * 2^12 + j)         (mod 2^64)
#     z   = splitmix64(key)
#     u_i = (z >> 40) * 2^-24 if i % 128 < 64 else ((z >> 16) mod 2^24) * 2^-24
# in [0, 1) with 24 bits, where splitmix64(x) is the output of a SplitMix64
# generator whose state was x before the step (state += golden gamma, then the
# 64-bit finaliser). Distinct bit fields of one output are independent
# uniforms to the generator's quality, so the u_i stay independent.

_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One SplitMix64 output for state x (pure Python integers)."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def rounding_key(seed: int, qid: int, list_id: int, j: int) -> int:
    """Counter of draw j of a (query, list) pair."""
    return (seed ^ ((qid << 40) + (list_id << 12) + j)) & _M64


def draw_index(i: int) -> int:
    """Coordinates i and i + 64 of each 128-coordinate block share draw j."""
    return ((i >> 7) << 6) | (i & 63)


def rounding_uniforms(seed: int, qid: int, list_id: int, dp: int) -> np.ndarray:
    """u_0..u_{Dp-1} for one (query, list) pair, in [0, 1) with 24 bits: one
    SplitMix64 output per draw gives two coordinates, bits 40..63 to the
    coordinate with bit 6 clear and bits 16..39 to its partner i + 64."""
    out = []
    for i in range(dp):
        z = splitmix64(rounding_key(seed, qid, list_id, draw_index(i)))
        v = (z >> 40) if (i & 64) == 0 else ((z >> 16) & 0xFFFFFF)
        out.append(v * 2.0 ** -24)
    return np.array(out)


def rounding_uniforms_fast(seed: int, qid: int, list_id: int, dp: int) -> np.ndarray:
    """Same numbers as `rounding_uniforms`, vectorised with uint64 NumPy arithmetic."""
    i = np.arange(dp, dtype=np.uint64)
    j = ((i >> np.uint64(7)) << np.uint64(6)) | (i & np.uint64(63))
    with np.errstate(over="ignore"):
        base = (np.uint64(qid) << np.uint64(40)) + (np.uint64(list_id) << np.uint64(12))
        z = np.uint64(seed) ^ (base + j)
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    hi = z >> np.uint64(40)
    mid = (z >> np.uint64(16)) & np.uint64(0xFFFFFF)
    v = np.where((i & np.uint64(64)) == 0, hi, mid)
    return v.astype(np.float64) * 2.0 ** -24


# ----------------------------------------------------------------------------
# Query phase, per (query, list) pair (Algorithm 2; Sec. 3.3.1).

class QuantizedQuery:
    """Per (query, list): b = ||q_r - c||, q' = P^{-1} q, and its B_q-bit code."""

    def __init__(self, b, qprime, vl, vr, delta, qu, sq):
        self.b = b
        self.qprime = qprime
        self.vl = vl
        self.vr = vr
        self.delta = delta
        self.qu = qu          # int64 [Dp], values 0 .. 2^Bq - 1
        self.sq = sq          # sum of qu


def quantize_query(q_raw, centroid, p, u, bq: int = BQ) -> QuantizedQuery:
    """Normalise against the list centroid (Sec. 3.1.1), inverse-rotate
    (Sec. 3.3: q' = P^{-1} q) and randomise-round to B_q-bit unsigned integers
    (Sec. 3.3.1): v_l = min q', v_r = max q', Delta = (v_r - v_l)/(2^Bq - 1),
    q_u[i] = floor((q'[i] - v_l)/Delta + u_i).

    Readings: u_i in [0, 1) and the result is clamped to 2^Bq - 1 (the floor at
    the maximum coordinate can only reach 2^Bq when u_i = 1); Delta = 0 (all
    coordinates equal) gives q_u = 0; q_r = c gives b = 0 and q' = 0.
    """
    dp = p.shape[0]
    d = np.asarray(q_raw, dtype=np.float64) - np.asarray(centroid, dtype=np.float64)
    b = math.sqrt(float((d * d).sum()))
    if b == 0.0:
        qp = np.zeros(dp)
    else:
        qp = inverse_rotate(p, pad(d / b, dp))[0]
    vl = float(qp.min())
    vr = float(qp.max())
    top = (1 << bq) - 1
    delta = (vr - vl) / top
    if delta == 0.0:
        qu = np.zeros(dp, dtype=np.int64)
    else:
        qu = np.floor((qp - vl) / delta + np.asarray(u, dtype=np.float64)).astype(np.int64)
        qu = np.minimum(qu, top)
    return QuantizedQuery(b, qp, vl, vr, delta, qu, int(qu.sum()))


# ----------------------------------------------------------------------------
# Sec. 3.3.2: three ways to get <x_b, q_u>.

def ip_naive(bits, qu) -> np.ndarray:
    """<x_b, q_u> = sum_i x_b[i] q_u[i] (rows of `bits` against one q_u)."""
    return (np.asarray(bits, dtype=np.int64) * np.asarray(qu, dtype=np.int64)).sum(-1)


def _popcount_rows(words: np.ndarray) -> np.ndarray:
    return np.unpackbits(words.view(np.uint8), axis=-1).sum(-1).astype(np.int64)


def ip_bitplanes(bits, qu, bq: int = BQ) -> np.ndarray:
    """Bitwise form: sum_j 2^j popcount(x_b AND q_u^(j)), q_u^(j) the j-th bit plane."""
    bits = np.atleast_2d(np.asarray(bits, dtype=np.uint8))
    code = np.packbits(bits, axis=-1)
    qu = np.asarray(qu, dtype=np.int64)
    total = np.zeros(bits.shape[0], dtype=np.int64)
    for j in range(bq):
        plane = np.packbits(((qu >> j) & 1).astype(np.uint8))
        total += (1 << j) * _popcount_rows(code & plane[None, :])
    return total


def ip_lut(bits, qu) -> np.ndarray:
    """Batch (fast-scan) form: D/4 look-up tables of 16 entries, one per 4-bit
    sub-segment; entry t of table s is the inner product of the pattern t with
    q_u[4s:4s+4]. The code's sub-segments index the tables and are summed."""
    bits = np.atleast_2d(np.asarray(bits, dtype=np.int64))
    qu = np.asarray(qu, dtype=np.int64)
    dp = qu.shape[0]
    nseg = dp // 4
    pat = (np.arange(16)[:, None] >> np.arange(4)[None, :]) & 1          # [16, 4]
    luts = pat @ qu.reshape(nseg, 4).T                                    # [16, nseg]
    idx = (bits.reshape(bits.shape[0], nseg, 4) << np.arange(4)).sum(-1)  # [N, nseg]
    return luts[idx, np.arange(nseg)[None, :]].sum(-1)


def popcount_code(bits) -> np.ndarray:
    """sum_i x_b[i] (a per-code constant, Sec. 3.3.2)."""
    return np.asarray(bits, dtype=np.int64).sum(-1)


# ----------------------------------------------------------------------------
# Sec. 3.3.2 decomposition, Theorem 3.2, Eq. (2).

def xbar_dot_qbar(ip, pc, vl, delta, sq, dp):
    """<x_bar, q_bar> = (2 Delta/sqrt D) <x_b, q_u> + (2 v_l/sqrt D) sum x_b
                        - (Delta/sqrt D) sum q_u - sqrt(D) v_l   (D = code length)."""
    rd = math.sqrt(dp)
    ip = np.asarray(ip, dtype=np.float64)
    pc = np.asarray(pc, dtype=np.float64)
    return (2.0 * delta / rd) * ip + (2.0 * vl / rd) * pc - (delta / rd) * sq - rd * vl


def estimate(xq, ipo, norm_o, norm_q, dp, eps0: float = EPS0):
    """Estimator and confidence interval (Theorem 3.2) turned into distances (Eq. 2).

    est     = <o_bar, q>/<o_bar, o>, with <o_bar, q> = <x_bar, q'> ~ <x_bar, q_bar>
    hw      = sqrt((1 - <o_bar,o>^2)/<o_bar,o>^2) * eps0/sqrt(D - 1)
    dist    = ||o_r-c||^2 + ||q_r-c||^2 - 2 ||o_r-c|| ||q_r-c|| est
    lb      = the same with est + hw (reading: the lower distance bound is Eq. (2)
              at the upper end of the interval, without clamping est + hw to 1)
    D is the code length. Returns (est, dist_est, lb).
    """
    ipo = np.asarray(ipo, dtype=np.float64)
    a = np.asarray(norm_o, dtype=np.float64)
    est = np.asarray(xq, dtype=np.float64) / ipo
    hw = np.sqrt(np.maximum(1.0 - ipo * ipo, 0.0)) / ipo * (eps0 / math.sqrt(dp - 1))
    base = a * a + norm_q * norm_q
    dist = base - 2.0 * a * norm_q * est
    lb = base - 2.0 * a * norm_q * (est + hw)
    return est, dist, lb


def pair_estimates(index: OracleIndex, list_id: int, qq: QuantizedQuery, eps0: float = EPS0,
                   ip_form: str = "naive"):
    """All per-code quantities of Algorithm 2's inner loop for one (query, list) pair.

    Returns dict of arrays over the list's members: ids, ip, pc, est, dist, lb.
    """
    ids = index.lists[list_id]
    bits = index.bits[ids]
    if ip_form == "naive":
        ip = ip_naive(bits, qq.qu)
    elif ip_form == "bitplanes":
        ip = ip_bitplanes(bits, qq.qu)
    else:
        ip = ip_lut(bits, qq.qu)
    pc = popcount_code(bits)
    if qq.b == 0.0:
        xq = np.zeros(len(ids))
    else:
        xq = xbar_dot_qbar(ip, pc, qq.vl, qq.delta, qq.sq, index.dp)
    est, dist, lb = estimate(xq, index.ipo[ids], index.norm[ids], qq.b, index.dp, eps0)
    return {"ids": ids, "ip": ip, "pc": pc, "est": est, "dist": dist, "lb": lb}


# ----------------------------------------------------------------------------
# Sec. 4: IVF probing and error-bound reranking.

def probe_lists(q_raw, centroids, nprobe: int) -> np.ndarray:
    """The nprobe lists whose centroids are nearest to the raw query (squared L2),
    nearest first. Reading: ties go to the lower list id."""
    c = np.asarray(centroids, dtype=np.float64)
    d = ((c - np.asarray(q_raw, dtype=np.float64)[None, :]) ** 2).sum(1)
    order = np.lexsort((np.arange(len(d)), d))
    return order[:nprobe]


def exact_sqdist(data_rows, q_raw) -> np.ndarray:
    diff = np.asarray(data_rows, dtype=np.float64) - np.asarray(q_raw, dtype=np.float64)[None, :]
    return (diff * diff).sum(1)


def exact_topk(data, q_raw, k: int, candidate_ids=None):
    """Plain definition of the search result: the k smallest exact squared
    distances among `candidate_ids` (all rows if None), ordered by (dist, id)."""
    ids = np.arange(len(data)) if candidate_ids is None else np.asarray(candidate_ids)
    d = exact_sqdist(np.asarray(data)[ids], q_raw)
    order = np.lexsort((ids, d))[:k]
    return ids[order], d[order]


def search(index: OracleIndex, q_raw, qid: int, k: int, nprobe: int, seed: int,
           eps0: float = EPS0, bq: int = BQ):
    """One query through Algorithm 2 and the Sec. 4 rerank rule.

    Lists are visited nearest first, codes in list order. tau is the k-th
    smallest exact distance found so far (+inf until k are known); a code is
    dropped when its distance lower bound exceeds tau (reading: equality keeps
    it), otherwise its exact distance is computed and the running top-k updated.
    Returns (ids, dists, info) with info = {'probed', 'reranked', 'violations'}:
    'violations' lists ids of the exact top-k among the probed lists whose lower
    bound exceeded their true distance (the only case where the result may
    differ from the exact top-k of the probed lists).
    """
    probed = probe_lists(q_raw, index.centroids, nprobe)
    best_d, best_i = [], []
    tau = math.inf
    reranked = 0
    all_ids, all_lb = [], []
    for lid in probed:
        u = rounding_uniforms_fast(seed, qid, int(lid), index.dp)
        qq = quantize_query(q_raw, index.centroids[lid], index.p, u, bq)
        pe = pair_estimates(index, int(lid), qq, eps0)
        all_ids.append(pe["ids"])
        all_lb.append(pe["lb"])
        for oid, lbv in zip(pe["ids"], pe["lb"]):
            if lbv > tau:
                continue
            d = float(exact_sqdist(index.data[oid:oid + 1], q_raw)[0])
            reranked += 1
            best_d.append(d)
            best_i.append(int(oid))
            order = np.lexsort((np.array(best_i), np.array(best_d)))[:k]
            best_d = [best_d[j] for j in order]
            best_i = [best_i[j] for j in order]
            if len(best_d) >= k:
                tau = best_d[k - 1]
    cand = np.concatenate(all_ids) if all_ids else np.zeros(0, np.int64)
    lbs = np.concatenate(all_lb) if all_lb else np.zeros(0)
    t_ids, t_d = exact_topk(index.data, q_raw, k, cand)
    lb_of = dict(zip(cand.tolist(), lbs.tolist()))
    viol = [int(i) for i, d in zip(t_ids, t_d) if lb_of[int(i)] > d]
    return (np.array(best_i, dtype=np.int64), np.array(best_d),
            {"probed": probed, "reranked": reranked, "violations": viol})


# ----------------------------------------------------------------------------
# Inner product and cosine similarity (conclusion, footnote): with c the list
# centroid,
#   <o_r, q_r> = ||o_r - c|| ||q_r - c|| <o, q> + <o_r, c> + <q_r, c> - ||c||^2
# where o, q are the unit vectors of Sec. 3.1.1, so the unbiased estimate of
# <o, q> (Theorem 3.2) gives an unbiased estimate of the inner product, and its
# confidence interval scaled by ||o_r - c|| ||q_r - c|| bounds it. Cosine
# similarity is the inner product of the unit-normalised raw vectors.
# Readings: the IVF probe takes the lists whose centroids have the largest
# inner product with the query (ties to the lower id); the sequential rerank
# drops a code whose upper bound is below the k-th largest exact inner product
# found so far (equality keeps it); results are ordered by (-inner product, id).

def ip_code_terms(index: OracleIndex) -> np.ndarray:
    """Per data vector: <o_r, c> - ||c||^2 = <o_r - c, c> for its list's centroid."""
    c = index.centroids[index.assign]
    return ((index.data - c) * c).sum(1)


def estimate_ip(xq, ipo, norm_o, norm_q, code_term, pair_term, dp, eps0: float = EPS0):
    """Inner product estimate and its upper bound (conclusion footnote with Theorem 3.2).

    est = <x_bar, q_bar>/<o_bar, o> estimates <o, q>;
    ip  = ||o_r-c|| ||q_r-c|| est + code_term + pair_term, with code_term =
          <o_r - c, c> and pair_term = <q_r, c>;
    ub  = ip + ||o_r-c|| ||q_r-c|| hw (hw the half-width of Theorem 3.2).
    Returns (est, ip, ub)."""
    ipo = np.asarray(ipo, dtype=np.float64)
    a = np.asarray(norm_o, dtype=np.float64)
    est = np.asarray(xq, dtype=np.float64) / ipo
    hw = np.sqrt(np.maximum(1.0 - ipo * ipo, 0.0)) / ipo * (eps0 / math.sqrt(dp - 1))
    ab = a * norm_q
    ip = ab * est + np.asarray(code_term, dtype=np.float64) + pair_term
    return est, ip, ip + ab * hw


def probe_lists_ip(q_raw, centroids, nprobe: int) -> np.ndarray:
    """The nprobe lists whose centroids have the largest inner product with the
    raw query, largest first, ties to the lower list id."""
    c = np.asarray(centroids, dtype=np.float64)
    s = c @ np.asarray(q_raw, dtype=np.float64)
    order = np.lexsort((np.arange(len(s)), -s))
    return order[:nprobe]


def exact_ip(data_rows, q_raw) -> np.ndarray:
    return np.asarray(data_rows, dtype=np.float64) @ np.asarray(q_raw, dtype=np.float64)


def exact_topk_ip(data, q_raw, k: int, candidate_ids=None):
    """Plain definition of the inner-product search result: the k largest exact
    inner products among `candidate_ids` (all rows if None), ordered by
    (-inner product, id)."""
    ids = np.arange(len(data)) if candidate_ids is None else np.asarray(candidate_ids)
    v = exact_ip(np.asarray(data)[ids], q_raw)
    order = np.lexsort((ids, -v))[:k]
    return ids[order], v[order]


def search_ip(index: OracleIndex, q_raw, qid: int, k: int, nprobe: int, seed: int,
              eps0: float = EPS0, bq: int = BQ):
    """Maximum inner product search: Algorithm 2's estimate turned into an
    inner product, lists probed by centroid inner product, the sequential rule
    of Sec. 4 with the bound reversed (drop a code whose upper bound is below
    tau, the k-th largest exact inner product so far, -inf until k are known).
    Returns (ids, inner products, info) like search(); 'violations' lists the
    exact top-k members of the probed lists whose upper bound fell below their
    inner product."""
    probed = probe_lists_ip(q_raw, index.centroids, nprobe)
    fo = ip_code_terms(index)
    best_v, best_i = [], []
    tau = -math.inf
    reranked = 0
    all_ids, all_ub = [], []
    q64 = np.asarray(q_raw, dtype=np.float64)
    for lid in probed:
        u = rounding_uniforms_fast(seed, qid, int(lid), index.dp)
        qq = quantize_query(q_raw, index.centroids[lid], index.p, u, bq)
        ids = index.lists[int(lid)]
        bits = index.bits[ids]
        if qq.b == 0.0:
            xq = np.zeros(len(ids))
        else:
            xq = xbar_dot_qbar(ip_naive(bits, qq.qu), popcount_code(bits), qq.vl, qq.delta, qq.sq, index.dp)
        g = float(index.centroids[lid] @ q64)
        _, _, ub = estimate_ip(xq, index.ipo[ids], index.norm[ids], qq.b, fo[ids], g, index.dp, eps0)
        all_ids.append(ids)
        all_ub.append(ub)
        for oid, ubv in zip(ids, ub):
            if ubv < tau:
                continue
            v = float(exact_ip(index.data[oid:oid + 1], q_raw)[0])
            reranked += 1
            best_v.append(v)
            best_i.append(int(oid))
            order = np.lexsort((np.array(best_i), -np.array(best_v)))[:k]
            best_v = [best_v[j] for j in order]
            best_i = [best_i[j] for j in order]
            if len(best_v) >= k:
                tau = best_v[k - 1]
    cand = np.concatenate(all_ids) if all_ids else np.zeros(0, np.int64)
    ubs = np.concatenate(all_ub) if all_ub else np.zeros(0)
    t_ids, t_v = exact_topk_ip(index.data, q_raw, k, cand)
    ub_of = dict(zip(cand.tolist(), ubs.tolist()))
    viol = [int(i) for i, v in zip(t_ids, t_v) if ub_of[int(i)] < v]
    return (np.array(best_i, dtype=np.int64), np.array(best_v),
            {"probed": probed, "reranked": reranked, "violations": viol})


# ----------------------------------------------------------------------------
# Closed forms used as pins (Appendix B and Lemma "Distribution").

def expected_ipo(dim: int) -> float:
    """E[<o_bar, o>] = sqrt(D/pi) * 2 Gamma(D/2) / ((D - 1) Gamma((D - 1)/2))  (Appendix B)."""
    lg = math.lgamma(dim / 2.0) - math.lgamma((dim - 1) / 2.0)
    return math.sqrt(dim / math.pi) * 2.0 * math.exp(lg) / (dim - 1)


def ipo_second_moment(dim: int) -> float:
    """E[<o_bar, o>^2] = (1 + 2 (D - 1)/pi)/D, from <o_bar, o> = ||P^{-1} o||_1/sqrt(D)
    (Appendix B) and E|x_1 x_2| = 2/(pi D) for a uniform unit vector."""
    return (1.0 + 2.0 * (dim - 1) / math.pi) / dim


def coordinate_density(x, dim: int):
    """p_D(x): density of one coordinate of a uniform unit vector in R^D (Appendix B)."""
    c = math.exp(math.lgamma(dim / 2.0) - math.lgamma((dim - 1) / 2.0)) / math.sqrt(math.pi)
    x = np.asarray(x, dtype=np.float64)
    return c * np.power(np.maximum(1.0 - x * x, 0.0), (dim - 3) / 2.0)


def bound_failure_probability(r: float, dim: int, eps0: float = EPS0) -> float:
    """Exact probability that the Theorem 3.2 interval misses <o, q> = r (exact q').

    By Lemma 3.1 the error is sqrt(1 - r^2) <o_bar, e1>/<o_bar, o>, and by the
    Lemma "Distribution" (Appendix B) <o_bar, e1> = sqrt(1 - <o_bar,o>^2) X1 with
    X1 ~ p_{D-1} independent of <o_bar, o>. The failure event is therefore
    sqrt(1 - r^2) |X1| > eps0/sqrt(D - 1), and X1^2 ~ Beta(1/2, (D - 2)/2).
    """
    from scipy.special import betainc
    if abs(r) >= 1.0:
        return 0.0
    t = eps0 / (math.sqrt(dim - 1) * math.sqrt(1.0 - r * r))
    if t >= 1.0:
        return 0.0
    return float(1.0 - betainc(0.5, (dim - 2) / 2.0, t * t))


def bit_entropy_fraction(bits) -> float:
    """Sum over code positions of the binary entropy of the fraction of 1s,
    divided by the code length (Appendix E, normalisation discussion)."""
    p = np.asarray(bits, dtype=np.float64).mean(0)
    with np.errstate(divide="ignore", invalid="ignore"):
        h = -(p * np.log2(p) + (1 - p) * np.log2(1 - p))
    h = np.nan_to_num(h, nan=0.0)
    return float(h.sum() / len(p))
