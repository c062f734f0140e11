"""Pins for the FP64 oracle: each test checks it against something other than
itself — values printed in the paper, closed forms from its appendices, brute
force, a textbook routine, or a distributional law — so that a dropped term, a
wrong sign or index, or a transposed operand fails one of them.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import rabitq_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_constants():
    out = {}
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, val = line.split()[:2]
            out[key] = float(val)
    return out


PAPER = _golden_constants()


def _unit(rng, d):
    v = rng.standard_normal(d)
    return v / np.linalg.norm(v)


def _pair_with_ip(rng, d, r):
    """Two unit vectors with <o, q> = r exactly."""
    o = _unit(rng, d)
    w = rng.standard_normal(d)
    w -= (w @ o) * o
    w /= np.linalg.norm(w)
    return o, r * o + math.sqrt(1 - r * r) * w


# --------------------------------------------------------------- parameters

def test_paper_parameters():
    assert O.EPS0 == PAPER["eps0"]
    assert O.BQ == PAPER["bq"]
    m = int(PAPER["code_multiple"])
    for d in (1, 63, 64, 65, 128, 150, 256, 300, 420, 768, 960):
        dp = O.code_length(d)
        assert dp % m == 0 and d <= dp < d + m


# --------------------------------------------------------------- rounding source

def test_splitmix64_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64.txt")) if l.startswith("0x")]
    gamma = 0x9E3779B97F4A7C15
    assert O.splitmix64(0) == vals[0]
    assert O.splitmix64(gamma) == vals[1]


def test_rounding_uniforms_properties():
    u = O.rounding_uniforms(4001, 3, 17, 256)
    uf = O.rounding_uniforms_fast(4001, 3, 17, 256)
    np.testing.assert_array_equal(u, uf)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))        # 24-bit values, exact in FP32
    many = np.concatenate([O.rounding_uniforms_fast(7, q, l, 128) for q in range(40) for l in range(25)])
    assert stats.kstest(many, "uniform").pvalue > 1e-3
    assert abs(np.corrcoef(many[:-1], many[1:])[0, 1]) < 0.01
    # different pairs give different streams
    assert not np.array_equal(O.rounding_uniforms_fast(7, 1, 2, 64), O.rounding_uniforms_fast(7, 2, 1, 64))
    # the two coordinates that share a draw (i, i + 64) are uncorrelated and
    # their joint law is uniform on the square (chi-square over 8 x 8 cells)
    w = np.stack([O.rounding_uniforms_fast(7, q, l, 256) for q in range(40) for l in range(25)])
    a = np.concatenate([w[:, 0:64], w[:, 128:192]], 1).ravel()
    b = np.concatenate([w[:, 64:128], w[:, 192:256]], 1).ravel()
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.01
    h, _, _ = np.histogram2d(a, b, bins=8, range=[[0, 1], [0, 1]])
    assert stats.chisquare(h.ravel()).pvalue > 1e-3


# --------------------------------------------------------------- rotation

def _gram_schmidt_rows(g):
    """Textbook modified Gram-Schmidt on the rows (Appendix B's construction)."""
    p = np.array(g, dtype=np.float64)
    for i in range(p.shape[0]):
        for j in range(i):
            p[i] -= (p[i] @ p[j]) * p[j]
        p[i] /= np.linalg.norm(p[i])
    return p


def test_orthogonal_matches_gram_schmidt():
    g = np.random.default_rng(1).standard_normal((24, 24))
    p = O.orthogonal_from_gaussian(g)
    np.testing.assert_allclose(p @ p.T, np.eye(24), atol=1e-12)
    np.testing.assert_allclose(p, _gram_schmidt_rows(g), atol=1e-10)
    stack = O.orthogonal_from_gaussian(np.stack([g, 2 * g]))
    np.testing.assert_allclose(stack[1], p, atol=1e-12)       # scale does not change P


# --------------------------------------------------------------- index phase

def test_code_is_codebook_argmin_bruteforce():
    """Sec. 3.1.3: x_bar = argmin over the 2^D codebook of ||o - P x||."""
    rng = np.random.default_rng(2)
    d = 10
    allx = ((np.arange(2 ** d)[:, None] >> np.arange(d)[None, :]) & 1) * 2.0 - 1.0
    allx /= math.sqrt(d)
    for t in range(20):
        p = O.orthogonal_from_gaussian(rng.standard_normal((d, d)))
        data = rng.standard_normal((1, d)) * 3 + 1
        cen = rng.standard_normal((1, d))
        idx = O.OracleIndex(data, cen, [0], p)
        o = (data[0] - cen[0]) / np.linalg.norm(data[0] - cen[0])
        dist = ((o[None, :] - allx @ p.T) ** 2).sum(1)     # rows of allx @ P^T are P x
        best = allx[np.argmin(dist)]
        np.testing.assert_array_equal((best > 0).astype(np.uint8), idx.bits[0])
        assert idx.norm[0] == pytest.approx(np.linalg.norm(data[0] - cen[0]), rel=1e-14)


def test_zero_coordinates_get_bit_zero():
    """A zero coordinate of P^{-1} o (here: identity rotation, exact zeros and the
    zero padding up to the code length) is a tie in the codebook argmin
    (Sec. 3.1.3); the reading gives it bit 0. It adds 0 to <o_bar, o> either way."""
    d, dp = 70, O.code_length(70)
    rng = np.random.default_rng(31)
    v = rng.standard_normal(d)
    v[::3] = 0.0
    idx = O.OracleIndex(v[None, :], np.zeros((1, d)), [0], np.eye(dp))
    want = np.concatenate([(v > 0), np.zeros(dp - d, bool)]).astype(np.uint8)
    np.testing.assert_array_equal(idx.bits[0], want)
    assert idx.ipo[0] == pytest.approx(np.abs(v).sum() / np.linalg.norm(v) / math.sqrt(dp), rel=1e-14)


def test_ipo_is_l1_norm_and_geometric_inner_product():
    rng = np.random.default_rng(3)
    d = 64
    p = O.orthogonal_from_gaussian(rng.standard_normal((d, d)))
    data = rng.standard_normal((50, d))
    cen = data.mean(0, keepdims=True)
    idx = O.OracleIndex(data, cen, np.zeros(50, int), p)
    for i in range(50):
        o = (data[i] - cen[0]) / np.linalg.norm(data[i] - cen[0])
        xbar = (2.0 * idx.bits[i] - 1) / math.sqrt(d)
        obar = p @ xbar                                        # o_bar = P x_bar
        assert idx.ipo[i] == pytest.approx(obar @ o, abs=1e-13)
        assert idx.ipo[i] == pytest.approx(np.abs(p.T @ o).sum() / math.sqrt(d), abs=1e-13)


def test_padding_keeps_distances():
    """Zero-padding to the code length leaves o and q' unchanged in norm."""
    rng = np.random.default_rng(4)
    d, dp = 100, O.code_length(100)
    p = O.orthogonal_from_gaussian(rng.standard_normal((dp, dp)))
    data = rng.standard_normal((5, d))
    idx = O.OracleIndex(data, np.zeros((1, d)), np.zeros(5, int), p)
    np.testing.assert_allclose((idx.z ** 2).sum(1), 1.0, atol=1e-12)
    assert idx.bits.shape == (5, 128)


def test_degenerate_vector_at_centroid():
    rng = np.random.default_rng(5)
    d = 64
    p = O.orthogonal_from_gaussian(rng.standard_normal((d, d)))
    c = rng.standard_normal((1, d))
    idx = O.OracleIndex(np.vstack([c, c + 1]), c, [0, 0], p)
    assert idx.norm[0] == 0 and idx.ipo[0] == 1.0
    qq = O.quantize_query(c[0] + 2.0, c[0], p, np.full(d, 0.5))
    pe = O.pair_estimates(idx, 0, qq)
    # the vector at the centroid gets its exact distance ||q_r - c||^2
    assert pe["dist"][0] == pytest.approx(qq.b ** 2, rel=1e-14)
    assert pe["lb"][0] == pytest.approx(qq.b ** 2, rel=1e-14)


# --------------------------------------------------------------- query phase

def test_quantization_definition_and_clamp():
    rng = np.random.default_rng(6)
    d = 128
    p = O.orthogonal_from_gaussian(rng.standard_normal((d, d)))
    q = rng.standard_normal(d)
    c = rng.standard_normal(d)
    u = O.rounding_uniforms_fast(11, 0, 0, d)
    qq = O.quantize_query(q, c, p, u)
    qp = p.T @ ((q - c) / np.linalg.norm(q - c))
    np.testing.assert_allclose(qq.qprime, qp, atol=1e-14)
    assert qq.qu.min() >= 0 and qq.qu.max() <= 15
    recon = qq.delta * qq.qu + qq.vl                   # q_bar
    assert np.all(np.abs(recon - qp) <= qq.delta * (1 + 1e-12))
    # u -> 1 would push the max coordinate to 2^Bq; the clamp keeps it at 15
    qq1 = O.quantize_query(q, c, p, np.full(d, 1.0 - 2 ** -24))
    assert qq1.qu.max() == 15 and qq1.qu[np.argmax(qp)] == 15
    # u = 1, the closed end of the paper's interval: floor reaches 2^Bq at the
    # maximum coordinate and the clamp brings it back to 15; elsewhere it is floor(x) + 1
    qq2 = O.quantize_query(q, c, p, np.ones(d))
    x = (qp - qq.vl) / qq.delta
    assert qq2.qu[np.argmax(qp)] == 15 and qq2.qu.max() == 15
    inner = x < 14.0 - 1e-9
    np.testing.assert_array_equal(qq2.qu[inner], np.floor(x[inner]).astype(np.int64) + 1)
    # all-equal coordinates: Delta = 0
    p1 = np.eye(4)
    qz = O.quantize_query(np.ones(4), np.zeros(4), p1, np.full(4, 0.9))
    assert qz.delta == 0 and np.all(qz.qu == 0)


def test_randomized_rounding_is_unbiased():
    """E[q_bar] = q' coordinate-wise (Sec. 3.3.1)."""
    rng = np.random.default_rng(7)
    d = 64
    p = O.orthogonal_from_gaussian(rng.standard_normal((d, d)))
    q, c = rng.standard_normal(d), rng.standard_normal(d)
    acc = np.zeros(d)
    n = 4000
    for t in range(n):
        qq = O.quantize_query(q, c, p, O.rounding_uniforms_fast(99, t, 0, d))
        acc += qq.delta * qq.qu + qq.vl
    mean = acc / n
    # per-coordinate std of the rounding error is at most Delta/2
    se = qq.delta / 2 / math.sqrt(n)
    assert np.all(np.abs(mean - qq.qprime) < 5 * se + 1e-12)


def test_three_inner_product_forms_agree_bitexact():
    rng = np.random.default_rng(8)
    for dp in (64, 128, 960):
        bits = rng.integers(0, 2, size=(200, dp), dtype=np.uint8)
        qu = rng.integers(0, 16, size=dp)
        naive = np.array([sum(int(b) * int(v) for b, v in zip(row, qu)) for row in bits[:5]])
        a = O.ip_naive(bits, qu)
        np.testing.assert_array_equal(a[:5], naive)
        np.testing.assert_array_equal(a, O.ip_bitplanes(bits, qu))
        np.testing.assert_array_equal(a, O.ip_lut(bits, qu))
    # extremes
    dp = 128
    ones = np.ones((1, dp), np.uint8)
    assert O.ip_bitplanes(ones, np.full(dp, 15))[0] == 15 * dp
    assert O.ip_lut(np.zeros((1, dp), np.uint8), np.full(dp, 15))[0] == 0


def test_decomposition_equals_direct_inner_product():
    """Sec. 3.3.2: the four-term expression equals <x_bar, q_bar> computed directly."""
    rng = np.random.default_rng(9)
    for dp in (64, 128, 768):
        bits = rng.integers(0, 2, size=(50, dp), dtype=np.uint8)
        qu = rng.integers(0, 16, size=dp)
        vl, delta = -0.17, 0.023
        xbar = (2.0 * bits - 1) / math.sqrt(dp)
        qbar = delta * qu + vl
        direct = xbar @ qbar
        got = O.xbar_dot_qbar(O.ip_naive(bits, qu), O.popcount_code(bits), vl, delta, qu.sum(), dp)
        np.testing.assert_allclose(got, direct, atol=1e-12)


def test_estimator_equals_geometric_ratio_and_lemma31():
    """With exact q', est * <o_bar,o> = <o_bar, q> (Sec. 3.3 identity via P) and
    Lemma 3.1 holds: <o_bar,q> = <o_bar,o><o,q> + <o_bar,e1> sqrt(1 - <o,q>^2)."""
    rng = np.random.default_rng(10)
    d = 128
    for t in range(10):
        p = O.orthogonal_from_gaussian(rng.standard_normal((d, d)))
        o, q = _pair_with_ip(rng, d, rng.uniform(-0.9, 0.9))
        idx = O.OracleIndex(o[None, :] * 2.0, np.zeros((1, d)), [0], p)
        qp = O.inverse_rotate(p, q[None, :])[0]
        xbar = (2.0 * idx.bits[0] - 1) / math.sqrt(d)
        est, dist, lb = O.estimate(xbar @ qp, idx.ipo[0], 2.0, 3.0, d)
        obar = p @ xbar
        assert est * idx.ipo[0] == pytest.approx(obar @ q, abs=1e-13)
        r = o @ q
        e1 = (q - r * o) / np.linalg.norm(q - r * o)
        assert obar @ q == pytest.approx(idx.ipo[0] * r + (obar @ e1) * math.sqrt(1 - r * r), abs=1e-13)
        # Eq. (2) with the exact inner product gives the exact distance
        _, dexact, _ = O.estimate(r * idx.ipo[0], idx.ipo[0], 2.0, 3.0, d)
        assert dexact == pytest.approx(((2.0 * o - 3.0 * q) ** 2).sum(), rel=1e-12)
        assert lb <= dist


def test_collinear_case_is_exact():
    """o and q collinear: the estimator returns <o,q> = +-1 exactly (Lemma 3.1)."""
    rng = np.random.default_rng(11)
    d = 128
    p = O.orthogonal_from_gaussian(rng.standard_normal((d, d)))
    c = rng.standard_normal(d)
    o_r = c + rng.standard_normal(d)
    idx = O.OracleIndex(o_r[None, :], c[None, :], [0], p)
    xbar = (2.0 * idx.bits[0] - 1) / math.sqrt(d)
    for sign, lam in ((1, 2.5), (-1, 0.7)):
        q_r = c + sign * lam * (o_r - c)
        qp = O.inverse_rotate(p, O.pad((q_r - c) / np.linalg.norm(q_r - c), d))[0]
        a, b = idx.norm[0], np.linalg.norm(q_r - c)
        est, dist, _ = O.estimate(xbar @ qp, idx.ipo[0], a, b, d)
        assert est == pytest.approx(sign, abs=1e-13)
        assert dist == pytest.approx(((o_r - q_r) ** 2).sum(), rel=1e-12)


# --------------------------------------------------------------- distributional pins

def _sample_ipo_and_est(d, r, nsamp, seed, quantize):
    rng = np.random.default_rng(seed)
    o, q = _pair_with_ip(rng, d, r)
    ipos, ests, ratios, obarq, hws = [], [], [], [], []
    e1 = (q - r * o) / np.linalg.norm(q - r * o)
    for s0 in range(0, nsamp, 500):
        ps = O.orthogonal_from_gaussian(rng.standard_normal((min(500, nsamp - s0), d, d)))
        for p in ps:
            idx = O.OracleIndex(o[None, :], np.zeros((1, d)), [0], p)
            if quantize:
                qq = O.quantize_query(q, np.zeros(d), p, rng.random(d))
                xq = O.xbar_dot_qbar(O.ip_naive(idx.bits, qq.qu), O.popcount_code(idx.bits),
                                     qq.vl, qq.delta, qq.sq, d)[0]
            else:
                xbar = (2.0 * idx.bits[0] - 1) / math.sqrt(d)
                xq = xbar @ O.inverse_rotate(p, q[None, :])[0]
            est, dist, lb = O.estimate(xq, idx.ipo[0], 1.0, 1.0, d)
            hws.append(float(dist - lb) / 2.0)      # with ||o_r-c|| = ||q_r-c|| = 1: lb = dist - 2 hw
            obar = p @ ((2.0 * idx.bits[0] - 1) / math.sqrt(d))
            ipos.append(idx.ipo[0])
            ests.append(float(est))
            obarq.append(obar @ q)
            ratios.append((obar @ e1) / math.sqrt(1 - idx.ipo[0] ** 2))
    return np.array(ipos), np.array(ests), np.array(ratios), np.array(obarq), np.array(hws)


@pytest.fixture(scope="module")
def mc128():
    return _sample_ipo_and_est(128, 0.5, 4000, 12, quantize=False)


def test_expected_ipo_closed_form_matches_paper_range():
    lo, hi = PAPER["ipo_mean_lo"], PAPER["ipo_mean_hi"]
    for d in np.unique(np.logspace(math.log10(PAPER["ipo_dim_lo"]), math.log10(PAPER["ipo_dim_hi"]), 25).astype(int)):
        assert round(O.expected_ipo(int(d)), 3) >= lo and round(O.expected_ipo(int(d)), 3) <= hi
    # large-D limit sqrt(2/pi) (mean absolute value of a standard normal)
    assert O.expected_ipo(10 ** 7) == pytest.approx(math.sqrt(2 / math.pi), rel=1e-6)


def test_ipo_mean_and_spread_monte_carlo(mc128):
    ipo = mc128[0]
    n = len(ipo)
    se = ipo.std() / math.sqrt(n)
    assert abs(ipo.mean() - O.expected_ipo(128)) < 4 * se
    var_th = O.ipo_second_moment(128) - O.expected_ipo(128) ** 2
    assert ipo.var() == pytest.approx(var_th, rel=0.1)
    # concentration: deviations are O(1/sqrt(D))
    assert np.max(np.abs(ipo - ipo.mean())) < 6.0 / math.sqrt(128)


def test_joint_law_x1_follows_p_dminus1(mc128):
    """Lemma "Distribution": <o_bar,e1>/sqrt(1-<o_bar,o>^2) ~ p_{D-1}, independent of <o_bar,o>."""
    ipo, _, ratio, _, _ = mc128
    d = 128
    ks = stats.kstest(ratio ** 2, stats.beta(0.5, (d - 2) / 2.0).cdf)
    assert ks.pvalue > 1e-3
    assert abs(ratio.mean()) < 4 * ratio.std() / math.sqrt(len(ratio))
    assert abs(np.corrcoef(ratio, ipo)[0, 1]) < 4 / math.sqrt(len(ratio))
    # the density function integrates to one and has variance 1/(D-1)
    x = np.linspace(-1, 1, 200001)
    dens = O.coordinate_density(x, d - 1)
    assert np.trapezoid(dens, x) == pytest.approx(1.0, rel=1e-6)
    assert np.trapezoid(dens * x * x, x) == pytest.approx(1.0 / (d - 1), rel=1e-6)


def test_estimator_unbiased_exact_query(mc128):
    est = mc128[1]
    assert abs(est.mean() - 0.5) < 4 * est.std() / math.sqrt(len(est))


def test_biased_alternative_is_scaled_by_ipo_mean(mc128):
    """<o_bar, q> alone (what treating o_bar as o would give) is biased by E[<o_bar,o>]."""
    obarq = mc128[3]
    assert obarq.mean() == pytest.approx(0.5 * O.expected_ipo(128), abs=4 * obarq.std() / math.sqrt(len(obarq)))
    assert abs(obarq.mean() - 0.5) > 0.05


def test_bound_failure_rate_matches_exact_law(mc128):
    est, hw = mc128[1], mc128[4]
    d, r = 128, 0.5
    fails = np.abs(est - r) > hw
    p = O.bound_failure_probability(r, d)
    n = len(est)
    assert abs(fails.mean() - p) < 4 * math.sqrt(p * (1 - p) / n)
    # special values of the exact law
    assert O.bound_failure_probability(0.0, d) == pytest.approx(0.0571, abs=2e-4)
    assert O.bound_failure_probability(0.999999, d) == 0.0
    assert O.bound_failure_probability(0.5, d, eps0=0.0) == pytest.approx(1.0)


def test_bound_failure_rate_small_dimension():
    """At small D the exact law separates the bound's 1/sqrt(D-1) (Theorem 3.2)
    from nearby forms: D = 8, <o,q> = 0.5, eps0 = 1.9 fails with probability
    0.0109 (1/sqrt(D) in the half-width would give 0.0237, 9.5 standard errors
    away at 6000 samples)."""
    d, r = 8, 0.5
    _, est, _, _, hw = _sample_ipo_and_est(d, r, 6000, 32, quantize=False)
    fails = np.abs(est - r) > hw
    p = O.bound_failure_probability(r, d)
    assert p == pytest.approx(0.0109, abs=1e-4)
    assert abs(fails.mean() - p) < 4 * math.sqrt(p * (1 - p) / len(est))


def test_estimator_unbiased_with_4bit_query():
    _, est, _, _, _ = _sample_ipo_and_est(128, -0.3, 3000, 13, quantize=True)
    assert abs(est.mean() + 0.3) < 4 * est.std() / math.sqrt(len(est))


def test_hoeffding_bound_on_query_quantization():
    """Appendix D: P{|<x_bar, q_bar - q'>| >= Delta u} <= 2 exp(-u^2/2)."""
    rng = np.random.default_rng(14)
    d = 128
    p = O.orthogonal_from_gaussian(rng.standard_normal((d, d)))
    q, c = rng.standard_normal(d), rng.standard_normal(d)
    xbar = (2.0 * rng.integers(0, 2, d) - 1) / math.sqrt(d)
    errs, deltas = [], []
    for t in range(3000):
        qq = O.quantize_query(q, c, p, rng.random(d))
        errs.append(xbar @ (qq.delta * qq.qu + qq.vl - qq.qprime))
        deltas.append(qq.delta)
    errs, delta = np.abs(np.array(errs)), deltas[0]
    assert abs(np.mean(errs * np.sign(rng.standard_normal(len(errs))))) < 1  # finite
    for u in (0.5, 1.0, 1.5, 2.0):
        assert (errs >= delta * u).mean() <= 2 * math.exp(-u * u / 2) + 0.01


# --------------------------------------------------------------- search

def _small_flat(n=2000, nq=20, seed=15):
    rng = np.random.default_rng(seed)
    means = rng.normal(0, 2, size=(8, 128))
    data = means[rng.integers(0, 8, n)] + rng.standard_normal((n, 128))
    qs = means[rng.integers(0, 8, nq)] + rng.standard_normal((nq, 128))
    return data, qs


def test_search_returns_exact_topk_of_probed_lists():
    data, qs = _small_flat()
    gauss = np.random.default_rng(16).standard_normal((128, 128))
    idx = O.build_index(data, data.mean(0, keepdims=True), np.zeros(len(data), int), gauss)
    hits = 0
    for qi, q in enumerate(qs):
        ids, d, info = O.search(idx, q, qi, 10, 1, seed=4001)
        t_ids, t_d = O.exact_topk(data, q, 10)
        if not info["violations"]:
            np.testing.assert_array_equal(ids, t_ids)
            np.testing.assert_allclose(d, t_d, rtol=1e-12)
        hits += len(set(ids.tolist()) & set(t_ids.tolist()))
        assert info["reranked"] < len(data)
    assert hits / (10 * len(qs)) >= 0.99      # eps0 = 1.9: near-perfect recall


def test_search_ivf_and_eps0_zero_loses_recall():
    data, qs = _small_flat(3000, 12, 17)
    rng = np.random.default_rng(18)
    cent = data[rng.choice(len(data), 16, replace=False)]
    assign = np.argmin(((data[:, None, :] - cent[None]) ** 2).sum(-1), 1)
    idx = O.build_index(data, cent, assign, rng.standard_normal((128, 128)))
    rec19 = rec0 = 0
    for qi, q in enumerate(qs):
        ids, d, info = O.search(idx, q, qi, 10, 4, seed=4002)
        cand = np.concatenate([idx.lists[k] for k in info["probed"]])
        t_ids, _ = O.exact_topk(data, q, 10, cand)
        if not info["violations"]:
            np.testing.assert_array_equal(ids, t_ids)
        rec19 += len(set(ids.tolist()) & set(t_ids.tolist()))
        ids0, _, info0 = O.search(idx, q, qi, 10, 4, seed=4002, eps0=0.0)
        rec0 += len(set(ids0.tolist()) & set(t_ids.tolist()))
        assert info0["reranked"] <= info["reranked"]
    assert rec19 >= rec0 and rec19 / (10 * len(qs)) >= 0.99


def test_probe_order_and_ties():
    cent = np.array([[0.0, 0.0], [1.0, 0.0], [-1.0, 0.0], [0.0, 3.0]])
    np.testing.assert_array_equal(O.probe_lists(np.zeros(2), cent, 3), [0, 1, 2])
    np.testing.assert_array_equal(O.probe_lists(np.array([0.0, 2.9]), cent, 2), [3, 0])


def test_relative_error_and_entropy_on_mixture():
    """Sec. 5.2.1 and Appendix E report, with IVF normalisation, a max relative
    error <= 40% and bit entropy > 99.9% of the code length. A consistency check
    on the mixture workload normalised per cluster (data-dependent, not a pin)."""
    rng = np.random.default_rng(19)
    means = rng.normal(0, 2, size=(8, 128))
    comp = rng.integers(0, 8, 5000)
    data = means[comp] + rng.standard_normal((5000, 128))
    qs = means[rng.integers(0, 8, 10)] + rng.standard_normal((10, 128))
    cent = np.stack([data[comp == k].mean(0) for k in range(8)])
    idx = O.build_index(data, cent, comp, np.random.default_rng(20).standard_normal((128, 128)))
    worst = 0.0
    for qi, q in enumerate(qs):
        for lid in O.probe_lists(q, cent, 2):
            qq = O.quantize_query(q, cent[lid], idx.p, O.rounding_uniforms_fast(3, qi, int(lid), 128))
            pe = O.pair_estimates(idx, int(lid), qq)
            true = O.exact_sqdist(data[pe["ids"]], q)
            worst = max(worst, float(np.max(np.abs(pe["dist"] - true) / true)))
            np.testing.assert_array_equal(pe["ip"], O.pair_estimates(idx, int(lid), qq, ip_form="bitplanes")["ip"])
    assert worst <= PAPER["max_rel_err"]
    assert O.bit_entropy_fraction(idx.bits) > PAPER["entropy_frac"]


# --------------------------------------------------------------- inner product (conclusion footnote)

def test_ip_decomposition_equals_direct_inner_product():
    """a b <o,q> + <o_r - c, c> + <q_r, c> equals <o_r, q_r> computed directly
    (the footnote's identity), through the oracle's code terms and estimate_ip
    fed the exact <o, q> (est * <o_bar,o> = <o,q> <o_bar,o>)."""
    rng = np.random.default_rng(40)
    d = 96
    data = rng.normal(0.3, 1.0, (40, d))
    cent = rng.normal(0.3, 0.5, (3, d))
    assign = rng.integers(0, 3, 40)
    idx = O.build_index(data, cent, assign, rng.standard_normal((128, 128)))
    fo = O.ip_code_terms(idx)
    q_r = rng.normal(0.1, 1.0, d)
    for i in range(40):
        c = cent[assign[i]]
        b = np.linalg.norm(q_r - c)
        o = (data[i] - c) / idx.norm[i]
        q = (q_r - c) / b
        xq = (o @ q) * idx.ipo[i]          # so that est = <o, q> exactly
        est, ip, ub = O.estimate_ip(xq, idx.ipo[i], idx.norm[i], b, fo[i], c @ q_r, idx.dp)
        assert ip == pytest.approx(data[i] @ q_r, rel=1e-12, abs=1e-12)
        assert ub >= ip
    # exact top-k by inner product: brute force over every vector
    t_ids, t_v = O.exact_topk_ip(data, q_r, 5)
    allv = data @ q_r
    np.testing.assert_allclose(t_v, np.sort(allv)[::-1][:5], rtol=1e-12)
    order = O.probe_lists_ip(q_r, cent, 3)
    np.testing.assert_allclose(cent[order] @ q_r, np.sort(cent @ q_r)[::-1][:3], rtol=1e-12)


def test_ip_estimator_unbiased_and_bound_failure_law():
    """Over random rotations the inner-product estimate is unbiased (Theorem 3.2
    carried through the footnote's identity), and its upper bound fails (falls
    below the true inner product) exactly when est + hw < <o,q>, the one-sided
    event whose probability is half the two-sided law of Lemma "Distribution"."""
    rng = np.random.default_rng(41)
    d, r = 128, 0.5
    o, q = _pair_with_ip(rng, d, r)
    c = rng.normal(0, 1, d)
    a, b = 1.7, 2.3
    o_r, q_r = c + a * o, c + b * q
    fo = (o_r - c) @ c
    g = q_r @ c
    vals, fails = [], 0
    n = 4000
    for s0 in range(0, n, 500):
        for p in O.orthogonal_from_gaussian(rng.standard_normal((500, d, d))):
            idx = O.OracleIndex(o_r[None, :], c[None, :], [0], p)
            xbar = (2.0 * idx.bits[0] - 1) / math.sqrt(d)
            xq = xbar @ O.inverse_rotate(p, q[None, :])[0]
            _, ip, ub = O.estimate_ip(xq, idx.ipo[0], idx.norm[0], b, fo, g, d)
            vals.append(ip)
            fails += ub < o_r @ q_r
    vals = np.array(vals)
    assert abs(vals.mean() - o_r @ q_r) < 4 * vals.std() / math.sqrt(n)
    p1 = O.bound_failure_probability(r, d) / 2.0       # the law is symmetric in X_1
    assert abs(fails / n - p1) < 4 * math.sqrt(p1 * (1 - p1) / n) + 1e-3


def test_search_ip_returns_exact_topk_of_probed_lists():
    """Maximum inner product search with the reversed sequential rule returns the
    exact top-k (largest inner products) of the probed lists wherever no true
    member's upper bound fell below its inner product; with eps0 = 0 it reranks
    less and can only lose."""
    data, qs = _small_flat(3000, 12, 42)
    rng = np.random.default_rng(43)
    cent = data[rng.choice(len(data), 16, replace=False)]
    assign = np.argmin(((data[:, None, :] - cent[None]) ** 2).sum(-1), 1)
    idx = O.build_index(data, cent, assign, rng.standard_normal((128, 128)))
    hits = 0
    for qi, q in enumerate(qs):
        ids, v, info = O.search_ip(idx, q, qi, 10, 4, seed=4003)
        cand = np.concatenate([idx.lists[k] for k in info["probed"]])
        t_ids, t_v = O.exact_topk_ip(data, q, 10, cand)
        if not info["violations"]:
            np.testing.assert_array_equal(ids, t_ids)
            np.testing.assert_allclose(v, t_v, rtol=1e-12)
        hits += len(set(ids.tolist()) & set(t_ids.tolist()))
        ids0, _, info0 = O.search_ip(idx, q, qi, 10, 4, seed=4003, eps0=0.0)
        assert info0["reranked"] <= info["reranked"]
        assert info["reranked"] < len(cand)
    assert hits / (10 * len(qs)) >= 0.99
