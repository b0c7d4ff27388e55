"""Pins of the oracle's general-sparse (noisy) decision rule against closed
forms.

The paper names the thresholds of the zero-ton and single-ton tests (Sect.
3.2, Subproblem 1) without values; the reading taken is
  zero-ton    iff |Y|^2 <= s_b^2 (n + zero_k sqrt(n)),
  single-ton  iff |Y - a v_f|^2 <= s_b^2 (n - 1 + single_k sqrt(n - 1)),
with s_b^2 = sigma^2 / B the noise variance of one bucket of B (a bucket is
the 1/B-scaled sum of B samples, each with variance sigma^2), and sigma^2
estimated from a quantile of the level-0 entries.  What the mathematics
fixes, independently of that reading:
  * for a class vector of n entries of complex white noise, |Y|^2 / s_b^2 is
    Gamma(n, 1) (a sum of n unit exponentials), so the zero-ton rate is
    P[Gamma(n, 1) <= n + zero_k sqrt(n)];
  * for one tone plus noise, located at its true position, the least-squares
    residual is the noise projected off the one-dimensional span of v_f, so
    residual / s_b^2 is Gamma(n - 1, 1) and the single-ton rate is
    P[Gamma(n - 1, 1) <= n - 1 + single_k sqrt(n - 1)];
  * B |yhat|^2 of a noise-only bucket is exponential with mean sigma^2; the
    k-th smallest of m such values is -sigma^2 ln(1 - U) with U ~ Beta(k,
    m + 1 - k), which gives the exact law of the quantile estimate.
Rates are compared with their binomial band, the estimate with its 99.9 %
interval.  Several widths are used so that a wrong width, or n written for
n - 1, moves a rate out of its band.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle

N, K, R, D = 2 ** 10, 4, 4, 2
B = 64
NOISE_VAR = 2.0           # time-domain sigma^2
SB2 = NOISE_VAR / B       # per-bucket variance


def cfg_with(zero_k=4.0, single_k=4.0, libpath=None):
    return oracle.config(N, K, R, D, seed=11, mode=oracle.NOISY, B0=B, zero_k=zero_k,
                         single_k=single_k, libpath=libpath)


def cnoise(rng, shape, var):
    return math.sqrt(var / 2.0) * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def within_band(hits, trials, p, z=5.0):
    sd = math.sqrt(trials * p * (1 - p))
    return abs(hits - trials * p) <= z * sd + 1.0


def zero_rate(cfg, trials, seed, libpath=None):
    rng = np.random.default_rng(seed)
    n = cfg.R * cfg.D
    Ys = cnoise(rng, (trials, n), SB2)
    return sum(oracle.classify_tree(cfg, Y, 5, B, 0.0, NOISE_VAR, libpath=libpath)[0] == oracle.ZERO
               for Y in Ys)


def single_rate(cfg, trials, seed, libpath=None):
    """Unit tones at a random position of class 5, noise at 30 dB per bucket:
    located exactly, so the residual is the projected noise alone."""
    rng = np.random.default_rng(seed)
    n = cfg.R * cfg.D
    taus = np.array([(cfg.shift[r] + d) % N for r in range(cfg.R) for d in range(cfg.D)],
                    dtype=np.int64)
    hits, located = 0, 0
    L = N // B
    for _ in range(trials):
        f = 5 + B * int(rng.integers(L))
        a = np.exp(2j * np.pi * rng.uniform())
        Y = a * np.exp(2j * np.pi * ((f * taus) % N) / N) + cnoise(rng, n, SB2)
        code, fo, _ = oracle.classify_tree(cfg, Y, 5, B, 0.0, NOISE_VAR, libpath=libpath)
        located += fo == f
        hits += code == oracle.SINGLE
    return hits, located


@pytest.mark.parametrize("zero_k", [0.5, 1.0, 4.0])
def test_zero_ton_rate_is_gamma_n(zero_k):
    cfg = cfg_with(zero_k=zero_k)
    n = R * D
    trials = 20000
    p = stats.gamma.cdf(n + zero_k * math.sqrt(n), n)
    hits = zero_rate(cfg, trials, 100 + int(10 * zero_k))
    assert within_band(hits, trials, p), (hits / trials, p)


@pytest.mark.parametrize("single_k", [0.5, 1.0, 4.0])
def test_single_ton_rate_is_gamma_n_minus_1(single_k):
    cfg = cfg_with(single_k=single_k)
    n = R * D
    trials = 20000
    p = stats.gamma.cdf(n - 1 + single_k * math.sqrt(n - 1), n - 1)
    hits, located = single_rate(cfg, trials, 200 + int(10 * single_k))
    assert located == trials
    assert within_band(hits, trials, p), (hits / trials, p)


def _estimate_interval(p_rank, m_noise, denom, alpha=1e-3):
    """99.9 % interval of q_(k) / denom, q_(k) the k-th smallest of m_noise
    unit exponentials."""
    lo, hi = stats.beta.ppf([alpha / 2, 1 - alpha / 2], p_rank, m_noise + 1 - p_rank)
    return -math.log1p(-lo) / denom, -math.log1p(-hi) / denom


@pytest.mark.parametrize("phi", [1.0, 0.6])
def test_noise_estimate_within_quantile_interval(phi):
    """Pure noise (phi = 1) and a mix in which a fraction 1 - phi of the
    entries are occupied buckets far above the noise: the estimate is the
    (p/phi)-quantile of the noise entries divided by -ln(1 - p/phi)."""
    cnt = 4096
    p = min(0.25, phi / 2)
    at = int(p * (cnt - 1))
    m_noise = int(round(phi * cnt))
    lo, hi = _estimate_interval(at + 1, m_noise, -math.log(1 - p / phi))
    rng = np.random.default_rng(7)
    inside = 0
    for trial in range(200):
        pw = np.concatenate([rng.exponential(NOISE_VAR, m_noise),
                             1e6 * NOISE_VAR * (1 + rng.uniform(size=cnt - m_noise))])
        rng.shuffle(pw)
        est = oracle.estimate_noise(pw, phi) / NOISE_VAR
        inside += lo <= est <= hi
    # 200 draws of a 99.9 % interval: at most a couple outside
    assert inside >= 197, inside
    # and the estimator is centred on sigma^2 (median of the order statistic)
    med = -math.log1p(-stats.beta.median(at + 1, m_noise + 1 - at)) / -math.log(1 - p / phi)
    assert abs(med - 1) < 0.02
