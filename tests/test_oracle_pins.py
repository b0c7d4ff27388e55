"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check uses an independent
computation (brute-force DFT, numpy's FFT, planted truth, closed forms,
printed worked examples and tables of the paper).
"""
import math

import numpy as np
import pytest

import oracle
import siggen
from tests.conftest import read_golden


def brute_dft(x):
    """xhat = F_N x of Eq. 1-2, as an explicit O(N^2) matrix product."""
    N = len(x)
    j = np.arange(N)
    W = np.exp(-2j * np.pi * np.outer(j, j) / N) / N
    return W @ x.astype(np.complex128)


# ---------------------------------------------------------------- Eq. 5-6
@pytest.mark.parametrize("N,B", [(64, 8), (64, 1), (64, 64), (60, 4), (60, 15), (48, 16)])
def test_aliasing_identity_bruteforce(N, B):
    """Eq. 6 (advance shift): bin sigma*c of the B-point transform of the
    shifted, permuted subsample equals sum_{f = c mod B} xhat_f e^{+2 pi i f tau/N}."""
    rng = np.random.default_rng(N * 1000 + B)
    x = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
    xh = brute_dft(x)
    sigmas = [s for s in range(1, N, 2 if N % 2 == 0 else 1) if math.gcd(s, B) == 1][:4]
    for sigma in sigmas:
        for tau in (0, 1, 2, 7, N - 1):
            for c in range(B):
                f = np.arange(c, N, B)
                want = np.sum(xh[f] * np.exp(2j * np.pi * f * tau / N))
                got = oracle.bin_value(x, N, B, sigma, tau, (sigma * c) % B)
                assert abs(got - want) < 1e-12 * max(1.0, abs(want)), (sigma, tau, c)


def test_relabeling_invariance():
    """A permutation only relabels buckets under the aliasing filter (Sect. 1:
    scaling is of no use): bin sigma*c with sigma equals bin c without it."""
    N, B = 1024, 32
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
    for sigma in (3, 5, 77, 1023):
        for c in (0, 1, 5, 31):
            a = oracle.bin_value(x, N, B, sigma, 5, (sigma * c) % B)
            b = oracle.bin_value(x, N, B, 1, 5, c)
            assert abs(a - b) < 1e-12


def test_tree_additivity():
    """A bucket of B splits into its two children of 2B (Sect. 3.3, layer
    structure): yhat_B[c] = yhat_2B[c] + yhat_2B[c + B]."""
    N = 4096
    rng = np.random.default_rng(4)
    x = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
    for B in (1, 2, 16, 256, 2048):
        for c in (0, 1, B - 1):
            p = oracle.bin_value(x, N, B, 1, 9, c)
            k0 = oracle.bin_value(x, N, 2 * B, 1, 9, c)
            k1 = oracle.bin_value(x, N, 2 * B, 1, 9, c + B)
            assert abs(p - (k0 + k1)) < 1e-11


def test_level0_table_matches_numpy_fft():
    """Level-0 class table of a tree plan: entry (c, r, d) is the alias sum of
    numpy.fft(x)/N over f = c mod B0 with phase e^{+2 pi i f (s_r + d)/N}."""
    N, K = 4096, 16
    sp = siggen.make_spec(N, K, seed=11)
    x = siggen.synth(sp)
    cfg = oracle.config(N, K, 3, 2, seed=99, B0=32)
    Y = oracle.level0(cfg, x)
    xh = np.fft.fft(x.astype(np.complex128)) / N
    for c in range(32):
        f = np.arange(c, N, 32)
        for r in range(3):
            for d in range(2):
                tau = (cfg.shift[r] + d) % N
                want = np.sum(xh[f] * np.exp(2j * np.pi * ((f * tau) % N) / N))
                assert abs(Y[c, r * 2 + d] - want) < 1e-11


# ------------------------------------------------------------ plan draws
def test_splitmix64_reference_vectors():
    for line in open(__file__.replace("test_oracle_pins.py", "golden/splitmix64.txt")):
        if line.startswith("#") or not line.strip():
            continue
        seed, *vals = [int(v) for v in line.split()]
        assert oracle.splitmix64(seed, 3) == vals


def test_plan_draws_and_factoring():
    cfg = oracle.config(10800, 10, 3, 2)
    assert cfg.kind == oracle.FFAST
    assert [cfg.stageB[j] for j in range(3)] == [16, 27, 25]
    with pytest.raises(ValueError):
        oracle.config(10800, 10, 2, 2)   # three prime powers, two stages
    with pytest.raises(ValueError):
        oracle.config(1024, 10, 2, 1)    # exact mode needs two delays
    cfg = oracle.config(2 ** 20, 256, 4, 2, seed=7)
    assert cfg.B0 == 512 and cfg.max_levels == 11
    for r in range(4):
        assert cfg.sigma[r] % 2 == 1 and cfg.sigma[r] < 2 ** 20 and cfg.shift[r] < 2 ** 20
    cfg1 = oracle.config(2 ** 14, 8, 1, 2, seed=7, identity_round0=True)
    assert cfg1.sigma[0] == 1 and cfg1.shift[0] == 0


# ------------------------------------------------- exact recovery (Sect. 2.1)
def _check_exact(N, K, stages, D, seed, **kw):
    sp = siggen.make_spec(N, K, seed)
    x = siggen.synth(sp)
    cfg = oracle.config(N, K, stages, D, seed=seed, **kw)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    sup, vals = siggen.truth(sp)
    return sp, x, idx, val, cnt, tr, sup, vals


@pytest.mark.parametrize("seed", range(12))
def test_ffast_config1_exact_recovery(seed):
    sp, x, idx, val, cnt, tr, sup, vals = _check_exact(10800, 10, 3, 2, seed)
    if tr.status == oracle.OK:
        assert cnt == 10
        np.testing.assert_array_equal(idx, sup)
        assert np.max(np.abs(val - vals)) < 1e-6


@pytest.mark.parametrize("N,K,R,B0,seed", [
    (2 ** 12, 8, 1, 8, 1), (2 ** 14, 64, 2, 128, 2), (2 ** 16, 100, 4, 256, 3),
    (2 ** 16, 300, 4, 512, 4), (2 ** 10, 1, 1, 1, 5), (2 ** 13, 7, 3, 16, 6)])
def test_tree_exact_recovery(N, K, R, B0, seed):
    sp, x, idx, val, cnt, tr, sup, vals = _check_exact(N, K, R, 2, seed, B0=B0)
    assert tr.status == oracle.OK
    assert cnt == K
    np.testing.assert_array_equal(idx, sup)
    assert np.max(np.abs(val - vals)) < 1e-6
    # independent reference: the K largest coefficients of numpy's FFT
    xh = np.fft.fft(x.astype(np.complex128)) / N
    top = np.sort(np.argsort(-np.abs(xh))[:K])
    np.testing.assert_array_equal(idx, top)
    # aliased complex64 rounding of x bounds the difference (~1e-8 here)
    assert np.max(np.abs(val - xh[top])) < 1e-6


def test_tree_three_delays_and_identity_round():
    sp, x, idx, val, cnt, tr, sup, vals = _check_exact(2 ** 12, 20, 1, 3, 8, B0=32,
                                                       identity_round0=True)
    np.testing.assert_array_equal(idx, sup)


def test_more_than_K_keeps_largest():
    """Goal of Sect. 2.1: the K largest coefficients; ties go to the lower index."""
    N = 1024
    sup = np.array([3, 100, 200, 900])
    vals = np.array([1.0, 3.0, 2.0, 0.5]) * np.exp(1j * np.array([0.1, 0.2, 0.3, 0.4]))
    sp = siggen.make_spec(N, 4, 0, support=sup, values=vals)
    x = siggen.synth(sp)
    cfg = oracle.config(N, 2, 1, 2, B0=64)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    assert cnt == 2 and tr.n_found == 4
    np.testing.assert_array_equal(idx, [100, 200])


def test_empty_and_padding():
    N = 2048
    x = np.zeros(N, np.complex64)
    cfg = oracle.config(N, 5, 2, 2, B0=16)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    assert cnt == 0 and tr.status == oracle.OK
    assert np.all(idx == -1) and np.all(val == 0)


# ------------------------------------------------ worked examples of the paper
def test_n20_peeling_example():
    g = read_golden("n20_peeling.txt")
    N = int(g["N"][0])
    sup = [int(v) for v in g["support"]]
    stages = [int(v) for v in g["stages"]]
    sp = siggen.make_spec(N, len(sup), 1, support=sup)
    x = siggen.synth(sp)
    for D in (2, 3):   # the paper's R = 3 delays {0, 1, 2} and the two-delay form
        cfg = oracle.config(N, len(sup), len(stages), D, stageB=stages)
        idx, val, cnt, tr = oracle.solve(cfg, x)
        assert tr.status == oracle.OK
        assert [tr.n_zero[0], tr.n_single[0], tr.n_multi[0]] == \
            [int(v) for v in g["round1_zero_single_multi"]]
        assert [tr.ident[i] for i in range(tr.levels)] == [int(v) for v in g["identifications"]]
        order = [tr.order[i] for i in range(tr.n_found)]
        assert sorted(order[:3]) == [int(v) for v in g["found_round1"]]
        assert sorted(order[3:]) == [int(v) for v in g["found_round2"]]
        np.testing.assert_array_equal(idx, sorted(sup))


def test_n64_tree_example():
    g = read_golden("n64_tree.txt")
    N = int(g["N"][0])
    sup = [int(v) for v in g["support"]]
    sp = siggen.make_spec(N, len(sup), 2, support=sup)
    x = siggen.synth(sp)
    cfg = oracle.config(N, len(sup), 1, 2, B0=1, identity_round0=True)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    occ = [int(v) for v in g["occupied"]]
    assert tr.levels == len(occ) - 1
    assert [tr.occupied[i] for i in range(len(occ))] == occ
    np.testing.assert_array_equal(idx, sorted(sup))
    assert sorted(set(int(f) % 8 for f in idx)) == [int(v) for v in g["last_layer_buckets"]]


def test_small_support_separates_at_level3():
    """Sect. 3.3: eight consecutive frequencies fall into eight distinct
    buckets of B = 8, so the search ends at the fourth layer."""
    N = 1024
    sup = np.arange(400, 408)
    sp = siggen.make_spec(N, 8, 3, support=sup)
    x = siggen.synth(sp)
    cfg = oracle.config(N, 8, 1, 2, B0=1, identity_round0=True)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    assert tr.levels == 3 and tr.occupied[3] == 8 and tr.n_multi[3] == 0
    np.testing.assert_array_equal(idx, sup)


def test_worst_case_pair_separates_only_at_full_depth():
    """Sect. 3.3, Subproblem 2: xhat_0 and xhat_{N/2} stay aliased until
    the layer of N buckets."""
    N = 256
    sp = siggen.make_spec(N, 2, 4, support=[0, N // 2])
    x = siggen.synth(sp)
    cfg = oracle.config(N, 2, 1, 2, B0=1, identity_round0=True)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    assert tr.levels == 8 and tr.status == oracle.OK
    np.testing.assert_array_equal(idx, [0, N // 2])
    cfg = oracle.config(N, 2, 1, 2, B0=1, identity_round0=True, max_levels=5)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    assert tr.status == oracle.PARTIAL and cnt == 0


# ------------------------------------------------------------- Table 1 (Sect. 4.3)
def _p_no_collision(N, K, B):
    """Product formula of Sect. 4.3: prod_{j=1}^{K-1} (N - jL)/(N - j)."""
    L = N // B
    p = 1.0
    for j in range(1, K):
        p *= (N - j * L) / (N - j)
    return p


def test_table1_closed_form_limit():
    g = read_golden("table1.txt")
    Ks = [1, 2, 4, 6, 8]
    for row, mult in (("B=1K", 1), ("B=2K", 2), ("B=4K", 4), ("B=8K", 8)):
        for K, printed in zip(Ks, g[row]):
            B = mult * K
            lim = math.factorial(B) / (math.factorial(B - K) * B ** K)
            assert abs(lim - float(printed)) < 6e-5, (row, K)
            assert abs(_p_no_collision(2 ** 30, K, B) - lim) < 1e-6


@pytest.mark.parametrize("K,mult", [(4, 2), (4, 4), (8, 2), (8, 8)])
def test_table1_monte_carlo(K, mult):
    """Level-0 occupancy of the oracle's tree: P(no multi-ton at B) over seeds
    matches the closed form within a 4-sigma binomial band."""
    N, B = 2 ** 12, mult * K
    trials = 600
    hits = 0
    for s in range(trials):
        sp = siggen.make_spec(N, K, 50000 + s)
        x = siggen.synth(sp)
        cfg = oracle.config(N, K, 1, 2, B0=B, identity_round0=True)
        _, _, _, tr = oracle.solve(cfg, x)
        hits += tr.n_multi[0] == 0
    p = _p_no_collision(N, K, B)
    sd = math.sqrt(p * (1 - p) / trials)
    assert abs(hits / trials - p) < 4 * sd + 1e-9


def test_theorem5_ffast_success_rate():
    """Theorem 5: with K < N^{1/3} and co-prime B_i, FFAST succeeds with
    probability at least 1 - 1/K."""
    K, trials, ok = 10, 200, 0
    for s in range(trials):
        sp = siggen.make_spec(10800, K, 70000 + s)
        x = siggen.synth(sp)
        cfg = oracle.config(10800, K, 3, 2)
        idx, val, cnt, tr = oracle.solve(cfg, x)
        ok += tr.status == oracle.OK and np.array_equal(idx, siggen.truth(sp)[0])
    assert ok / trials >= 1 - 1 / K


# ------------------------------------------------------------------ noisy mode
def test_noisy_mode_noiseless_limit_equals_exact():
    N, K = 2 ** 14, 40
    sp = siggen.make_spec(N, K, 21)
    x = siggen.synth(sp)
    ce = oracle.config(N, K, 4, 2, seed=5)
    cn = oracle.config(N, K, 4, 2, seed=5, mode=oracle.NOISY, noise_var=1e-9)
    ie, ve, _, _ = oracle.solve(ce, x)
    i_n, vn, _, _ = oracle.solve(cn, x)
    np.testing.assert_array_equal(ie, i_n)
    assert np.max(np.abs(ve - vn)) < 1e-9


@pytest.mark.parametrize("window", [0, 64])
def test_noisy_mode_recovers_at_20db(window):
    N, K = 2 ** 16, 32
    sp = siggen.make_spec(N, K, 31, snr_db=20.0)
    x = siggen.synth(sp)
    cfg = oracle.config(N, K, 4, 2, seed=8, mode=oracle.NOISY, window=window)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    sup, vals = siggen.truth(sp)
    np.testing.assert_array_equal(idx, sup)
    # a value is the mean of R*D = 8 bucket measurements, each with noise
    # variance sigma^2 / B (B >= B0 = 64 here)
    sv = math.sqrt(sp.noise_var / (cfg.B0 * 8))
    assert np.max(np.abs(val - vals)) < 6 * sv
    # estimated noise level within 25% of the planted one
    assert abs(tr.noise_var / sp.noise_var - 1) < 0.25
