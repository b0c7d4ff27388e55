"""Pins of the oracle's two-ton solve: the moment preserving problem of
Sect. 3.1 with a = 2 (Eq. 12-14, Method 1 roots, Vandermonde values of
Eq. 9) applied to the multi-tons of the binary tree search (Sect. 3.3).

Each check uses something other than the oracle's own arithmetic: the planted
spectrum, numpy's FFT, and the residue arithmetic that decides which
frequencies share a class (f = c mod B) level by level.
"""
import numpy as np
import pytest

import oracle
import siggen
from tests.conftest import read_golden


def pair_solvable(f0, f1, N, D, shifts):
    """The stacked moment equations determine the pair's polynomial when one
    round gives two of them (D >= 4), or when two rounds r, r' see the pair
    with different relative phases: (f1 - f0)(s_r - s_r') != 0 mod N."""
    if D >= 4:
        return True
    return any(((f1 - f0) * (a - b)) % N for a in shifts for b in shifts)


def expected_tree(support, B0, N, two_tons=True, D=4, shifts=()):
    """Per-level (singles, doubles, multis) of the tree from the residues
    alone: a class holds the support members f = c (mod B); with the two-ton
    solve a class of two is closed (if its moment equations have full rank),
    otherwise only a class of one is."""
    out = []
    open_cls = None
    B = B0
    while True:
        members = {}
        for f in support:
            members.setdefault(int(f) % B, []).append(int(f))
        if open_cls is not None:
            members = {c: m for c, m in members.items() if c in open_cls}
        ns = sum(1 for m in members.values() if len(m) == 1)
        dbl = [c for c, m in members.items()
               if two_tons and len(m) == 2 and pair_solvable(m[0], m[1], N, D, shifts)]
        nd = len(dbl)
        multi = [c for c, m in members.items() if len(m) > 1 and c not in dbl]
        out.append((ns, nd, len(multi)))
        if not multi or B >= N:
            return out
        open_cls = set()
        for c in multi:
            open_cls.update((c, c + B))
        B *= 2


def trace_counts(tr):
    return [(tr.n_single[l], tr.n_double[l], tr.n_multi[l]) for l in range(tr.levels + 1)]


def test_n64_example_two_tons():
    """The Sect. 3.3 example (1, 6, 13, 20, 59 at N = 64): with B0 = 4 the
    pair {1, 13} shares class 1 and is solved at once; with B0 = 2 class 0
    holds {6, 20} (solved) and class 1 holds {1, 13, 59}, which opens
    children 1 = {1, 13} (solved) and 3 = {59}."""
    g = read_golden("n64_tree.txt")
    N = int(g["N"][0])
    sup = [int(v) for v in g["support"]]
    sp = siggen.make_spec(N, len(sup), 2, support=sup)
    x = siggen.synth(sp)
    cfg = oracle.config(N, 5, 1, 4, B0=4, identity_round0=True, mpp=2)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    assert trace_counts(tr) == [(3, 1, 0)]
    np.testing.assert_array_equal(idx, sorted(sup))
    np.testing.assert_allclose(val, sp.values[np.argsort(sup)], atol=1e-6)
    cfg = oracle.config(N, 5, 1, 4, B0=2, identity_round0=True, mpp=2)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    assert trace_counts(tr) == [(0, 1, 1), (1, 1, 0)]
    np.testing.assert_array_equal(idx, sorted(sup))


def test_worst_case_pair_solved_at_level0():
    """Sect. 3.3, Subproblem 2: xhat_0 and xhat_{N/2} share every class down to
    the layer of N buckets; the moment preserving solve of Sect. 3.1 separates
    them in the first class."""
    N = 256
    sp = siggen.make_spec(N, 2, 4, support=[0, N // 2])
    x = siggen.synth(sp)
    cfg = oracle.config(N, 2, 1, 4, B0=1, identity_round0=True, mpp=2)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    assert tr.levels == 0 and tr.n_double[0] == 1 and tr.status == oracle.OK
    np.testing.assert_array_equal(idx, [0, N // 2])
    np.testing.assert_allclose(val, sp.values, atol=1e-6)
    cfg.mpp = 0
    idx, val, cnt, tr = oracle.solve(cfg, x)
    assert tr.levels == 8


@pytest.mark.parametrize("R,D", [(1, 4), (2, 3), (3, 4), (1, 6)])
@pytest.mark.parametrize("N,K,B0", [(256, 12, 4), (256, 20, 8), (1024, 40, 16)])
def test_class_structure_follows_residues(N, K, B0, R, D):
    """Level by level, the classes the oracle reports as single / two-ton /
    multi-ton are exactly those the residues f mod B predict."""
    for seed in range(6):
        sp = siggen.make_spec(N, K, 100 + seed)
        x = siggen.synth(sp)
        cfg = oracle.config(N, K, R, D, seed=seed, B0=B0, identity_round0=(R == 1), mpp=2)
        idx, val, cnt, tr = oracle.solve(cfg, x)
        shifts = [cfg.shift[r] for r in range(R)]
        assert trace_counts(tr) == expected_tree(sp.support, B0, N, D=D, shifts=shifts), seed
        assert tr.status == oracle.OK
        np.testing.assert_array_equal(idx, sp.support)
        np.testing.assert_allclose(val, sp.values, atol=1e-6)
        # and without the two-ton solve the tree follows the singles-only rule
        cfg.mpp = 0
        idx2, val2, cnt2, tr2 = oracle.solve(cfg, x)
        assert trace_counts(tr2) == [(s, 0, m) for s, _, m in expected_tree(sp.support, B0, N, False)]
        assert tr.samples <= tr2.samples


def test_three_tons_are_never_taken_for_two():
    """Three frequencies of one class (f = c + kB for three k) fit no
    two-root polynomial: the class must open its children."""
    N, B0 = 4096, 16
    for seed in range(40):
        rng = np.random.default_rng(seed)
        c = int(rng.integers(B0))
        ks = rng.choice(N // B0, size=3, replace=False)
        sup = np.sort(c + ks * B0)
        sp = siggen.make_spec(N, 3, seed, support=sup)
        x = siggen.synth(sp)
        cfg = oracle.config(N, 3, 2, 4, seed=seed, B0=B0, mpp=2)
        idx, val, cnt, tr = oracle.solve(cfg, x)
        assert tr.n_double[0] == 0 and tr.n_multi[0] == 1, seed
        assert trace_counts(tr) == expected_tree(sup, B0, N)
        np.testing.assert_array_equal(idx, sup)
        np.testing.assert_allclose(val, sp.values, atol=1e-6)


@pytest.mark.parametrize("N,K,R,D,B0", [(2 ** 16, 64, 4, 4, 128), (2 ** 16, 64, 2, 3, 64),
                                         (2 ** 18, 256, 1, 4, 256)])
def test_exact_recovery_matches_numpy_fft(N, K, R, D, B0):
    """Random exactly sparse signals: the result equals the K largest entries
    of numpy.fft(x)/N, with fewer samples than the tree without the solve."""
    for seed in range(3):
        sp = siggen.make_spec(N, K, 500 + seed)
        x = siggen.synth(sp)
        xh = np.fft.fft(x.astype(np.complex128)) / N
        want = np.sort(np.argsort(-np.abs(xh))[:K])
        cfg = oracle.config(N, K, R, D, seed=seed, B0=B0, mpp=2)
        idx, val, cnt, tr = oracle.solve(cfg, x)
        assert cnt == K and tr.status == oracle.OK
        np.testing.assert_array_equal(idx, want)
        np.testing.assert_allclose(val, xh[want], atol=1e-6)
        assert sum(tr.n_double[l] for l in range(tr.levels + 1)) > 0
        cfg.mpp = 0
        _, _, _, tr0 = oracle.solve(cfg, x)
        assert tr.samples < tr0.samples and tr.levels <= tr0.levels


@pytest.mark.parametrize("kw", [dict(N=1024, R=2, D=2),                 # no moment equation
                                dict(N=1024, R=1, D=3),                 # one equation, two unknowns
                                dict(N=1024, R=2, D=4, mode=oracle.NOISY),
                                dict(N=10800, R=3, D=4)])               # FFAST
def test_two_ton_solve_preconditions(kw):
    N = kw["N"]
    cfg = oracle.config(N, 4, kw["R"], kw["D"], mode=kw.get("mode", oracle.EXACT), mpp=2)
    x = siggen.synth(siggen.make_spec(N, 4, 1))
    assert oracle.solve(cfg, x)[2] == -1
