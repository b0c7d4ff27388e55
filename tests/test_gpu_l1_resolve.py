"""Parity of the level-1 column pass (plan field l1_resolve) with the FP64
oracle's level-by-level tree search (Sect. 3.3), and with the gathering path
of the same plan.

The column pass measures every level-0 multi-ton's coefficients M_c(t) from
one read of x and classifies each later level's class vectors from them; the
oracle gathers those vectors level by level.  Bar: indices bit-exact (padding
included), counts and status equal, values within relative L2 1e-5.
Shapes cover the five widths B0 = 512 ... 8192, the smallest stride each
takes (L = 32768 / B0), both modes, the two-ton solve, the FP32 decisions, a
depth cap, and a batch that mixes the widths with signals that gather.
"""
import numpy as np
import pytest

import oracle
import siggen
from tests.test_gpu_parity import assert_parity, oracle_cfg, rel_l2, solve_both, to_dev, VAL_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfft():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2011_05749_amd as m
    return m


EXACT_CASES = [
    # N, K, rounds, delays, B0, seed
    (2 ** 15, 300, 2, 2, 2048, 1),    # L = 16: one item pair per signal
    (2 ** 15, 700, 4, 2, 1024, 2),    # L = 32, 16 columns per item
    (2 ** 16, 1500, 3, 2, 4096, 3),   # L = 16, 4 columns per item, groups of 4
    (2 ** 18, 900, 4, 2, 2048, 4),
    (2 ** 17, 500, 2, 3, 1024, 5),
    (2 ** 20, 2000, 3, 2, 4096, 6),
    (2 ** 17, 3000, 2, 2, 8192, 7),   # L = 16, 2 columns per item, groups of 8
    (2 ** 15, 150, 4, 2, 512, 9),     # L = 64, 32 columns per item
    (2 ** 20, 256, 4, 2, 512, 10),
    (2 ** 18, 4000, 4, 2, 8192, 8),
]


@pytest.mark.parametrize("N,K,R,D,B0,seed", EXACT_CASES)
def test_exact_matches_oracle(sfft, N, K, R, D, B0, seed):
    x = siggen.synth(siggen.make_spec(N, K, seed))
    g, o = solve_both(sfft, x, N, K, R, D, seed=seed, B0=B0)
    assert_parity(g, o)
    p = sfft.Plan(N, K, R, D, seed=seed, B0=B0)
    assert p.info.l1_resolve == 1
    st = g[3]
    # level 0 reads n B0 samples, the column pass all N of them
    if g[2] > 0 and (st["level_mask"] >> 1) & 1:
        assert st["samples"] == R * D * B0 + N


@pytest.mark.parametrize("N,K,R,D,B0,seed", EXACT_CASES[:4])
def test_same_as_gathering_path(sfft, N, K, R, D, B0, seed):
    x = to_dev(siggen.synth(siggen.make_spec(N, K, seed + 100)))
    a = sfft.Plan(N, K, R, D, seed=seed, B0=B0)
    b = sfft.Plan(N, K, R, D, seed=seed, B0=B0, l1_resolve=0)
    assert a.info.l1_resolve == 1 and b.info.l1_resolve == 0
    ia, va, ca = a.exec(x)
    ib, vb, cb = b.exec(x)
    assert ca == cb
    np.testing.assert_array_equal(ia.cpu().numpy(), ib.cpu().numpy())
    m = ia.cpu().numpy() >= 0
    if m.any():
        assert rel_l2(va.cpu().numpy()[m].astype(np.complex128),
                      vb.cpu().numpy()[m].astype(np.complex128)) <= VAL_TOL
    assert a.stats()["status"] == b.stats()["status"]


@pytest.mark.parametrize("seed", [11, 12])
def test_noisy_matches_oracle(sfft, seed):
    N, K, B0 = 2 ** 18, 400, 1024
    x = siggen.synth(siggen.make_spec(N, K, seed, snr_db=25.0))
    g, o = solve_both(sfft, x, N, K, 4, 2, seed=seed, B0=B0, mode=1)
    assert_parity(g, o)


def test_two_ton_solve_matches_oracle(sfft):
    N, K, B0 = 2 ** 16, 900, 1024
    x = siggen.synth(siggen.make_spec(N, K, 21))
    g, o = solve_both(sfft, x, N, K, 2, 3, seed=21, B0=B0, mpp=2)
    assert_parity(g, o)


def test_fp32_decisions_match_oracle(sfft):
    N, K, B0 = 2 ** 17, 800, 2048
    x = siggen.synth(siggen.make_spec(N, K, 22))
    g, o = solve_both(sfft, x, N, K, 4, 2, seed=22, B0=B0, precision=1)
    assert_parity(g, o)


@pytest.mark.parametrize("cap", [1, 2, 3])
def test_depth_cap_matches_oracle(sfft, cap):
    """A multi-ton still open at the deepest allowed level leaves the solve
    partial, as in the oracle."""
    N, K, B0 = 2 ** 16, 1200, 1024
    x = siggen.synth(siggen.make_spec(N, K, 30 + cap))
    g, o = solve_both(sfft, x, N, K, 2, 2, seed=30 + cap, B0=B0, max_levels=cap)
    assert_parity(g, o)


def test_no_multiton_reads_nothing_more(sfft):
    """A signal whose level-0 buckets all close takes no column items."""
    N, K, B0 = 2 ** 16, 3, 1024
    sp = siggen.make_spec(N, K, 40, support=[5, 77, 1030])
    x = siggen.synth(sp)
    g, o = solve_both(sfft, x, N, K, 2, 2, seed=40, B0=B0)
    assert_parity(g, o)
    assert g[3]["samples"] == 2 * 2 * B0


def test_unsupported_widths_fall_back(sfft):
    assert sfft.Plan(2 ** 16, 100, 2, 2, B0=512).info.l1_resolve == 1
    assert sfft.Plan(2 ** 16, 100, 2, 2, B0=256).info.l1_resolve == 0
    assert sfft.Plan(2 ** 17, 100, 2, 2, B0=8192).info.l1_resolve == 1
    assert sfft.Plan(2 ** 16, 100, 2, 2, B0=8192).info.l1_resolve == 0   # L = 8 < 16
    assert sfft.Plan(2 ** 15, 100, 2, 2, B0=4096).info.l1_resolve == 0   # L = 8 < 16
    assert sfft.Plan(2 ** 14, 100, 2, 2, B0=2048).info.l1_resolve == 0   # L = 8 < 16
    assert sfft.Plan(2 ** 16, 100, 2, 2, B0=2048, max_levels=0).info.l1_resolve == 0


def test_mixed_batch_matches_oracle(sfft):
    """All five widths beside signals that gather level by level, in one
    batch, eager and graph-replayed."""
    shapes = [(2 ** 16, 500, 1024), (2 ** 17, 900, 2048), (2 ** 15, 1500, 4096),
              (2 ** 16, 120, 256), (2 ** 18, 700, 2048), (2 ** 14, 200, 512),
              (2 ** 17, 1000, 1024), (2 ** 16, 800, 4096), (2 ** 17, 2500, 8192),
              (2 ** 16, 150, 512), (2 ** 18, 3000, 8192)]
    plans, xs, host, cfgs = [], [], [], []
    for i, (N, K, B0) in enumerate(shapes):
        seed = 700 + i
        x = siggen.synth(siggen.make_spec(N, K, seed))
        plans.append(sfft.Plan(N, K, 3, 2, seed=seed, B0=B0))
        cfgs.append(oracle_cfg(N, K, 3, 2, seed=seed, B0=B0))
        host.append(x)
        xs.append(to_dev(x))
    for graph in (False, True, True):
        b = sfft.Batch(plans, xs)
        b.run(graph=graph)
        torch.cuda.synchronize()
        counts = b.counts.cpu().numpy()
        status = b.status.cpu().numpy()
        for i, (x, cfg) in enumerate(zip(host, cfgs)):
            oi, ov, oc, tr = oracle.solve(cfg, x)
            gi = b.idxs[i].cpu().numpy()
            gv = b.vals[i].cpu().numpy()
            assert counts[i] == oc and status[i] == tr.status, i
            np.testing.assert_array_equal(gi, oi)
            m = oi >= 0
            if m.any():
                assert rel_l2(gv[m].astype(np.complex128), ov[m]) <= VAL_TOL
        torch.cuda.synchronize()
        _ = (xs[0].abs() * 2).sum().item()


@pytest.mark.parametrize("N,B0,gap", [
    (2 ** 16, 1024, 32 * 1024),        # L = 64: the pair splits at depth 6
    (2 ** 17, 2048, 32 * 2048),        # L = 64, width 2048
    (2 ** 22, 1024, 2048 * 1024),      # L = 4096: the pair splits at depth 12
])
def test_deep_pairs_match_oracle(sfft, N, B0, gap):
    """Pairs of tones in one level-0 class that agree on every level down to
    depth d - 1 (f2 = f1 + gap, gap = B0 2^(d-1)) keep their class open past
    depth 5, where the whole wave shares each class-vector sum."""
    rng = np.random.default_rng(N + B0)
    base = [int(f) for f in rng.choice(N - gap, 6, replace=False)]
    sup = sorted(set(base + [f + gap for f in base]))
    x = siggen.synth(siggen.make_spec(N, len(sup), 50, support=sup))
    g, o = solve_both(sfft, x, N, len(sup), 4, 2, seed=51, B0=B0)
    assert_parity(g, o)
    assert g[2] == len(sup)


@pytest.mark.parametrize("form", [2, 3])
@pytest.mark.parametrize("N,K,R,D,seed,mode,snr", [
    (2 ** 15, 300, 2, 2, 81, 0, None),      # L = 16: one item (form 3) or two (form 2) per signal
    (2 ** 18, 900, 4, 2, 82, 0, None),
    (2 ** 20, 1500, 3, 3, 83, 0, None),
    (2 ** 18, 600, 4, 2, 84, 1, 25.0),
])
def test_col_form_matches_oracle(sfft, form, N, K, R, D, seed, mode, snr):
    """The 16-row form (1024-thread work-groups, 16-, 8- and 16-point
    transforms) and the 16-column form (128-byte row segments, 64- and
    32-point transforms in two halves) of the B0 = 2048 column pass against
    the oracle, and equal to the 32-row form up to FP32 rounding."""
    x = siggen.synth(siggen.make_spec(N, K, seed, snr_db=snr))
    g, o = solve_both(sfft, x, N, K, R, D, seed=seed, B0=2048, mode=mode, col_form=form)
    assert_parity(g, o)
    p = sfft.Plan(N, K, R, D, seed=seed, B0=2048, mode=mode, col_form=form)
    assert p.info.col_form == form and p.info.l1_resolve == 1
    q = sfft.Plan(N, K, R, D, seed=seed, B0=2048, mode=mode)
    xd = to_dev(x)
    ia, va, ca = p.exec(xd)
    ib, vb, cb = q.exec(xd)
    assert ca == cb
    np.testing.assert_array_equal(ia.cpu().numpy(), ib.cpu().numpy())


def test_col_forms_batch_mixed(sfft):
    """All three forms, both sample formats and other widths in one captured batch."""
    from tests.test_gpu_fp16 import EPS16, np_pack
    shapes = [(2 ** 17, 900, 2048, 2, 0), (2 ** 17, 900, 2048, 1, 0), (2 ** 18, 700, 2048, 2, 1),
              (2 ** 16, 500, 1024, 0, 0), (2 ** 15, 300, 2048, 2, 0), (2 ** 16, 120, 256, 0, 0),
              (2 ** 17, 800, 2048, 3, 0), (2 ** 15, 250, 2048, 3, 0), (2 ** 18, 650, 2048, 3, 1),
              (2 ** 17, 2000, 8192, 0, 0), (2 ** 16, 400, 2048, 3, 0)]
    plans, xs, cfgs, decs = [], [], [], []
    for i, (N, K, B0, form, f16) in enumerate(shapes):
        x = siggen.synth(siggen.make_spec(N, K, 90 + i))
        kw = dict(eps0=EPS16, eps1=EPS16) if f16 else {}
        if f16:
            buf, dec = np_pack(x)
            xs.append(to_dev(buf))
        else:
            dec = x
            xs.append(to_dev(x))
        plans.append(sfft.Plan(N, K, 3, 2, seed=90 + i, B0=B0, col_form=form, sample_format=f16, **kw))
        cfgs.append(oracle_cfg(N, K, 3, 2, seed=90 + i, B0=B0, **kw))
        decs.append(dec)
    b = sfft.Batch(plans, xs)
    for graph in (False, True, True):
        b.run(graph=graph)
        torch.cuda.synchronize()
        for i in range(len(plans)):
            oi, ov, oc, tr = oracle.solve(cfgs[i], decs[i])
            assert int(b.counts[i].item()) == oc, i
            np.testing.assert_array_equal(b.idxs[i].cpu().numpy(), oi)
            m = oi >= 0
            if m.any():
                assert rel_l2(b.vals[i].cpu().numpy()[m].astype(np.complex128), ov[m]) <= VAL_TOL
    del b
    sfft.release_batches()


def test_enum_share_changes_nothing(sfft):
    """Noisy solves with the enumeration in teams of lanes from 1, 2, 16 or
    64 blocks of 32 candidates on: every candidate's statistic is the same
    number, so indices and values are identical, and equal to the oracle."""
    N, K, B0 = 2 ** 18, 160, 512
    x = siggen.synth(siggen.make_spec(N, K, 77, snr_db=20.0))
    xd = to_dev(x)
    outs = []
    for es in (64, 16, 2, 1):
        p = sfft.Plan(N, K, 4, 2, seed=77, B0=B0, mode=1, enum_share=es)
        assert p.info.enum_share == es
        idx, val, cnt = p.exec(xd)
        outs.append((idx.cpu().numpy(), val.cpu().numpy(), cnt))
    for o in outs[1:]:
        np.testing.assert_array_equal(o[0], outs[0][0])
        np.testing.assert_array_equal(o[1], outs[0][1])
        assert o[2] == outs[0][2]
    g, o = solve_both(sfft, x, N, K, 4, 2, seed=77, B0=B0, mode=1, enum_share=1)
    assert_parity(g, o)


def test_l0_spread_changes_nothing(sfft):
    """Noisy solves with the level-0 classes spread over 1, 2, 4 or 8 lanes
    each (64, 32, 16 or 8 classes a wave; the extra lanes join the team
    enumeration): indices and values are identical at every spread and under
    the batch's own choice, and equal to the oracle."""
    N, K, B0 = 2 ** 18, 160, 512
    x = siggen.synth(siggen.make_spec(N, K, 78, snr_db=20.0))
    xd = to_dev(x)
    outs = []
    for sp in (1, 2, 4, 8, 0):
        p = sfft.Plan(N, K, 4, 2, seed=78, B0=B0, mode=1, enum_share=2, l0_spread=sp)
        assert p.info.l0_spread == sp
        idx, val, cnt = p.exec(xd)
        outs.append((idx.cpu().numpy(), val.cpu().numpy(), cnt))
    for o in outs[1:]:
        np.testing.assert_array_equal(o[0], outs[0][0])
        np.testing.assert_array_equal(o[1], outs[0][1])
        assert o[2] == outs[0][2]
    g, o = solve_both(sfft, x, N, K, 4, 2, seed=78, B0=B0, mode=1, enum_share=2, l0_spread=8)
    assert_parity(g, o)


@pytest.mark.parametrize("pairs", [128, 140])
def test_column_rows_overflow_reports_partial(sfft, pairs):
    """The column pass reserves rows for the expected level-0 multi-tons with a
    margin: for K = 256 tones in B0 = 512 classes, 1.5 x 46.2 + 64 -> 134 rows
    (of multi_cap = 256).  Tone pairs k B0 apart in `pairs` distinct classes
    (N = 2^20) make that many level-0 multi-tons: 128 (the K tones) fit and
    the solve equals the oracle's; with 140 the GPU leaves the classes past its
    rows unresolved and reports PARTIAL, returning only planted tones with
    their values, while the oracle, which reserves nothing, resolves every one
    (280 tones of equal magnitude against K = 256: which 256 the top-K keeps
    depends on rounding, so only the planted set is checked)."""
    N, B0, K = 2 ** 20, 512, 256
    ws, sig = sfft.workspace([sfft.Plan(N, K, 4, 2, seed=4, B0=B0)])
    assert sig[0]["l1"] == 1 and sig[0]["col_rows"] == 134 and sig[0]["multi_cap"] == 256
    rng = np.random.default_rng(11)
    cls = rng.choice(B0, size=pairs, replace=False)
    k = rng.integers(0, N // B0 - 1, size=pairs)
    support = np.sort(np.concatenate([cls + B0 * k, cls + B0 * (k + 1)]))
    sp = siggen.make_spec(N, 2 * pairs, 4, support=support)
    x = siggen.synth(sp)
    g, o = solve_both(sfft, x, N, K, 4, 2, seed=4, B0=B0)
    gi, gv, gc, st = g
    oi, ov, oc, tr = o
    if pairs <= 134:
        assert_parity(g, o)
        return
    assert tr.status == 0                          # the oracle resolves every tone
    assert st["status"] == sfft.STATUS_PARTIAL     # the GPU ran out of rows
    got = gi[gi >= 0]
    assert 0 < len(got) <= K and set(got.tolist()) <= set(support.tolist())
    truth = dict(zip(sp.support.tolist(), sp.values.tolist()))
    for f, v in zip(got.tolist(), gv[gi >= 0].tolist()):
        assert abs(v - truth[f]) <= 1e-4 * abs(truth[f])


def test_open_list_overflow_reports_partial(sfft):
    """200 tones in one level-0 class (N = 2^20, B0 = 512, L = 2048), in 100
    pairs 1024 positions apart whose members share their low 10 bits, the pairs
    with distinct residues mod 128: from depth 7 to depth 10 each pair is a
    multi-ton subclass of its own, so every depth there needs 200 open
    subclasses next, more than the resolution's open list holds (128).  The
    GPU reports PARTIAL and returns only planted tones, each with its value;
    the oracle, which keeps no such list, resolves all."""
    N, B0, c = 2 ** 20, 512, 37
    rng = np.random.default_rng(5)
    res = np.sort(rng.choice(128, size=100, replace=False))
    r = res + 128 * rng.integers(0, 8, size=100)
    ks = np.concatenate([r, r + 1024])
    support = np.sort(c + B0 * ks)
    assert len(np.unique(support)) == 200
    sp = siggen.make_spec(N, 200, 3, support=support)
    x = siggen.synth(sp)
    g, o = solve_both(sfft, x, N, 200, 4, 2, seed=3, B0=B0)
    gi, gv, gc, st = g
    oi, ov, oc, tr = o
    assert tr.status == 0 and oc == 200          # the oracle resolves every tone
    assert st["status"] == sfft.STATUS_PARTIAL   # the GPU's open list overflowed
    got = gi[gi >= 0]
    assert 0 < len(got) < 200 and set(got.tolist()) <= set(support.tolist())
    truth = dict(zip(sp.support.tolist(), sp.values.tolist()))
    for f, v in zip(got.tolist(), gv[gi >= 0].tolist()):
        assert abs(v - truth[f]) <= 1e-4 * abs(truth[f])
