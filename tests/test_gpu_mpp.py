"""Parity of the two-ton moment preserving solve (Sect. 3.1, a = 2) inside the
HIP tree search with the FP64 oracle, through the C-ABI.

Bar as for the rest of the tree: indices bit-exact, counts and status equal,
values within relative L2 <= 1e-5; the tree's depth and samples equal the
oracle's at these sizes (close pairs resolve in FP32 buckets as in FP64)."""
import numpy as np
import pytest

import oracle
import siggen
from tests.test_gpu_parity import assert_parity, solve_both, to_dev, oracle_cfg, rel_l2, VAL_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfft():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2011_05749_amd as m
    return m


@pytest.mark.parametrize("jump", [0, 64, 128])
@pytest.mark.parametrize("N,K,R,D,B0,seed,ident", [
    (2 ** 12, 8, 1, 4, 4, 1, 1), (2 ** 14, 64, 2, 3, 64, 2, 0), (2 ** 16, 300, 4, 4, 256, 4, 0),
    (2 ** 16, 100, 2, 4, 64, 3, 0), (2 ** 13, 7, 3, 3, 2, 6, 0), (2 ** 18, 256, 1, 4, 256, 7, 1),
    (2 ** 20, 256, 4, 4, 512, 8, 0), (2 ** 17, 37, 2, 4, 16, 9, 0)])
def test_mpp_tree_exact(sfft, N, K, R, D, B0, seed, ident, jump):
    sp = siggen.make_spec(N, K, seed)
    x = siggen.synth(sp)
    g, o = solve_both(sfft, x, N, K, R, D, seed=seed, B0=B0, identity_round0=ident, jump_L=jump,
                      mpp=2, l1_resolve=0)
    assert_parity(g, o)
    assert g[3]["levels"] == o[3].levels
    if jump == 0:
        assert g[3]["samples"] == o[3].samples
    np.testing.assert_array_equal(g[0], siggen.truth(sp)[0])
    assert sum(o[3].n_double[l] for l in range(o[3].levels + 1)) > 0 or K < 8


def test_mpp_worst_pair_level0(sfft):
    N = 2 ** 12
    sp = siggen.make_spec(N, 2, 4, support=[0, N // 2])
    x = siggen.synth(sp)
    g, o = solve_both(sfft, x, N, 2, 1, 4, B0=1, identity_round0=1, mpp=2)
    assert_parity(g, o)
    assert g[3]["levels"] == o[3].levels == 0 and o[3].n_double[0] == 1


def test_mpp_n64_example(sfft):
    sup = [1, 6, 13, 20, 59]
    x = siggen.synth(siggen.make_spec(64, 5, 2, support=sup))
    for B0 in (2, 4):
        g, o = solve_both(sfft, x, 64, 5, 1, 4, B0=B0, identity_round0=1, mpp=2)
        assert_parity(g, o)
        assert g[3]["levels"] == o[3].levels
        np.testing.assert_array_equal(g[0], sup)


def test_mpp_three_tons_open_children(sfft):
    N, B0 = 4096, 16
    for seed in range(12):
        rng = np.random.default_rng(seed)
        c = int(rng.integers(B0))
        sup = np.sort(c + rng.choice(N // B0, size=3, replace=False) * B0)
        x = siggen.synth(siggen.make_spec(N, 3, seed, support=sup))
        g, o = solve_both(sfft, x, N, 3, 2, 4, seed=seed, B0=B0, mpp=2)
        assert_parity(g, o)
        assert o[3].n_multi[0] == 1 and g[3]["levels"] == o[3].levels >= 1


def test_mpp_validation(sfft):
    for args, kw, code in [((1024, 8, 2, 2), {"mpp": 2}, -1), ((1024, 8, 1, 3), {"mpp": 2}, -1),
                           ((1024, 8, 2, 4), {"mpp": 2, "mode": "noisy"}, -2),
                           ((10800, 8, 3, 4), {"mpp": 2}, -2), ((1024, 8, 2, 4), {"mpp": 1}, -1)]:
        with pytest.raises(sfft.SfftError) as e:
            sfft.Plan(*args, **kw)
        assert e.value.code == code


def test_mpp_batch_mixed_with_plain_tree(sfft):
    """Two-ton plans and plain tree plans in one captured batch."""
    plans, xs, cfgs, hx = [], [], [], []
    for i in range(12):
        N, K = 2 ** (14 + i % 4), 16 + 8 * i
        mpp = 2 if i % 2 == 0 else 0
        D = 4 if mpp else 2
        B0 = 1
        while B0 < K:
            B0 *= 2
        x = siggen.synth(siggen.make_spec(N, K, 3000 + i))
        plans.append(sfft.Plan(N, K, 2, D, seed=3000 + i, B0=B0, mpp=mpp))
        cfgs.append(oracle_cfg(N, K, 2, D, seed=3000 + i, B0=B0, mpp=mpp))
        hx.append(x)
        xs.append(to_dev(x))
    for graph in (False, True, True):
        b = sfft.Batch(plans, xs)
        b.run(graph=graph)
        torch.cuda.synchronize()
        counts = b.counts.cpu().numpy()
        for i, cfg in enumerate(cfgs):
            oi, ov, oc, tr = oracle.solve(cfg, hx[i])
            gi = b.idxs[i].cpu().numpy()
            gv = b.vals[i].cpu().numpy()
            assert counts[i] == oc
            np.testing.assert_array_equal(gi, oi)
            m = oi >= 0
            assert rel_l2(gv[m].astype(np.complex128), ov[m]) <= VAL_TOL
        torch.cuda.synchronize()
        _ = (xs[0].abs() * 2).sum().item()


def test_mpp_headline_shape_sampled(sfft):
    """N = 2^22, K = 1024, B0 = 2048, 4 rounds x 4 delays with the two-ton
    solve: two signals against the oracle and the planted spectrum."""
    N, K = 2 ** 22, 1024
    for seed in (9000, 9001):
        sp = siggen.make_spec(N, K, seed)
        x = siggen.synth(sp)
        g, o = solve_both(sfft, x, N, K, 4, 4, seed=seed, B0=2048, mpp=2)
        assert_parity(g, o)
        np.testing.assert_array_equal(g[0], siggen.truth(sp)[0])
        print(f"mpp headline seed {seed}: levels gpu {g[3]['levels']} oracle {o[3].levels}, "
              f"samples gpu {g[3]['samples']} oracle {o[3].samples}", flush=True)
