"""Parity of the packet-erasure peeling schedule (Sect. 3.2, Subproblem 3,
method 2) in the HIP FFAST kernel with the FP64 oracle, through the C-ABI:
indices bit-exact, values within relative L2 <= 1e-5, the same number of
peeling rounds and bucket identifications."""
import numpy as np
import pytest

import oracle
import siggen
from tests.conftest import read_golden
from tests.test_gpu_parity import assert_parity, solve_both, to_dev, oracle_cfg, rel_l2, VAL_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfft():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2011_05749_amd as m
    return m


def _ident(tr):
    return sum(tr.ident[r] for r in range(tr.levels))


def test_n20_six_identifications(sfft):
    g = read_golden("n20_packet_erasure.txt")
    sup = [int(v) for v in g["support"]]
    starts = [int(v) for v in g["starts"]]
    x = siggen.synth(siggen.make_spec(20, 5, 1, support=sup))
    gg, o = solve_both(sfft, x, 20, 5, 2, 2, stage_B=[4, 5], peel_start_f=starts)
    assert_parity(gg, o)
    assert gg[3]["ident"] == _ident(o[3]) == 6
    assert gg[3]["levels"] == o[3].levels == 3
    np.testing.assert_array_equal(gg[0], sup)


def test_start_in_empty_buckets_falls_back(sfft):
    sup = [1, 3, 5, 10, 13]
    x = siggen.synth(siggen.make_spec(20, 5, 1, support=sup))
    gg, o = solve_both(sfft, x, 20, 5, 2, 2, stage_B=[4, 5], peel_start_f=[12])
    assert_parity(gg, o)
    assert gg[3]["ident"] == _ident(o[3]) and gg[3]["levels"] == o[3].levels


@pytest.mark.parametrize("S", [1, 4, 10])
def test_config1_schedule(sfft, S):
    for seed in range(20):
        x = siggen.synth(siggen.make_spec(10800, 10, seed))
        gg, o = solve_both(sfft, x, 10800, 10, 3, 2, seed=seed, peel_starts=S)
        assert_parity(gg, o)
        assert gg[3]["ident"] == _ident(o[3]) and gg[3]["levels"] == o[3].levels


def test_schedule_in_a_mixed_batch(sfft):
    plans, xs, hx, cfgs = [], [], [], []
    for i in range(8):
        x = siggen.synth(siggen.make_spec(10800, 10, 500 + i))
        S = (0, 2, 5, 10)[i % 4]
        kw = {"peel_starts": S} if S else {}
        plans.append(sfft.Plan(10800, 10, 3, 2, seed=500 + i, **kw))
        cfgs.append(oracle_cfg(10800, 10, 3, 2, seed=500 + i, **kw))
        hx.append(x)
        xs.append(to_dev(x))
    for graph in (False, True):
        b = sfft.Batch(plans, xs)
        b.run(graph=graph)
        torch.cuda.synchronize()
        for i, cfg in enumerate(cfgs):
            oi, ov, oc, tr = oracle.solve(cfg, hx[i])
            np.testing.assert_array_equal(b.idxs[i].cpu().numpy(), oi)
            m = oi >= 0
            assert rel_l2(b.vals[i].cpu().numpy()[m].astype(np.complex128), ov[m]) <= VAL_TOL
            assert b.stats(i)["ident"] == _ident(tr)
