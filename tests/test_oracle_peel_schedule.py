"""Pins of the oracle's packet-erasure peeling schedule (Sect. 3.2,
Subproblem 3, method 2) against the paper's worked example and against the
genie-assisted schedule (method 1), whose final support it must reproduce."""
import numpy as np
import pytest

import oracle
import siggen
from tests.conftest import read_golden


def test_n20_packet_erasure_example():
    """Fig. 5 text: start points xhat_2 and xhat_7 recover all five
    frequencies with 6 = 4 + 4 - 2 identifications (method 1 needs 13)."""
    g = read_golden("n20_packet_erasure.txt")
    sup = [int(v) for v in g["support"]]
    stages = [int(v) for v in g["stages"]]
    starts = [int(v) for v in g["starts"]]
    x = siggen.synth(siggen.make_spec(20, 5, 1, support=sup))
    cfg = oracle.config(20, 5, 2, 2, stageB=stages, start_f=starts)
    idx, val, cnt, tr = oracle.solve(cfg, x)
    ident = [tr.ident[r] for r in range(tr.levels)]
    assert ident == [int(v) for v in g["identifications"]]
    assert sum(ident) == 6
    np.testing.assert_array_equal(idx, sup)
    assert tr.status == oracle.OK
    order = [tr.order[i] for i in range(tr.n_found)]
    r1 = [int(v) for v in g["found_round1"]]
    r2 = [int(v) for v in g["found_round2"]]
    r3 = [int(v) for v in g["found_round3"]]
    assert sorted(order[:2]) == r1 and sorted(order[2:4]) == r2 and order[4:] == r3
    # method 1 on the same signal: 9 + 3 + 1
    cfg1 = oracle.config(20, 5, 2, 2, stageB=stages)
    idx1, _, _, tr1 = oracle.solve(cfg1, x)
    assert [tr1.ident[r] for r in range(tr1.levels)] == [9, 3, 1]
    np.testing.assert_array_equal(idx1, idx)


def test_start_points_in_empty_buckets_fall_back():
    """Start points whose buckets hold nothing grow no tree; the buckets never
    reached then join the next peeling and decoding completes."""
    sup = [1, 3, 5, 10, 13]
    x = siggen.synth(siggen.make_spec(20, 5, 1, support=sup))
    # 2 -> buckets (4,2) = {10} single, (5,2) empty; 16 -> (4,0) empty, (5,1) = {1} single
    # 12 -> (4,0) empty, (5,2) empty: a start with no live bucket at all
    cfg = oracle.config(20, 5, 2, 2, stageB=[4, 5], start_f=[12])
    idx, val, cnt, tr = oracle.solve(cfg, x)
    assert tr.ident[0] == 2 and tr.ident[1] == 7
    np.testing.assert_array_equal(idx, sup)
    assert tr.status == oracle.OK


@pytest.mark.parametrize("starts", [1, 4, 10])
def test_schedule_support_equals_method1(starts):
    """Config-1 signals (N = 10800, K = 10, stages 16, 27, 25): with random
    start frequencies the schedule finds the same support as method 1 with no
    more identifications."""
    fewer = 0
    for seed in range(60):
        sp = siggen.make_spec(10800, 10, seed)
        x = siggen.synth(sp)
        c1 = oracle.config(10800, 10, 3, 2)
        i1, v1, n1, t1 = oracle.solve(c1, x)
        c2 = oracle.config(10800, 10, 3, 2, seed=seed, peel_starts=starts)
        i2, v2, n2, t2 = oracle.solve(c2, x)
        if t1.status == oracle.OK:
            np.testing.assert_array_equal(i2, i1)
            np.testing.assert_allclose(v2, v1, atol=1e-9)
            assert t2.status == oracle.OK
        id1 = sum(t1.ident[r] for r in range(t1.levels))
        id2 = sum(t2.ident[r] for r in range(t2.levels))
        assert id2 <= id1
        fewer += id2 < id1
    assert fewer >= 40


def test_drawn_start_points_are_splitmix64():
    cfg = oracle.config(10800, 10, 3, 2, seed=1234567, peel_starts=3)
    draws = oracle.splitmix64(1234567, 3)
    assert [cfg.start_f[i] for i in range(3)] == [d % 10800 for d in draws]
