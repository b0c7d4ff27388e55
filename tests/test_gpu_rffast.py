"""Parity of the R-FFAST delay set and singleton estimator (Sect. 3.2,
Subproblem 2, general case; Kay's weights, Eq. 21-22) in the HIP FFAST kernel
with the FP64 oracle, through the C-ABI: indices bit-exact, values within
relative L2 <= 1e-5, same peeling rounds."""
import math

import numpy as np
import pytest

import oracle
import siggen
from tests.test_gpu_parity import assert_parity, solve_both, to_dev, oracle_cfg, rel_l2, VAL_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C1 = math.ceil(math.log2(675)) + 1      # config 1: L_max = 10800 / 16 = 675


@pytest.fixture(scope="module")
def sfft():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2011_05749_amd as m
    return m


def test_every_position_n20(sfft):
    for f in range(20):
        x = siggen.synth(siggen.make_spec(20, 1, 0, support=[f], values=[1.0 - 0.25j]))
        g, o = solve_both(sfft, x, 20, 1, 2, 2, seed=f, stage_B=[4, 5], rf_iters=4, rf_m=2)
        assert_parity(g, o)
        assert g[0][0] == f


@pytest.mark.parametrize("m", [2, 3])
def test_config1_exact(sfft, m):
    for seed in range(20):
        sp = siggen.make_spec(10800, 10, seed)
        x = siggen.synth(sp)
        g, o = solve_both(sfft, x, 10800, 10, 3, 2, seed=seed, rf_iters=C1, rf_m=m)
        assert_parity(g, o)
        assert g[3]["levels"] == o[3].levels


@pytest.mark.parametrize("snr", [40.0, 25.0])
def test_config1_noisy(sfft, snr):
    for seed in range(20):
        sp = siggen.make_spec(10800, 10, seed, snr_db=snr)
        x = siggen.synth(sp)
        g, o = solve_both(sfft, x, 10800, 10, 3, 2, seed=seed, mode=oracle.NOISY,
                          rf_iters=C1, rf_m=4)
        assert_parity(g, o)


def test_rffast_with_schedule_in_a_batch(sfft):
    plans, xs, hx, cfgs = [], [], [], []
    for i in range(6):
        x = siggen.synth(siggen.make_spec(10800, 10, 700 + i, snr_db=30.0))
        kw = {"rf_iters": C1, "rf_m": 4, "mode": oracle.NOISY}
        if i % 2:
            kw["peel_starts"] = 5
        plans.append(sfft.Plan(10800, 10, 3, 2, seed=700 + i, **kw))
        okw = {"rffast": (C1, 4)}
        if i % 2:
            okw["peel_starts"] = 5
        cfgs.append(oracle_cfg(10800, 10, 3, 2, seed=700 + i, mode=oracle.NOISY, **okw))
        hx.append(x)
        xs.append(to_dev(x))
    b = sfft.Batch(plans, xs)
    b.run(graph=True)
    torch.cuda.synchronize()
    for i, cfg in enumerate(cfgs):
        oi, ov, oc, tr = oracle.solve(cfg, hx[i])
        np.testing.assert_array_equal(b.idxs[i].cpu().numpy(), oi)
        m = oi >= 0
        assert rel_l2(b.vals[i].cpu().numpy()[m].astype(np.complex128), ov[m]) <= VAL_TOL
