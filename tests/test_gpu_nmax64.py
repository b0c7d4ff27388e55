"""Class vectors of 17..64 measurements (the widest kernel instances, NMAX =
64) against the FP64 oracle: tree plans with up to 16 rounds x 4 delays on
the level-1 column pass and on the gathering path, and one batch that holds
a column-pass tree signal beside an R-FFAST signal of 44 delays, which puts
every kernel of that batch in its 64-measurement form.  Bar: indices
bit-exact, counts and status equal, values within relative L2 1e-5."""
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


@pytest.mark.parametrize("R,D", [(8, 4), (16, 4), (6, 3)])
@pytest.mark.parametrize("path", ["column", "gather", "dense"])
def test_wide_class_vectors_match_oracle(sfft, R, D, path):
    N, K, B0, seed = 2 ** 16, 600, 1024, 40 + R
    kw = {"column": {}, "gather": {"l1_resolve": 0, "jump_L": 0},
          "dense": {"l1_resolve": 0, "jump_L": 64}}[path]
    x = siggen.synth(siggen.make_spec(N, K, seed))
    p = sfft.Plan(N, K, R, D, seed=seed, B0=B0, **kw)
    assert p.info.l1_resolve == (1 if path == "column" else 0)
    g, o = solve_both(sfft, x, N, K, R, D, seed=seed, B0=B0, **kw)
    assert_parity(g, o)
    np.testing.assert_array_equal(g[0], siggen.truth(siggen.make_spec(N, K, seed))[0])


def test_noisy_wide_matches_oracle(sfft):
    N, K, B0, seed = 2 ** 16, 200, 1024, 77
    x = siggen.synth(siggen.make_spec(N, K, seed, snr_db=25.0))
    g, o = solve_both(sfft, x, N, K, 8, 4, seed=seed, B0=B0, mode=1)
    assert_parity(g, o)


def test_column_pass_beside_rffast_signal(sfft):
    """nmax = 44: the column pass, its resolve, level-0 classify and the FFAST
    kernel all run their 64-measurement instances in one captured batch."""
    jobs = [
        (dict(N=2 ** 16, K=600, stages=4, delays=2, seed=7), dict(B0=1024), 0.0),
        (dict(N=10800, K=10, stages=3, delays=2, seed=31), dict(mode="noisy", rf_iters=11, rf_m=4), 25.0),
        (dict(N=2 ** 15, K=300, stages=2, delays=2, seed=8), dict(B0=2048), 0.0),
        (dict(N=2 ** 14, K=40, stages=4, delays=2, seed=9), dict(B0=128), 0.0),
    ]
    plans, xs, cfgs = [], [], []
    for spec, kw, snr in jobs:
        sp = siggen.make_spec(spec["N"], spec["K"], spec["seed"], snr_db=snr or None)
        x = siggen.synth(sp)
        plans.append(sfft.Plan(spec["N"], spec["K"], spec["stages"], spec["delays"], seed=spec["seed"],
                               **kw))
        okw = {}
        if "rf_iters" in kw:
            okw["rffast"] = (kw["rf_iters"], kw["rf_m"])
        cfgs.append(oracle_cfg(spec["N"], spec["K"], spec["stages"], spec["delays"], seed=spec["seed"],
                               mode=1 if kw.get("mode") == "noisy" else 0, B0=kw.get("B0", 0), **okw))
        xs.append(x)
    ws, _ = sfft.workspace(plans)
    assert ws["nmax"] == 44
    assert plans[0].info.l1_resolve == 1 and plans[2].info.l1_resolve == 1
    b = sfft.Batch(plans, [to_dev(x) for x in xs])
    for graph in (False, True, True):
        b.run(graph=graph)
        torch.cuda.synchronize()
        counts, status = b.counts.cpu().numpy(), b.status.cpu().numpy()
        for i, (cfg, x) in enumerate(zip(cfgs, xs)):
            oi, ov, oc, tr = oracle.solve(cfg, x)
            assert counts[i] == oc and status[i] == tr.status, i
            gi = b.idxs[i].cpu().numpy()
            np.testing.assert_array_equal(gi, oi)
            m = oi >= 0
            if m.any():
                assert rel_l2(b.vals[i].cpu().numpy()[m].astype(np.complex128), ov[m]) <= VAL_TOL
    del b
    sfft.release_batches()
