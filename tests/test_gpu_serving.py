"""Serving loop (sfft_server_*): requests of mixed shapes released at Poisson
times are batched as lanes and memory free up, and each result equals the
same request solved alone by sfft_exec (indices, counts and status
bit-exact, values within relative L2 1e-5); a sample also matches the FP64
oracle.  Admission by HBM footprint bounds every batch's workspace by the
lane's share; a request larger than a lane's share is refused at submit."""
import numpy as np
import pytest

import oracle
import siggen
from tests.test_gpu_parity import oracle_cfg, rel_l2, VAL_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfft():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2011_05749_amd as m
    return m


POOL = [
    # (N, K, rounds, delays, seed, plan keywords, SNR dB or None)
    (2 ** 16, 64, 4, 2, 1, dict(B0=128), None),
    (2 ** 18, 300, 4, 2, 2, dict(B0=1024, mode="noisy"), 25.0),
    (2 ** 20, 256, 4, 2, 3, dict(B0=512, mode="noisy"), 20.0),
    (2 ** 22, 1024, 4, 2, 4, dict(B0=2048), None),
    (10800, 10, 3, 2, 5, {}, None),
    (2 ** 16, 64, 2, 4, 6, dict(B0=64, mpp=2), None),
    (2 ** 17, 500, 4, 2, 7, dict(B0=1024), None),
    (2 ** 15, 40, 1, 2, 8, dict(B0=64, identity_round0=1), None),
]


def make_pool(sfft, dev):
    pool = []
    for N, K, R, D, seed, kw, snr in POOL:
        sp = siggen.make_spec(N, K, seed, snr_db=snr)
        pool.append((sfft.Plan(N, K, R, D, seed=seed, **kw), siggen.synth_torch(sp, dev), sp,
                     (N, K, R, D, seed, kw)))
    return pool


def test_serving_results_equal_alone(sfft):
    dev = torch.device("cuda")
    pool = make_pool(sfft, dev)
    alone = []
    for plan, x, _, _ in pool:
        i, v, c = plan.exec(x)
        alone.append((i.cpu().numpy(), v.cpu().numpy().astype(np.complex128), c, plan.stats()["status"]))
    rng = np.random.default_rng(77)
    n = 120
    pick = rng.integers(0, len(pool), n)
    plans = [pool[j][0] for j in pick]
    xs = [pool[j][1] for j in pick]
    idxs = [torch.full((p.K,), -7, dtype=torch.int64, device=dev) for p in plans]
    vals = [torch.zeros(p.K, dtype=torch.complex64, device=dev) for p in plans]
    counts = torch.full((n,), -1, dtype=torch.int64, device=dev)
    status = torch.full((n,), -1, dtype=torch.int32, device=dev)
    # 2 lanes of 64 MiB: a batch holds at most ten of the headline-shape requests (6 MiB each)
    srv = sfft.Server(hbm_bytes=128 << 20, lanes=2, max_batch=16)
    t0 = srv.clock_ns() + 2_000_000
    rel = t0 + np.cumsum(rng.exponential(150_000.0, n)).astype(np.int64)   # ~6.7 k requests/s
    first = srv.submit(plans, xs, idxs, vals, counts, status, release_ns=rel)
    srv.drain()
    torch.cuda.synchronize()
    rq = srv.requests(first, n)
    assert np.all(rq["status"] == 1)
    assert np.all(rq["release_ns"] == rel)
    assert np.all(rq["launch_ns"] >= rq["release_ns"]) and np.all(rq["done_ns"] >= rq["launch_ns"])
    assert rq["batch"].max() > 1 and rq["batch"].max() <= 16
    cnt, stt = counts.cpu().numpy(), status.cpu().numpy()
    for r in range(n):
        ai, av, ac, ast = alone[pick[r]]
        gi = idxs[r].cpu().numpy()
        assert cnt[r] == ac and stt[r] == ast, r
        np.testing.assert_array_equal(gi, ai)
        m = ai >= 0
        if m.any():
            assert rel_l2(vals[r].cpu().numpy()[m].astype(np.complex128), av[m]) <= VAL_TOL
    # the oracle agrees with a sample of the served results
    for j in (0, 2, 4, 7):
        rs = np.nonzero(pick == j)[0]
        if len(rs) == 0:
            continue
        N, K, R, D, seed, kw = pool[j][3]
        okw = {k: v for k, v in kw.items() if k == "mpp"}
        cfg = oracle_cfg(N, K, R, D, seed=seed, mode=1 if kw.get("mode") == "noisy" else 0,
                         B0=kw.get("B0", 0), identity_round0=bool(kw.get("identity_round0", 0)), **okw)
        oi, ov, oc, tr = oracle.solve(cfg, pool[j][1].cpu().numpy())
        np.testing.assert_array_equal(idxs[rs[0]].cpu().numpy(), oi)
    srv.close()


def test_serving_batches_fit_the_lane(sfft):
    """Every batch's workspace fits the lane's share: with 15 MiB lanes and
    requests of about 6 MiB each, no batch holds more than two of them."""
    dev = torch.device("cuda")
    N, K = 2 ** 22, 1024
    sp = siggen.make_spec(N, K, 9)
    x = siggen.synth_torch(sp, dev)
    plan = sfft.Plan(N, K, 4, 2, seed=9, B0=2048)
    ws, _ = sfft.workspace([plan])
    assert 5 << 20 < ws["bytes"] < 7 << 20
    n = 12
    idxs = [torch.empty(K, dtype=torch.int64, device=dev) for _ in range(n)]
    vals = [torch.empty(K, dtype=torch.complex64, device=dev) for _ in range(n)]
    counts = torch.zeros(n, dtype=torch.int64, device=dev)
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    srv = sfft.Server(hbm_bytes=30 << 20, lanes=2, max_batch=64)
    first = srv.submit([plan] * n, [x] * n, idxs, vals, counts, status)
    srv.drain()
    rq = srv.requests(first, n)
    assert np.all(rq["status"] == 1)
    assert rq["batch"].max() <= 2
    truth = siggen.truth(sp)[0]
    for r in range(n):
        np.testing.assert_array_equal(idxs[r].cpu().numpy(), truth)
    srv.close()


def test_serving_refuses_oversized_request(sfft):
    dev = torch.device("cuda")
    plan = sfft.Plan(2 ** 22, 1024, 4, 2, seed=1, B0=2048)
    x = torch.zeros(plan.N, dtype=torch.complex64, device=dev)
    srv = sfft.Server(hbm_bytes=4 << 20, lanes=1, max_batch=4)  # the request's workspace: about 6 MiB
    with pytest.raises(sfft.SfftError) as e:
        srv.submit([plan], [x], [torch.empty(plan.K, dtype=torch.int64, device=dev)],
                   [torch.empty(plan.K, dtype=torch.complex64, device=dev)],
                   torch.zeros(1, dtype=torch.int64, device=dev),
                   torch.zeros(1, dtype=torch.int32, device=dev))
    assert e.value.code == -5
    srv.close()
