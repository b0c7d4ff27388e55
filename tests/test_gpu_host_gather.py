"""Host-gather solves (sfft_exec_host): a host-resident signal is solved with
only the samples each step reads copied to the device.  Parity with the
device-resident path and with the FP64 oracle: indices bit-exact, values
within relative L2 <= 1e-5; bytes copied = samples read x 8."""
import ctypes

import numpy as np
import pytest

import oracle
import siggen
from tests.test_gpu_parity import assert_parity, to_dev, oracle_cfg, rel_l2, VAL_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfft():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2011_05749_amd as m
    return m


def check(sfft, x, N, K, R, D, seed=0, okw=None, **kw):
    plan = sfft.Plan(N, K, R, D, seed=seed, **kw)
    hi, hv, hc, hs = plan.exec_host(x)
    # device-resident path of the same plan without the dense pass
    dplan = sfft.Plan(N, K, R, D, seed=seed, **dict(kw, jump_L=0, l1_resolve=0) if plan.info.kind == 0 else kw)
    di, dv, dc = dplan.exec(to_dev(x))
    ds = dplan.stats()
    np.testing.assert_array_equal(hi, di.cpu().numpy())
    assert hc == dc and hs["status"] == ds["status"] and hs["levels"] == ds["levels"]
    m = hi >= 0
    if m.any():
        assert rel_l2(hv[m].astype(np.complex128), dv.cpu().numpy()[m].astype(np.complex128)) <= 1e-6
    assert hs["h2d_bytes"] == 8 * hs["samples"] == 8 * ds["samples"]
    cfg = oracle_cfg(N, K, R, D if "rf_iters" not in kw else 2, seed=seed, mode=kw.get("mode", 0),
                     B0=kw.get("B0", 0), stage_B=kw.get("stage_B"), **(okw or {}))
    oi, ov, oc, tr = oracle.solve(cfg, x)
    assert_parity((hi, hv, hc, hs), (oi, ov, oc, tr))
    return hs, tr


@pytest.mark.parametrize("N,K,R,D,B0,mpp,seed", [
    (2 ** 12, 8, 1, 2, 8, 0, 1), (2 ** 16, 100, 4, 2, 256, 0, 3), (2 ** 16, 100, 2, 4, 128, 2, 4),
    (2 ** 18, 256, 4, 2, 512, 0, 5), (2 ** 20, 256, 2, 4, 512, 2, 6), (2 ** 14, 64, 3, 3, 64, 2, 7)])
def test_tree_exact(sfft, N, K, R, D, B0, mpp, seed):
    sp = siggen.make_spec(N, K, seed)
    x = siggen.synth(sp)
    okw = {"mpp": mpp} if mpp else {}
    hs, tr = check(sfft, x, N, K, R, D, seed=seed, okw=okw, B0=B0, mpp=mpp)
    assert hs["samples"] == tr.samples


def test_tree_noisy(sfft):
    sp = siggen.make_spec(2 ** 16, 32, 31, snr_db=20.0)
    x = siggen.synth(sp)
    check(sfft, x, 2 ** 16, 32, 4, 2, seed=8, okw={"window": 64}, mode=oracle.NOISY, window=64)


@pytest.mark.parametrize("kw,okw", [({}, {}), ({"peel_starts": 5}, {"peel_starts": 5}),
                                    ({"rf_iters": 11, "rf_m": 3}, {"rffast": (11, 3)})])
def test_ffast(sfft, kw, okw):
    for seed in range(6):
        x = siggen.synth(siggen.make_spec(10800, 10, seed))
        hs, tr = check(sfft, x, 10800, 10, 3, 2, seed=seed, okw=okw, **kw)
        assert hs["h2d_bytes"] == 8 * (16 + 27 + 25) * (2 if not kw.get("rf_iters") else 33)


def test_plan_reuse_and_shallower_signal(sfft):
    """The device image keeps samples of earlier calls: a later, shallower
    solve must read only what it wrote itself."""
    N, K = 2 ** 16, 64
    plan = sfft.Plan(N, K, 2, 2, seed=11, B0=64)
    deep = siggen.synth(siggen.make_spec(N, 2, 1, support=[5, 5 + N // 2]))
    shallow_sp = siggen.make_spec(N, K, 12)
    shallow = siggen.synth(shallow_sp)
    for x, sup in ((deep, [5, 5 + N // 2]), (shallow, shallow_sp.support), (deep, [5, 5 + N // 2])):
        idx, val, cnt, st = plan.exec_host(x)
        np.testing.assert_array_equal(idx[:cnt], sup)


def test_device_pointers_rejected(sfft):
    plan = sfft.Plan(1024, 4, 1, 2)
    xd = torch.zeros(1024, dtype=torch.complex64, device="cuda")
    idx = np.empty(4, dtype=np.int64)
    val = np.empty(4, dtype=np.complex64)
    rc = sfft._lib.sfft_exec_host(plan.handle, ctypes.c_void_p(xd.data_ptr()), idx.ctypes.data,
                                  val.ctypes.data, None)
    assert rc == -1
