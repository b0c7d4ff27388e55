"""sfft_exec_noalloc (workspace in the library's static device scratch)
against sfft_exec_async (workspace allocated per plan) on the same plans and
signals, called through the C-ABI: two calls in a row, the second with a
smaller input; indices, counts and status bit-exact, values within relative
L2 1e-5.  A plan whose workspace exceeds the scratch is rejected before any
launch."""
import numpy as np
import pytest

import siggen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VAL_TOL = 1e-5


@pytest.fixture(scope="module")
def sfft():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2011_05749_amd as m
    return m


def run_both(sfft, plan, x):
    dev = x.device
    outs = []
    for form in ("async", "noalloc"):
        idx = torch.full((plan.K,), -7, dtype=torch.int64, device=dev)
        val = torch.full((plan.K,), 9.0 + 9.0j, dtype=torch.complex64, device=dev)
        cnt = torch.full((1,), -1, dtype=torch.int64, device=dev)
        st = torch.full((1,), -1, dtype=torch.int32, device=dev)
        if form == "async":
            plan.exec_async(x, idx, val, cnt, st)
        else:
            plan.exec_noalloc(x, idx, val, cnt, st)
        torch.cuda.synchronize()
        outs.append((idx.cpu().numpy(), val.cpu().numpy().astype(np.complex128),
                     int(cnt.item()), int(st.item())))
    return outs


def check_equal(a, b):
    assert a[2] == b[2] and a[3] == b[3], (a[2:], b[2:])
    np.testing.assert_array_equal(a[0], b[0])
    m = a[0] >= 0
    if m.any():
        nb = np.linalg.norm(a[1][m])
        assert np.linalg.norm(a[1][m] - b[1][m]) / max(nb, 1e-30) <= VAL_TOL
    np.testing.assert_array_equal(b[1][~m], 0)


def test_noalloc_two_calls_second_smaller(sfft):
    dev = torch.device("cuda")
    cases = [
        # headline shape: level-1 column pass, 6 MiB of workspace
        (dict(N=2 ** 22, K=1024, stages=4, delays=2, seed=9000), dict(B0=2048)),
        # smaller: level-by-level tree with the dense pass
        (dict(N=2 ** 16, K=300, stages=4, delays=2, seed=4), dict(B0=512)),
    ]
    for spec, kw in cases:
        sp = siggen.make_spec(spec["N"], spec["K"], spec["seed"])
        x = siggen.synth_torch(sp, dev)
        plan = sfft.Plan(spec["N"], spec["K"], spec["stages"], spec["delays"], seed=spec["seed"], **kw)
        a, b = run_both(sfft, plan, x)
        check_equal(a, b)
        np.testing.assert_array_equal(b[0], siggen.truth(sp)[0])
        plan.close()


def test_noalloc_mixed_kinds_and_repeat(sfft):
    """FFAST, noisy tree and a repeated large call after small ones: every
    call starts from whatever the previous call left in the scratch."""
    dev = torch.device("cuda")
    seq = [
        (dict(N=10800, K=10, stages=3, delays=2, seed=0), {}, 0.0),
        (dict(N=2 ** 20, K=256, stages=4, delays=2, seed=1000), dict(B0=512, mode="noisy"), 20.0),
        (dict(N=2 ** 14, K=40, stages=4, delays=2, seed=1), dict(B0=128), 0.0),
        (dict(N=2 ** 20, K=256, stages=4, delays=2, seed=1000), dict(B0=512, mode="noisy"), 20.0),
    ]
    for spec, kw, snr in seq:
        sp = siggen.make_spec(spec["N"], spec["K"], spec["seed"], snr_db=snr if snr else None)
        x = siggen.synth_torch(sp, dev)
        plan = sfft.Plan(spec["N"], spec["K"], spec["stages"], spec["delays"], seed=spec["seed"], **kw)
        a, b = run_both(sfft, plan, x)
        check_equal(a, b)
        plan.close()


def test_noalloc_rejects_oversized_workspace(sfft):
    # column-pass rows of 1889 slots x 8192 samples: 124 MB > the scratch
    plan = sfft.Plan(2 ** 24, 4096, 4, 2, seed=1, B0=2048)
    ws, _ = sfft.workspace([plan])
    assert ws["bytes"] > sfft.NOALLOC_SCRATCH_MIB << 20
    dev = torch.device("cuda")
    x = torch.zeros(plan.N, dtype=torch.complex64, device=dev)
    idx = torch.empty(plan.K, dtype=torch.int64, device=dev)
    val = torch.empty(plan.K, dtype=torch.complex64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    with pytest.raises(sfft.SfftError) as e:
        plan.exec_noalloc(x, idx, val, cnt, st)
    assert e.value.code == -5
