"""Single-precision variant of locate / value / residual (plan field
precision = 1) against the FP64 oracle.  Exact mode: the FP32 phase and snap
reach the same decisions (the snap needs an angle error below pi / L, far
above FP32's), indices bit-exact, values within relative L2 <= 1e-5.  The
N = 2^24, K = 4096 noisy workload: both variants against the planted
spectrum, with L0 / L1 / L2 reported."""
import numpy as np
import pytest

import oracle
import siggen
from tests.test_gpu_parity import assert_parity, solve_both, _l_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfft():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2011_05749_amd as m
    return m


@pytest.mark.parametrize("jump", [0, 128])
@pytest.mark.parametrize("N,K,R,D,B0,seed,mpp", [
    (2 ** 14, 64, 2, 2, 128, 2, 0), (2 ** 16, 300, 4, 2, 512, 4, 0), (2 ** 20, 256, 4, 2, 512, 8, 0),
    (2 ** 18, 200, 2, 4, 256, 7, 2), (2 ** 22, 1024, 4, 2, 2048, 9000, 0)])
def test_fp32_exact(sfft, N, K, R, D, B0, seed, mpp, jump):
    sp = siggen.make_spec(N, K, seed)
    x = siggen.synth(sp)
    g, o = solve_both(sfft, x, N, K, R, D, seed=seed, B0=B0, jump_L=jump, mpp=mpp, precision=1)
    assert_parity(g, o)
    np.testing.assert_array_equal(g[0], siggen.truth(sp)[0])


def test_fp32_noisy_shape_of_the_large_workload(sfft):
    """N = 2^24, K = 4096, magnitudes 10^U[0,2], 30 dB, B0 = 8192, 4 x 2 noisy:
    the FP64 and FP32 variants against the planted spectrum."""
    N, K = 2 ** 24, 4096
    sp = siggen.make_spec(N, K, 5001, mag="loguniform", mag_lo=0.0, mag_hi=2.0, snr_db=30.0)
    x = torch.from_numpy(siggen.synth(sp)).to("cuda")
    errs = {}
    for prec in (0, 1):
        plan = sfft.Plan(N, K, 4, 2, seed=5001, B0=8192, mode="noisy", precision=prec)
        gi, gv, gc = plan.exec(x)
        errs[prec] = _l_errors(gi.cpu().numpy(), gv.cpu().numpy(), *siggen.truth(sp))
    print(f"precision study: FP64 L0={errs[0][0]} L1={errs[0][1]:.3e} L2={errs[0][2]:.3e}; "
          f"FP32 L0={errs[1][0]} L1={errs[1][1]:.3e} L2={errs[1][2]:.3e}")
    assert errs[0][2] < 0.05 and errs[1][2] < 0.05
    assert abs(errs[1][0] - errs[0][0]) <= 4


def test_fp32_rejected_for_ffast(sfft):
    with pytest.raises(sfft.SfftError) as e:
        sfft.Plan(10800, 10, 3, 2, precision=1)
    assert e.value.code == -2
