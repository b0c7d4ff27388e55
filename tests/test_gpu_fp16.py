"""Packed FP16 signal storage (plan field sample_format = SAMPLES_F16): the
samples the bucketization of Eq. 5-6 reads are binary16 pairs with a
per-signal power-of-two scale, every sum stays FP32.  The pack routine is
checked bit for bit against numpy's binary16 rounding; solves of a packed
signal (built by numpy, so no oracle input comes from the GPU) against the
FP64 oracle on the same decoded samples: indices bit-exact, counts and status
equal, values within relative L2 1e-5 -- on the column pass, the gathering
path with the VALU and matrix-core dense passes, the per-bin sums, noisy
mode, and one batch that mixes both storage forms.

Binary16 rounding leaves a relative error of up to 2^-11 in every component,
so a stored signal is no longer exactly sparse: exact-mode solves of packed
signals use thresholds above that floor (eps0 = eps1 = EPS16); with the
default 1e-4 every empty level-0 bucket fails the zero-ton bound and the
multi-ton lists overflow.  The configuration that stores samples in FP16 is
the noisy one (SNR 30 dB), whose thresholds follow the noise."""
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


def np_pack(x):
    """(packed bytes, decoded complex64): scale s = 2^(e - 15) with 2^(e-1) <=
    m < 2^e for the largest component magnitude m (1 when x = 0); binary16
    of re / s and im / s, rounded to nearest even."""
    x = np.ascontiguousarray(x, dtype=np.complex64)
    m = np.float32(max(np.abs(x.real).max(initial=0), np.abs(x.imag).max(initial=0)))
    s = np.float32(np.ldexp(np.float32(1.0), int(np.frexp(m)[1]) - 15)) if m > 0 else np.float32(1.0)
    re = (x.real / s).astype(np.float16)
    im = (x.imag / s).astype(np.float16)
    buf = np.zeros(16 + 4 * x.size, dtype=np.uint8)
    buf[:4] = np.frombuffer(np.float32(s).tobytes(), dtype=np.uint8)
    pairs = np.empty(2 * x.size, dtype=np.float16)
    pairs[0::2], pairs[1::2] = re, im
    buf[16:] = pairs.view(np.uint8)
    dec = (re.astype(np.float32) * s + 1j * (im.astype(np.float32) * s)).astype(np.complex64)
    return buf, dec


def test_pack_matches_numpy(sfft):
    rng = np.random.default_rng(5)
    base = siggen.synth(siggen.make_spec(2 ** 16, 64, 3))
    cases = [base, base * np.float32(1e6), base * np.float32(1e-6),
             np.zeros(4096, np.complex64),
             ((rng.standard_normal(5000) + 1j * rng.standard_normal(5000)) *
              1e-3 ** rng.integers(0, 3, 5000)).astype(np.complex64)]   # some components far below the scale
    for x in cases:
        want, _ = np_pack(x)
        got = sfft.pack_fp16(torch.from_numpy(x).cuda()).cpu().numpy()
        # header word 1 is the routine's scratch
        np.testing.assert_array_equal(got[:4], want[:4])
        np.testing.assert_array_equal(got[16:], want[16:])


EPS16 = 3e-3


def solve_f16(sfft, x, N, K, R, D, seed, **kw):
    buf, dec = np_pack(x)
    plan = sfft.Plan(N, K, R, D, seed=seed, sample_format=sfft.SAMPLES_F16, **kw)
    assert plan.info.sample_format == 1
    gi, gv, gc = plan.exec(torch.from_numpy(buf).cuda())
    st = plan.stats()
    okw = {k: v for k, v in kw.items() if k in ("max_levels", "eps0", "eps1")}
    cfg = oracle_cfg(N, K, R, D, seed=seed, mode=1 if kw.get("mode") == "noisy" else 0,
                     B0=kw.get("B0", 0), identity_round0=bool(kw.get("identity_round0", 0)), **okw)
    oi, ov, oc, tr = oracle.solve(cfg, dec)
    return plan, (gi.cpu().numpy(), gv.cpu().numpy().astype(np.complex128), gc, st), (oi, ov, oc, tr)


CASES = [
    # name, N, K, R, D, seed, plan keywords, SNR
    ("column 2048", 2 ** 18, 900, 4, 2, 1, dict(B0=2048, eps0=EPS16, eps1=EPS16), None),
    ("column 8192", 2 ** 18, 4000, 4, 2, 2, dict(B0=8192, eps0=EPS16, eps1=EPS16), None),
    ("dense VALU", 2 ** 16, 300, 4, 2, 3, dict(B0=512, l1_resolve=0, jump_L=64, eps0=EPS16, eps1=EPS16), None),
    ("dense MFMA", 2 ** 17, 300, 4, 2, 4, dict(B0=512, l1_resolve=0, jump_L=128, eps0=EPS16, eps1=EPS16),
     None),
    ("levels only", 2 ** 16, 300, 4, 2, 5, dict(B0=512, l1_resolve=0, jump_L=0, eps0=EPS16, eps1=EPS16),
     None),
    ("noisy column", 2 ** 18, 400, 4, 2, 6, dict(B0=1024, mode="noisy"), 25.0),
    ("noisy 8192 30 dB", 2 ** 18, 3000, 4, 2, 11, dict(B0=8192, mode="noisy"), 30.0),
    ("noisy levels", 2 ** 16, 200, 4, 2, 12, dict(B0=512, mode="noisy", l1_resolve=0), 25.0),
]


@pytest.mark.parametrize("name,N,K,R,D,seed,kw,snr", CASES, ids=[c[0] for c in CASES])
def test_fp16_solve_matches_oracle(sfft, name, N, K, R, D, seed, kw, snr):
    x = siggen.synth(siggen.make_spec(N, K, seed, snr_db=snr))
    plan, g, o = solve_f16(sfft, x, N, K, R, D, seed, **kw)
    gi, gv, gc, st = g
    oi, ov, oc, tr = o
    assert gc == oc and st["status"] == tr.status
    np.testing.assert_array_equal(gi, oi)
    m = oi >= 0
    assert rel_l2(gv[m], ov[m]) <= VAL_TOL


def test_fp16_per_bin_sums_match_oracle(sfft):
    """A pair that separates only at L = 1: the levels past B' = 4096 with one
    parent take the per-bin partial sums (k_expand_direct)."""
    N = 2 ** 18
    x = siggen.synth(siggen.make_spec(N, 2, 7, support=[5, 5 + N // 2]))
    plan, g, o = solve_f16(sfft, x, N, 2, 1, 2, 7, B0=2, identity_round0=1, l1_resolve=0, jump_L=0,
                           eps0=EPS16, eps1=EPS16)
    assert g[2] == o[2] == 2 and g[3]["levels"] == 17
    np.testing.assert_array_equal(g[0], o[0])
    assert rel_l2(g[1], o[1]) <= VAL_TOL


def test_fp16_and_c64_in_one_batch(sfft):
    shapes = [(2 ** 18, 900, 2048, 1), (2 ** 16, 300, 512, 0), (2 ** 17, 500, 1024, 1), (2 ** 16, 64, 128, 0)]
    plans, xs, cfgs, decs = [], [], [], []
    for i, (N, K, B0, f16) in enumerate(shapes):
        x = siggen.synth(siggen.make_spec(N, K, 50 + i))
        if f16:
            buf, dec = np_pack(x)
            xs.append(torch.from_numpy(buf).cuda())
        else:
            dec = x
            xs.append(torch.from_numpy(x).cuda())
        plans.append(sfft.Plan(N, K, 4, 2, seed=50 + i, B0=B0, sample_format=f16, eps0=EPS16, eps1=EPS16))
        cfgs.append(oracle_cfg(N, K, 4, 2, seed=50 + i, B0=B0, eps0=EPS16, eps1=EPS16))
        decs.append(dec)
    b = sfft.Batch(plans, xs)
    for graph in (False, True, True):
        b.run(graph=graph)
        torch.cuda.synchronize()
        for i in range(len(plans)):
            oi, ov, oc, tr = oracle.solve(cfgs[i], decs[i])
            np.testing.assert_array_equal(b.idxs[i].cpu().numpy(), oi)
            assert int(b.counts[i].item()) == oc
            m = oi >= 0
            assert rel_l2(b.vals[i].cpu().numpy()[m].astype(np.complex128), ov[m]) <= VAL_TOL
    del b
    sfft.release_batches()


def test_fp16_refused_where_unsupported(sfft):
    with pytest.raises(sfft.SfftError):
        sfft.Plan(10800, 10, 3, 2, sample_format=sfft.SAMPLES_F16)
    plan = sfft.Plan(2 ** 14, 8, 2, 2, B0=16, sample_format=sfft.SAMPLES_F16)
    with pytest.raises(sfft.SfftError):
        plan.exec_host(np.zeros(2 ** 14, np.complex64))
