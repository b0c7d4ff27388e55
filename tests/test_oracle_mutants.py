"""The pins must be able to fail: plant plausible mistakes in a copy of the
oracle (a flipped sign, a dropped scale, a wrong index, a transposed operand,
a wrong constant), compile each copy on the CPU and check that a battery of
pins rejects it while accepting the real oracle."""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import siggen
from tests.conftest import read_golden

SRC = os.path.join(os.path.dirname(oracle.__file__), "sfft_oracle.c")

MUTANTS = {
    "bucket_twiddle_conjugated": ("acc += load(x, (int64_t)pos) * tw[t];",
                                  "acc += load(x, (int64_t)pos) * conj(tw[t]);"),
    "dropped_1_over_B": ("return acc / (double)B;", "return acc;"),
    "shift_off_by_one": ("uint64_t pos = tau % (uint64_t)N;",
                         "uint64_t pos = (tau + 1) % (uint64_t)N;"),
    "snap_truncates": ("floor((u - (double)c) / (double)B + 0.5)",
                       "floor((u - (double)c) / (double)B)"),
    "phase_pair_transposed": ("P += Y[r * cf->D + d + 1] * conj(Y[r * cf->D + d]);",
                              "P += conj(Y[r * cf->D + d + 1]) * Y[r * cf->D + d];"),
    "value_derotation_sign": ("a += Y[i] * unit(t, N, -1);", "a += Y[i] * unit(t, N, +1);"),
    "residual_sign": ("cplx e = Y[i] - a * unit(t, N, +1);", "cplx e = Y[i] - a * unit(t, N, -1);"),
    "child_index": ("next[nnext++] = cls[q] + B;", "next[nnext++] = cls[q] + 2 * B;"),
    "peel_subtract_sign": ("Y[b * D + d] -= na[i] * unit(t, N, +1);",
                           "Y[b * D + d] -= na[i] * unit(t, N, -1);"),
    "peel_no_retire": ("active[b] = modified[b] && !detected[b];", "active[b] = modified[b];"),
    "splitmix_constant": ("0xBF58476D1CE4E5B9ULL", "0xBF58476D1CE4E5B8ULL"),
    "topk_order": ("return a->mag2 > b->mag2 ? -1 : 1;", "return a->mag2 > b->mag2 ? 1 : -1;"),
    "noise_quantile": ("return pw[at] / -log(1.0 - p / phi);", "return pw[at] / log(4.0 / 3.0);"),
    "mpp_moment_index": ("rhs = -Y[r * D + d + 2];", "rhs = -Y[r * D + d + 1];"),
    "mpp_gram_unconjugated": ("g01 += conj(m0) * m1;", "g01 += m0 * m1;"),
    "mpp_root_sign": ("cplx z0 = (-c1 - disc) / 2.0, z1 = (-c1 + disc) / 2.0;",
                      "cplx z0 = (c1 - disc) / 2.0, z1 = (c1 + disc) / 2.0;"),
    "schedule_start_stage": ("active[off[j] + c->start_f[i] % c->stageB[j]] = 1;",
                             "active[off[j] + c->start_f[i] % c->stageB[0]] = 1;"),
    "schedule_no_stop_at_K": ("if (schedule && fl.n >= c->K) {", "if (schedule && fl.n > c->K) {"),
    "kay_weight_center": ("double u = (2.0 * t - m + 2.0) / (double)m;",
                          "double u = (2.0 * t - m) / (double)m;"),
    "rffast_decision_flipped": ("if (th >= TWO_PI / 2) lo += len;", "if (th < TWO_PI / 2) lo += len;"),
    "rffast_delay_spacing": ("return (c->rf_off[it] + ((uint64_t)t << it)) % (uint64_t)c->N;",
                             "return (c->rf_off[it] + ((uint64_t)t << (it + 1))) % (uint64_t)c->N;"),
    "zero_width_x3": ("T0sq = sb2 * ((double)n + cf->zero_k * sqrt((double)n));",
                      "T0sq = sb2 * ((double)n + 3.0 * cf->zero_k * sqrt((double)n));"),
    "single_width_x3": ("T1sq = sb2 * ((double)(n - 1) + cf->single_k * sqrt((double)(n - 1)));",
                        "T1sq = sb2 * ((double)(n - 1) + 3.0 * cf->single_k * sqrt((double)(n - 1)));"),
    "single_n_for_n_minus_1": ("T1sq = sb2 * ((double)(n - 1) + cf->single_k * sqrt((double)(n - 1)));",
                               "T1sq = sb2 * ((double)n + cf->single_k * sqrt((double)n));"),
    "single_n_and_width_x3": ("T1sq = sb2 * ((double)(n - 1) + cf->single_k * sqrt((double)(n - 1)));",
                              "T1sq = sb2 * ((double)n + 3.0 * cf->single_k * sqrt((double)n));"),
    "bucket_noise_without_1_over_B": ("double sb2 = x->noise_var / (double)B;",
                                      "double sb2 = x->noise_var;"),
    "noise_estimate_ignores_phi": ("return pw[at] / -log(1.0 - p / phi);",
                                   "return pw[at] / -log(1.0 - p);"),
    "mpp_value_cross_term": ("cplx a0 = (nn * q0 - s01 * q1) / dv;",
                             "cplx a0 = (nn * q0 + s01 * q1) / dv;"),
}


def battery(libpath):
    """Names of the pins that fail for the oracle at ``libpath``."""
    failed = []

    def check(name, fn):
        try:
            ok = fn()
        except Exception:
            ok = False
        if not ok:
            failed.append(name)

    def aliasing():
        N, B = 64, 8
        rng = np.random.default_rng(1)
        x = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
        j = np.arange(N)
        xh = (np.exp(-2j * np.pi * np.outer(j, j) / N) / N) @ x.astype(np.complex128)
        for sigma in (1, 3):
            for tau in (0, 5):
                for c in range(B):
                    f = np.arange(c, N, B)
                    want = np.sum(xh[f] * np.exp(2j * np.pi * f * tau / N))
                    got = oracle.bin_value(x, N, B, sigma, tau, (sigma * c) % B, libpath=libpath)
                    if abs(got - want) > 1e-12:
                        return False
        return True

    def exact_tree():
        sp = siggen.make_spec(2 ** 12, 20, 5)
        x = siggen.synth(sp)
        cfg = oracle.config(2 ** 12, 20, 2, 2, seed=3, B0=32, libpath=libpath)
        idx, val, cnt, tr = oracle.solve(cfg, x, libpath=libpath)
        sup, vals = siggen.truth(sp)
        return tr.status == 0 and np.array_equal(idx, sup) and np.max(np.abs(val - vals)) < 1e-6

    def n20():
        g = read_golden("n20_peeling.txt")
        sup = [int(v) for v in g["support"]]
        x = siggen.synth(siggen.make_spec(20, 5, 1, support=sup))
        cfg = oracle.config(20, 5, 2, 2, stageB=[4, 5], libpath=libpath)
        idx, val, cnt, tr = oracle.solve(cfg, x, libpath=libpath)
        return ([tr.ident[i] for i in range(tr.levels)] == [9, 3, 1]
                and np.array_equal(idx, sup))

    def n64():
        sup = [1, 6, 13, 20, 59]
        x = siggen.synth(siggen.make_spec(64, 5, 2, support=sup))
        cfg = oracle.config(64, 5, 1, 2, B0=1, identity_round0=True, libpath=libpath)
        idx, val, cnt, tr = oracle.solve(cfg, x, libpath=libpath)
        return [tr.occupied[i] for i in range(4)] == [1, 2, 4, 5] and np.array_equal(idx, sup)

    def splitmix():
        return oracle.splitmix64(1234567, 3, libpath=libpath) == [
            6457827717110365317, 3203168211198807973, 9817491932198370423]

    def topk():
        sup = np.array([3, 100, 200, 900])
        vals = np.array([1.0, 3.0, 2.0, 0.5]) * np.exp(1j * np.array([0.1, 0.2, 0.3, 0.4]))
        x = siggen.synth(siggen.make_spec(1024, 4, 0, support=sup, values=vals))
        cfg = oracle.config(1024, 2, 1, 2, B0=64, libpath=libpath)
        idx, val, cnt, tr = oracle.solve(cfg, x, libpath=libpath)
        return list(idx) == [100, 200]

    def noisy():
        sp = siggen.make_spec(2 ** 14, 16, 31, snr_db=20.0)
        x = siggen.synth(sp)
        cfg = oracle.config(2 ** 14, 16, 4, 2, seed=8, mode=oracle.NOISY, libpath=libpath)
        idx, val, cnt, tr = oracle.solve(cfg, x, libpath=libpath)
        return (np.array_equal(idx, siggen.truth(sp)[0])
                and abs(tr.noise_var / sp.noise_var - 1) < 0.25)

    def two_tons():
        sup = [1, 6, 13, 20, 59]
        sp = siggen.make_spec(64, 5, 2, support=sup)
        x = siggen.synth(sp)
        ok = True
        for B0, want in ((4, [(3, 1, 0)]), (2, [(0, 1, 1), (1, 1, 0)])):
            cfg = oracle.config(64, 5, 1, 4, B0=B0, identity_round0=True, mpp=2, libpath=libpath)
            idx, val, cnt, tr = oracle.solve(cfg, x, libpath=libpath)
            got = [(tr.n_single[l], tr.n_double[l], tr.n_multi[l]) for l in range(tr.levels + 1)]
            ok = ok and got == want and np.array_equal(idx, sup)
            ok = ok and np.max(np.abs(val - sp.values)) < 1e-6
        return ok

    def packet_erasure():
        sup = [1, 3, 5, 10, 13]
        x = siggen.synth(siggen.make_spec(20, 5, 1, support=sup))
        cfg = oracle.config(20, 5, 2, 2, stageB=[4, 5], start_f=[2, 7], libpath=libpath)
        idx, val, cnt, tr = oracle.solve(cfg, x, libpath=libpath)
        return [tr.ident[r] for r in range(tr.levels)] == [3, 2, 1] and np.array_equal(idx, sup)

    def rffast():
        rng = np.random.default_rng(5)
        y = np.exp(1j * 0.7 * np.arange(8))[None, :] + (rng.standard_normal((4000, 8))
                                                         + 1j * rng.standard_normal((4000, 8))) * 0.02236
        est = np.array([oracle.kay_phase(r, libpath=libpath) for r in y])
        crlb = 6.0 / (1000.0 * 8 * 63)
        if not (0.8 * crlb < np.var(est - 0.7) < 1.2 * crlb):
            return False
        for f in range(20):
            x = siggen.synth(siggen.make_spec(20, 1, 0, support=[f], values=[1.0]))
            cfg = oracle.config(20, 1, 2, 2, stageB=[4, 5], rffast=(4, 2), seed=f, libpath=libpath)
            idx, val, cnt, tr = oracle.solve(cfg, x, libpath=libpath)
            if idx[0] != f:
                return False
        return True

    def noisy_rules():
        from tests import test_oracle_noisy_pins as nz
        import math
        from scipy import stats
        n, trials = nz.R * nz.D, 4000
        cfg = nz.cfg_with(zero_k=1.0, single_k=1.0, libpath=libpath)
        p0 = stats.gamma.cdf(n + math.sqrt(n), n)
        if not nz.within_band(nz.zero_rate(cfg, trials, 3, libpath=libpath), trials, p0):
            return False
        p1 = stats.gamma.cdf(n - 1 + math.sqrt(n - 1), n - 1)
        hits, located = nz.single_rate(cfg, trials, 4, libpath=libpath)
        if located != trials or not nz.within_band(hits, trials, p1):
            return False
        rng = np.random.default_rng(9)
        cnt, phi = 4096, 0.6
        m_noise = int(round(phi * cnt))
        p = min(0.25, phi / 2)
        lo, hi = nz._estimate_interval(int(p * (cnt - 1)) + 1, m_noise, -math.log(1 - p / phi))
        pw = np.concatenate([rng.exponential(1.0, m_noise), 1e6 * (1 + rng.uniform(size=cnt - m_noise))])
        return lo <= oracle.estimate_noise(pw, phi, libpath=libpath) <= hi

    for name, fn in [("noisy_rules", noisy_rules), ("rffast", rffast), ("packet_erasure", packet_erasure), ("aliasing", aliasing), ("exact_tree", exact_tree), ("n20", n20),
                     ("n64", n64), ("splitmix", splitmix), ("topk", topk), ("noisy", noisy),
                     ("two_tons", two_tons)]:
        check(name, fn)
    return failed


def test_real_oracle_passes_battery():
    assert battery(None) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    msrc = tmp_path / "sfft_oracle.c"
    msrc.write_text(src.replace(old, new))
    hdr = os.path.join(os.path.dirname(SRC), "sfft_oracle.h")
    (tmp_path / "sfft_oracle.h").write_text(open(hdr).read())
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", str(so), str(msrc), "-lm"],
                   check=True)
    assert battery(str(so)) != [], f"mutant {name} passed every pin"
