"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/sfft.h declares, its structs match the binding, and its
plan logic (factoring, SplitMix64 draws, validation) agrees with the
oracle's independent implementation."""
import ctypes
import os
import re
import subprocess

import pytest

import oracle
import paper_2011_05749_amd as sfft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "sfft.h")


def header_functions():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sfft_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", sfft.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(sfft.LIB_PATH)
    for n in names:
        getattr(lib, n)
    assert sorted(sfft.EXPORTS) == names


def test_struct_layouts_match_binding(tmp_path):
    prog = tmp_path / "layout.c"
    fields = {
        "sfft_params_t": sfft.Params, "sfft_plan_info_t": sfft.PlanInfo, "sfft_stats_t": sfft.Stats,
        "sfft_workspace_t": sfft.Workspace, "sfft_workspace_signal_t": sfft.WorkspaceSignal,
        "sfft_server_params_t": sfft.ServerParams, "sfft_request_t": sfft.Request}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HDR}"', "int main(void){"]
    for cname, py in fields.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(prog)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    for line in out.splitlines():
        cname, f, v = line.split()
        py = fields[cname]
        if f == "size":
            assert ctypes.sizeof(py) == int(v), cname
        else:
            assert getattr(py, f).offset == int(v), (cname, f)


def test_plan_factoring_matches_oracle():
    p = sfft.Plan(10800, 10, 3, 2)
    c = oracle.config(10800, 10, 3, 2)
    assert p.info.kind == sfft.KIND_FFAST
    assert [p.info.stage_B[j] for j in range(3)] == [c.stageB[j] for j in range(3)] == [16, 27, 25]
    p = sfft.Plan(20, 5, 2, 3, stage_B=[4, 5])
    assert [p.info.stage_B[j] for j in range(2)] == [4, 5]


@pytest.mark.parametrize("N,K,R,seed,B0,ident", [
    (2 ** 22, 1024, 4, 9000, 2048, 0), (2 ** 20, 256, 4, 1000, 0, 0), (2 ** 14, 8, 1, 7, 0, 1),
    (2 ** 24, 4096, 4, 5000, 8192, 0), (2 ** 16, 100, 16, 3, 256, 1)])
def test_plan_draws_match_oracle(N, K, R, seed, B0, ident):
    p = sfft.Plan(N, K, R, 2, seed=seed, B0=B0, identity_round0=ident)
    c = oracle.config(N, K, R, 2, seed=seed, B0=B0, identity_round0=bool(ident))
    assert p.info.B0 == c.B0 and p.info.max_levels == c.max_levels
    for r in range(R):
        assert p.info.sigma[r] == c.sigma[r] and p.info.shift[r] == c.shift[r]


@pytest.mark.parametrize("args,kw,code", [
    ((10800, 10, 2, 2), {}, -2),           # three prime powers, two stages
    ((1024, 10, 2, 1), {}, -1),            # exact mode needs >= 2 delays
    ((1024, 0, 2, 2), {}, -1),             # K < 1
    ((1024, 2000, 2, 2), {}, -1),          # K > N
    ((1024, 10, 2, 2), {"B0": 24}, -1),    # B0 not a power of two
    ((1024, 10, 2, 2), {"B0": 2048}, -1),  # B0 > N
    ((2 ** 20, 10, 2, 2), {"B0": 16384}, -2),  # beyond the LDS FFT
    ((60, 4, 2, 2), {"stage_B": [4, 6]}, -1),  # stages not co-prime
    ((60, 4, 2, 2), {"stage_B": [7, 5]}, -1),  # stage does not divide N
    ((1024, 10, 17, 2), {}, -1),           # too many rounds
    ((1024, 10, 2, 2), {"jump_L": 48}, -1),   # subtree stride not a power of two
    ((1024, 10, 2, 2), {"jump_L": 256}, -1),  # beyond the dense-pass width
    ((1024, 10, 2, 2), {"l1_resolve": 2}, -1),  # the column pass is on or off
])
def test_plan_validation(args, kw, code):
    with pytest.raises(sfft.SfftError) as e:
        sfft.Plan(*args, **kw)
    assert e.value.code == code


@pytest.mark.parametrize("S,seed", [(1, 0), (4, 77), (64, 1234567)])
def test_peel_start_draws_match_oracle(S, seed):
    p = sfft.Plan(10800, 10, 3, 2, seed=seed, peel_starts=S)
    c = oracle.config(10800, 10, 3, 2, seed=seed, peel_starts=S)
    assert p.info.peel_starts == c.n_starts == S
    assert [p.info.peel_start_f[i] for i in range(S)] == [c.start_f[i] for i in range(S)]
    q = sfft.Plan(20, 5, 2, 2, stage_B=[4, 5], peel_start_f=[2, 7])
    assert q.info.peel_starts == 2 and list(q.info.peel_start_f[:2]) == [2, 7]


@pytest.mark.parametrize("kw,code", [
    ({"peel_starts": 3}, -2),                                   # tree plan: no schedule
])
def test_peel_schedule_tree_unsupported(kw, code):
    with pytest.raises(sfft.SfftError) as e:
        sfft.Plan(1024, 10, 2, 2, **kw)
    assert e.value.code == code


def test_peel_schedule_validation():
    for kw in ({"peel_starts": 65}, {"peel_starts": -1}, {"peel_start_f": [2, 25]}):
        with pytest.raises(sfft.SfftError) as e:
            sfft.Plan(20, 5, 2, 2, stage_B=[4, 5], **kw)
        assert e.value.code == -1
    p = sfft.Params()
    sfft._lib.sfft_params_init(ctypes.byref(p), 20, 5, 2, 2, 0)
    p.nstage_B = 2
    p.stage_B[0], p.stage_B[1] = 4, 5
    p.peel_starts = 2
    p.peel_start_f[0] = 3      # one given, one drawn: rejected
    assert not sfft._lib.sfft_plan_ex(ctypes.byref(p))
    assert sfft._lib.sfft_last_error() == -1


def test_rffast_plan_matches_oracle_and_validates():
    p = sfft.Plan(10800, 10, 3, 2, seed=99, rf_iters=5, rf_m=3, peel_starts=2)
    c = oracle.config(10800, 10, 3, 2, seed=99, rffast=(5, 3), peel_starts=2)
    assert p.info.D == c.D == 15 and p.info.rf_iters == 5 and p.info.rf_m == 3
    assert [p.info.rf_off[i] for i in range(5)] == [c.rf_off[i] for i in range(5)]
    assert [p.info.peel_start_f[i] for i in range(2)] == [c.start_f[i] for i in range(2)]
    for kw, code in [({"rf_iters": 17, "rf_m": 2}, -1), ({"rf_iters": 4, "rf_m": 1}, -1),
                     ({"rf_iters": 11, "rf_m": 6}, -1)]:
        with pytest.raises(sfft.SfftError) as e:
            sfft.Plan(10800, 10, 3, 2, **kw)
        assert e.value.code == code
    with pytest.raises(sfft.SfftError) as e:
        sfft.Plan(1024, 10, 2, 2, rf_iters=4, rf_m=2)
    assert e.value.code == -2


def test_noisy_plan_allows_one_delay_and_window():
    p = sfft.Plan(2 ** 16, 32, 4, 1, seed=1, mode="noisy", window=16)
    assert p.info.mode == sfft.NOISY and p.info.D == 1 and p.info.window == 16


def test_column_pass_shapes():
    """The level-1 column pass is taken for B0 = 512 ... 8192 with at
    least 32768 / B0 columns and one tree level, never for FFAST plans."""
    assert sfft.Plan(2 ** 22, 1024, 4, 2, B0=2048).info.l1_resolve == 1
    assert sfft.Plan(2 ** 15, 300, 2, 2, B0=2048).info.l1_resolve == 1
    assert sfft.Plan(2 ** 14, 300, 2, 2, B0=2048).info.l1_resolve == 0
    assert sfft.Plan(2 ** 15, 300, 2, 2, B0=1024).info.l1_resolve == 1
    assert sfft.Plan(2 ** 14, 300, 2, 2, B0=1024).info.l1_resolve == 0
    assert sfft.Plan(2 ** 16, 300, 2, 2, B0=4096).info.l1_resolve == 1
    assert sfft.Plan(2 ** 15, 300, 2, 2, B0=4096).info.l1_resolve == 0   # L = 8 < 16
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=512).info.l1_resolve == 1
    assert sfft.Plan(2 ** 14, 300, 2, 2, B0=512).info.l1_resolve == 0
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=256).info.l1_resolve == 0
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=8192).info.l1_resolve == 1
    assert sfft.Plan(2 ** 14, 300, 2, 2, B0=8192).info.l1_resolve == 0
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=2048, l1_resolve=0).info.l1_resolve == 0
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=2048, max_levels=0).info.l1_resolve == 0
    assert sfft.Plan(10800, 10, 3, 2).info.l1_resolve == 0


def test_column_pass_forms():
    """Forms 2 (16 rows) and 3 (16 columns) of the column pass exist at
    B0 = 2048 only; a plan without the pass reports form 0."""
    for f in (1, 2, 3):
        assert sfft.Plan(2 ** 20, 300, 2, 2, B0=2048, col_form=f).info.col_form == f
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=2048).info.col_form == 3
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=4096).info.col_form == 1
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=1024, col_form=1).info.col_form == 1
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=2048, col_form=3, l1_resolve=0).info.col_form == 0
    for bad in (dict(B0=1024, col_form=2), dict(B0=4096, col_form=3), dict(B0=2048, col_form=4),
                dict(B0=2048, col_form=-1)):
        with pytest.raises(sfft.SfftError):
            sfft.Plan(2 ** 20, 300, 2, 2, **bad)


def test_enum_share_bounds():
    """The wave-sharing threshold of the noisy enumeration below level 0:
    1 .. 64 blocks, 0 = 4; FFAST plans ignore it."""
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=512, mode="noisy").info.enum_share == 4
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=512, mode="noisy", enum_share=4).info.enum_share == 4
    for bad in (-1, 65):
        with pytest.raises(sfft.SfftError):
            sfft.Plan(2 ** 20, 300, 2, 2, B0=512, mode="noisy", enum_share=bad)


def test_l0_spread_bounds():
    """Level-0 lanes per class: 1, 2, 4 or 8, 0 = the batch's choice."""
    assert sfft.Plan(2 ** 20, 300, 2, 2, B0=512, mode="noisy").info.l0_spread == 0
    for ok in (1, 2, 4, 8):
        assert sfft.Plan(2 ** 20, 300, 2, 2, B0=512, mode="noisy", l0_spread=ok).info.l0_spread == ok
    for bad in (-1, 3, 6, 16):
        with pytest.raises(sfft.SfftError):
            sfft.Plan(2 ** 20, 300, 2, 2, B0=512, mode="noisy", l0_spread=bad)


def test_one_hip_runtime_per_process():
    """Importing the binding maps exactly one HIP and one HSA runtime: the
    library's runtime dependency binds to the copy torch already loaded (two
    runtimes on one device would not see each other's allocations)."""
    prog = ("import paper_2011_05749_amd\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "for lib in ('libamdhip64', 'libhsa-runtime64'):\n"
            "    print(lib, len(set(l.split()[-1] for l in maps if lib in l)))\n")
    out = subprocess.run(["python", "-c", prog], capture_output=True, text=True, check=True,
                         cwd=ROOT).stdout.split()
    assert out == ["libamdhip64", "1", "libhsa-runtime64", "1"], out
