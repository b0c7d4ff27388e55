"""Autotuner of the launch shape of a solve (host-side; every candidate runs
the library's own kernels).

For a problem shape (N, K, rounds, delays, B0, mode) it times the candidate
settings of the knobs that change how the bucketization of Sect. 2.2 (one
round costs B samples and a B log B transform) is laid out on the device,
not what it computes:

* the level-1 path: the column pass (every level-0 multi-ton's coefficients
  from one read of x; at B0 = 2048 in any of its three forms, col_form) or
  level-by-level gathers, and for the latter the stride at which the dense
  subtree pass takes over (jump_L);
* fft_tile_lg: log2 of the sub-FFT size of the level-0 transform (the B0-point
  DFT is taken as B0 / 2^fft_tile_lg LDS-resident sub-FFTs; smaller tiles use
  less LDS per work-group, so more work-groups share a CU);
* gather_unroll: samples each thread has in flight in the strided gathers
  (2, 4 or 8 load batches per thread);
* enum_share (noisy mode): from how many blocks of 32 candidates on the
  subtree levels' enumerations (Sect. 3.1, Method 2) run in teams of a wave's
  lanes instead of one lane a class; l0_spread (noisy mode): lanes per
  class of the level-0 classification (1 .. 8; the extra lanes join the
  teams).

Each candidate runs a captured batch of synthetic signals of the shape
(random K-sparse spectra, unit magnitudes, generated on the device), as many
as the batches the caller will run: how the work spreads over the 256 CUs
depends on the batch, and so does the fastest setting.  The sweep keeps the
median of a few replays per candidate; the default and the sweep's fastest
few are then timed again in alternating rounds, and a setting replaces the
default only if it is faster there by more than a noise margin.  Results go
to a JSON cache keyed by the device, the library build (sha256 of
libsfft.so), the shape and the batch class (the batch rounded up to a power
of two), so a rebuilt library or another device re-tunes; lookup() returns
the stored knobs (or {}), ready to pass to Plan(...).
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

CACHE_VERSION = 2


def cache_path() -> str:
    return os.environ.get("SFFT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "sfft_tune.json"))


def _lib_sha16() -> str:
    from . import LIB_PATH
    h = hashlib.sha256()
    with open(LIB_PATH, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()[:16]


def device_tag() -> str:
    import torch
    if not torch.cuda.is_available():
        return "cpu"
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch.split(':')[0]}-{p.multi_processor_count}cu"


def batch_class(batch) -> int:
    """The batch rounded up to a power of two (batches of one class share
    tuned knobs)."""
    return 1 << max(0, (int(batch) - 1).bit_length())


def shape_key(N, K, rounds, delays, B0, mode, device=None, lib=None, batch=1) -> str:
    return (f"{device or device_tag()}|{lib or _lib_sha16()}|N={int(N)}|K={int(K)}|R={int(rounds)}"
            f"|D={int(delays)}|B0={int(B0)}|mode={int(mode)}|batch={batch_class(batch)}")


def _load(path):
    try:
        with open(path) as f:
            c = json.load(f)
        if c.get("version") == CACHE_VERSION and isinstance(c.get("entries"), dict):
            return c
    except (OSError, ValueError):
        pass
    return {"version": CACHE_VERSION, "entries": {}}


def _store(path, cache):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(N, K, rounds, delays, B0=0, mode=0, path=None, device=None, lib=None, batch=1) -> dict:
    """Stored knobs for the shape and batch class on this device and library
    build, or {}.  B0 as the plan resolves it (0 is looked up as the default
    B0)."""
    mode = {"exact": 0, "noisy": 1}.get(mode, mode)
    if not B0:
        B0 = min(1 << max(0, (2 * int(K) - 1).bit_length()), int(N))
    e = _load(path or cache_path())["entries"].get(shape_key(N, K, rounds, delays, B0, mode, device, lib, batch))
    return dict(e["best"]) if e else {}


def default_knobs(B0, delays, l1_eligible) -> dict:
    """The knobs a plan takes when none is given."""
    lgB = int(B0).bit_length() - 1
    top = min(lgB, 13 - (0 if delays <= 1 else (1 if delays <= 2 else 2)))
    path = {"l1_resolve": 1} if l1_eligible else {"l1_resolve": 0, "jump_L": 128}
    return {**path, "fft_tile_lg": top, "gather_unroll": 4}


def candidates(N, B0, delays, l1_eligible, mode=0):
    """Knob settings tried for a shape (each a dict of Plan keywords), the
    default first; noisy shapes also try the team enumeration from other
    range lengths on (enum_share) and other level-0 spreads (l0_spread)."""
    lgB = int(B0).bit_length() - 1
    top = min(lgB, 13 - (0 if delays <= 1 else (1 if delays <= 2 else 2)))
    tiles = sorted({t for t in (top, top - 1, top - 2) if t >= 5}, reverse=True) or [top]
    paths = ([{"l1_resolve": 1}] if l1_eligible else []) + (
        [{"l1_resolve": 1, "col_form": f} for f in (1, 2)] if l1_eligible and int(B0) == 2048 else []) + [
        {"l1_resolve": 0, "jump_L": j} for j in (128, 64, 32, 0)]
    out = [default_knobs(B0, delays, l1_eligible)]
    for path, tile, u in itertools.product(paths, tiles, (4, 2, 8)):
        c = {**path, "fft_tile_lg": tile, "gather_unroll": u}
        if c not in out:
            out.append(c)
    if mode in (1, "noisy"):
        out += [{**out[0], "enum_share": e} for e in (64, 16, 1)]
        out += [{**out[0], "l0_spread": sp} for sp in (1, 2, 4, 8)]
    return out


def _signals(N, K, n, seed, dev):
    """n random K-sparse complex64 signals of length N on the device (unit
    magnitudes, uniform phases, distinct uniform positions)."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    xs = []
    for _ in range(n):
        pos = torch.randperm(N, generator=g)[:K]
        ph = torch.rand(K, generator=g, dtype=torch.float64) * (2 * torch.pi)
        xh = torch.zeros(N, dtype=torch.complex128)
        xh[pos] = torch.polar(torch.ones(K, dtype=torch.float64), ph)
        xs.append((torch.fft.ifft(xh.to(dev)) * N).to(torch.complex64))
    return xs


def choose(meds, margin) -> int:
    """Index of the setting kept, given the confirmation medians with the
    default's first: the fastest, unless it is not faster than the default by
    more than the fraction `margin` (then the default, 0)."""
    bi = min(range(len(meds)), key=lambda i: meds[i])
    return bi if meds[bi] < meds[0] * (1.0 - margin) else 0


def tune(N, K, rounds, delays, B0=0, mode=0, batch=32, reps=5, seed=1, path=None, verbose=False,
         timer=None, limit=None, finalists=3, confirm=3, margin=0.02) -> dict:
    """Time every candidate on a captured batch of `batch` synthetic signals,
    time the default and the `finalists` fastest again in `confirm`
    alternating rounds, and store the winner in the cache: the fastest of
    those by median, unless it beats the default by no more than `margin`
    (then the default).  Returns the cache entry."""
    import torch

    from . import Batch, Plan, release_batches
    dev = torch.device("cuda")
    mode = {"exact": 0, "noisy": 1}.get(mode, mode)
    base = Plan(N, K, rounds, delays, seed=seed, B0=B0, mode=mode)
    B0 = int(base.info.B0)
    eligible = bool(base.info.l1_resolve)
    xs = _signals(N, K, batch, seed, dev)
    cands = candidates(N, B0, delays, eligible, mode)
    if limit is not None:
        cands = cands[:limit]
    default = default_knobs(B0, delays, eligible)

    def replays(cand, n):
        plans = [Plan(N, K, rounds, delays, seed=seed + i, B0=B0, mode=mode, **cand) for i in range(batch)]
        b = Batch(plans, xs)
        for _ in range(2):
            b.run(graph=True)
        torch.cuda.synchronize()
        ts = []
        for _ in range(n):
            t0 = time.perf_counter()
            b.run(graph=True)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        del b, plans
        release_batches()
        return ts

    def median(ts):
        ts = sorted(ts)
        return ts[len(ts) // 2]

    results = []
    for cand in cands:
        ts = replays(cand, reps)
        med = median(ts) if timer is None else timer(cand, ts)
        results.append((med, cand))
        if verbose:
            print(f"tune N={N} K={K} B0={B0} batch={batch} {cand}: {med * 1e3:.3f} ms", flush=True)
    results.sort(key=lambda r: r[0])
    final = [default] + [c for _, c in results if c != default][:finalists]
    times = {i: [] for i in range(len(final))}
    for _ in range(confirm):
        for i, cand in enumerate(final):
            times[i] += replays(cand, reps)
    meds = [median(times[i]) if timer is None else timer(final[i], times[i]) for i in range(len(final))]
    bi = choose(meds, margin)
    if verbose:
        for c, m in zip(final, meds):
            print(f"tune confirm {c}: {m * 1e3:.3f} ms", flush=True)
    entry = {"best": final[bi], "ms_per_batch": round(meds[bi] * 1e3, 4), "batch": batch,
             "default": default, "default_ms_per_batch": round(meds[0] * 1e3, 4),
             "tried": len(results), "finalists": len(final) - 1, "timestamp": int(time.time())}
    p = path or cache_path()
    cache = _load(p)
    cache["entries"][shape_key(N, K, rounds, delays, B0, mode, batch=batch)] = entry
    _store(p, cache)
    return entry


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="tune the launch knobs of one problem shape")
    ap.add_argument("--N", type=int, required=True)
    ap.add_argument("--K", type=int, required=True)
    ap.add_argument("--rounds", type=int, default=4)
    ap.add_argument("--delays", type=int, default=2)
    ap.add_argument("--B0", type=int, default=0)
    ap.add_argument("--mode", default="exact")
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--confirm", type=int, default=3)
    a = ap.parse_args(argv)
    e = tune(a.N, a.K, a.rounds, a.delays, a.B0, a.mode, a.batch, a.reps, verbose=True, confirm=a.confirm)
    print(json.dumps(e))


if __name__ == "__main__":
    main()
