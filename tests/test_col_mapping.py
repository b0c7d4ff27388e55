"""Work mapping of the level-1 column pass (host logic, no GPU).

The column pass walks a batch-wide prefix of items (signal, TC adjacent
columns).  Persistent work-groups, eight XCDs apart, take the G adjacent
items of an aligned group in step; each signal's item range is padded to a
multiple of 8 so that no group straddles two signals' ranges unaligned and
the whole prefix is a multiple of every G.  This model of the mapping checks
that every real item of every signal is taken exactly once, for mixes of
widths and grid sizes, and that padding items are the only ones skipped.
"""
import itertools
import random

ALIGN = 8


def col_items(N, B0):
    L = N // B0
    TC = 512 * 32 // B0
    return L // TC


def group_of(B0, form16=False):
    if form16:
        return 2
    TC = 512 * 32 // B0
    LTC = TC.bit_length() - 1
    return 2 if LTC >= 3 else 1 << (4 - LTC)


def visited(prefix, real, grid, G):
    npairs = prefix[-1] // G
    nwp = grid // G
    per = (npairs + nwp - 1) // nwp
    seen = []
    for b in range(grid):
        wp = ((b >> (3 + (G.bit_length() - 1))) << 3) + (b & 7)
        hf = (b >> 3) & (G - 1)
        ip0 = wp * per
        ip1 = min(ip0 + per, npairs)
        for ip in range(ip0, ip1):
            item = G * ip + hf
            s = max(i for i in range(len(real)) if prefix[i] <= item and item < prefix[i + 1])
            if item - prefix[s] < real[s]:
                seen.append((s, item - prefix[s]))
    return seen


def test_every_item_taken_once():
    rng = random.Random(5)
    widths = [512, 1024, 2048, 4096, 8192]
    for trial in range(40):
        sigs = []
        for _ in range(rng.randint(1, 9)):
            B0 = rng.choice(widths + [256])
            N = B0 * rng.choice([16, 32, 64, 128, 256]) if B0 != 256 else 2 ** 16
            if B0 == 512:
                N = max(N, 512 * 64)
            sigs.append((N, B0))
        real = [col_items(N, B0) if B0 != 256 else 0 for N, B0 in sigs]
        padded = [(r + ALIGN - 1) // ALIGN * ALIGN for r in real]
        prefix = [0] + list(itertools.accumulate(padded))
        for grid in (64, 128, 256):
            for B0 in widths:
                G = group_of(B0)
                mine = [i for i, (N, b) in enumerate(sigs) if b == B0]
                seen = [v for v in visited(prefix, real, grid, G) if v[0] in mine]
                want = [(s, k) for s in mine for k in range(real[s])]
                assert sorted(seen) == sorted(want), (trial, grid, B0)
                assert len(seen) == len(set(seen))
            G = group_of(2048, form16=True)
            mine = [i for i, (N, b) in enumerate(sigs) if b == 2048]
            seen = [v for v in visited(prefix, real, grid, G) if v[0] in mine]
            assert sorted(seen) == sorted((s, k) for s in mine for k in range(real[s]))


def visited_t16(prefix, real, mine, grid):
    """The 16-column form: work-group b walks the contiguous range
    [b per, (b + 1) per) of the prefix and takes only its own items."""
    total = prefix[-1]
    per = (total + grid - 1) // grid
    seen = []
    for b in range(grid):
        i0, i1 = b * per, min(b * per + per, total)
        it, s = i0, 0
        while it < i1:
            while it >= prefix[s + 1]:
                s += 1
            if s in mine and it - prefix[s] < real[s]:
                seen.append((s, it - prefix[s]))
                it += 1
            else:
                it = prefix[s + 1]
    return seen


def test_t16_form_takes_every_item_once():
    rng = random.Random(7)
    for trial in range(60):
        n = rng.randint(1, 9)
        forms = [rng.choice([1, 3, 0]) for _ in range(n)]
        Ls = [rng.choice([16, 32, 64, 128, 2048]) for _ in range(n)]
        real = [(L // 16 if f == 3 else L // 8) if f else 0 for f, L in zip(forms, Ls)]
        padded = [(r + ALIGN - 1) // ALIGN * ALIGN for r in real]
        prefix = [0] + list(itertools.accumulate(padded))
        mine = {i for i, f in enumerate(forms) if f == 3}
        for grid in (1, 7, 64, 256):
            seen = visited_t16(prefix, real, mine, grid)
            assert sorted(seen) == sorted((s, k) for s in mine for k in range(real[s])), (trial, grid)
            assert len(seen) == len(set(seen))


def test_unpadded_prefix_loses_items():
    """Why the padding: with a width-1024 signal of 4 items ahead of a
    width-8192 signal (groups of 8), an unpadded prefix of 4 + 16 items
    leaves the last 4 items of the second signal untaken."""
    real = [4, 16]
    prefix = [0, 4, 20]
    seen = [v for v in visited(prefix, real, 64, 8) if v[0] == 1]
    assert len(seen) < 16
