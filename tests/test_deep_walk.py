"""Round-by-round subtree walk of the deep column resolution (host logic, no GPU).

The deep resolution classifies, in one round, every node of the subtrees
below its open subclasses down to as many levels as its node budget allows
(node l = 2^r - 1 + u of subtree o is subclass kappa_o + u 2^dd at depth
dd + r), then walks the round's levels from the subtrees' roots, a level at a
time with one thread per node (a node is reached when it is a root or its
parent was reached as a multi-ton), so that only children of multi-tons count.
This model of that indexing and walk must visit exactly the nodes the
depth-by-depth tree search visits, with the same decisions, flags and deepest
level, whatever the decisions are.
"""
import random

ZERO, SINGLE, MULTI, DOUBLE = 0, 1, 2, 3
NODES, CAP = 512, 128


def sequential(open0, dd0, dmax, decide):
    seen, flags, levels = [], 0, 0
    open_, dd = list(open0), dd0
    while open_:
        nxt = []
        for k in open_:
            v = decide(dd, k)
            seen.append((dd, k, v))
            levels = max(levels, dd)
            if v == MULTI:
                if dd >= dmax:
                    flags = 1
                else:
                    nxt += [k, k + (1 << dd)]
        if len(nxt) > CAP:
            flags, nxt = 1, nxt[:CAP]
        open_, dd = nxt, dd + 1
    return sorted(seen), flags, levels


def rounds(open0, dd0, dmax, decide):
    seen, flags, levels = [], 0, 0
    open_, dd = list(open0), dd0
    while open_:
        sl = 1
        while dd + sl <= dmax and len(open_) * ((2 << sl) - 1) <= NODES:
            sl += 1
        per = (1 << sl) - 1
        nodes = []
        for o in range(len(open_)):
            for l in range(per):
                r = (l + 1).bit_length() - 1
                u = l + 1 - (1 << r)
                nodes.append((dd + r, open_[o] + (u << dd)))
        dec = [decide(*nd) for nd in nodes]
        reached = [False] * len(nodes)
        nxt = []
        # level-major, as the kernel's threads take them: level r holds the
        # nopen 2^r nodes e = (o, u) of every subtree, and reads level r - 1
        for r in range(sl):
            for e in range(len(open_) << r):
                o, u = e >> r, e & ((1 << r) - 1)
                base = o * per
                q = base + (1 << r) - 1 + u
                if r == 0:
                    reach = True
                else:
                    pl = base + (1 << (r - 1)) - 1 + (u & ((1 << (r - 1)) - 1))
                    reach = reached[pl] and dec[pl] == MULTI and dd + r - 1 < dmax
                reached[q] = reach
                if not reach:
                    continue
                ddn, k = nodes[q]
                assert ddn == dd + r
                v = dec[q]
                seen.append((ddn, k, v))
                levels = max(levels, ddn)
                if v == MULTI:
                    if ddn >= dmax:
                        flags = 1
                    elif r == sl - 1:
                        nxt += [k, k + (1 << ddn)]
        if len(nxt) > CAP:
            flags, nxt = 1, nxt[:CAP]
        open_, dd = nxt, dd + sl
    return sorted(seen), flags, levels


def test_round_walk_equals_sequential_descent():
    rng = random.Random(11)
    for trial in range(300):
        dz = rng.randint(1, 5)
        lgL = rng.randint(dz + 1, 13)
        dmax = min(lgL, rng.randint(dz + 1, 14))
        p_multi = rng.choice([0.2, 0.5, 0.8, 0.95])
        table = {}

        def decide(dd, k):
            if (dd, k) not in table:
                x = rng.random()
                table[(dd, k)] = MULTI if x < p_multi else rng.choice([ZERO, SINGLE, DOUBLE])
            return table[(dd, k)]

        bits = rng.sample(range(1 << (dz + 1)), rng.randint(1, min(8, 1 << (dz + 1))))
        a = sequential(sorted(bits), dz + 1, dmax, decide)
        b = rounds(sorted(bits), dz + 1, dmax, decide)
        if a[1] == 0:   # no open-list overflow: visits must agree exactly
            assert a == b, trial
        else:
            assert b[1] == 1


def test_node_indexing_covers_each_subtree_once():
    for dd in (3, 6):
        for sl in range(1, 7):
            per = (1 << sl) - 1
            kap = 5
            got = set()
            for l in range(per):
                r = (l + 1).bit_length() - 1
                u = l + 1 - (1 << r)
                got.add((dd + r, kap + (u << dd)))
            want = {(dd + r, kap + (u << dd)) for r in range(sl) for u in range(1 << r)}
            assert got == want and len(got) == per
