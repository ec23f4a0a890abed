"""Host simulation of the persistent raytrace's tile scheduling: workgroups take
tickets from per-XCD tile lists that keep schedule order (tile diagonals in
turn), claim their next tile before they sweep the current one, and a tile
sweeps only once every upstream tile (the up to seven tiles whose faces,
edges or corner it reads) has swept.  The claim ahead means a workgroup holds
a tile it has not started; the argument that no cycle of waits can form is
that a held tile waits only on the tile its workgroup works on, which is
earlier in schedule order, as every upstream tile is.  The simulation runs the
protocol with random integration and sweep times on few workgroups (where a
wrong argument would show first) and checks that every tile sweeps; a list
that breaks schedule order must be able to deadlock it, which shows that the
check can fail."""
import itertools
import random

import pytest

NXCD = 8


def schedule(dims, octants):
    """Tiles of the given octants in schedule order: tile diagonal by tile
    diagonal, each diagonal's tiles of every octant (x-major inside)."""
    tiles = [(o, x, y, z) for o in range(octants)
             for x, y, z in itertools.product(*(range(d) for d in dims))]
    return sorted(tiles, key=lambda t: (t[1] + t[2] + t[3], t[0], t[3], t[2], t[1]))


def deal(order, nlists):
    """One list per XCD, tiles dealt by their 4-tile-wide line (x // 4),
    each list in schedule order."""
    lists = [[] for _ in range(nlists)]
    for t in order:
        o, x, y, z = t
        lists[hash((o, x // 4, y, z)) % nlists].append(t)
    return lists


def upstream(t):
    o, x, y, z = t
    for dx, dy, dz in itertools.product((0, 1), repeat=3):
        if dx or dy or dz:
            u = (o, x - dx, y - dy, z - dz)
            if min(u[1:]) >= 0:
                yield u


def simulate(lists, nwg, rng):
    """Event simulation of the claim-ahead protocol; returns the number of tiles
    that never swept (0: all done, > 0: the workgroups deadlocked)."""
    ticket = [0] * len(lists)
    done = set()
    total = sum(len(l) for l in lists)

    def claim(b):
        li = b % len(lists)
        k = ticket[li]
        ticket[li] += 1
        return lists[li][k] if k < len(lists[li]) else None

    # workgroup state: (current tile, next tile or None, phase, time of phase end)
    wg = []
    for b in range(nwg):
        cur = claim(b)
        wg.append([cur, None, "integrate", rng.uniform(1.0, 3.0)] if cur else None)
    now = 0.0
    while True:
        live = [b for b in range(nwg) if wg[b] is not None]
        if not live:
            break
        progressed = False
        # finish phases in time order
        for b in sorted(live, key=lambda b: wg[b][3]):
            cur, nxt, phase, end = wg[b]
            if phase == "integrate":
                now = max(now, end)
                wg[b] = [cur, claim(b), "wait", now]   # the next ticket is claimed here
                progressed = True
            elif phase == "wait":
                if all(u in done for u in upstream(cur)):
                    wg[b] = [cur, nxt, "sweep", max(now, end) + rng.uniform(0.1, 0.5)]
                    progressed = True
            elif phase == "sweep":
                now = max(now, end)
                done.add(cur)
                wg[b] = [nxt, None, "integrate", now + rng.uniform(1.0, 3.0)] if nxt else None
                progressed = True
            if progressed:
                break
        if not progressed:
            break   # every live workgroup waits on a tile that never sweeps
    return total - len(done)


@pytest.mark.parametrize("dims,octants,nwg", [((4, 4, 4), 8, 8), ((5, 3, 6), 8, 9),
                                              ((8, 8, 8), 2, 16), ((3, 7, 2), 4, 8)])
def test_claim_ahead_never_deadlocks(dims, octants, nwg):
    lists = deal(schedule(dims, octants), NXCD)
    for seed in range(20):
        assert simulate(lists, nwg, random.Random(seed)) == 0, seed


def test_lists_out_of_schedule_order_can_deadlock():
    lists = deal(schedule((4, 4, 4), 8), NXCD)
    stuck = 0
    for seed in range(20):
        rng = random.Random(seed)
        shuffled = [l[:] for l in lists]
        for l in shuffled:
            rng.shuffle(l)
        stuck += simulate(shuffled, 8, rng) > 0
    assert stuck > 0
