"""CPU emulation of the coarsest-level Gauss-Seidel solve's dataflow
protocol (Section 5.2's sweep, executed by the library without grid
barriers):

* every cell (or 2 x 2 x 2 brick) counts its completed updates; update
  c = 8 sweep + (position of the octant in the order) of a cell may start
  once the cell's own counter equals c and every upwind neighbour's counter
  (downwind for the adjoint) is at least c + 1;
* the updates are dealt round-robin, in the order of their dependency step,
  to lists that each run their updates one after the other.

Under random interleavings of the lists, every update must read exactly
the data the sequential sweep reads -- the inflow of its octant from each
upwind neighbour after that neighbour's update in the same octant sweep
and not a later one -- and the lists must never deadlock.  The emulation
follows the protocol as stated above, independently of the library's
code."""
import itertools

import numpy as np
import pytest

GRAY = (0, 1, 3, 2, 6, 7, 5, 4)


def _units(n):
    return list(itertools.product(range(n[0]), range(n[1]), range(n[2])))


def _upwind(u, o, n, adj):
    """Neighbours a unit receives its inflow from in octant o (sign bit d set:
    the direction runs towards decreasing index d)."""
    out = []
    for d in range(3):
        step = -1 if not ((o >> d) & 1) else 1   # forward: upwind is at index - 1 for s_d > 0
        if adj:
            step = -step
        v = list(u)
        v[d] += step
        if 0 <= v[d] < n[d]:
            out.append(tuple(v))
    return out


def _schedule(n, nu, order, adj):
    """(step, unit, c) of every update: one step after the latest of the
    unit's previous update and its upwind neighbours' updates in the same
    octant sweep (the order a sequential sweep would respect)."""
    last = {u: -1 for u in _units(n)}
    items = []
    for sweep in range(nu):
        for pos, o in enumerate(order):
            c = 8 * sweep + pos
            sign = [(-1 if (o >> d) & 1 else 1) * (-1 if adj else 1) for d in range(3)]
            # cells in upwind plane order of this octant
            units = sorted(_units(n), key=lambda u: sum((u[d] if sign[d] > 0 else n[d] - 1 - u[d]) for d in range(3)))
            step_of = {}
            for u in units:
                t = last[u] + 1
                for v in _upwind(u, o, n, adj):
                    t = max(t, step_of[v] + 1)
                step_of[u] = t
                last[u] = t
                items.append((t, u, c, o))
    items.sort(key=lambda it: it[0])
    return items


def _emulate(n, nu, order, adj, nlists, seed):
    items = _schedule(n, nu, order, adj)
    lists = [[] for _ in range(nlists)]
    for i, it in enumerate(items):
        lists[i % nlists].append(it)
    cnt = {u: 0 for u in _units(n)}
    version = {(u, o): 0 for u in _units(n) for o in range(8)}   # updates of (unit, octant) done
    heads = [0] * nlists
    rng = np.random.default_rng(seed)
    done = 0
    while done < len(items):
        runnable = []
        for w in range(nlists):
            if heads[w] == len(lists[w]):
                continue
            _, u, c, o = lists[w][heads[w]]
            if cnt[u] == c and all(cnt[v] >= c + 1 for v in _upwind(u, o, n, adj)):
                runnable.append(w)
        assert runnable, "the lists deadlocked"
        w = runnable[int(rng.integers(len(runnable)))]
        _, u, c, o = lists[w][heads[w]]
        sweep = c // 8
        # the inflow of octant o from every upwind neighbour: exactly its
        # update of this octant sweep
        for v in _upwind(u, o, n, adj):
            assert version[(v, o)] == sweep + 1, (u, c, v, version[(v, o)])
        # the unit's own data: every earlier update of it done, no later one
        assert cnt[u] == c
        version[(u, o)] += 1
        cnt[u] += 1
        heads[w] += 1
        done += 1
    assert all(cnt[u] == 8 * nu for u in cnt)


@pytest.mark.parametrize("n", [(3, 4, 2), (2, 2, 2), (5, 1, 3)])
@pytest.mark.parametrize("adj", [False, True])
def test_dataflow_reads_the_sequential_data(n, adj):
    for seed in range(3):
        for nlists in (1, 3, 8):
            _emulate(n, 3, GRAY, adj, nlists, seed)


def test_dataflow_with_identity_octant_order():
    _emulate((3, 3, 3), 2, tuple(range(8)), False, 5, 11)


def test_schedule_steps_respect_every_dependency():
    """Each update's step exceeds those of the updates it waits for."""
    n = (3, 2, 4)
    items = _schedule(n, 2, GRAY, False)
    when = {(u, c): t for t, u, c, o in items}
    for t, u, c, o in items:
        if c > 0:
            assert when[(u, c - 1)] < t
        for v in _upwind(u, o, n, False):
            assert when[(v, c)] < t
