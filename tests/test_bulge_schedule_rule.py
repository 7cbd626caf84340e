"""The ordering rules of the bulge-chasing schedules (tgba_band.hip), checked on
exact task footprints.

Task (i, k) of sweep i works on rows r = i + 1 + 64 k .. of the band: the bulge
block E (rows r.., columns col..col+63, col = i for k = 0 where only column i is
touched, else r - 64), the lower triangle of the diagonal block D and the block F
below it, each clipped to the order n.  The sets below are the entries the
kernel's index formulas read or write.

* Sweep schedule: before task k, sweep i - 1 of the same sector has completed
  min(k + 3, all) tasks.  Every two tasks of different sweeps that share an entry
  must then run in the sequential order; the check follows each pair through the
  chain of waits (i2 waits on i2 - 1, which waits on i2 - 2, ...).  The weaker
  rule (k + 2) must fail, so the rule is tight.
* Step schedule: the pair (i, kap) = tasks 2 kap, 2 kap + 1 runs at step
  2 i + kap; pairs of one step share no entry, and every shared entry is met in
  the sequential order of the steps.
Pure index arithmetic, no oracle and no GPU.
"""
import pytest

BW = 64


def tasks(n, i):
    return (n - 3 - i) // BW + 1


def footprint(n, i, k):
    r = i + 1 + k * BW
    ln = min(n - r, BW)
    ln2 = max(0, min(n - r - ln, BW))
    col = i if k == 0 else r - BW
    s = set()
    for l in range(ln):
        if k > 0:
            s.update((r + l, col + j) for j in range(BW))
        else:
            s.add((r + l, col))
        s.update((r + l, r + j) for j in range(min(l, ln - 1) + 1))
    for l in range(ln2):
        s.update((r + ln + l, r + j) for j in range(ln))
    return s


def owners(n):
    """entry -> {sweep: (first task, last task)} over the whole reduction"""
    own = {}
    for i in range(n - 2):
        for k in range(tasks(n, i)):
            for e in footprint(n, i, k):
                d = own.setdefault(e, {})
                lo, hi = d.get(i, (k, k))
                d[i] = (min(lo, k), max(hi, k))
    return own


def reach(n, i1, i2, k2, lead):
    """last task of sweep i1 complete when task (i2, k2) starts, with the wait rule
    'sweep i - 1 has completed min(k + lead, all) tasks'"""
    k = k2
    for i in range(i2 - 1, i1 - 1, -1):
        k = min(k + lead - 1, tasks(n, i) - 1)
    return k


def violations(n, lead, own):
    bad = 0
    for d in own.values():
        sw = sorted(d)
        for i1, i2 in zip(sw, sw[1:]):  # consecutive sweeps meeting an entry; the rest follows by chaining
            if d[i1][1] > reach(n, i1, i2, d[i2][0], lead):
                bad += 1
    return bad


@pytest.mark.parametrize("n", [3, 4, 5, 66, 67, 129, 130, 131, 200])
def test_sweep_schedule_wait_rule_orders_every_shared_entry(n):
    own = owners(n)
    assert violations(n, 3, own) == 0


def test_sweep_schedule_wait_rule_is_tight():
    assert violations(200, 2, owners(200)) > 0


@pytest.mark.parametrize("n", [5, 67, 130, 200])
def test_step_schedule_pairs_of_a_step_are_disjoint_and_ordered(n):
    step = {}
    for i in range(n - 2):
        for k in range(tasks(n, i)):
            step[(i, k)] = 2 * i + k // 2
    own = {}
    for (i, k), t in step.items():
        for e in footprint(n, i, k):
            own.setdefault(e, []).append((i, k, t))
    for lst in own.values():
        lst.sort()  # sequential order: sweep, then task; steps must increase along it (transitively: all pairs)
        for (i1, k1, t1), (i2, k2, t2) in zip(lst, lst[1:]):
            if (i1, k1 // 2) == (i2, k2 // 2):
                continue  # the two tasks of one pair run in order inside one workgroup
            assert t1 < t2, ((i1, k1), (i2, k2))
