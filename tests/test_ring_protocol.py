"""Model check of the state ring of the persistent kernels (CPU).

The persistent year and reverse-sweep kernels publish the state of step t
into slot t mod 2K of a ring that holds a sentinel until the owner writes it;
every K steps the domains hand over (each publishes its phase counter and
waits for the counters of its neighbours), and after hand-over p a domain
resets its rows of the slots of states (p+1)K .. (p+2)K-1.  This test runs
the same rules in a sequentially consistent model with domains advancing in
random order (an event per action, a domain blocked while what it waits for
is not there yet) and checks that

* a read of a neighbour's state t never returns another state's value (a
  stale slot), only the sentinel (then it waits) or state t itself;
* every schedule runs to completion (no deadlock).

It checks the slot-reuse logic, not the hardware memory model; that part of
the argument (single-copy atomic 8-byte accesses, release/acquire at the
hand-over) is in the kernel's header comment.
"""

import random

import pytest

SENT = None


class Domain:
    def __init__(self, d, deps):
        self.d = d
        self.deps = deps          # neighbours read and waited for (symmetric)
        self.jj = 0               # next step to take
        self.stage = 0            # 0: hand-over/resets, 1: read halo, 2: write
        self.flag = 0


def run(G, K, nsteps, seed):
    rng = random.Random(seed)
    ring = {(d, s): SENT for d in range(G) for s in range(2 * K)}
    for d in range(G):
        ring[(d, 0)] = ("y", 0)                        # slot 0: the launch's initial state
    deps = {d: sorted({(d - 1) % G, (d + 1) % G} - {d}) for d in range(G)}
    doms = [Domain(d, deps[d]) for d in range(G)]
    done = 0
    events = 0
    while done < G:
        events += 1
        assert events < 200 * G * (nsteps + 2), "no progress: deadlock"
        dm = rng.choice([x for x in doms if x.jj < nsteps])
        jj = dm.jj
        if dm.stage == 0:
            if jj % K == 0:
                ph = jj // K
                if ph > 0:
                    dm.flag = max(dm.flag, ph)
                    if any(doms[e].flag < ph for e in dm.deps):
                        continue                           # waits at the hand-over
                for i in range(K):                         # resets of the phase after next
                    ring[(dm.d, (jj + K + i) % (2 * K))] = SENT
            dm.stage = 1
        elif dm.stage == 1:
            ok = True
            for e in dm.deps:
                v = ring[(e, jj % (2 * K))]
                if v is SENT:
                    ok = False                             # not published yet: read again later
                    break
                assert v == ("y", jj), f"stale read: domain {dm.d} step {jj} saw {v} in the slot of {e}"
            if ok:
                dm.stage = 2
        else:
            if jj + 1 < nsteps:
                ring[(dm.d, (jj + 1) % (2 * K))] = ("y", jj + 1)
            dm.jj += 1
            dm.stage = 0
            if dm.jj == nsteps:
                done += 1
    return events


@pytest.mark.parametrize("G,K,nsteps", [(2, 1, 7), (3, 2, 17), (5, 4, 33), (8, 4, 40), (6, 8, 100),
                                        (7, 64, 300), (4, 64, 24), (3, 3, 2)])
def test_ring_reads_are_never_stale_and_every_schedule_completes(G, K, nsteps):
    for seed in range(40):
        run(G, K, nsteps, seed)


def test_model_catches_a_ring_that_is_too_short():
    """The check has teeth: with resets one phase too early (slots of the next
    phase instead of the one after) some schedule reads a reset or stale slot."""
    def run_early(G, K, nsteps, seed):
        rng = random.Random(seed)
        ring = {(d, s): SENT for d in range(G) for s in range(2 * K)}
        for d in range(G):
            ring[(d, 0)] = ("y", 0)
        doms = [Domain(d, sorted({(d - 1) % G, (d + 1) % G} - {d})) for d in range(G)]
        done, events = 0, 0
        while done < G:
            events += 1
            if events > 200 * G * (nsteps + 2):
                return "deadlock"
            dm = rng.choice([x for x in doms if x.jj < nsteps])
            jj = dm.jj
            if dm.stage == 0:
                if jj % K == 0:
                    ph = jj // K
                    if ph > 0:
                        dm.flag = max(dm.flag, ph)
                        if any(doms[e].flag < ph for e in dm.deps):
                            continue
                    for i in range(1, K + 1):              # wrong: states jj+1 .. jj+K
                        ring[(dm.d, (jj + i) % (2 * K))] = SENT
                dm.stage = 1
            elif dm.stage == 1:
                ok = True
                for e in dm.deps:
                    v = ring[(e, jj % (2 * K))]
                    if v is SENT:
                        ok = False
                        break
                    if v != ("y", jj):
                        return "stale"
                if ok:
                    dm.stage = 2
            else:
                if jj + 1 < nsteps:
                    ring[(dm.d, (jj + 1) % (2 * K))] = ("y", jj + 1)
                dm.jj += 1
                dm.stage = 0
                if dm.jj == nsteps:
                    done += 1
        return "ok"
    outcomes = {run_early(4, 2, 20, seed) for seed in range(200)}
    assert outcomes & {"stale", "deadlock"}
