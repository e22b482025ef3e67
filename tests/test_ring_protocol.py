"""Model check of the state ring of the persistent kernels (CPU).

The persistent year and reverse-sweep kernels publish the state of step t
into slot t mod 2K of a ring that holds a sentinel until the owner writes it.
Every K steps the domains hand over (each publishes its phase counter and
waits for the counters of its neighbours); in step jj, after publishing state
jj + 1, a domain resets its rows of the slot of state jj + K.  This test runs
the same rules in a sequentially consistent model with domains advancing in
random order (one event per action, a domain blocked while what it waits for
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


def run(G, K, nsteps, seed, reset_offset=None):
    """One random schedule; returns "ok", "stale" or "deadlock".

    reset_offset: the state whose slot step jj resets is jj + reset_offset
    (the kernels use K)."""
    off = K if reset_offset is None else reset_offset
    rng = random.Random(seed)
    # before the launch: slot 0 the initial state, slots 1 .. K-1 the sentinel;
    # slots K .. 2K-1 keep whatever an earlier launch left (here: stale values)
    ring = {(d, s): (SENT if s < K else ("y", -1 - s)) for d in range(G) for s in range(2 * K)}
    for d in range(G):
        ring[(d, 0)] = ("y", 0)
    deps = {d: sorted({(d - 1) % G, (d + 1) % G} - {d}) for d in range(G)}
    jj = [0] * G
    stage = [0] * G                                    # 0: hand-over, 1: read halo, 2: publish and reset
    flag = [0] * G
    done = events = 0
    while done < G:
        events += 1
        if events > 200 * G * (nsteps + 2):
            return "deadlock"
        d = rng.choice([x for x in range(G) if jj[x] < nsteps])
        j = jj[d]
        if stage[d] == 0:
            if j % K == 0 and j > 0:
                flag[d] = max(flag[d], j // K)
                if any(flag[e] < j // K for e in deps[d]):
                    continue                           # waits at the hand-over
            stage[d] = 1
        elif stage[d] == 1:
            ready = True
            for e in deps[d]:
                v = ring[(e, j % (2 * K))]
                if v is SENT:
                    ready = False                      # not published yet: read again later
                    break
                if v != ("y", j):
                    return "stale"
            if ready:
                stage[d] = 2
        else:
            if j + 1 < nsteps:
                ring[(d, (j + 1) % (2 * K))] = ("y", j + 1)
            ring[(d, (j + off) % (2 * K))] = SENT
            jj[d] += 1
            stage[d] = 0
            if jj[d] == nsteps:
                done += 1
    return "ok"


@pytest.mark.parametrize("G,K,nsteps", [(2, 2, 7), (3, 2, 17), (5, 4, 33), (8, 4, 40), (6, 8, 100),
                                        (7, 64, 300), (4, 64, 24), (3, 3, 2), (5, 2, 64)])
def test_ring_reads_are_never_stale_and_every_schedule_completes(G, K, nsteps):
    for seed in range(40):
        assert run(G, K, nsteps, seed) == "ok", seed


@pytest.mark.parametrize("K,offset", [(1, 1), (4, 1), (4, 0), (8, 0)])
def test_model_catches_wrong_reset_rules(K, offset):
    """The check has teeth: a phase of one step (the reset hits the slot just
    published), or a reset of the slot of state jj (still being read) or of
    state jj + 1 (just published), makes some schedule read a reset or stale
    slot, or wait for ever.  (Offsets between 2 and 2K - 1 other than K are
    safe in this sequentially consistent model; the kernels use K because only
    then a hand-over, with its release and acquire, lies between the reads of
    a slot's previous state and its reset, and between the reset and the reads
    of the new state.)"""
    outcomes = {run(4, K, 24, seed, reset_offset=offset) for seed in range(200)}
    assert outcomes & {"stale", "deadlock"}, outcomes
