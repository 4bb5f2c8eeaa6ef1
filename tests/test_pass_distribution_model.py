"""Host model of the particle pass's dynamic work distribution (pass_dyn_kernel: ring_start,
next_sub, ring_wait in csrc/pic_kernels.hip), run under random interleavings of its waves.

Blocks of 4096 slots come from a per-species counter; a workgroup's waves take 4-iteration
sub-blocks of 64 consecutive slots from an LDS counter; the wave holding a block's first
sub-block fetches the workgroup's block two ahead once the block one ahead is published in
an 8-entry tagged ring.  The model checks what the kernel relies on: every slot is taken
exactly once, no wait is left unsatisfied (no deadlock), and no ring entry is overwritten
while a wave still needs it.  The static mode (a workgroup's own range, sub-blocks from the
LDS counter only) is checked the same way.
"""
import random

import pytest

SUB_ITERS, BLOCK_SUBS, RING = 4, 16, 8
SUB_SLOTS = 64 * SUB_ITERS
BLOCK_SLOTS = SUB_SLOTS * BLOCK_SUBS
NOBLOCK = 0xFFFFFFFF


def run_dynamic(ns, n_wg, n_waves, seed):
    rng = random.Random(seed)
    nblk = (ns + BLOCK_SLOTS - 1) // BLOCK_SLOTS
    counter = [0]
    taken = [0] * ns
    wgs = []
    for _ in range(n_wg):   # ring_start: blocks 0 and 1 with one atomic, other tags unreachable
        b = counter[0]
        counter[0] += 2
        ring = [(-1, 0)] * RING
        ring[0] = (0, b if b < nblk else NOBLOCK)
        ring[1] = (1, b + 1 if b + 1 < nblk else NOBLOCK)
        wgs.append({"ring": ring, "sub": 0})

    def wave(L):
        def wait(j):
            for _ in range(100_000):
                tag, val = L["ring"][j % RING]
                if tag == j:
                    return val
                assert tag < j, "ring entry overwritten before it was read"
                yield
            raise AssertionError("wait never satisfied")

        def next_sub():
            s = L["sub"]
            L["sub"] += 1
            yield
            j, q = divmod(s, BLOCK_SUBS)
            if q == 0:   # fetch block j + 2 once block j + 1 is published
                prev = yield from wait(j + 1)
                bid = NOBLOCK
                if prev != NOBLOCK:
                    b = counter[0]
                    counter[0] += 1
                    yield
                    if b < nblk:
                        bid = b
                L["ring"][(j + 2) % RING] = (j + 2, bid)
                yield
            bid = yield from wait(j)
            if bid == NOBLOCK:
                return -1
            base = bid * BLOCK_SLOTS + q * SUB_SLOTS
            return base if base < ns else -1

        while True:
            base = yield from next_sub()
            if base < 0:
                return
            for k in range(SUB_ITERS):
                for lane in range(64):
                    i = base + 64 * k + lane
                    if i < ns:
                        taken[i] += 1
                if rng.random() < 0.5:
                    yield

    waves = [wave(wgs[w // n_waves]) for w in range(n_wg * n_waves)]
    alive = list(range(len(waves)))
    while alive:
        k = rng.choice(alive)
        try:
            next(waves[k])
        except StopIteration:
            alive.remove(k)
    assert all(t == 1 for t in taken)


def run_static(ns, n_wg, n_waves, seed):
    rng = random.Random(seed)
    per = (ns + n_wg - 1) // n_wg if n_wg else 0
    taken = [0] * ns
    for g in range(n_wg):
        b, e = min(g * per, ns), min(g * per + per, ns)
        sub = [0]

        def wave():
            while True:
                s = sub[0]
                sub[0] += 1
                yield
                base = b + s * SUB_SLOTS
                if base >= e:
                    return
                for k in range(SUB_ITERS):
                    for lane in range(64):
                        i = base + 64 * k + lane
                        if i < e:
                            taken[i] += 1
                    yield

        ws = [wave() for _ in range(n_waves)]
        alive = list(range(n_waves))
        while alive:
            k = rng.choice(alive)
            try:
                next(ws[k])
            except StopIteration:
                alive.remove(k)
    assert all(t == 1 for t in taken)


@pytest.mark.parametrize("ns,n_wg,n_waves", [(0, 1, 16), (1, 1, 16), (255, 2, 4), (4096, 3, 16), (4097, 3, 16),
                                             (50_000, 5, 16), (3 * 8192 + 17, 1, 16), (123_457, 16, 4)])
def test_every_slot_once_and_every_wait_satisfied(ns, n_wg, n_waves):
    for seed in range(3):
        run_dynamic(ns, n_wg, n_waves, seed)
        run_static(ns, n_wg, n_waves, seed)
