"""A model of the job board of the D1 workgroup pass's cooperative merges, on
the CPU.

A workgroup whose column needs a long full merge cuts it into parts and posts
it as a job in a slot of a small board; idle workgroups take parts of open
jobs. Per slot the kernel keeps four words: W0 = (sequence << 32 | parts
taken), W1 = parts finished, W2 = slot claimed, W3 = (sequence << 32 | number
of parts), next to the job's fields (pointers and sizes). The owner claims a
slot, writes W1, W3 and the fields, opens the job by writing W0 with an odd
sequence, takes parts with fetch-and-add on W0, waits until W1 counts every
part, closes the job (even sequence) and frees the slot. A helper checks W0
and W3 for an open job with parts left, takes one with fetch-and-add on W0,
re-reads W3, and merges the part only when the sequence it took is the one W3
names and the part index is below the part count; then it reads the fields and
counts the part in W1.

Each shared-memory operation of that sequence is one step here, and random
schedules interleave several owners (each running jobs one after another) and
helpers over few slots. The checks: every part of every job is merged exactly
once, by a workgroup that read that job's fields, while the job is open, and
no job closes before all its parts are merged. It shares no code with the
kernel.
"""
import random

import pytest

M32 = (1 << 32) - 1


class Board:
    def __init__(self, nslots):
        self.w = [[0, 0, 0, 0] for _ in range(nslots)]
        self.fields = [None] * nslots
        self.open_jobs = 0
        self.done = {}  # (job, part) -> times merged
        self.open = set()  # jobs open now
        self.closed = set()


def owner(B, jobs, log):
    """Generator: one step per shared-memory operation."""
    for job, nparts in jobs:
        slot = -1
        for s in range(len(B.w)):
            yield
            if B.w[s][2] == 0:  # compare-and-swap 0 -> 1
                B.w[s][2] = 1
                slot = s
                break
        if slot < 0:  # no free slot: the owner merges every part alone
            for k in range(nparts):
                yield
                B.done[(job, k)] = B.done.get((job, k), 0) + 1
            continue
        w = B.w[slot]
        yield
        seq = (w[0] >> 32) + 1  # odd: open
        yield
        w[1] = 0
        yield
        w[3] = (seq << 32) | nparts
        yield
        B.fields[slot] = job
        yield
        w[0] = seq << 32  # exchange: the job opens
        B.open.add(job)
        yield
        B.open_jobs += 1
        while True:
            yield
            r = w[0]
            w[0] = r + 1  # fetch-and-add
            k = r & M32
            if k >= nparts:
                break
            assert job in B.open
            B.done[(job, k)] = B.done.get((job, k), 0) + 1
            yield
            w[1] += 1
        while True:  # every part taken by a helper ends
            yield
            if w[1] >= nparts:
                break
        for k in range(nparts):
            assert B.done.get((job, k), 0) == 1, (job, k, B.done.get((job, k)))
        yield
        s2 = w[0] >> 32
        yield
        w[0] = (s2 + 1) << 32  # exchange: even, closed
        B.open.discard(job)
        B.closed.add(job)
        yield
        B.open_jobs -= 1
        yield
        w[2] = 0  # the slot is free again
        log.append(job)


def helper(B, start, stop):
    while not stop[0]:
        yield
        if B.open_jobs == 0:
            continue
        n = len(B.w)
        for i in range(n):  # one slot per lane of the first wave, from a rotating start
            s = (start + i) % n
            yield
            c = B.w[s][0]
            yield
            sp = B.w[s][3]
            if ((c >> 32) & 1) and (c >> 32) == (sp >> 32) and (c & M32) < (sp & M32):
                break
        else:
            continue
        w = B.w[s]
        yield
        r = w[0]
        w[0] = r + 1  # fetch-and-add
        if not ((r >> 32) & 1):
            continue
        yield
        sp2 = w[3]
        if (sp2 >> 32) != (r >> 32) or (r & M32) >= (sp2 & M32):
            continue
        part = r & M32
        yield
        job = B.fields[s]
        # the fields belong to the job whose sequence the part was taken under
        assert job in B.open and job not in B.closed, (job, part)
        assert part < dict(JOBS_N)[job]
        yield
        B.done[(job, part)] = B.done.get((job, part), 0) + 1
        assert job in B.open, (job, part)
        yield
        w[1] += 1


JOBS_N = []


@pytest.mark.parametrize("seed", range(200))
def test_every_part_once_and_jobs_close_after_their_parts(seed):
    rng = random.Random(seed)
    nslots = rng.choice([1, 2, 3])
    nowners = rng.choice([1, 2, 3, 4])
    nhelpers = rng.choice([1, 2, 3, 5])
    JOBS_N.clear()
    per_owner = []
    jid = 0
    for o in range(nowners):
        jobs = []
        for _ in range(rng.choice([1, 2, 3])):
            nparts = rng.choice([1, 2, 3, 5, 9])
            jobs.append((jid, nparts))
            JOBS_N.append((jid, nparts))
            jid += 1
        per_owner.append(jobs)
    B = Board(nslots)
    log = []
    stop = [False]
    owners = [owner(B, jobs, log) for jobs in per_owner]
    helpers = [helper(B, rng.randrange(nslots), stop) for _ in range(nhelpers)]
    live = owners + helpers
    steps = 0
    while any(o is not None for o in owners):
        i = rng.randrange(len(live))
        g = live[i]
        if g is None:
            continue
        try:
            next(g)
        except StopIteration:
            if i < len(owners):
                owners[i] = None
            live[i] = None
        steps += 1
        assert steps < 2_000_000, "no progress"
    stop[0] = True
    for jid_, nparts in JOBS_N:
        for k in range(nparts):
            assert B.done.get((jid_, k), 0) == 1, (jid_, k)
    assert B.open_jobs == 0 and not B.open
    assert all(w[2] == 0 and not ((w[0] >> 32) & 1) for w in B.w)
