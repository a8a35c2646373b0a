"""The tile hand-over of the wave-specialised rollout (rollout_pipe.hip) as a host model: eight
walkers and four state waves under random interleavings, with the kernel's rules for which tiles a
walker reads and releases, the counters it waits on, and the state waves' order of generation,
variance reads and meetings.  Every schedule must finish (no wait can block for good), every walker
read of tile c in slot e must see the tile as written for slot e, no tile may be rewritten while a
walker still has to read it in the earlier slot, and no row of the four-slot ring of variance
partials may be rewritten before every state wave has read it."""
import random

import pytest

NT = 32          # column tiles at M_pad = 1024
WALKERS = 8
STATE = 4
VROWS = 4        # slots of variance partials kept


def users(c):
    """Walkers that read tile c in a slot (the kernel's pipe_users)."""
    return 8 if c <= 17 else (31 - c) // 2 + 1


def walker_reads(w):
    """Walker w's reads in one slot: (tile, last read of that tile in the slot)."""
    hi, lo = NT // 2 - 1 - w, w
    seq = []
    for pair_index, u in enumerate((hi, lo)):
        for it in range(2 * u + 1, -1, -1):          # columns descending
            last = pair_index == 1 or it > 2 * lo + 1
            seq.append((it, last))
    return seq


def state_tiles(g):
    return [NT - 1 - g - STATE * n for n in range(NT // STATE)]


def test_users_count_the_walkers_that_read_a_tile():
    for c in range(NT):
        readers = sum(any(t == c for t, _ in walker_reads(w)) for w in range(WALKERS))
        assert readers == users(c)
        # every reader releases the tile exactly once per slot
        releases = sum(sum(1 for t, last in walker_reads(w) if t == c and last) for w in range(WALKERS))
        assert releases == users(c)
    # and the last read of a tile by a walker comes after all its other reads of it
    for w in range(WALKERS):
        seq = walker_reads(w)
        for i, (t, last) in enumerate(seq):
            if last:
                assert all(t2 != t for t2, _ in seq[i + 1:])


class Sim:
    def __init__(self, T, seed):
        self.T, self.nslot = T, 2 * T
        self.rng = random.Random(seed)
        self.ready = [0] * NT
        self.freed = [0] * NT
        self.vdone = [0] * WALKERS
        self.sbar = 0
        self.tile_slot = [None] * NT      # slot whose kernel vector tile c holds
        self.pending = [0] * NT           # walkers still to read tile c in the slot it holds
        self.vrow = [[None] * WALKERS for _ in range(VROWS)]   # slot whose partial each row holds
        self.vread = {}                   # slot -> state waves that have read its partials

    def walker(self, w):
        seq = walker_reads(w)
        for e in range(self.nslot):
            for c, last in seq:
                while self.ready[c] < e + 1:                  # need(c, e)
                    yield
                assert self.tile_slot[c] == e, (w, c, e, self.tile_slot[c])
                if last:
                    self.pending[c] -= 1
                    self.freed[c] += 1
                yield
            r = e % VROWS
            if e >= VROWS:
                assert self.vread.get(e - VROWS, 0) == STATE, (w, e)
            self.vrow[r][w] = e
            self.vdone[w] = e + 1
            yield

    def gen(self, g, e):
        for jt in state_tiles(g):
            if e > 0:
                while self.freed[jt] < users(jt) * e:         # pipe_wait(freed)
                    yield
            assert self.pending[jt] == 0, (g, jt, e)          # no walker still to read the old tile
            self.tile_slot[jt] = e
            self.pending[jt] = users(jt)
            self.ready[jt] = e + 1
            yield

    def state(self, g):
        met = 0
        for k in range(self.T):
            yield from self.gen(g, 2 * k)
            if k > 0:
                yield from self.variances(k - 1)
            yield                                             # sample step, constraint loops
            yield from self.gen(g, 2 * k + 1)
            met += STATE
            self.sbar += 1
            while self.sbar < met:                            # the state waves meet
                yield
        yield from self.variances(self.T - 1)

    def variances(self, k):
        while min(self.vdone) < 2 * k + 2:
            yield
        for e in (2 * k, 2 * k + 1):
            assert self.vrow[e % VROWS] == [e] * WALKERS, (k, e, self.vrow[e % VROWS])
            self.vread[e] = self.vread.get(e, 0) + 1
        yield

    def run(self, max_steps=10 ** 6):
        agents = [self.walker(w) for w in range(WALKERS)] + [self.state(g) for g in range(STATE)]
        # uneven speeds: each agent moves with a weight drawn once per schedule
        speed = [self.rng.expovariate(1.0) + 0.01 for _ in agents]
        live = list(range(len(agents)))
        steps = 0
        while live:
            i = self.rng.choices(live, weights=[speed[j] for j in live])[0]
            try:
                next(agents[i])
            except StopIteration:
                live.remove(i)
            steps += 1
            assert steps < max_steps, "no progress: a wait that never ends"
        assert self.vdone == [self.nslot] * WALKERS
        assert all(f == users(c) * self.nslot for c, f in enumerate(self.freed))
        assert all(self.vread[e] == STATE for e in range(self.nslot))


@pytest.mark.parametrize("seed", range(24))
def test_random_interleavings_finish_and_read_the_right_slot(seed):
    Sim(T=4, seed=seed).run()


def test_a_walker_ahead_of_the_others_waits_for_the_tiles_they_still_read():
    # the first walker of each SIMD runs far ahead: schedule it whenever it can move
    sim = Sim(T=3, seed=99)
    agents = [sim.walker(w) for w in range(WALKERS)] + [sim.state(g) for g in range(STATE)]
    live = list(range(len(agents)))
    steps = 0
    while live:
        fast = [i for i in live if i < 4]
        i = fast[0] if fast and sim.rng.random() < 0.9 else sim.rng.choice(live)
        try:
            next(agents[i])
        except StopIteration:
            live.remove(i)
        steps += 1
        assert steps < 10 ** 6
    assert sim.vdone == [sim.nslot] * WALKERS
