"""Host model of the persistent sweep's tile protocol (single-launch formal solution).

The persistent kernel runs a whole formal solution (section 3.1: the tiles of one
octant are swept in upwind-to-downwind order; octants and frequency bins are
independent) in one launch.  Workgroup b serves octant b & 7; thread 0 of the
workgroup publishes the tile it finished last and draws the next ticket from the
octant's counter; ticket t is tile tiles[t % ntiles] of bin t // ntiles; before a
tile reads the outgoing faces of its upwind neighbours, thread 0 waits until their
completion flags carry the sweep's epoch.

Here every wave is a Python generator that yields at each workgroup barrier and at
each poll of a flag, and a seeded scheduler interleaves the waves of the resident
workgroups at random, with a bounded number of workgroups resident at once (the
rest start, in block order, as resident ones exit).  Every index the kernel forms
is bounds-checked.  The model checks that every tile of every live bin and octant
is swept once, that a tile's upwind neighbours are complete when it reads their
faces, that all waves of a workgroup agree on each ticket, that no wait runs out
and that the launch ends, also for two launches in a row on the same flags (the
epoch) and with frozen bins.

The batched form (one launch over the members of a batch class) is modelled the same
way: its work list runs stage by stage over all members, bins and tiles, each member
keeps its own completion flags and epoch (advanced before every sweep, so flags left by
the member's single solves are stale), and the octants' counters are shared.

It also models the control flow the compiler once produced for this loop, when the
ticket lived in a vector register: after a tile's last barrier lane 0 of wave 0
(the only lane that publishes and draws) waited for lanes 1..63 to leave the
loop, while they and the other waves went round again on the old ticket.  In that
form the workgroup sweeps its first tile over and over, which the model reports.
"""
import random

import pytest

T = 8   # tile edge of the sweep kernels


def tile_schedule(n):
    """Tiles in hyperplane order: stage s holds tiles with tx + ty + tz = s."""
    nt = [(v + T - 1) // T for v in n]
    tiles = []
    for s in range(nt[0] + nt[1] + nt[2] - 2):
        for tz in range(nt[2]):
            for ty in range(nt[1]):
                tx = s - ty - tz
                if 0 <= tx < nt[0]:
                    tiles.append(tx | (ty << 10) | (tz << 20))
    return nt, tiles


class Livelock(Exception):
    """A workgroup swept a ticket it had swept before in the same launch."""


class Checked(list):
    """A device array whose every access is bounds-checked."""

    def _ix(self, i):
        if not 0 <= i < len(self):
            raise IndexError(f"index {i} outside [0, {len(self)})")
        return i

    def __getitem__(self, i):
        return list.__getitem__(self, self._ix(i))

    def __setitem__(self, i, v):
        list.__setitem__(self, self._ix(i), v)


class Launch:
    def __init__(self, n, nf, waves, bpo, resident, frozen=(), seed=0, split=False, poll_limit=20000,
                 done=None, epoch=1):
        self.nt, tiles = tile_schedule(n)
        self.ntiles = len(tiles)
        assert self.ntiles == self.nt[0] * self.nt[1] * self.nt[2]
        self.tiles = Checked(tiles)
        self.nf, self.W, self.epoch = nf, waves, epoch
        self.frozen = Checked([1 if f in frozen else 0 for f in range(nf)])
        self.counter = Checked([0] * 8)
        self.done = done if done is not None else Checked([0] * (nf * 8 * self.ntiles))
        assert len(self.done) == nf * 8 * self.ntiles
        self.err = 0
        self.rng = random.Random(seed)
        self.split = split
        self.poll_limit = poll_limit
        self.grid = 8 * bpo
        self.resident = resident
        self.faces = {}       # (f, oct, tile id) -> waves that wrote their outgoing faces
        self.swept = {}       # (f, oct, tile id) -> times swept
        self.violations = []

    def tile_id(self, tx, ty, tz):
        assert 0 <= tx < self.nt[0] and 0 <= ty < self.nt[1] and 0 <= tz < self.nt[2]
        return (tz * self.nt[1] + ty) * self.nt[0] + tx

    def flag(self, f, oct, tid):
        return ((f * 8) + oct) * self.ntiles + tid

    # one wave of workgroup b; yields "bar" at each workgroup barrier, "poll" at each
    # poll of a completion flag
    def wave(self, b, w, wg):
        oct = b & 7
        items = self.ntiles * self.nf
        done_f = done_tile = -1
        first = True
        seen = set()
        while True:
            thread0 = w == 0 and (first or not self.split)
            if thread0:
                if done_tile >= 0:
                    self.done[self.flag(done_f, oct, done_tile)] = self.epoch
                wg["ticket"] = self.counter[oct]
                self.counter[oct] += 1
            yield "bar"
            t = wg["ticket"]
            wg.setdefault("reads", {}).setdefault(wg["iter"][w], set()).add(t)
            wg["iter"][w] += 1
            yield "bar"
            if t >= items:
                return
            f, tile = divmod(t, self.ntiles)
            packed = self.tiles[tile]
            done_tile = -1
            if self.frozen[f] or packed < 0:
                first = False
                continue
            if t in seen:
                raise Livelock(f"workgroup {b} swept ticket {t} twice")
            seen.add(t)
            tx, ty, tz = packed & 1023, (packed >> 10) & 1023, (packed >> 20) & 1023
            tid = self.tile_id(tx, ty, tz)
            ups = []
            if tx > 0:
                ups.append(self.tile_id(tx - 1, ty, tz))
            if ty > 0:
                ups.append(self.tile_id(tx, ty - 1, tz))
            if tz > 0:
                ups.append(self.tile_id(tx, ty, tz - 1))
            # staging loads of chi and S (inputs: no dependency), then thread 0 waits
            if thread0:
                for u in ups:
                    polls = 0
                    while self.done[self.flag(f, oct, u)] != self.epoch:
                        if self.err:
                            break
                        polls += 1
                        if polls > self.poll_limit:
                            self.err = 1
                            break
                        yield "poll"
            yield "bar"
            # every wave reads the upwind faces of its rays
            for u in ups:
                if self.faces.get((f, oct, u), 0) != self.W:
                    self.violations.append((b, t, u))
            yield "bar"      # staged tile and shells in LDS
            yield "poll"     # the rays of the wave (no workgroup barrier)
            yield "bar"      # partial sums of all waves in LDS
            key = (f, oct, tid)
            self.faces[key] = self.faces.get(key, 0) + 1     # this wave's outgoing faces
            if w == 0:
                self.swept[key] = self.swept.get(key, 0) + 1
            yield "bar"      # every wave's stores complete; thread 0 releases at the loop top
            done_f, done_tile = f, tid
            first = False

    def run(self, max_steps=3_000_000):
        pending = list(range(self.grid))      # blocks not yet started, in block order
        running = {}
        steps = 0

        def start(b):
            wg = {"iter": [0] * self.W, "blocked": set()}
            wg["gens"] = {w: self.wave(b, w, wg) for w in range(self.W)}
            running[b] = wg

        while pending and len(running) < self.resident:
            start(pending.pop(0))
        while running:
            steps += 1
            if steps > max_steps:
                raise Livelock(f"no end after {max_steps} steps")
            b = self.rng.choice(list(running))
            wg = running[b]
            live = [w for w in wg["gens"] if w not in wg["blocked"]]
            w = self.rng.choice(live)
            try:
                ev = next(wg["gens"][w])
            except StopIteration:
                del wg["gens"][w]
                wg["blocked"].discard(w)
                ev = None
            if ev == "bar":
                wg["blocked"].add(w)
            # a barrier opens when every wave still running has arrived
            if wg["gens"] and wg["blocked"] == set(wg["gens"]):
                wg["blocked"] = set()
            if not wg["gens"]:
                del running[b]
                for it, ts in wg.get("reads", {}).items():
                    if len(ts) != 1:
                        self.violations.append(("tickets differ", b, it, sorted(ts)))
                if pending:
                    start(pending.pop(0))
        return steps


CASES = [
    # shape, bins, waves, workgroups per octant, resident workgroups, frozen bins
    ((19, 13, 11), 2, 3, 24, 192, ()),
    ((19, 13, 11), 2, 3, 24, 40, ()),
    ((19, 13, 11), 2, 1, 5, 8, ()),
    ((24, 24, 24), 1, 3, 2, 3, ()),
    ((24, 24, 24), 1, 2, 27, 216, ()),
    ((9, 17, 8), 3, 3, 4, 16, (1,)),
    ((40, 8, 16), 2, 4, 10, 1, ()),
    ((8, 8, 8), 4, 3, 3, 24, (0, 2)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_persistent_protocol_sweeps_every_tile_once_in_dependency_order(case):
    shape, nf, waves, bpo, resident, frozen = CASES[case]
    for seed in range(3):
        L = Launch(shape, nf, waves, bpo, resident, frozen=frozen, seed=1000 * case + seed)
        L.run()
        assert L.violations == []
        assert L.err == 0
        for f in range(nf):
            for oct in range(8):
                for tid in range(L.ntiles):
                    want = 0 if f in frozen else 1
                    assert L.swept.get((f, oct, tid), 0) == want, (f, oct, tid)
                    flag = L.done[L.flag(f, oct, tid)]
                    assert flag == (0 if f in frozen else L.epoch)
        # every workgroup drew one ticket past the end
        assert all(c >= L.ntiles * nf for c in L.counter)


def test_epochs_keep_two_launches_apart():
    """A second launch on the same flags (epoch 2) waits for its own publications."""
    shape, nf = (19, 13, 11), 2
    first = Launch(shape, nf, 3, 6, 48, seed=7, epoch=1)
    first.run()
    second = Launch(shape, nf, 3, 6, 48, seed=8, epoch=2, done=first.done)
    second.run()
    assert second.violations == [] and second.err == 0
    assert all(v == 2 for v in second.done)


def test_stale_flags_would_be_caught():
    """The checks of the model are live: with flags left at the current epoch by a
    previous launch, tiles read neighbours that are not yet complete."""
    shape, nf = (24, 24, 24), 1
    nt, tiles = tile_schedule(shape)
    stale = Checked([1] * (nf * 8 * len(tiles)))
    L = Launch(shape, nf, 3, 27, 216, seed=3, epoch=1, done=stale)
    L.run()
    assert L.violations


def test_split_lane_loop_sweeps_its_first_tile_again():
    """The control flow compiled from a ticket held in a vector register: lanes
    1..63 of wave 0 and the other waves go round again without a new ticket."""
    with pytest.raises(Livelock):
        Launch((19, 13, 11), 2, 3, 24, 192, seed=5, split=True).run()


def test_schedule_indices_stay_in_bounds():
    for shape in [(1, 1, 1), (8, 8, 8), (9, 8, 8), (127, 3, 200), (1023 * 8, 8, 8)]:
        nt, tiles = tile_schedule(shape)
        assert len(tiles) == nt[0] * nt[1] * nt[2]
        ids = set()
        for p in tiles:
            tx, ty, tz = p & 1023, (p >> 10) & 1023, (p >> 20) & 1023
            assert p >= 0 and tx < nt[0] and ty < nt[1] and tz < nt[2]
            ids.add((tz * nt[1] + ty) * nt[0] + tx)
        assert ids == set(range(len(tiles)))
        # upwind neighbours come earlier in the list
        pos = {p: i for i, p in enumerate(tiles)}
        for p in tiles[: 2000]:
            tx, ty, tz = p & 1023, (p >> 10) & 1023, (p >> 20) & 1023
            for q in [(tx - 1, ty, tz), (tx, ty - 1, tz), (tx, ty, tz - 1)]:
                if min(q) >= 0:
                    assert pos[q[0] | (q[1] << 10) | (q[2] << 20)] < pos[p]


def batch_work_list(members):
    """Items (member, bin, position in the member's tile list), stage by stage, then
    member, bin and tile: the list the host builds for a persistent batch class."""
    sched = []
    for shape, nf in members:
        nt, tiles = tile_schedule(shape)
        stage_off = [0] * (nt[0] + nt[1] + nt[2] - 1)
        for i, p in enumerate(tiles):
            st = (p & 1023) + ((p >> 10) & 1023) + ((p >> 20) & 1023)
            stage_off[st + 1] = i + 1
        for k in range(1, len(stage_off)):
            stage_off[k] = max(stage_off[k], stage_off[k - 1])
        sched.append((nt, tiles, stage_off))
    items = []
    for st in range(max(len(o) - 1 for _, _, o in sched)):
        for j, ((shape, nf), (nt, tiles, off)) in enumerate(zip(members, sched)):
            if st >= len(off) - 1:
                continue
            for f in range(nf):
                for z in range(off[st], off[st + 1]):
                    items.append((j, f, z))
    return sched, items


class BatchLaunch(Launch):
    """One persistent launch over several members of different shapes and bins."""

    def __init__(self, members, waves, bpo, resident, frozen=None, seed=0, poll_limit=20000, stale=None):
        self.members = members
        self.sched, items = batch_work_list(members)
        self.items = Checked(items)
        self.W = waves
        self.frozen = [Checked([1 if (frozen and f in frozen.get(j, ())) else 0 for f in range(nf)])
                       for j, (_, nf) in enumerate(members)]
        self.rng = random.Random(seed)
        # flags left by earlier sweeps of each member (its single solves included): any
        # value up to the member's last epoch; the batch sweep runs with the next one
        self.epochs = []
        self.done = []
        for j, (shape, nf) in enumerate(members):
            ntiles = len(self.sched[j][1])
            last = stale[j] if stale else self.rng.randrange(0, 50)
            self.done.append(Checked([self.rng.randrange(0, last + 1) for _ in range(nf * 8 * ntiles)]))
            self.epochs.append(last + 1)
        self.counter = Checked([0] * 8)
        self.err = 0
        self.split = False
        self.poll_limit = poll_limit
        self.grid = 8 * bpo
        self.resident = resident
        self.faces, self.swept, self.violations = {}, {}, []

    def wave(self, b, w, wg):
        oct = b & 7
        pub = None            # (member, flag index) of the tile finished last, and its epoch
        seen = set()
        while True:
            if w == 0:
                if pub is not None:
                    j0, i0, e0 = pub
                    self.done[j0][i0] = e0
                wg["ticket"] = self.counter[oct]
                self.counter[oct] += 1
            yield "bar"
            t = wg["ticket"]
            wg.setdefault("reads", {}).setdefault(wg["iter"][w], set()).add(t)
            wg["iter"][w] += 1
            yield "bar"
            if t < 0 or t >= len(self.items):
                return
            j, f, z = self.items[t]
            nt, tiles, _ = self.sched[j]
            packed = Checked(tiles)[z]
            epoch = self.epochs[j]
            pub = None
            if self.frozen[j][f] or packed < 0:
                continue
            if t in seen:
                raise Livelock(f"workgroup {b} swept ticket {t} twice")
            seen.add(t)
            tx, ty, tz = packed & 1023, (packed >> 10) & 1023, (packed >> 20) & 1023
            assert tx < nt[0] and ty < nt[1] and tz < nt[2]
            tid = (tz * nt[1] + ty) * nt[0] + tx
            ntiles = len(tiles)
            ups = []
            if tx > 0:
                ups.append(tid - 1)
            if ty > 0:
                ups.append(tid - nt[0])
            if tz > 0:
                ups.append(tid - nt[0] * nt[1])
            if w == 0:
                for u in ups:
                    polls = 0
                    while self.done[j][(f * 8 + oct) * ntiles + u] != epoch:
                        if self.err:
                            break
                        polls += 1
                        if polls > self.poll_limit:
                            self.err = 1
                            break
                        yield "poll"
            yield "bar"
            for u in ups:
                if self.faces.get((j, f, oct, u), 0) != self.W:
                    self.violations.append((b, t, j, u))
            yield "bar"
            yield "poll"
            yield "bar"
            key = (j, f, oct, tid)
            self.faces[key] = self.faces.get(key, 0) + 1
            if w == 0:
                self.swept[key] = self.swept.get(key, 0) + 1
            yield "bar"
            pub = (j, (f * 8 + oct) * ntiles + tid, epoch)


BATCH_CASES = [
    # members (shape, bins), waves, workgroups per octant, resident workgroups, frozen bins per member
    ([((19, 13, 11), 2), ((8, 8, 8), 1), ((24, 9, 17), 3)], 3, 12, 96, {}),
    ([((19, 13, 11), 2), ((8, 8, 8), 1), ((24, 9, 17), 3)], 2, 3, 10, {2: (1,)}),
    ([((40, 8, 16), 1), ((9, 17, 8), 2)], 1, 6, 8, {0: (0,)}),
    ([((16, 16, 16), 1)] * 4, 3, 20, 160, {}),
    ([((7, 7, 7), 1), ((33, 25, 9), 2)], 4, 2, 3, {}),
]


@pytest.mark.parametrize("case", range(len(BATCH_CASES)))
def test_persistent_batch_sweeps_every_member_tile_once_in_order(case):
    members, waves, bpo, resident, frozen = BATCH_CASES[case]
    for seed in range(3):
        L = BatchLaunch(members, waves, bpo, resident, frozen=frozen, seed=100 * case + seed)
        L.run()
        assert L.violations == [] and L.err == 0
        for j, (shape, nf) in enumerate(members):
            ntiles = len(L.sched[j][1])
            for f in range(nf):
                off = f in frozen.get(j, ())
                for oct in range(8):
                    for tid in range(ntiles):
                        assert L.swept.get((j, f, oct, tid), 0) == (0 if off else 1), (j, f, oct, tid)
                        if not off:
                            assert L.done[j][(f * 8 + oct) * ntiles + tid] == L.epochs[j]
        assert all(c >= len(L.items) for c in L.counter)


def test_persistent_batch_work_list_order():
    """Every tile of every member and bin is listed once, and a tile's upwind
    neighbours (same member and bin) are listed before it."""
    members = [((19, 13, 11), 2), ((8, 8, 8), 1), ((24, 9, 17), 3), ((1, 1, 1), 2)]
    sched, items = batch_work_list(members)
    pos = {}
    for i, (j, f, z) in enumerate(items):
        nt, tiles, _ = sched[j]
        p = tiles[z]
        key = (j, f, p & 1023, (p >> 10) & 1023, (p >> 20) & 1023)
        assert key not in pos
        pos[key] = i
    assert len(items) == sum(nf * len(sched[j][1]) for j, (_, nf) in enumerate(members))
    for (j, f, tx, ty, tz), i in pos.items():
        for q in [(tx - 1, ty, tz), (tx, ty - 1, tz), (tx, ty, tz - 1)]:
            if min(q) >= 0:
                assert pos[(j, f) + q] < i


def test_persistent_batch_stale_epoch_would_be_caught():
    """The epoch check is live: flags of one member left at the epoch of the batch sweep
    (an epoch not advanced) let its tiles read upwind faces not yet written."""
    members = [((24, 24, 24), 1), ((16, 8, 8), 1)]
    L = BatchLaunch(members, 3, 27, 216, seed=4, stale=[5, 5])
    L.done[0] = Checked([L.epochs[0]] * len(L.done[0]))
    L.run()
    assert L.violations
