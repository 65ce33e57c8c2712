"""CPU model of the protocol of the batch's single-launch (persistent) form.

Work items are handed out in dependency order by an atomic ticket; a
finished item publishes a completion flag with a release store; a waiting
workgroup polls the flags it needs with relaxed device-coherent loads, then
acquires before reading the producers' data; every wait is bounded and
gives up at once when another workgroup has set the error word; the last
workgroup to leave clears the ticket, the exit count and the flags.

Only items that waited acquire, and only items whose output another item
of the launch reads (value gathers; numeric items of a product whose C is
another product's A or B) publish a flag.

Workgroups are coroutines stepped by a seeded random scheduler.  Each sits
on one of several "XCDs", each with a write-back cache of its own, in lines
of several values filled whole on a miss: a plain store dirties its value,
a release writes the dirty values back, an acquire drops the clean lines, a
plain load is served from the cache when the line is there; a launch starts
with an acquire and ends with a release on every XCD.  Relaxed device-coherent loads, release stores and returning atomics
act on memory itself (the forms the chained scans and work queues of the
library already rely on).

The model shows that the protocol drains and computes the sequential result
on every interleaving tried, including replays whose caches still hold the
previous replay's lines; that leaving out the release or the acquire lets a
consumer read stale values; that completion counts posted into the
issuing XCD's cache (a model of a count kept with atomic adds that are not
performed at the coherence point, the form an earlier version of the kernel
used, whose waits never completed) make the waits run out; and that a flag
that never arrives ends in the error word rather than a hang."""

import random

import pytest


LINE = 4  # values per cache line


def line_of(a):
    if a[0] in ("A", "B", "At", "C"):
        return (a[0], a[1], a[2] // LINE)
    return a


def members(line):
    if line[0] in ("A", "B", "At", "C"):
        return [(line[0], line[1], line[2] * LINE + i) for i in range(LINE)]
    return [line]


class Memory:
    """Memory and one write-back cache per XCD, in lines of LINE values.  A
    line is filled whole from memory on a miss (loads and stores alike), so
    a line holds values that other XCDs may overwrite later; dirty values
    are written back value by value (byte-masked)."""

    def __init__(self, xcds):
        self.glob = {}
        self.cache = [dict() for _ in range(xcds)]  # line -> {"v": {addr: val}, "d": set()}

    def _line(self, x, a):
        ln = line_of(a)
        c = self.cache[x]
        if ln not in c:
            c[ln] = {"v": {m: self.glob.get(m, 0) for m in members(ln)}, "d": set()}
        return c[ln]

    def load(self, x, a):
        return self._line(x, a)["v"][a]

    def store(self, x, a, v):
        ln = self._line(x, a)
        ln["v"][a] = v
        ln["d"].add(a)

    def release(self, x):
        for ln in self.cache[x].values():
            for a in ln["d"]:
                self.glob[a] = ln["v"][a]
            ln["d"].clear()

    def acquire(self, x):
        c = self.cache[x]
        for k in [k for k, ln in c.items() if not ln["d"]]:
            del c[k]

    def coherent_load(self, a):
        return self.glob.get(a, 0)

    def store_through(self, x, a, v):
        """A store at the coherence point (the issuing XCD's copy, if any,
        is updated too)."""
        self.glob[a] = v
        ln = self.cache[x].get(line_of(a))
        if ln is not None:
            ln["v"][a] = v
            ln["d"].discard(a)

    def release_store(self, x, a, v, with_release=True):
        if with_release:
            self.release(x)
        self.store_through(x, a, v)

    def atomic_add(self, a, v):
        old = self.glob.get(a, 0)
        self.glob[a] = old + v
        return old

    def posted_add(self, x, a, v):
        """An add merged into the issuing XCD's cache line, written back
        only at that XCD's next release."""
        self.store(x, a, self.load(x, a) + v)


def make_dag(rng, nprod):
    """Products with their dependencies; `in_place` products read their A
    values where they lie (A~ holds all of A) and so have no gathers."""
    prods = []
    for t in range(nprod):
        dep_a = rng.randrange(-1, t) if t else -1
        dep_b = rng.randrange(-1, t) if t else -1
        prods.append({"dep_A": dep_a, "dep_B": dep_b, "in_place": rng.random() < 0.4})
    return prods


def sequential(prods, width, inputs):
    """C_t[j] = sum_i A_t[i] * B_t[(i + j) % width]; A_t and B_t are an
    earlier product's C or the product's own input."""
    C = []
    for t, p in enumerate(prods):
        A = C[p["dep_A"]] if p["dep_A"] >= 0 else inputs[("A", t)]
        B = C[p["dep_B"]] if p["dep_B"] >= 0 else inputs[("B", t)]
        C.append([sum(A[i] * B[(i + j) % width] for i in range(width)) for j in range(width)])
    return C


def items_of(prods, width, tile):
    """Items in dependency order: per depth, every product's gathers, then
    every product's numeric tiles.  Returns the items and, per product, the
    first ticket and count of its gathers and of its numeric items."""
    depth = []
    for p in prods:
        d = 0
        for dep in (p["dep_A"], p["dep_B"]):
            if dep >= 0:
                d = max(d, depth[dep] + 1)
        depth.append(d)
    items = []
    span = {t: {} for t in range(len(prods))}
    for d in range(max(depth) + 1):
        lvl = [t for t in range(len(prods)) if depth[t] == d]
        for kind in ("gather", "numeric"):
            for t in lvl:
                if kind == "gather" and prods[t].get("in_place"):
                    span[t][kind] = (len(items), 0)
                    continue
                span[t][kind] = (len(items), len(range(0, width, tile)))
                for f in range(0, width, tile):
                    items.append((kind, t, f))
    return items, span


T, EXIT, ERR = ("ticket",), ("exit",), ("error",)


def run_launch(mem, prods, width, tile, inputs, n_wg, xcds, rng, release=True, acquire=True,
               publish="flag", lost=None, wait_bound=3000, give_up_on_error=True):
    """One launch; returns (error word, scheduler steps)."""
    items, span = items_of(prods, width, tile)

    def flag(i):
        return ("flag", i)

    def cnt(t, kind):
        return ("cnt", t, kind)

    for (kind, t), vec in inputs.items():  # written by the caller before the launch
        for i, v in enumerate(vec):
            mem.glob[(kind, t, i)] = v
    # products whose C another product reads: only their numeric items publish
    readers = {p[d] for p in prods for d in ("dep_A", "dep_B") if p[d] >= 0}
    # kernel start: every XCD drops its clean lines
    for x in range(xcds):
        mem.acquire(x)

    def ready(t, kind):
        first, n = span[t][kind]
        if publish == "flag":
            return all(mem.coherent_load(flag(first + i)) for i in range(n))
        return mem.coherent_load(cnt(t, kind)) >= n

    def wg(g):
        x = g % xcds
        while True:
            it = mem.atomic_add(T, 1)
            yield
            if it >= len(items):
                break
            kind, t, f = items[it]
            p = prods[t]
            need = []
            if kind == "gather":
                if p["dep_A"] >= 0:
                    need.append((p["dep_A"], "numeric"))
            else:
                if not p.get("in_place"):
                    need.append((t, "gather"))
                elif p["dep_A"] >= 0:  # A values read in place: dep_A's C
                    need.append((p["dep_A"], "numeric"))
                if p["dep_B"] >= 0:
                    need.append((p["dep_B"], "numeric"))
            ok = True
            waited = bool(need)
            for dep in need:
                spins = 0
                while ok and not ready(*dep):
                    spins += 1
                    if spins > wait_bound or (give_up_on_error and mem.coherent_load(ERR)):
                        ok = False
                    yield
            if not ok:
                mem.release_store(x, ERR, 1)
            if acquire and waited:
                mem.acquire(x)
            yield
            if kind == "gather":
                for i in range(f, min(width, f + tile)):
                    src = ("C", p["dep_A"], i) if p["dep_A"] >= 0 else ("A", t, i)
                    mem.store(x, ("At", t, i), mem.load(x, src))
                    yield
            else:
                for j in range(f, min(width, f + tile)):
                    s = 0
                    for i in range(width):
                        if p.get("in_place"):
                            asrc = ("C", p["dep_A"], i) if p["dep_A"] >= 0 else ("A", t, i)
                        else:
                            asrc = ("At", t, i)
                        a = mem.load(x, asrc)
                        b = ("C", p["dep_B"], (i + j) % width) if p["dep_B"] >= 0 \
                            else ("B", t, (i + j) % width)
                        s += a * mem.load(x, b)
                    mem.store(x, ("C", t, j), s)
                    yield
            read_later = kind == "gather" or t in readers
            if it != lost and read_later:
                if publish == "flag":
                    mem.release_store(x, flag(it), 1, with_release=release)
                else:
                    if release:
                        mem.release(x)
                    mem.posted_add(x, cnt(t, kind), 1)
            yield
        # leaving: the last workgroup clears the ticket, the exit count and
        # the flags (or counts) at the coherence point
        mem.release(x)
        if mem.atomic_add(EXIT, 1) == n_wg - 1:
            mem.store_through(x, T, 0)
            mem.store_through(x, EXIT, 0)
            for i in range(len(items)):
                mem.store_through(x, flag(i), 0)
            for t in range(len(prods)):
                for kind in ("gather", "numeric"):
                    mem.store_through(x, cnt(t, kind), 0)

    live = [wg(g) for g in range(n_wg)]
    steps = 0
    while live:
        k = rng.randrange(len(live))
        try:
            next(live[k])
        except StopIteration:
            live.pop(k)
        steps += 1
        assert steps < 5 * 10 ** 6, "the launch did not drain"
    # kernel end: every XCD's dirty lines reach memory
    for x in range(xcds):
        mem.release(x)
    return mem.glob.get(ERR, 0), steps


def c_of(mem, t, width):
    return [mem.glob.get(("C", t, j), 0) for j in range(width)]


def setup(seed, nprod=6, width=6):
    rng = random.Random(seed)
    prods = make_dag(rng, nprod)
    inputs = {}
    for t in range(nprod):
        inputs[("A", t)] = [rng.randint(-3, 3) for _ in range(width)]
        inputs[("B", t)] = [rng.randint(-3, 3) for _ in range(width)]
    return rng, prods, inputs


def chained(prods):
    return any(p["dep_A"] >= 0 or p["dep_B"] >= 0 for p in prods)


@pytest.mark.parametrize("seed", range(40))
def test_protocol_drains_and_matches_sequential_over_replays(seed):
    rng, prods, inputs = setup(seed)
    width, tile = 6, 2
    mem = Memory(xcds=3)
    for replay in range(3):
        # new input values between replays; the caches keep the old lines
        scaled = {k: [v * (replay + 1) for v in vec] for k, vec in inputs.items()}
        n_wg = rng.choice([1, 2, 3, 5, 8])
        err, _ = run_launch(mem, prods, width, tile, scaled, n_wg, 3, rng)
        assert err == 0
        ref = sequential(prods, width, scaled)
        for t in range(len(prods)):
            assert c_of(mem, t, width) == ref[t], (seed, replay, t)
        n_items = len(items_of(prods, width, tile)[0])
        assert mem.glob[T] == 0 and mem.glob[EXIT] == 0
        assert all(mem.glob.get(("flag", i), 0) == 0 for i in range(n_items))


def _wrong_result_seen(**kw):
    for seed in range(60):
        rng, prods, inputs = setup(seed)
        if not chained(prods):
            continue
        mem = Memory(xcds=3)
        for replay in range(2):
            scaled = {k: [v * (replay + 2) for v in vec] for k, vec in inputs.items()}
            err, _ = run_launch(mem, prods, 6, 2, scaled, 4, 3, rng, **kw)
            ref = sequential(prods, 6, scaled)
            if err or any(c_of(mem, t, 6) != ref[t] for t in range(len(prods))):
                return True
    return False


def test_without_release_consumers_read_stale_values():
    assert _wrong_result_seen(release=False)


def test_without_acquire_consumers_read_stale_values():
    assert _wrong_result_seen(acquire=False)


def test_counts_posted_into_the_xcd_cache_make_the_waits_run_out():
    seen = False
    for seed in range(20):
        rng, prods, inputs = setup(seed)
        if not chained(prods):
            continue
        mem = Memory(xcds=3)
        err, _ = run_launch(mem, prods, 6, 2, inputs, 6, 3, rng, publish="posted_counter",
                            wait_bound=400)
        seen |= err > 0
    assert seen


def test_a_flag_that_never_arrives_sets_the_error_word_and_the_launch_ends():
    rng, prods, inputs = setup(3)
    prods[1]["dep_B"] = 0  # product 1 reads product 0's C
    items, span = items_of(prods, 6, 2)
    lost = span[0]["numeric"][0]
    mem = Memory(xcds=2)
    err, steps = run_launch(mem, prods, 6, 2, inputs, 4, 2, rng, lost=lost, wait_bound=50)
    assert err > 0
    # once the error word is set the other waits give up at once: the launch
    # takes a bounded number of steps, not one bound per waiting item
    _, clean_steps = run_launch(Memory(xcds=2), prods, 6, 2, inputs, 4, 2, random.Random(3))
    assert steps < clean_steps + 4 * 60


def test_waits_that_ignore_the_error_word_add_up_item_after_item():
    """Why the earlier kernel's bounded waits did not end its launch: its
    counts were posted into the XCD caches (so waits ran out), each wait had
    its own bound and none looked at the error word, so every waiting item
    waited out a full bound, one after another on each workgroup.  The launch
    then lasts about (items per workgroup) x (waits per item) x (bound):
    minutes on the GPU for a bound of about a second per wait.  Giving up as
    soon as the error word is set ends it after about one bound."""
    rng, prods, inputs = setup(3)
    prods[1]["dep_B"] = 0
    for t in range(2, len(prods)):  # every later product waits on product 1
        prods[t]["dep_B"] = 1
    bound = 200
    for n_wg in (2, 4):
        kw = dict(publish="posted_counter", wait_bound=bound)
        e_old, steps_old = run_launch(Memory(xcds=2), prods, 6, 2, inputs, n_wg, 2,
                                      random.Random(5), give_up_on_error=False, **kw)
        e_new, steps_new = run_launch(Memory(xcds=2), prods, 6, 2, inputs, n_wg, 2,
                                      random.Random(5), give_up_on_error=True, **kw)
        assert e_old and e_new
        # many full bounds in a row against about one
        assert steps_old > 5 * n_wg * bound
        assert steps_new < 2 * n_wg * bound
        assert steps_old > 5 * steps_new
