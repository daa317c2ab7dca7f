"""CPU model of the radix sort's one-sweep pass (k_onesweep in
csrc/csr_build.hip) and of its decoupled look-back: workgroups take tiles from
a counter one ahead of the tile they work on, publish each digit's count
(state "aggregate"), add up the counts of earlier tiles back to the first one
that published an inclusive count, and publish their own inclusive count.
Status words carry a pass tag, so words left by the previous pass read as not
ready.  Workgroups are stepped in random orders; the model asserts that the
offsets equal the exact exclusive prefix over tiles, that the stable scatter
they give equals a stable sort by digit, and that at every moment some
workgroup can make progress (no schedule leaves all of them waiting)."""
import random

AGG, INCL = 1, 2


def word(tag, state, count):
    return (tag, state, count)


def run_pass(keys, tile, radix, nwg, tag, status, rng):
    """One pass over keys (digits already extracted); returns the output order."""
    ntiles = (len(keys) + tile - 1) // tile
    counts = [[0] * radix for _ in range(ntiles)]
    for i, d in enumerate(keys):
        counts[i // tile][d] += 1
    total = [sum(counts[t][d] for t in range(ntiles)) for d in range(radix)]
    dstart = [sum(total[:d]) for d in range(radix)]
    ctr = [0]
    out = [None] * len(keys)
    excl_seen = {}

    def grab():
        v = ctr[0]
        ctr[0] += 1
        return v

    def workgroup():
        cur = grab()
        yield "step"
        while cur < ntiles:
            nxt = grab()  # the next tile, taken at the top of this one
            yield "step"
            for d in range(radix):  # publish this tile's counts
                status[(cur, d)] = word(tag, INCL if cur == 0 else AGG, counts[cur][d])
                yield "step"
            base = []
            for d in range(radix):
                excl = 0
                if cur != 0:
                    k = cur - 1
                    while True:
                        wtag, state, c = status.get((k, d), (0, 0, 0))
                        if wtag != tag or state == 0:
                            yield ("wait", k, d)  # not ready: poll again
                            continue
                        excl += c
                        if state == INCL or k == 0:
                            break
                        k -= 1
                        yield "step"
                    status[(cur, d)] = word(tag, INCL, excl + counts[cur][d])
                    yield "step"
                base.append(dstart[d] + excl)
                excl_seen[(cur, d)] = excl
            # stable scatter of the tile: within a digit, keys keep their order
            seen = [0] * radix
            for i in range(cur * tile, min(len(keys), (cur + 1) * tile)):
                d = keys[i]
                out[base[d] + seen[d]] = i
                seen[d] += 1
            yield "step"
            cur = nxt

    wgs = [workgroup() for _ in range(nwg)]
    state = {id(g): "step" for g in wgs}
    live = list(wgs)
    def can_move(g):
        st = state[id(g)]
        if st == "step":
            return True
        _, k, d = st  # waiting: can it move now, i.e. is that word ready?
        wtag, s, _ = status.get((k, d), (0, 0, 0))
        return wtag == tag and s != 0

    while live:
        if not any(can_move(g) for g in live):
            raise AssertionError("every workgroup waits on a word nobody will publish")
        g = rng.choice(live)
        try:
            state[id(g)] = next(g)
        except StopIteration:
            live.remove(g)
    for t in range(ntiles):
        for d in range(radix):
            assert excl_seen[(t, d)] == sum(counts[s][d] for s in range(t)), (t, d)
    return out


def test_onesweep_model():
    rng = random.Random(7)
    for trial in range(60):
        radix = rng.choice([2, 4, 16])
        tile = rng.choice([1, 3, 8])
        n = rng.randint(1, 120)
        nwg = rng.randint(1, 9)
        keys = [rng.randrange(radix) for _ in range(n)]
        status = {}
        # pass 1 leaves its words behind; pass 2 reuses the same status words
        out1 = run_pass(keys, tile, radix, nwg, 1, status, rng)
        assert out1 == sorted(range(n), key=lambda i: keys[i])
        keys2 = [rng.randrange(radix) for _ in range(n)]
        out2 = run_pass(keys2, tile, radix, nwg, 2, status, rng)
        assert out2 == sorted(range(n), key=lambda i: keys2[i])


def test_stale_words_read_as_not_ready():
    # a word of the previous pass with an inclusive count must not be used
    rng = random.Random(3)
    keys = [1, 0, 1, 1, 0, 0, 1, 0]
    status = {(t, d): word(1, INCL, 99) for t in range(8) for d in range(2)}
    out = run_pass(keys, 2, 2, 3, 2, status, rng)
    assert out == sorted(range(len(keys)), key=lambda i: keys[i])
