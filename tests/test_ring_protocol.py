"""Model check of the draw-ring protocol between an event-loop lane and its
producer lane (the 512-thread kernel, ssa_kernel_pc).

The two agents are modelled as step machines whose steps are the kernel's LDS
operations, in the kernel's order and with its 32-bit arithmetic: a counter
word is (low 24 bits of an event index) << 8 | epoch byte. A random scheduler interleaves them; a step is atomic
and the waits the kernel places (lgkmcnt 0) make each agent's steps take effect
in program order, which is what the model assumes. Each ring slot stores the
identity (trajectory id, event index) of the draw written to it, so the check is direct:
whenever the event-loop lane takes a draw from the ring, it must be the draw of
its current trajectory and event. Runs cover slow and fast producers, short
trajectories that cycle the 255 epochs many times, event indices crossing the
24-bit wrap, and a producer that sees claims late (it then skips ahead).

Conversion fields: when a lane's counts pass the exact-integer limit its wave
enters a conversion version and sets the request word (once, at that step; a
claim clears it); the producer then also forms each draw's conversion fields
into the slot and marks the draw. In an event that needs them the lane reads
the current draw's fields from its slot (before it publishes done) if that
draw came from the ring with the mark, and forms them itself otherwise; fields
it reads must be its own draw's.

Two producers (PLACE_TWO0): producer k makes only the draws of event index
with parity k and publishes its own made word; the lane reads the made word of
its next draw's parity. The same checks apply, with both producers scheduled
against the lane.

This checks the protocol as designed; the GPU tests check the kernel's results.
"""
import random

import pytest

M32 = 0xFFFFFFFF


def word(idx, e):
    """Counter word of event index idx in epoch e."""
    return ((idx << 8) | e) & M32


def sra8(v):
    """(i32)v >> 8: arithmetic shift of a 32-bit word."""
    v &= M32
    return (v - (1 << 32) if v & 0x80000000 else v) >> 8


def rotr8(v):
    v &= M32
    return ((v >> 8) | (v << 24)) & M32


class Shared:
    def __init__(self, D):
        self.made = [0, 0]          # [parity class]; class 1 only with two producers
        self.done = 0
        self.req_e = 0
        self.req_id = 0
        self.req_lo = 0
        self.req_hi = 0
        self.convw = 0
        self.ring = [None] * D      # (trajectory, event) of the draw
        self.conv = [None] * D      # (trajectory, event) of the conversion fields


def consumer(sh, D, rng, n_traj, start_n, log, lengths, p_need=0.0, two=False):
    """Generator: one step per LDS operation (plus the local work between).
    p_need: per trajectory, the chance that its counts pass the exact-integer
    limit (from a random event on, until it ends). two: the made word is the
    one of the next draw's parity class."""
    eb = 0
    for uid in range(1, n_traj + 1):     # uid: the trajectory's id (draws are keyed by it)
        n = start_n(rng)
        log["claim_step"] = log["step"]
        # claim: done = made = word(n + 1); request words; wait; epoch
        eb = eb % 255 + 1
        dw = word(n + 1, eb)
        sh.done = dw
        yield
        sh.made[0] = dw
        sh.made[1] = dw
        yield
        sh.req_id, sh.req_lo, sh.req_hi = uid, n & 0xFFFFFFFF, n >> 32
        sh.convw = 0
        yield
        sh.req_e = eb
        yield
        length = lengths(rng)
        need_from = rng.randint(0, max(length, 1)) if rng.random() < p_need else None
        cur_mark = False                                      # the claim forms its draw itself
        for ev in range(length):
            want = n + 1
            mw = sh.made[(dw >> 8) & 1 if two else 0]         # top of the event
            yield
            if need_from is not None and ev == need_from:     # entering a conversion version
                sh.convw = 1                                  # the request word, once
                yield
            if need_from is not None and ev >= need_from:     # conversion path: fields of draw n
                fields = sh.conv[(((dw - 256) & M32) >> 8) % D]
                yield
                if cur_mark:
                    log["conv_ring"] += 1
                    assert fields == (uid, n), f"stale conversion fields: got {fields}, wanted {(uid, n)}"
                else:
                    log["conv_self"] += 1
            sh.done = dw                                      # after the wait: done, then ring words
            yield
            data = sh.ring[(dw >> 8) % D]
            yield
            nxt = (dw + 256) & M32
            hit = rotr8(mw - nxt) < D
            dw = nxt
            if hit:
                log["hits"] += 1
                assert data is not None and data[:2] == (uid, want), f"stale draw: got {data}, wanted {(uid, want)}"
                cur_mark = data[2]
            else:
                log["misses"] += 1                            # formed by the lane itself
                cur_mark = False
            n = want                                          # the event fires
    log["consumer_done"] = True


def producer(sh, D, batch, rng, log, skip=True, start=1, cls=0, stride=1):
    """start: free slots before a batch begins (in the kernel another lane's
    free slots may start it, so start = 1 covers every lane's case).
    stride 2: one of two producers, making the draws of parity cls."""
    e, p, uid = 0, 0, 0
    while not log.get("consumer_done"):
        re = sh.req_e
        yield
        dw = sh.done                                          # after the wait
        yield
        if re != e:
            e = re
            uid = sh.req_id
            p = ((sh.req_hi << 32) | sh.req_lo) + 1
            if stride == 2:
                p += (p ^ cls) & 1
            yield
        cw = sh.convw
        yield
        mine = e != 0 and (dw & 0xFF) == e
        if skip:
            ahead = sra8((p << 8) - (dw & ~0xFF))
            if mine and ahead < 0:
                p += -ahead
                ahead = 0
                if stride == 2:
                    fix = (p ^ cls) & 1
                    p += fix
                    ahead = fix
        else:   # the unsigned distance without the skip: behind reads as a full ring
            ahead = (((p << 8) - (dw & ~0xFF)) & M32) >> 8
        span = D - ahead if (mine and ahead < D) else 0
        room = (span + 1) // 2 if stride == 2 else span
        if room < start:
            yield                                             # sleep
            continue
        k = min(room, batch)
        mark = bool(mine and cw)
        for b in range(k):
            q = p + stride * b
            if mark:
                sh.conv[q % D] = (uid, q)
                yield
            sh.ring[q % D] = (uid, q, mark)
            yield
        p += stride * k
        sh.made[cls if stride == 2 else 0] = word(p, e)       # after the wait for the stores
        yield
        log["made"] += k


def mixed_lengths(r):
    return r.choice([0, 1, 2, 3, r.randint(4, 60)])


def run(seed, D=16, batch=8, p_producer=0.5, n_traj=300, start=None, skip=True, lengths=mixed_lengths,
        hold_after_claim=0, batch_start=1, p_need=0.0, two=False):
    """hold_after_claim: the producers do not run for that many steps after each
    claim (they see the claim late, after the lane has formed draws itself)."""
    rng = random.Random(seed)
    sh = Shared(D)
    log = {"hits": 0, "misses": 0, "made": 0, "step": 0, "claim_step": 0, "conv_ring": 0, "conv_self": 0}
    start = start or (lambda r: r.randint(0, 50))
    c = consumer(sh, D, rng, n_traj, start, log, lengths, p_need, two)
    live = {"c": c}
    if two:
        live["p"] = producer(sh, D, batch, rng, log, skip, batch_start, cls=0, stride=2)
        live["p1"] = producer(sh, D, batch, rng, log, skip, batch_start, cls=1, stride=2)
    else:
        live["p"] = producer(sh, D, batch, rng, log, skip, batch_start)
    while "c" in live:
        held = log["step"] - log["claim_step"] < hold_after_claim
        prods = [k for k in live if k != "c"]
        who = rng.choice(prods) if (prods and not held and rng.random() < p_producer) else "c"
        log["step"] += 1
        try:
            next(live[who])
        except StopIteration:
            del live[who]
    return log


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("p_producer", [0.15, 0.5, 0.85])
def test_ring_hits_are_always_the_wanted_draw(seed, p_producer):
    log = run(seed, p_producer=p_producer)     # the stale-draw check is inside
    if p_producer >= 0.5:
        assert log["hits"] > log["misses"]


@pytest.mark.parametrize("seed", range(4))
def test_epoch_wrap_with_short_trajectories(seed):
    # 2,000 claims (the 255 epochs cycle about 8 times), mostly trajectories of
    # 0-3 events, with a producer slow enough to leave made words of old epochs
    # behind: none may read as a hit for a later epoch with the same byte
    log = run(100 + seed, p_producer=0.2, n_traj=2000,
              lengths=lambda r: r.choice([0, 0, 1, 2, 3, r.randint(10, 30)]))
    assert log["hits"] > 0 and log["misses"] > 0


def bursts_of_finished(r, state):
    """Runs of 254 trajectories without an event (finished trajectories claimed
    again in a later window stop at once), then a short one with events, so
    the lane's epoch byte returns to a value its made word may still hold."""
    state["i"] = state.get("i", 0) + 1
    return 3 if state["i"] % 255 == 1 else 0


def epoch_reuse_run(run_fn, bursts, seed):
    # every trajectory starts at event 5; the producer sees claims only 10
    # steps late, so it never sees the empty ones (a claim takes 4 steps)
    st = {}
    return run_fn(seed, p_producer=0.5, n_traj=255 * 8 + 1, start=lambda r: 5,
                  lengths=lambda r: bursts(r, st), hold_after_claim=10)


def test_epoch_byte_reuse_after_bursts_of_empty_claims():
    for seed in range(20):
        epoch_reuse_run(run, bursts_of_finished, 400 + seed)


def test_the_made_reset_at_claim_is_what_prevents_stale_hits():
    # the same runs against a copy of the model whose claim does not reset
    # made: a made word left from 255 claims earlier then reads as a hit and
    # hands the lane another trajectory's draw
    src = open(__file__).read()
    variant = src.replace("        sh.made[0] = dw\n        sh.made[1] = dw\n        yield\n        sh.req_id", "        sh.req_id")
    assert variant != src
    ns = {"__name__": "variant"}
    exec(compile(variant, "variant", "exec"), ns)
    stale = 0
    for seed in range(20):
        try:
            epoch_reuse_run(ns["run"], ns["bursts_of_finished"], 400 + seed)
        except AssertionError:
            stale += 1
    assert stale > 0


@pytest.mark.parametrize("seed", range(4))
def test_event_index_crosses_the_24_bit_wrap(seed):
    log = run(200 + seed, start=lambda r: (1 << 24) - r.randint(1, 40), n_traj=200)
    assert log["hits"] > 0


@pytest.mark.parametrize("D,batch,batch_start", [(2, 2, 1), (4, 4, 1), (8, 4, 1), (16, 8, 1), (16, 6, 6),
                                                 (16, 8, 4), (8, 4, 4), (2, 1, 1)])
def test_ring_depths_and_batches(D, batch, batch_start):
    for seed in range(3):
        log = run(300 + seed, D=D, batch=batch, batch_start=batch_start)
        assert log["hits"] > 0


def test_a_late_producer_skips_ahead_and_keeps_up():
    # the producer sees each claim only after the lane has formed a few draws
    # itself; without the skip it stays behind for the rest of the trajectory
    long_runs = lambda r: r.randint(80, 120)
    fast = run(7, p_producer=0.5, n_traj=100, lengths=long_runs, hold_after_claim=40)
    stuck = run(7, p_producer=0.5, n_traj=100, lengths=long_runs, hold_after_claim=40, skip=False)
    assert fast["hits"] > 5 * max(stuck["hits"], 1)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("p_producer,D,batch", [(0.5, 16, 6), (0.2, 8, 4), (0.85, 8, 4), (0.5, 2, 1)])
def test_conversion_fields_from_the_ring_are_the_lanes_own(seed, p_producer, D, batch):
    # trajectories that pass the exact-integer limit part way through; fields
    # taken from the ring must be those of the lane's current draw
    log = run(500 + seed, D=D, batch=batch, p_producer=p_producer, n_traj=400, p_need=0.6,
              lengths=lambda r: r.choice([1, 3, r.randint(10, 80)]))
    assert log["conv_self"] > 0
    if p_producer >= 0.5:    # a slow producer may never get ahead of a lane's request
        assert log["conv_ring"] > 0


def test_conversion_fields_across_epoch_reuse():
    # short trajectories and late claims cycle the epoch byte: a stale mark or
    # stale fields from 255 claims earlier must never be taken
    for seed in range(10):
        st = {}
        run(600 + seed, p_producer=0.5, n_traj=255 * 4 + 1, start=lambda r: 5, p_need=0.5,
            lengths=lambda r: bursts_of_finished(r, st) or r.randint(0, 2), hold_after_claim=10)


def test_the_mark_check_is_what_keeps_stale_fields_out():
    # a copy of the model whose lane takes ring fields without checking the
    # draw's mark reads fields of another draw
    src = open(__file__).read()
    variant = src.replace("                if cur_mark:\n                    log[\"conv_ring\"]",
                          "                if True:\n                    log[\"conv_ring\"]")
    assert variant != src
    ns = {"__name__": "variant"}
    exec(compile(variant, "variant", "exec"), ns)
    stale = 0
    for seed in range(6):
        try:
            ns["run"](500 + seed, D=8, batch=4, p_producer=0.2, n_traj=400, p_need=0.6,
                      lengths=lambda r: r.choice([1, 3, r.randint(10, 80)]))
        except AssertionError:
            stale += 1
    assert stale > 0


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("p_producer,D,batch,batch_start", [(0.5, 16, 4, 4), (0.2, 16, 4, 1), (0.85, 8, 2, 2),
                                                            (0.5, 4, 1, 1)])
def test_two_producers_split_by_parity(seed, p_producer, D, batch, batch_start):
    # both producers against one lane: every hit is the lane's own draw, and
    # both parity classes come from the ring
    log = run(700 + seed, D=D, batch=batch, batch_start=batch_start, p_producer=p_producer, n_traj=300,
              two=True, p_need=0.5, lengths=lambda r: r.choice([0, 1, 3, r.randint(10, 80)]))
    assert log["hits"] > 0
    if p_producer >= 0.5 and D >= 8:    # a ring of 4 holds two draws per producer
        assert log["hits"] > log["misses"]
        assert log["conv_ring"] > 0


@pytest.mark.parametrize("seed", range(3))
def test_two_producers_epoch_reuse_and_wrap(seed):
    for s in range(4):
        st = {}
        run(800 + 10 * seed + s, p_producer=0.5, n_traj=255 * 4 + 1, start=lambda r: 5, p_need=0.5, two=True,
            batch=4, lengths=lambda r: bursts_of_finished(r, st) or r.randint(0, 2), hold_after_claim=10)
    log = run(900 + seed, start=lambda r: (1 << 24) - r.randint(1, 40), n_traj=200, two=True, batch=4)
    assert log["hits"] > 0


def test_the_parity_of_the_made_word_matters():
    # a copy of the model whose lane reads producer 0's made word for every
    # draw takes odd draws that producer 1 has not made
    src = open(__file__).read()
    variant = src.replace("mw = sh.made[(dw >> 8) & 1 if two else 0]", "mw = sh.made[0]")
    assert variant != src
    ns = {"__name__": "variant"}
    exec(compile(variant, "variant", "exec"), ns)
    stale = 0
    for seed in range(6):
        try:
            ns["run"](700 + seed, D=16, batch=4, p_producer=0.3, n_traj=300, two=True,
                      lengths=lambda r: r.choice([1, 3, r.randint(10, 80)]))
        except AssertionError:
            stale += 1
    assert stale > 0
