"""Model of the serving work ring's space rule, checked on the CPU with random interleavings.

The ring (host-pinned, capacity CAP) holds work items; the host publishes item k into slot
k mod CAP only while tail + n - claimed <= CAP, where `claimed` is the claim count that waves
publish.  A wave reads slot h and then claims h with a compare-and-swap on the head counter;
after a successful claim it publishes h + 1 as the claim count with a plain store, which may land
late and out of order.  Every step of every wave and of the host is taken in a random order, and
the test checks that every wave ran exactly the item it claimed: no slot is reused while a wave
that claimed it has not read it.  The same model with the claim taken before the read (the
order the kernel used before) is shown to fail, so the check has teeth.
"""
import random

CAP = 8


def run(read_first: bool, seed: int, n_waves: int = 6, n_items: int = 400) -> bool:
    rnd = random.Random(seed)
    ring = [None] * CAP
    head = 0                 # device claim counter
    tail = 0                 # items published
    claimed_seen = 0         # the claim count as the host sees it
    pending_stores = []      # claim-count stores in flight
    # wave state: (phase, h, value)
    waves = [("idle", None, None) for _ in range(n_waves)]
    ran = []
    ok = True
    steps = 0
    while (len(ran) < n_items or any(w[0] != "idle" for w in waves)) and steps < 200000:
        steps += 1
        actor = rnd.randrange(n_waves + 2)
        if actor == n_waves:                                   # host publishes a batch
            n = rnd.randint(1, 3)
            if tail < n_items and tail + n - claimed_seen <= CAP:
                for k in range(n):
                    if tail < n_items:
                        ring[tail % CAP] = tail
                        tail += 1
            continue
        if actor == n_waves + 1:                               # a claim-count store lands
            if pending_stores:
                claimed_seen = pending_stores.pop(rnd.randrange(len(pending_stores)))
            continue
        phase, h, val = waves[actor]
        if phase == "idle":
            if head < tail:
                h = head
                if read_first:
                    waves[actor] = ("read", h, ring[h % CAP])
                else:
                    waves[actor] = ("claim_first", h, None)
        elif phase == "read":                                  # CAS after the read
            if head == h:
                head += 1
                pending_stores.append(h + 1)
                waves[actor] = ("run", h, val)
            else:
                waves[actor] = ("idle", None, None)            # lost the race: drop the value
        elif phase == "claim_first":                           # CAS, then the read later
            if head == h:
                head += 1
                pending_stores.append(h + 1)
                waves[actor] = ("read_late", h, None)
            else:
                waves[actor] = ("idle", None, None)
        elif phase == "read_late":
            waves[actor] = ("run", h, ring[h % CAP])
        elif phase == "run":
            ok = ok and val == h
            ran.append(h)
            waves[actor] = ("idle", None, None)
    return ok and sorted(ran) == list(range(len(ran)))


def test_read_before_claim_never_runs_an_overwritten_item():
    assert all(run(True, seed) for seed in range(150))


def test_claim_before_read_is_caught_by_the_model():
    assert not all(run(False, seed) for seed in range(20))
