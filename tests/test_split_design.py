"""The repeat finder's order independence, on a host model of its table.

The device table (csrc/hashsplit.hpp, k_hdup) inserts 32-bit tags by linear
probing with compare-and-swap, from a first slot that is a function of the
tag alone, and marks a slot when a tag finds itself there.  The claim is that
the marked slots are exactly the tags that occur twice or more, whatever the
order of the insertions: every copy of a tag walks the same probe sequence,
slots are never emptied, so each later copy meets the first one before any
empty slot.  This model replays bucket contents in many orders (one insertion
at a time, which is what the atomic compare-and-swap serialises to) and
checks the marked set.  It also shows why the first slot must come from the
tag: with a first slot taken from other hash bits, two distinct hashes with
one tag are marked in some orders and not in others.
"""
import random

SLOTS = 97  # small, so that probe runs and collisions are common


def insert_all(hashes, tag_of, slot_of):
    tab = [None] * SLOTS
    marked = set()
    for h in hashes:
        t = tag_of(h)
        s = slot_of(h)
        for _ in range(SLOTS):
            if tab[s] is None:
                tab[s] = t
                break
            if tab[s] == t:
                marked.add(t)
                break
            s = (s + 1) % SLOTS
        else:
            raise AssertionError("table full")
    return marked


def tag_of(h):
    return (h >> 8) & 0xFF  # a narrow tag: distinct hashes share tags often


def test_marks_do_not_depend_on_the_order():
    rng = random.Random(5)
    for trial in range(200):
        n = rng.randrange(2, 60)
        pool = [rng.getrandbits(32) for _ in range(n)]
        hashes = [rng.choice(pool) for _ in range(n)]  # repeats
        want = {t for t in map(tag_of, hashes) if list(map(tag_of, hashes)).count(t) >= 2}
        for _ in range(10):
            rng.shuffle(hashes)
            got = insert_all(hashes, tag_of, lambda h: (tag_of(h) * 37) % SLOTS)
            assert got == want, (trial, sorted(got), sorted(want))


def test_first_slot_from_other_bits_depends_on_the_order():
    # two distinct hashes a, b with one tag but first slots 1 and 3, and two
    # other tags with first slots 1 and 2: when the others come first, a is
    # pushed to slot 3 and b meets it (marked); when a comes first, the
    # others fill slots 2 and 3 and b lands at 4 (not marked)
    a = (5 << 8) | 1
    b = (5 << 8) | 3
    f1 = (20 << 8) | 1
    f2 = (21 << 8) | 2
    slot = lambda h: h & 0xFF  # noqa: E731  (first slot from bits outside the tag)
    assert 5 in insert_all([f1, f2, a, b], tag_of, slot)
    assert 5 not in insert_all([a, f1, f2, b], tag_of, slot)
    # with the first slot a function of the tag, both orders mark it
    tslot = lambda h: (tag_of(h) * 37) % SLOTS  # noqa: E731
    assert 5 in insert_all([f1, f2, a, b], tag_of, tslot)
    assert 5 in insert_all([a, f1, f2, b], tag_of, tslot)
