"""Pin of the SR random-field layout (Sec. 3.3; the layout is this build's
reading): every field the 16-bit trajectory code reads is rebuilt here from
Philox words with Python integer bit slicing, an independent construction.

Field width B = 13 (fp16) or 16 (bf16). Main slots: floor(80/B) fields of the
80-bit string [word 2, word 3, low byte of word 0, low byte of word 1] of the
event's stream-0 draw, then floor(128/B) fields of each further stream's
128-bit string. Conversion slots: fields of streams 2^31, 2^31 + 1, ..."""
import numpy as np
import pytest

SEED = 0x1234_5678_9ABC_DEF0


def words(orc, tid, n, stream):
    ctr = np.array([[n & 0xFFFFFFFF, n >> 32, tid, stream]], np.uint32)
    key = np.array([[SEED & 0xFFFFFFFF, SEED >> 32]], np.uint32)
    return [int(w) for w in orc.philox(ctr, key)[0]]


def field(bits, r, B):
    return (bits >> (r * B)) & ((1 << B) - 1)


def expected(orc, B, tid, n, slot, conv):
    F0, F1 = 80 // B, 128 // B
    if conv:
        w = words(orc, tid, n, 0x80000000 + slot // F1)
        return field(w[0] | w[1] << 32 | w[2] << 64 | w[3] << 96, slot % F1, B)
    if slot < F0:
        w = words(orc, tid, n, 0)
        return field(w[2] | w[3] << 32 | (w[0] & 0xFF) << 64 | (w[1] & 0xFF) << 72, slot, B)
    q, r = divmod(slot - F0, F1)
    w = words(orc, tid, n, q + 1)
    return field(w[0] | w[1] << 32 | w[2] << 64 | w[3] << 96, r, B)


@pytest.mark.parametrize("fmt,B", [("F16", 13), ("BF16", 16)])
def test_fields_match_bit_slicing(orc, fmt, B):
    rng = np.random.default_rng(5)
    count = 600
    ids = rng.integers(0, 2**32, count, dtype=np.uint64).astype(np.uint32)
    ns = rng.integers(0, 2**40, count, dtype=np.uint64)
    slots = np.concatenate([np.arange(40), rng.integers(0, 120, count - 40)]).astype(np.int32)
    conv = (np.arange(count) % 3 == 0).astype(np.int32)
    got = orc.sr_fields(fmt, SEED, ids, ns, slots, conv)
    for i in range(count):
        f = expected(orc, B, int(ids[i]), int(ns[i]), int(slots[i]), int(conv[i]))
        assert got[i] == f << (16 - B), (i, int(slots[i]), int(conv[i]))


def test_fields_are_uniform(orc):
    # every main and conversion slot position carries uniform B-bit values
    B = 13
    count = 60000
    rng = np.random.default_rng(9)
    ids = rng.integers(0, 2**32, count, dtype=np.uint64).astype(np.uint32)
    ns = rng.integers(0, 2**20, count, dtype=np.uint64)
    for slot, conv in ((4, 0), (5, 0), (6, 0), (14, 0), (8, 1)):
        f = orc.sr_fields("F16", SEED, ids, ns, np.full(count, slot, np.int32), np.full(count, conv, np.int32))
        hist = np.bincount((f >> (16 - B)) >> 7, minlength=64)   # top 6 bits of the field
        chi2 = ((hist - count / 64) ** 2 / (count / 64)).sum()
        assert chi2 < 130, (slot, conv, chi2)       # 63 degrees of freedom; P(chi2 > 130) ~ 1e-6
