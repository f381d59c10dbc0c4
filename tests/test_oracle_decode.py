"""Oracle decode of the synthetic super-pixel banks.

Pins: the round trip through the generator's encoder (independent numpy code)
returns the generated pixels exactly; hand-built words decode to the pixels
their fields name; each malformation (reserved bits, empty pattern, a set bit
outside the sensor) drops its word and flags its event; a pixel decoded twice
is kept and flags its event; under a capacity limit the planes that fit are
written, the others not, and the offsets stay complete.
"""
import numpy as np
import pytest

import oracle
from paper_2412_05041_amd import gen

SIDE = 1454


def word(pattern, spr, spc, extra=0):
    return np.uint32(pattern | (spr << 8) | (spc << 17) | (extra << 27))


def one_plane_bank(words, plane=0):
    off = np.zeros(27, np.int32)
    off[plane + 1:] = len(words)
    return off, np.array(words, np.uint32)


@pytest.mark.parametrize("name,n", [("tiny", None), ("nominal", 40), ("heavy_ion", 1)])
def test_round_trip_through_the_encoder(name, n):
    w = gen.WORKLOADS[name]
    b = gen.generate(w if n is None else w.with_events(n, 77))
    off, bank = gen.raw_banks(b, seed=5)
    assert bank.size < b.n_pix or b.n_pix == 0  # words carry several pixels
    pix_off, pix_id, flags, total = oracle.decode(off, bank, b.n_events)
    assert total == b.n_pix
    assert np.array_equal(pix_off, b.pix_off)
    assert np.array_equal(pix_id, b.pix_id)
    assert not flags.any()


def test_hand_words():
    # pattern bits (dr, dc): bit 0 = (0,0), bit 1 = (0,1), bit 7 = (3,1)
    off, bank = one_plane_bank([word(0b10000011, 10, 20), word(0b00000100, 0, 0)], plane=3)
    pix_off, pix_id, flags, total = oracle.decode(off, bank, 1)
    exp = sorted([40 * SIDE + 40, 40 * SIDE + 41, 43 * SIDE + 41, 1 * SIDE + 0])
    assert total == 4 and pix_id.tolist() == exp
    assert pix_off[3] == 0 and pix_off[4] == 4 and pix_off[-1] == 4
    assert flags[0] == 0


@pytest.mark.parametrize("bad", [word(1, 5, 5, extra=1), word(0, 5, 5), word(1, 364, 0), word(0b10000, 363, 0),
                                 word(1, 0, 727), word(0b10, 0, 1023)])
def test_malformed_word_is_dropped_and_flagged(bad):
    good = word(0b1, 2, 3)
    off, bank = one_plane_bank([good, bad])
    pix_off, pix_id, flags, total = oracle.decode(off, bank, 1)
    assert total == 1 and pix_id.tolist() == [8 * SIDE + 6]
    assert flags[0] == 2


def test_last_rows_and_columns_are_valid():
    off, bank = one_plane_bank([word(0b11, 363, 726)])  # rows 1452, columns 1452/1453
    _, pix_id, flags, total = oracle.decode(off, bank, 1)
    assert pix_id.tolist() == [1452 * SIDE + 1452, 1452 * SIDE + 1453] and not flags.any()


def test_duplicate_pixel_is_kept_and_flagged():
    off, bank = one_plane_bank([word(0b11, 1, 1), word(0b10, 1, 1)])
    _, pix_id, flags, total = oracle.decode(off, bank, 1)
    assert total == 3 and pix_id.tolist() == [4 * SIDE + 2, 4 * SIDE + 3, 4 * SIDE + 3]
    assert flags[0] == 2


def test_capacity_keeps_offsets():
    b = gen.generate(gen.WORKLOADS["tiny"].with_events(3, 9))
    off, bank = gen.raw_banks(b)
    cap = b.n_pix - 5
    pix_off, pix_id, flags, total = oracle.decode(off, bank, 3, pix_cap=cap)
    assert total == b.n_pix and np.array_equal(pix_off, b.pix_off)
    fit = int(b.pix_off[b.pix_off <= cap].max())  # planes that fit entirely are written
    assert np.array_equal(pix_id[:fit], b.pix_id[:fit])
    assert flags[2] == 1 and flags[0] == 0
