"""Pins of the oracle's packed code stream (the paper's 512-bit output words
of floor(512/n) codes, each quartet starting on a new word): a hand-worked
12-bit word, word counts per block, field boundaries that straddle 64-bit
lanes, the zero padding, and the round trip for every width."""
import numpy as np
import pytest

import oracle as O


def _u64(words, i):
    return int.from_bytes(bytes(words[8 * i: 8 * i + 8]), "little")


def test_hand_worked_12bit_word():
    # codes 1, -1, 2047, -2048 as 12-bit fields: 0x001, 0xFFF, 0x7FF, 0x800
    packed, woff = O.pack(12, [1, -1, 2047, -2048], [0, 4])
    assert list(woff) == [0, 1] and len(packed) == 64
    assert _u64(packed, 0) == 0x001 | (0xFFF << 12) | (0x7FF << 24) | (0x800 << 36)
    assert not packed[8:].any()


def test_words_per_block_and_alignment():
    # 12 bits: 42 codes per word (504 bits, 8 unused); blocks start on a word
    sizes = [1, 42, 43, 84, 85, 0, 10]
    off = np.concatenate([[0], np.cumsum(sizes)])
    codes = np.arange(off[-1]) % 2000 - 1000
    packed, woff = O.pack(12, codes, off)
    assert list(np.diff(woff)) == [1, 1, 2, 2, 3, 0, 1]
    # the 43rd code of block 2 is the first field of its second word
    b2 = int(woff[2])
    assert _u64(packed, 8 * (b2 + 1)) & 0xFFF == int(codes[off[2] + 42]) & 0xFFF
    # the last 8 bits of every 12-bit word are zero
    assert all(packed[64 * w + 63] == 0 for w in range(int(woff[-1])))


def test_field_straddles_lanes():
    # 12-bit code 5 starts at bit 60: 4 bits in lane 0, 8 bits in lane 1
    codes = [0, 0, 0, 0, 0, 0xABC - 4096]
    packed, _ = O.pack(12, codes, [0, 6])
    assert _u64(packed, 0) >> 60 == 0xC
    assert _u64(packed, 1) & 0xFF == 0xAB


@pytest.mark.parametrize("bits", [2, 3, 7, 8, 11, 12, 13, 16, 17, 24, 31, 32])
def test_round_trip(bits):
    rng = np.random.default_rng(bits)
    qmax = (1 << (bits - 1)) - 1
    sizes = rng.integers(0, 150, size=9)
    off = np.concatenate([[0], np.cumsum(sizes)])
    codes = rng.integers(-qmax, qmax + 1, size=off[-1])
    packed, woff = O.pack(bits, codes, off)
    per = 512 // bits
    assert len(packed) == 64 * int(np.sum((sizes + per - 1) // per))
    assert np.array_equal(O.unpack(bits, packed, off), codes)
