"""Integer identities the packing kernels rely on, checked on the CPU.

* The second heuristic draws criterion t of a permutation packing as digit
  t+1 of u / 2^32 in base 3: floor(3u / 2^32), then u = 3u mod 2^32.  A
  forced criterion c runs the same iteration from a word whose digits are all
  c (0, 2^31, 2^32 - 1), for up to six placements.
* The byte offset of a criterion's key constants is 16 times that digit,
  taken as floor(48u / 2^32) with the low four bits cleared.
* The Worst Fit key of the one-word bin encoding, (A ^ ~1023) + XW with
  XW = (32767 + w - (2^22 - 1)) << 10, equals (32767 - room + w) << 10 | tag
  and is below 2^25 exactly when the item fits.
* Rule 5 in the second heuristic's kernel: with H = (floor(cap/2) + 1) << 10,
  a bin divides at the placement whose bin word before it is >= H and after
  it is < H.  Since rooms only fall, that is the one placement at which the
  bin's load first reaches half its capacity, the division the oracle
  records with an explicit mark.
"""
import numpy as np

M32 = (1 << 32) - 1


def digits(u, n):
    out = []
    for _ in range(n):
        out.append((3 * u) >> 32)
        u = (3 * u) & M32
    return out


def test_forced_criterion_words():
    for c, u in ((0, 0), (1, 1 << 31), (2, M32)):
        assert digits(u, 6) == [c] * 6


def test_digits_are_the_base3_expansion():
    rng = np.random.default_rng(5)
    for u in list(rng.integers(0, 1 << 32, size=2000, dtype=np.uint64)) + [0, 1, M32]:
        u = int(u)
        exp = [(3 ** (t + 1) * u >> 32) % 3 for t in range(6)]
        assert digits(u, 6) == exp


def test_key_table_offset():
    rng = np.random.default_rng(6)
    edge = [0, 1, M32, 1 << 31, (1 << 32) // 3, (1 << 32) // 3 + 1,
            (1 << 33) // 3, (1 << 33) // 3 + 1]
    for u in list(rng.integers(0, 1 << 32, size=20000, dtype=np.uint64)) + edge:
        u = int(u)
        assert ((48 * u) >> 32) & 0x30 == 16 * ((3 * u) >> 32)


def test_worst_fit_key_of_one_word_bins():
    rng = np.random.default_rng(7)
    r5 = 32767
    for _ in range(20000):
        room = int(rng.integers(0, r5 + 1))
        w = int(rng.integers(1, r5 + 1))
        tag = int(rng.integers(0, 1024))
        a = (room << 10) | tag
        xw = ((r5 + w - ((1 << 22) - 1)) << 10) & M32
        key = ((a ^ 0xFFFFFC00) + xw) & M32
        assert key == ((r5 - room + w) << 10) | tag
        assert (key < (1 << 25)) == (w <= room)


def test_rule5_crossing_test_equals_the_divided_mark():
    rng = np.random.default_rng(8)
    for _ in range(4000):
        cap = int(rng.integers(1, 32768))
        tag = int(rng.integers(0, 1024))
        h = ((cap >> 1) + 1) << 10
        load, divided = 0, False
        word = (cap << 10) | tag          # an empty bin: room = cap
        while True:
            room = cap - load
            if room < 1:
                break
            w = int(rng.integers(1, room + 1))
            after = word - (w << 10)      # the kernel's new word
            kernel_split = after < h and after + (w << 10) >= h
            load += w
            oracle_split = (not divided) and 2 * load >= cap
            divided = divided or oracle_split
            assert kernel_split == oracle_split, (cap, load, w)
            assert after == ((cap - load) << 10) | tag
            word = after
