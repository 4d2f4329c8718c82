"""The edit-encoding reference (oracle/edits_ref.py) against a hand-worked
stream, brute-force optimal prefix codes, and round trips (no GPU)."""
import itertools
import json
import os
import struct

import numpy as np
import pytest

from oracle import edits_ref as E

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "edits_tiny.json")


def test_hand_worked_stream():
    g = json.load(open(GOLDEN))
    x = np.zeros(g["n"], dtype=np.float32)
    x[g["indices"]] = g["value"]
    glen = [0] * E.GAP_SYMS
    vlen = [0] * E.VAL_SYMS
    for k, v in g["gap_lengths"].items():
        glen[int(k)] = v
    for k, v in g["value_lengths"].items():
        vlen[int(k)] = v
    head = struct.pack("<6I", 0x455A534D, 1, g["n"], len(g["indices"]), 1, 256) + bytes(glen) + bytes(vlen)
    head += bytes(576 - len(head))
    want = head + b"".join(struct.pack("<Ii", w, i) for w, i in g["chunk_table"])
    want += b"".join(struct.pack("<I", w) for w in g["stream_words"])
    assert E.encode(x) == want
    assert (E.decode(want, g["n"]).view(np.uint32) == x.view(np.uint32)).all()


def _cost(freq, lengths):
    return sum(f * L for f, L in zip(freq, lengths))


@pytest.mark.parametrize("seed", range(40))
def test_huffman_lengths_are_optimal(seed):
    """Against every prefix-code length vector (Kraft sum <= 1) of up to 5 symbols."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 6))
    freq = [int(v) for v in rng.integers(1, 50, size=k)]
    L = E.huffman_lengths(freq)
    best = min(_cost(freq, c) for c in itertools.product(range(1, k), repeat=k)
               if sum(2.0 ** -l for l in c) <= 1.0)
    assert _cost(freq, L) == best
    assert sum(2.0 ** -l for l in L) == 1.0


def test_huffman_length_limit():
    fib = [1, 1]
    while len(fib) < 32:
        fib.append(fib[-1] + fib[-2])
    L = E.huffman_lengths(fib)  # unlimited, the longest code would be 31 bits
    assert max(L) <= E.MAX_LEN and sum(2.0 ** -l for l in L) <= 1.0
    assert max(E.huffman_lengths(fib, max_len=64)) == 31
    assert E.huffman_lengths([0, 0, 7, 0]) == [0, 0, 1, 0]
    assert E.huffman_lengths([0, 0]) == [0, 0]


def test_canonical_codes_are_prefix_free():
    rng = np.random.default_rng(3)
    freq = [int(v) for v in rng.integers(0, 1000, size=E.VAL_SYMS)]
    codes = E.canonical_codes(E.huffman_lengths(freq))
    words = sorted(format(c, f"0{L}b") for c, L in codes.values())
    for a, b in zip(words, words[1:]):
        assert not b.startswith(a)
    by_len = sorted(codes.items(), key=lambda t: (t[1][1], t[0]))
    for (s0, (c0, l0)), (s1, (c1, l1)) in zip(by_len, by_len[1:]):
        assert c1 == (c0 + 1) << (l1 - l0)


def _random_edits(rng, n, m):
    x = np.zeros(n, dtype=np.float32)
    idx = rng.choice(n, size=m, replace=False) if m else np.zeros(0, np.int64)
    x[idx] = -rng.exponential(1e-3, size=m).astype(np.float32)
    return x


@pytest.mark.parametrize("n,m", [(1, 0), (1, 1), (100, 0), (257, 257), (4097, 4097), (20000, 9000), (3_000_000, 5000)])
def test_round_trip(n, m):
    rng = np.random.default_rng(n + m)
    x = _random_edits(rng, n, m)
    blob = E.encode(x)
    assert struct.unpack_from("<I", blob, 12)[0] == m
    assert (E.decode(blob, n).view(np.uint32) == x.view(np.uint32)).all()


def test_round_trip_extremes():
    n = (1 << 21) + 5
    x = np.zeros(n, dtype=np.float32)
    x[[0, 1, 2, 1 << 20, n - 1]] = [-1e-40, -0.0, -3.0e38, -1.0, np.float32(-2.0 ** -149)]
    blob = E.encode(x)
    assert (E.decode(blob, n).view(np.uint32) == x.view(np.uint32)).all()
    with pytest.raises(ValueError):
        E.decode(blob, n + 1)
    with pytest.raises(ValueError):
        E.decode(blob[:-4], n)
