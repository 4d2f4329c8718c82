"""Reference (test infrastructure) of the lossless edit encoding, Sec. 6.3.

Plain Python and numpy, written from the stream format that include/msz.h
states, for checking the GPU encoder byte for byte and its decoder value for
value.  Only tests/ use it.

The paper stores every edit as a key-value pair: the keys (vertex indices)
sorted ascending and kept as their differences, which run-length and Huffman
coding then shrink, and the values compressed separately.  This format keeps
the sorted differences and Huffman-codes them by bit length (bucket
b = floor(log2 d) followed by the b low bits of d; a run of neighbouring
edits costs one short code per edit), and codes each value's sign and
exponent with a second Huffman code followed by the raw mantissa.
"""
from __future__ import annotations

import heapq
import struct

import numpy as np

GAP_SYMS, VAL_SYMS, MAX_LEN = 32, 512, 20
CHUNK = 256
HEADER = 576
MAGIC, VERSION = 0x455A534D, 1


def huffman_lengths(freq, max_len: int = MAX_LEN) -> list:
    """Code lengths of a Huffman code for the counts (0 = absent symbol).

    The two lightest nodes merge first; equal weights go to the older node
    (leaves, numbered by symbol, before merged nodes, numbered in order of
    creation).  While a code is longer than max_len, every count is halved,
    rounding up, and the code is built again.
    """
    f = [int(x) for x in freq]
    present = [s for s, x in enumerate(f) if x > 0]
    lengths = [0] * len(f)
    if not present:
        return lengths
    if len(present) == 1:
        lengths[present[0]] = 1
        return lengths
    while True:
        heap = [(f[s], s) for s in present]
        heapq.heapify(heap)
        parent = {}
        next_id = len(f)
        while len(heap) > 1:
            wa, a = heapq.heappop(heap)
            wb, b = heapq.heappop(heap)
            parent[a] = parent[b] = next_id
            heapq.heappush(heap, (wa + wb, next_id))
            next_id += 1
        for s in present:
            d, x = 0, s
            while x in parent:
                x = parent[x]
                d += 1
            lengths[s] = d
        if max(lengths) <= max_len:
            return lengths
        f = [(x + 1) // 2 if x > 0 else 0 for x in f]


def canonical_codes(lengths) -> dict:
    """symbol -> (code, length): by increasing length, then symbol, each code
    one more than the previous, shifted left when the length grows."""
    order = sorted((L, s) for s, L in enumerate(lengths) if L > 0)
    codes, code, prev = {}, 0, None
    for L, s in order:
        if prev is not None:
            code = (code + 1) << (L - prev)
        prev = L
        codes[s] = (code, L)
    return codes


class _Bits:
    """Emitted bit j lands in bit j of a little-endian integer."""

    def __init__(self):
        self.acc, self.pos = 0, 0

    def put(self, v: int, w: int):
        for t in range(w):  # most significant bit first
            self.acc |= ((v >> (w - 1 - t)) & 1) << self.pos
            self.pos += 1

    def words(self) -> bytes:
        nw = (self.pos + 31) // 32
        return self.acc.to_bytes(4 * nw, "little")


def edits_of(edits: np.ndarray):
    """(indices, value bits) of the entries that are not +0, in index order."""
    bits = np.ascontiguousarray(edits, dtype=np.float32).reshape(-1).view(np.uint32)
    idx = np.nonzero(bits)[0]
    return idx.astype(np.int64), bits[idx].astype(np.int64)


def encode(edits: np.ndarray) -> bytes:
    n = int(np.asarray(edits).size)
    idx, val = edits_of(edits)
    m = len(idx)
    nchunks = (m + CHUNK - 1) // CHUNK
    gaps = np.zeros(m, dtype=np.int64)
    first = np.arange(m) % CHUNK == 0
    gaps[1:] = idx[1:] - idx[:-1]
    buckets = np.full(m, -1, dtype=np.int64)  # the position of the highest set bit of each gap
    for k in np.nonzero(~first)[0]:
        buckets[k] = int(gaps[k]).bit_length() - 1
    gfreq = np.bincount(buckets[~first], minlength=GAP_SYMS)[:GAP_SYMS] if m else np.zeros(GAP_SYMS, np.int64)
    vfreq = np.bincount(val >> 23, minlength=VAL_SYMS)[:VAL_SYMS] if m else np.zeros(VAL_SYMS, np.int64)
    glen, vlen = huffman_lengths(gfreq), huffman_lengths(vfreq)
    gcode, vcode = canonical_codes(glen), canonical_codes(vlen)
    chunks, table, word = [], [], 0
    for c in range(nchunks):
        bw = _Bits()
        for k in range(c * CHUNK, min(m, (c + 1) * CHUNK)):
            if k % CHUNK:
                b = int(buckets[k])
                bw.put(*gcode[b])
                bw.put(int(gaps[k]) - (1 << b), b)
            v = int(val[k])
            bw.put(*vcode[v >> 23])
            bw.put(v & 0x7FFFFF, 23)
        data = bw.words()
        table.append((word, int(idx[c * CHUNK])))
        chunks.append(data)
        word += len(data) // 4
    head = struct.pack("<6I", MAGIC, VERSION, n, m, nchunks, CHUNK) + bytes(glen) + bytes(vlen)
    head += bytes(HEADER - len(head))
    tab = b"".join(struct.pack("<Ii", w, i) for w, i in table)
    return head + tab + b"".join(chunks)


def decode(blob: bytes, n: int) -> np.ndarray:
    """Dense float32 edits from an encoded blob (raises ValueError if malformed)."""
    blob = bytes(blob)
    if len(blob) < HEADER:
        raise ValueError("short blob")
    magic, version, n_h, m, nchunks, chunk = struct.unpack_from("<6I", blob, 0)
    if (magic, version, n_h, chunk) != (MAGIC, VERSION, n, CHUNK) or nchunks != (m + CHUNK - 1) // CHUNK:
        raise ValueError("header mismatch")
    glen = list(blob[24:24 + GAP_SYMS])
    vlen = list(blob[24 + GAP_SYMS:24 + GAP_SYMS + VAL_SYMS])
    gdec = {(c, L): s for s, (c, L) in canonical_codes(glen).items()}
    vdec = {(c, L): s for s, (c, L) in canonical_codes(vlen).items()}
    table = [struct.unpack_from("<Ii", blob, HEADER + 8 * c) for c in range(nchunks)]
    stream = blob[HEADER + 8 * nchunks:]
    nwords = len(stream) // 4
    out = np.zeros(n, dtype=np.uint32)
    for c in range(nchunks):
        w0 = table[c][0]
        w1 = table[c + 1][0] if c + 1 < nchunks else nwords
        acc = int.from_bytes(stream[4 * w0:4 * w1], "little")
        limit = 32 * (w1 - w0)
        pos = 0

        def bit():
            nonlocal pos
            if pos >= limit:
                raise ValueError("read past the chunk")
            b = (acc >> pos) & 1
            pos += 1
            return b

        def bits(w):
            v = 0
            for _ in range(w):
                v = (v << 1) | bit()
            return v

        def symbol(dec):
            code = 0
            for L in range(1, MAX_LEN + 1):
                code = (code << 1) | bit()
                if (code, L) in dec:
                    return dec[(code, L)]
            raise ValueError("bad code")

        i = table[c][1]
        for k in range(c * CHUNK, min(m, (c + 1) * CHUNK)):
            if k % CHUNK:
                b = symbol(gdec)
                i += (1 << b) + bits(b)
            e = symbol(vdec)
            mant = bits(23)
            if not 0 <= i < n:
                raise ValueError("index out of range")
            out[i] = (e << 23) | mant
    return out.view(np.float32)
