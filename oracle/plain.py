"""Plaintext side of the oracle (TEST INFRASTRUCTURE).

* ``comp_s_bits`` -- Algorithm 2 (HomCompS) evaluated on booleans, gate by
  gate: t0 = 0; optional NOT of both MSBs; for each bit from the LSB,
  t1 = XNOR(a_i, b_i), t0 = MUX(t1, t0, b_i).
* ``bbox_circuit_bits`` -- Algorithm 3 (LocPIR) with Algorithm 4
  (bitwiseAND) and Algorithm 5 (HomAddXOR, as a balanced XOR tree) on
  booleans.
* ``predicate`` -- the plain bounding-box predicate on integers: the XOR of
  the payloads of every box with x1 <= x < x2 and y1 <= y < y2.  With
  disjoint boxes this is the payload of the box holding the point, or 0
  (Sec. 4.4).

The first two are the circuit; the last is what the circuit must compute.
Tests check one against the other exhaustively and at random.
"""
from __future__ import annotations


def to_bits(v: int, l: int) -> list[int]:
    """l-bit two's-complement bits of v, LSB first."""
    return [(v >> i) & 1 for i in range(l)]


def from_bits(bits) -> int:
    return sum(int(b) << i for i, b in enumerate(bits))


def as_signed(v: int, l: int) -> int:
    v &= (1 << l) - 1
    return v - (1 << l) if v >> (l - 1) else v


def xnor(a: int, b: int) -> int:
    return 1 - (a ^ b)


def mux(sel: int, t: int, f: int) -> int:
    return t if sel else f


def comp_s_bits(a_bits, b_bits, is_signed: bool) -> int:
    """Algorithm 2 on plaintext bits: 1 iff a < b."""
    a = list(a_bits)
    b = list(b_bits)
    l = len(a)
    t0 = 0
    if is_signed:
        a[l - 1] ^= 1
        b[l - 1] ^= 1
    for i in range(l):
        t1 = xnor(a[i], b[i])
        t0 = mux(t1, t0, b[i])
    return t0


def comp_le_bits(a_bits, b_bits, is_signed: bool) -> int:
    """HomCompLE(a, b) = NOT HomCompS(b, a): 1 iff a <= b."""
    return 1 - comp_s_bits(b_bits, a_bits, is_signed)


def xor_tree(vals):
    """Balanced XOR reduction, pairs left to right, odd element carried."""
    cur = list(vals)
    while len(cur) > 1:
        nxt = [cur[2 * k] ^ cur[2 * k + 1] for k in range(len(cur) // 2)]
        if len(cur) % 2:
            nxt.append(cur[-1])
        cur = nxt
    return cur[0]


def bbox_circuit_bits(x: int, y: int, boxes, payloads, l: int, m: int, is_signed: bool) -> int:
    """Algorithms 3-5 on plaintext bits; boxes are (x1, x2, y1, y2) integers."""
    xb, yb = to_bits(x, l), to_bits(y, l)
    masked = []
    for (x1, x2, y1, y2), s in zip(boxes, payloads):
        xl = comp_le_bits(to_bits(x1, l), xb, is_signed)
        xr = comp_s_bits(xb, to_bits(x2, l), is_signed)
        yl = comp_le_bits(to_bits(y1, l), yb, is_signed)
        yr = comp_s_bits(yb, to_bits(y2, l), is_signed)
        f = (xl & xr) & (yl & yr)
        masked.append([f & b for b in to_bits(s, m)])
    out = [xor_tree([mb[j] for mb in masked]) for j in range(m)]
    return from_bits(out)


def predicate(x: int, y: int, boxes, payloads, l: int, m: int, is_signed: bool) -> int:
    """XOR of the payloads of all boxes with x1 <= x < x2 and y1 <= y < y2."""
    conv = (lambda v: as_signed(v, l)) if is_signed else (lambda v: v & ((1 << l) - 1))
    X, Y = conv(x), conv(y)
    r = 0
    for (x1, x2, y1, y2), s in zip(boxes, payloads):
        if conv(x1) <= X < conv(x2) and conv(y1) <= Y < conv(y2):
            r ^= s & ((1 << m) - 1)
    return r
