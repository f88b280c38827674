"""Seeded synthetic inputs for the LocPIR bounding-box workloads.

Holds none of the encryption or bootstrapping arithmetic: it only draws
plaintext inputs (bits, coordinates, boxes, payloads) and quantizes
coordinates to the fixed-point integers of Sec. 4.1.  Both the GPU path and
the CPU oracle consume what it returns.

Recipes (all numpy PCG64, seeded):
* fixed point, 16 bit: two's complement of floor(deg * 2^7) -- 9 integer
  bits (room for +-180 degrees) and 7 fraction bits, the paper's default;
* fixed point, 32 bit: two's complement of floor(deg * 10^6);
* 8 bit: raw uniform unsigned integers;
* boxes: a random guillotine tiling of a region (split the largest box at a
  uniform position along a random axis until N boxes exist), so boxes are
  disjoint with random widths; tilings that quantize to an empty box are
  redrawn;
* points: uniform over the region grown by 10 % on each side, so some points
  fall in no box.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KOREA = (33.0, 38.7, 124.5, 131.0)          # lat0, lat1, lon0, lon1
ZERO_STRADDLE = (-5.0, 5.0, -8.0, 8.0)


def quantize(deg: float, l: int) -> int:
    """Fixed-point code of a coordinate (l-bit two's complement, as unsigned)."""
    if l == 16:
        v = math.floor(deg * 128.0)
    elif l == 32:
        v = math.floor(deg * 1e6)
    else:  # 9 integer bits (signed degrees), l - 9 fraction bits; fewer than 9 bits scale down
        v = math.floor(deg * 2.0 ** (l - 9))
    lo, hi = -(1 << (l - 1)), (1 << (l - 1)) - 1
    if not lo <= v <= hi:
        raise ValueError(f"{deg} does not fit {l}-bit fixed point")
    return v & ((1 << l) - 1)


def bits_lsb(v: int, l: int) -> np.ndarray:
    return np.array([(v >> i) & 1 for i in range(l)], np.uint8)


def from_bits(bits) -> int:
    return int(sum(int(b) << i for i, b in enumerate(bits)))


@dataclass
class BBoxQuery:
    """One plaintext query: a point, N boxes (x1, x2, y1, y2) and payloads."""
    l: int
    m: int
    is_signed: bool
    x: int
    y: int
    boxes: list = field(default_factory=list)     # [(x1, x2, y1, y2)] as l-bit codes
    payloads: list = field(default_factory=list)  # m-bit integers

    @property
    def n_boxes(self) -> int:
        return len(self.boxes)

    def plain_bits(self):
        """Bits in ciphertext order: x (l), y (l), bounds (N*4*l), payload (N*m)."""
        xb = bits_lsb(self.x, self.l)
        yb = bits_lsb(self.y, self.l)
        bb = np.concatenate([bits_lsb(v, self.l) for box in self.boxes for v in box]) \
            if self.boxes else np.zeros(0, np.uint8)
        pb = np.concatenate([bits_lsb(s, self.m) for s in self.payloads]) \
            if self.payloads else np.zeros(0, np.uint8)
        return xb, yb, bb, pb


def guillotine(rng: np.random.Generator, region, n: int):
    boxes = [tuple(region)]
    while len(boxes) < n:
        areas = [(b[1] - b[0]) * (b[3] - b[2]) for b in boxes]
        k = int(np.argmax(areas))
        a0, a1, b0, b1 = boxes.pop(k)
        if rng.random() < 0.5:
            c = a0 + (a1 - a0) * rng.uniform(0.05, 0.95)
            boxes += [(a0, c, b0, b1), (c, a1, b0, b1)]
        else:
            c = b0 + (b1 - b0) * rng.uniform(0.05, 0.95)
            boxes += [(a0, a1, b0, c), (a0, a1, c, b1)]
    return boxes


def _signed(v: int, l: int) -> int:
    return v - (1 << l) if v >> (l - 1) else v


def random_query(seed: int, l: int, n_boxes: int, m: int, region=KOREA,
                 force_inside: bool | None = None) -> BBoxQuery:
    """Signed fixed-point query over a guillotine tiling of `region`."""
    rng = np.random.default_rng(seed)
    for _ in range(100):
        boxes_deg = guillotine(rng, region, n_boxes)
        boxes = [tuple(quantize(v, l) for v in b) for b in boxes_deg]
        if all(_signed(b[0], l) < _signed(b[1], l) and _signed(b[2], l) < _signed(b[3], l) for b in boxes):
            break
    else:
        raise RuntimeError("could not draw a non-degenerate tiling")
    la0, la1, lo0, lo1 = region
    if force_inside:
        b = boxes_deg[int(rng.integers(n_boxes))]
        px, py = rng.uniform(b[0], b[1]), rng.uniform(b[2], b[3])
    else:
        gx, gy = 0.1 * (la1 - la0), 0.1 * (lo1 - lo0)
        px, py = rng.uniform(la0 - gx, la1 + gx), rng.uniform(lo0 - gy, lo1 + gy)
    payloads = [int(v) for v in rng.integers(0, 1 << m, size=n_boxes, dtype=np.uint64)]
    return BBoxQuery(l, m, True, quantize(px, l), quantize(py, l), boxes, payloads)


def random_query_u8(seed: int, force_inside: bool | None = None, m: int = 8) -> BBoxQuery:
    """Unsigned 8-bit query against one box (two sorted distinct values per axis)."""
    rng = np.random.default_rng(seed)

    def axis():
        a, b = sorted(int(v) for v in rng.choice(256, size=2, replace=False))
        return a, b
    x1, x2 = axis()
    y1, y2 = axis()
    if force_inside:
        x, y = int(rng.integers(x1, x2)), int(rng.integers(y1, y2))
    else:
        x, y = int(rng.integers(0, 256)), int(rng.integers(0, 256))
    payload = int(rng.integers(0, 1 << m))
    return BBoxQuery(8, m, False, x, y, [(x1, x2, y1, y2)], [payload])


def random_bits(seed: int, count: int) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 2, size=count, dtype=np.uint8)


def table1_query(point_deg, rows, l: int = 16, m: int = 9) -> BBoxQuery:
    """Query against the boxes printed in the paper's Table 1."""
    boxes = [tuple(quantize(v, l) for v in (r[1], r[2], r[3], r[4])) for r in rows]
    payloads = [int(r[5]) for r in rows]
    return BBoxQuery(l, m, True, quantize(point_deg[0], l), quantize(point_deg[1], l), boxes, payloads)
