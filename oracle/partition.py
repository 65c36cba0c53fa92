"""Partition of the STEM image under a residency budget M (Sec. 4.2.4). TEST INFRASTRUCTURE ONLY.

For a set S of probes, I_{f,S,L} is the union of the L-nearest translate sets of its
probes. Computing the parts P_1..P_l in order, keeping each part's translates resident
and reusing those shared with the next part, costs

    T = sum_j |I_{f,P_j,L}| - sum_{j<l} |I_{f,P_j,L} intersect I_{f,P_{j+1},L}|

multislice runs. Of the paper's three strategies only the rectangle one is written here
(the row strategy is not used by the library, and the greedy one draws a random start).

Reading of the rectangle strategy ("rectangles of the same size, as large as possible
while every part keeps at most M solutions; smaller rectangles fill the rest; row-major or
column-major order"): the parts are taken row-major, so the rectangles are made as wide
as possible first, up to the whole region width, and then as tall as possible at that
width; edge rectangles are clipped. The paper fixes this reading through its second
example (Fig. lmastrategy_examples, bottom row): the rectangle partition stores about a
quarter of the trivial strategy's solutions, makes exactly its number of multislice
calls, and has l = 48 parts on the 48 x 48 sub-image. A largest-area reading cannot do
that: at a quarter of the memory it picks squares, whose row-major order recomputes the
translates shared between rows of rectangles.
"""
from __future__ import annotations


def union(sets_by_probe, probes) -> set:
    out = set()
    for p in probes:
        out.update(sets_by_probe[p])
    return out


def multislice_calls(sets_by_probe, parts) -> int:
    """T_{P_1..P_l} of Sec. 4.2.4."""
    unions = [union(sets_by_probe, part) for part in parts]
    t = sum(len(u) for u in unions)
    t -= sum(len(unions[j] & unions[j + 1]) for j in range(len(unions) - 1))
    return t


def _fits(sets_by_probe, region, w, h, M) -> bool:
    return all(len(union(sets_by_probe, part)) <= M for part in tiling(region, w, h))


def rectangles(sets_by_probe, region, M: int):
    """The rectangle strategy (reading in the module docstring); ``region`` = (a0, b0, width,
    height) in probe indices. Returns the parts in row-major order."""
    a0, b0, wd, ht = region
    for w in range(wd, 0, -1):
        for h in range(ht, 0, -1):
            if _fits(sets_by_probe, region, w, h, M):
                return tiling(region, w, h)
    raise ValueError("M smaller than one probe's translate set")


def tiling(region, w, h):
    """Row-major tiling of the region by w x h rectangles, clipped at its right and bottom."""
    a0, b0, wd, ht = region
    parts = []
    for by in range(0, ht, h):
        for bx in range(0, wd, w):
            parts.append([(a0 + a, b0 + b) for b in range(by, min(by + h, ht))
                          for a in range(bx, min(bx + w, wd))])
    return parts
