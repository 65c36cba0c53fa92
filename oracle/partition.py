"""Partition of the STEM image under a residency budget M (Sec. 4.2.4). TEST INFRASTRUCTURE ONLY.

For a set S of probes, I_{f,S,L} is the union of the L-nearest translate sets of its
probes. Computing the parts P_1..P_l in order, keeping each part's translates resident
and reusing those shared with the next part, costs

    T = sum_j |I_{f,P_j,L}| - sum_{j<l} |I_{f,P_j,L} intersect I_{f,P_{j+1},L}|

multislice runs. Two of the paper's strategies are written here: row by row and
rectangles (the greedy one draws a random start and is not reproducible from the text).

Reading of the rectangle strategy: among all rectangle shapes w x h, take the one of
largest area (ties: the wider one) whose every tile in the row-major tiling of the
region, edge tiles clipped, satisfies |I_{f,P_j,L}| <= M. A device may restrict the
shapes to sides that are multiples of a granule (gx, gy), or the whole region side;
granule (1, 1) is the strategy as the paper states it.
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


def row_by_row(sets_by_probe, region, M: int):
    """Strategy 1: walk the region row-major, start a new part when the next probe would
    push the part's translate count above M. ``region`` = (a0, b0, width, height)."""
    a0, b0, wd, ht = region
    order = [(a0 + a, b0 + b) for b in range(ht) for a in range(wd)]
    parts, cur, cur_u = [], [], set()
    for p in order:
        nu = cur_u | set(sets_by_probe[p])
        if cur and len(nu) > M:
            parts.append(cur)
            cur, cur_u = [p], set(sets_by_probe[p])
        else:
            cur.append(p)
            cur_u = nu
    if cur:
        parts.append(cur)
    return parts


def rectangles(sets_by_probe, region, M: int, granule=(1, 1)):
    """Strategy 2 (reading in the module docstring). Returns the parts, row-major."""
    a0, b0, wd, ht = region
    gx, gy = granule
    best = None
    for h in range(1, ht + 1):
        if h % gy and h != ht:
            continue
        for w in range(1, wd + 1):
            if w % gx and w != wd:
                continue
            if best is not None and w * h < best[0] * best[1]:
                continue
            parts = _tiling(region, w, h)
            if all(len(union(sets_by_probe, part)) <= M for part in parts):
                if best is None or w * h > best[0] * best[1] or (w * h == best[0] * best[1] and w > best[0]):
                    best = (w, h)
    if best is None:
        raise ValueError("M smaller than one probe's translate set")
    return _tiling(region, *best)


def _tiling(region, w, h):
    a0, b0, wd, ht = region
    parts = []
    for by in range(0, ht, h):
        for bx in range(0, wd, w):
            parts.append([(a0 + a, b0 + b) for b in range(by, min(by + h, ht))
                          for a in range(bx, min(bx + w, wd))])
    return parts
