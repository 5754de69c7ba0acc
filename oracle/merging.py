"""Small-cell merging (Sec. 4.2: theta-proper cells, MAP-1/MAP-3 and the
BFS fallback of the CellMerging algorithm).

Reading used here (the paper leaves tie-breaking and the fallback's host
open):
  * a cut cell with |C| < theta h^3 is absorbed into the face neighbour,
    among theta-proper ones with positive common open-face area, whose
    common face is largest; areas within a relative 1e-10 of the largest
    tie and the smallest linear index wins;
  * a small cell without such a neighbour grows its own group by a
    breadth-first search over face neighbours with positive common area
    (neighbour order -x,+x,-y,+y,-z,+z), absorbing each visited cell's
    whole group, until the group volume reaches theta h^3; it becomes the
    group's host.  Such cells are processed in increasing index order.
Multi-component cells (MAP-2) cannot occur for the supported obstacles.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from .geometry import CUT, EXTERIOR, GeometryError

THETA = 0.1
TIE = 1e-10
NEIGH = ((0, -1), (0, 1), (1, -1), (1, 1), (2, -1), (2, 1))


def _neighbour(geo, p, d, s):
    ijk = list(geo.ijk(p))
    ijk[d] += s
    if not (0 <= ijk[d] < geo.n):
        return -1
    return geo.idx(*ijk)


def merge_cells(geo, theta: float = THETA) -> np.ndarray:
    """Returns host[n^3]: -1 for exterior cells, p for a cell that carries
    its own unknown (alone or as a host), and the host index for a cell
    absorbed into another."""
    n3 = geo.n ** 3
    h3 = geo.h ** 3
    host = np.arange(n3, dtype=np.int64)
    host[geo.cls == EXTERIOR] = -1
    small = [p for p in sorted(geo.cut) if geo.vol[p] < theta * h3]
    pending = []
    for p in small:
        best, best_a = -1, 0.0
        cands = []
        for d, s in NEIGH:
            q = _neighbour(geo, p, d, s)
            if q < 0 or geo.cls[q] == EXTERIOR or geo.vol[q] < theta * h3:
                continue
            a = geo.face_area(p, d, s)
            if a > 0:
                cands.append((a, q))
        if cands:
            amax = max(a for a, _ in cands)
            best = min(q for a, q in cands if a >= amax * (1.0 - TIE))
            host[p] = best
        else:
            pending.append(p)
    for p in pending:
        group = {q for q in range(n3) if host[q] == p} | {p}
        vol = sum(geo.vol[q] for q in group)
        seen = {p}
        queue = deque([p])
        while queue and vol < theta * h3:
            u = queue.popleft()
            for d, s in NEIGH:
                v = _neighbour(geo, u, d, s)
                if v < 0 or v in seen or geo.cls[v] == EXTERIOR:
                    continue
                if geo.face_area(u, d, s) <= 0:
                    continue
                seen.add(v)
                queue.append(v)
                w = host[v]
                members = set(np.nonzero(host == w)[0].tolist()) | {w, v}
                for q in members:
                    if q not in group:
                        group.add(q)
                        vol += geo.vol[q]
                    host[q] = p
                if vol >= theta * h3:
                    break
        if vol < theta * h3:
            raise GeometryError("merging could not reach a theta-proper cell")
        for q in group:
            host[q] = p
    return host


def groups(host: np.ndarray):
    """dict host -> sorted list of member cells (the host included)."""
    out = {}
    for q in np.nonzero(host >= 0)[0]:
        out.setdefault(int(host[q]), []).append(int(q))
    return out
