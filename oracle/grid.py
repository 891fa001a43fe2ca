"""Grid, boundary-ring ordering and the quadtree of boxes (oracle).

Section 2 of the paper: the grid is partitioned into 4^L boxes (the leaves),
L being the smallest integer for which every leaf is small enough; leaves are
merged four at a time into boxes of twice the side until the whole domain (the
root) is recovered.  Levels are numbered 0 (root) .. L (leaves).

Readings taken where the paper is silent:
* the leaf-size parameter is the maximum box side in nodes, `leaf`, and
  L = min{L >= 0 : ceil(n / 2^L) <= leaf}; a node interval [a, b) is split at
  a + floor((b - a) / 2), so boxes may be uneven by one node;
* children are listed SW, SE, NW, NE;
* a box ring is listed counter-clockwise starting at the box's SW corner
  (this is what makes the interface coupling blocks anti-diagonal, as stated
  in Section 6 Step 1).

Node (i, j) sits at (i h, j h), h = 1/(n-1); its linear index is i + n*j.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np


@dataclass
class Box:
    """A rectangle of nodes [x0, x1) x [y0, y1) and its children (SW, SE, NW, NE)."""
    x0: int
    x1: int
    y0: int
    y1: int
    level: int
    children: List["Box"] = field(default_factory=list)

    @property
    def sx(self) -> int:
        return self.x1 - self.x0

    @property
    def sy(self) -> int:
        return self.y1 - self.y0


def box_ring(x0: int, x1: int, y0: int, y1: int) -> List[Tuple[int, int]]:
    """Nodes on the ring of box [x0,x1)x[y0,y1), counter-clockwise from the SW corner.

    Side lengths (in steps) are sx-1 and sy-1, so the ring has 2(sx-1)+2(sy-1) nodes.
    """
    sx, sy = x1 - x0, y1 - y0
    assert sx >= 2 and sy >= 2
    out = []
    for t in range(sx - 1):          # south side, west -> east
        out.append((x0 + t, y0))
    for t in range(sy - 1):          # east side, south -> north
        out.append((x1 - 1, y0 + t))
    for t in range(sx - 1):          # north side, east -> west
        out.append((x1 - 1 - t, y1 - 1))
    for t in range(sy - 1):          # west side, north -> south
        out.append((x0, y1 - 1 - t))
    return out


def box_interior(x0: int, x1: int, y0: int, y1: int) -> List[Tuple[int, int]]:
    """Nodes of the box whose four neighbours all lie in the box (Section 3.1), row by row."""
    return [(i, j) for j in range(y0 + 1, y1 - 1) for i in range(x0 + 1, x1 - 1)]


def ring_nodes(n: int) -> List[Tuple[int, int]]:
    """The global boundary ring: nb = 4(n-1) nodes, counter-clockwise from (0, 0)."""
    return box_ring(0, n, 0, n)


def ring_index_of(n: int) -> dict:
    return {p: r for r, p in enumerate(ring_nodes(n))}


def num_levels(n: int, leaf: int) -> int:
    L = 0
    while -(-n // (2 ** L)) > leaf:
        L += 1
    return L


def build_tree(n: int, leaf: int) -> Box:
    """Quadtree over the n x n grid (Section 2) with leaves of side <= leaf."""
    if n < 3:
        raise ValueError("n must be >= 3")
    if leaf < 4:
        raise ValueError("leaf must be >= 4")
    L = num_levels(n, leaf)

    def make(x0, x1, y0, y1, lev):
        b = Box(x0, x1, y0, y1, lev)
        if lev < L:
            xm = x0 + (x1 - x0) // 2
            ym = y0 + (y1 - y0) // 2
            b.children = [make(x0, xm, y0, ym, lev + 1), make(xm, x1, y0, ym, lev + 1),
                          make(x0, xm, ym, y1, lev + 1), make(xm, x1, ym, y1, lev + 1)]
        return b

    return make(0, n, 0, n, 0)


def boxes_at_level(root: Box, level: int) -> List[Box]:
    out = []

    def walk(b):
        if b.level == level:
            out.append(b)
        else:
            for c in b.children:
                walk(c)

    walk(root)
    return out


def lin(n: int, nodes) -> np.ndarray:
    """Linear indices i + n*j of a list of (i, j) nodes."""
    return np.array([i + n * j for (i, j) in nodes], dtype=np.int64)
