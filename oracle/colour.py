"""Greedy element colouring (Sec. 5, the paragraph after Alg. 2).

The paper avoids the race of the accumulation in Alg. 2 (several elements adding into
the rate of one shared global node) by colouring: elements are the vertices of a graph,
two elements are joined when they share any global node, and a greedy vertex colouring
gives joined elements different colours. Elements of one colour can then be processed
in parallel; the colours are walked one after another.

Readings where the paper is silent:
  * "greedy" is the first-fit rule: the elements are visited in the current element
    order (the order the solver stores them in, e.g. the Hilbert order) and each takes
    the smallest colour not yet used by an already-visited element it shares a node
    with;
  * sharing "a global node" includes a single shared vertex, so on a quadrilateral grid
    the four elements around an interior vertex are pairwise joined.

FP64 is not involved: colours are integers.
"""
from __future__ import annotations

import numpy as np


def element_neighbours(conn):
    """For every element, the sorted array of other elements sharing a global node with
    it (brute force over the node incidence)."""
    conn = np.asarray(conn, dtype=np.int64)
    E = conn.shape[0]
    n_nodes = int(conn.max()) + 1
    around = [[] for _ in range(n_nodes)]
    for e in range(E):
        for nd in set(conn[e].tolist()):
            around[nd].append(e)
    out = []
    for e in range(E):
        s = set()
        for nd in set(conn[e].tolist()):
            s.update(around[nd])
        s.discard(e)
        out.append(np.array(sorted(s), dtype=np.int64))
    return out


def greedy_colours(conn, order=None):
    """Colour of every element (indexed by element id of ``conn``): elements are visited
    in ``order`` (default: ascending id) and each takes the smallest colour absent from
    its already-coloured neighbours."""
    conn = np.asarray(conn, dtype=np.int64)
    E = conn.shape[0]
    order = np.arange(E) if order is None else np.asarray(order, dtype=np.int64)
    nbrs = element_neighbours(conn)
    colour = np.full(E, -1, np.int64)
    for e in order.tolist():
        used = {int(colour[f]) for f in nbrs[e].tolist() if colour[f] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[e] = c
    return colour


def colour_classes(colour, order):
    """Elements of each colour, each class in the visiting order."""
    colour = np.asarray(colour)
    order = np.asarray(order, dtype=np.int64)
    n = int(colour.max()) + 1 if colour.size else 0
    return [order[colour[order] == c] for c in range(n)]
