"""Element and node reordering (Sec. 4.3) plus the comparison orders.

Element reordering along a generalized Hilbert curve, in the paper's four steps:
  1. element centroids;
  2. a bounding box of about sqrt(n_e) x sqrt(n_e)/r cells (r = mesh width / height)
     over which a generalized Hilbert curve (Cerveny 2020) is generated;
  3. walk the curve; at each cell append, once, the elements whose scaled centroid
     falls inside it, to a list L;
  4. L is the new element order.
Node reordering (Cuthill-McKee flavoured first touch): walk the elements in their new
order, collect each element's not-yet-seen nodes N^(e), sort them by ascending degree
and append them.

Readings where the paper is silent or garbled:
  * centroid of a quad = vertex average, evaluated as ((X0 + X1) + (X2 + X3)) * 0.25;
    of a triangle (the paper's element), ((X0 + X1) + X2) / 3;
  * the "bounding box of width sqrt(n_e)" is a W x H grid of cells with
    W = ceil(sqrt(E)), H = ceil(sqrt(E) / r); a centroid maps to cell
    clamp(floor((c - x_min) * W / w_m), 0, W - 1) (same for y with H / h_m);
  * curve index = 0-based position of a cell along the curve;
  * inside one cell, elements keep ascending original id;
  * node degree = number of distinct other nodes sharing at least one element with
    the node; equal degrees keep ascending local index q inside the element;
  * the generalized curve halves a side of odd length s into floor(s/2) and
    s - floor(s/2) cells before the parity adjustment described in ``gilbert_cells``.
Morton: cell x on even bits, cell y on odd bits. Lexicographic: generator order.
Random: stable sort by splitmix64(seed XOR element id).

The paper's two other strategies (Sec. 5, "Node Connectivity" and "Node Distance") walk
the mesh's nodes from a start node to connected nodes, appending each visited node's
elements (once) to the element list. Readings:
  * the walk runs over the mesh vertices (the nodes of the linear mesh), two vertices
    being connected when they share an element; "very similar to Cuthill-McKee" is read
    as the Cuthill-McKee breadth-first walk: visit the queue in order and append each
    visited vertex's unvisited neighbours in ascending priority;
  * priority: connectivity = vertex degree (distinct other vertices sharing an element),
    distance = squared distance (x - x0)^2 + (y - y0)^2 to the lower-left corner
    (x0, y0) = (min x, min y) of the vertices; ties by ascending vertex id;
  * the walk starts at the vertex of least priority and restarts there (among the
    unvisited vertices) if the mesh has several components;
  * a visited vertex appends its not-yet-listed elements in ascending element id.
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np

MASK64 = (1 << 64) - 1


# ----------------------------------------------------------------------------- step 1-2
def centroids(vxy, quads):
    X = vxy[quads]                                       # [E, 4, 2] or [E, 3, 2]
    if X.shape[1] == 3:
        return ((X[:, 0] + X[:, 1]) + X[:, 2]) / 3.0
    return ((X[:, 0] + X[:, 1]) + (X[:, 2] + X[:, 3])) * 0.25


def curve_grid(n_elements: int, vxy):
    """Bounding-box extent and the W x H cell grid of the curve."""
    xmin, ymin = float(vxy[:, 0].min()), float(vxy[:, 1].min())
    wm = float(vxy[:, 0].max()) - xmin
    hm = float(vxy[:, 1].max()) - ymin
    r = wm / hm
    s = math.sqrt(n_elements)
    W = max(1, math.ceil(s))
    H = max(1, math.ceil(s / r))
    return xmin, ymin, wm, hm, W, H


def centroid_cells(vxy, quads):
    """Cell (cx, cy) of every element centroid on the curve grid."""
    xmin, ymin, wm, hm, W, H = curve_grid(quads.shape[0], vxy)
    c = centroids(vxy, quads)
    sx = W / wm
    sy = H / hm
    cx = np.clip(np.floor((c[:, 0] - xmin) * sx), 0, W - 1).astype(np.int64)
    cy = np.clip(np.floor((c[:, 1] - ymin) * sy), 0, H - 1).astype(np.int64)
    return cx, cy, W, H


# ----------------------------------------------------------------------- Hilbert curve
def gilbert_cells(W: int, H: int):
    """All cells of a W x H grid in generalized-Hilbert order, as two int arrays.

    A region is an origin cell plus a major axis A (length w cells) and a minor axis
    B (length h cells). The curve enters the region at its origin and leaves at the far
    end of the first row along A. A region one cell thick is walked straight. A region
    much longer than it is wide (2w > 3h) is cut across A into two halves, each walked
    with the same axes. Otherwise it is cut into three: the near half of the first
    h/2 rows walked with the axes swapped (up the near side), the remaining rows at
    full width walked with the original axes, and the far half of the first rows
    walked back down with the axes swapped and reversed. A half-length that comes out
    odd is rounded up by one cell (when the side is longer than two) so the pieces
    keep even lengths where possible.
    """
    xs = np.empty(W * H, np.int64)
    ys = np.empty(W * H, np.int64)
    pos = 0

    def sgn(v):
        return (v > 0) - (v < 0)

    stack = []
    if W >= H:
        stack.append((0, 0, W, 0, 0, H))
    else:
        stack.append((0, 0, 0, H, W, 0))
    # explicit stack, children pushed in reverse so they pop in curve order
    while stack:
        x, y, ax, ay, bx, by = stack.pop()
        w = abs(ax + ay)
        h = abs(bx + by)
        dax, day = sgn(ax), sgn(ay)
        dbx, dby = sgn(bx), sgn(by)
        if h == 1:
            for i in range(w):
                xs[pos] = x + i * dax
                ys[pos] = y + i * day
                pos += 1
            continue
        if w == 1:
            for j in range(h):
                xs[pos] = x + j * dbx
                ys[pos] = y + j * dby
                pos += 1
            continue
        w2 = w // 2
        h2 = h // 2
        if 2 * w > 3 * h:
            if (w2 % 2) and w > 2:
                w2 += 1
            ax2, ay2 = w2 * dax, w2 * day
            stack.append((x + ax2, y + ay2, ax - ax2, ay - ay2, bx, by))
            stack.append((x, y, ax2, ay2, bx, by))
        else:
            if (h2 % 2) and h > 2:
                h2 += 1
            bx2, by2 = h2 * dbx, h2 * dby
            ax2, ay2 = w2 * dax, w2 * day
            third = (x + (ax - dax) + (bx2 - dbx), y + (ay - day) + (by2 - dby),
                     -bx2, -by2, -(ax - ax2), -(ay - ay2))
            second = (x + bx2, y + by2, ax, ay, bx - bx2, by - by2)
            first = (x, y, bx2, by2, ax2, ay2)
            stack.append(third)
            stack.append(second)
            stack.append(first)
    assert pos == W * H
    return xs, ys


def hilbert_index_grid(W: int, H: int):
    """idx[cy, cx] = position of cell (cx, cy) along the generalized Hilbert curve."""
    xs, ys = gilbert_cells(W, H)
    idx = np.empty((H, W), np.int64)
    idx[ys, xs] = np.arange(W * H)
    return idx


# --------------------------------------------------------------------- element orders
def hilbert_order(vxy, quads):
    """List L of the paper's step 3: walk the curve, append each cell's elements."""
    cx, cy, W, H = centroid_cells(vxy, quads)
    xs, ys = gilbert_cells(W, H)
    cell = cy * W + cx
    by_cell = {}
    for e in range(quads.shape[0]):           # ascending id inside each cell
        by_cell.setdefault(int(cell[e]), []).append(e)
    L = []
    for x, y in zip(xs.tolist(), ys.tolist()):
        L.extend(by_cell.get(y * W + x, ()))
    return np.asarray(L, dtype=np.int64)


def morton_key(cx, cy):
    """Interleave the bits of cx (even positions) and cy (odd positions)."""
    cx = np.asarray(cx, dtype=np.uint64)
    cy = np.asarray(cy, dtype=np.uint64)
    key = np.zeros(cx.shape, np.uint64)
    for bit in range(32):
        b = np.uint64(bit)
        key |= ((cx >> b) & np.uint64(1)) << np.uint64(2 * bit)
        key |= ((cy >> b) & np.uint64(1)) << np.uint64(2 * bit + 1)
    return key


def morton_order(vxy, quads):
    cx, cy, _, _ = centroid_cells(vxy, quads)
    return np.argsort(morton_key(cx, cy), kind="stable")


def splitmix64(state):
    """SplitMix64 output for the given 64-bit state(s): advance the state by the golden
    gamma 0x9E3779B97F4A7C15, then apply the two xor-shift-multiply rounds and a final
    xor-shift (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
    2014)."""
    with np.errstate(over="ignore"):
        z = (np.asarray(state, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def random_order(n_elements: int, seed: int):
    ids = np.arange(n_elements, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = splitmix64(np.uint64(seed) ^ ids)
    return np.argsort(key, kind="stable")


def vertex_adjacency(quads, n_vertices: int):
    """Sorted neighbour lists: vertices sharing at least one element, self excluded."""
    nb = [set() for _ in range(n_vertices)]
    for q in np.asarray(quads).tolist():
        for a in q:
            nb[a].update(q)
    return [sorted(s - {v}) for v, s in enumerate(nb)]


def vertex_elements(quads, n_vertices: int):
    """Elements of every vertex, ascending."""
    out = [[] for _ in range(n_vertices)]
    for e, q in enumerate(np.asarray(quads).tolist()):
        for a in set(q):
            out[a].append(e)
    return out


def walk_order(quads, n_vertices: int, priority):
    """Cuthill-McKee walk over the vertex graph with the given priority (smaller first,
    ties by vertex id). Returns (element new -> old order, vertex visit order)."""
    adj = vertex_adjacency(quads, n_vertices)
    v_el = vertex_elements(quads, n_vertices)
    key = lambda v: (priority[v], v)
    starts = sorted(range(n_vertices), key=key)
    visited = [False] * n_vertices
    listed = [False] * len(quads)
    elems, verts = [], []
    queue = deque()
    for s in starts:
        if visited[s]:
            continue
        visited[s] = True
        queue.append(s)
        while queue:
            v = queue.popleft()
            verts.append(v)
            for e in v_el[v]:
                if not listed[e]:
                    listed[e] = True
                    elems.append(e)
            fresh = sorted((w for w in adj[v] if not visited[w]), key=key)
            for w in fresh:
                visited[w] = True
                queue.append(w)
    return np.array(elems, np.int64), np.array(verts, np.int64)


def vertex_degree(quads, n_vertices: int):
    return np.array([len(a) for a in vertex_adjacency(quads, n_vertices)], np.int64)


def distance_priority(vxy):
    """Squared distance of every vertex to the lower-left corner of the vertex set."""
    vxy = np.asarray(vxy, dtype=np.float64)
    x0, y0 = vxy[:, 0].min(), vxy[:, 1].min()
    dx, dy = vxy[:, 0] - x0, vxy[:, 1] - y0
    return dx * dx + dy * dy


def element_order(kind: str, vxy, quads, seed: int = 3):
    """new -> old element permutation for 'hilbert' | 'morton' | 'lex' | 'random' |
    'connectivity' | 'distance'."""
    if kind == "connectivity":
        nv = np.asarray(vxy).shape[0]
        return walk_order(quads, nv, vertex_degree(quads, nv))[0]
    if kind == "distance":
        return walk_order(quads, np.asarray(vxy).shape[0], distance_priority(vxy))[0]
    if kind == "hilbert":
        return hilbert_order(vxy, quads)
    if kind == "morton":
        return morton_order(vxy, quads)
    if kind == "lex":
        return np.arange(quads.shape[0], dtype=np.int64)
    if kind == "random":
        return random_order(quads.shape[0], seed)
    raise ValueError(kind)


# ------------------------------------------------------------------- node reordering
def node_degree(conn, n_nodes: int, chunk: int = 1 << 20):
    """Number of distinct other nodes that share at least one element with each node."""
    E, nq = conn.shape
    flat = conn.ravel()
    order = np.argsort(flat, kind="stable")
    inc_elem = (order // nq).astype(np.int64)                 # incident elements, node-sorted
    counts = np.bincount(flat, minlength=n_nodes)
    starts = np.concatenate([[0], np.cumsum(counts)])
    deg = np.empty(n_nodes, np.int64)
    for c in np.unique(counts):
        nodes = np.nonzero(counts == c)[0]
        for lo in range(0, nodes.size, max(1, chunk // max(1, c))):
            nd = nodes[lo:lo + max(1, chunk // max(1, c))]
            els = inc_elem[starts[nd][:, None] + np.arange(c)[None, :]]   # [k, c]
            nb = np.sort(conn[els].reshape(nd.size, c * nq), axis=1)
            distinct = 1 + np.count_nonzero(np.diff(nb, axis=1), axis=1)
            deg[nd] = distinct - 1
    return deg


def first_touch_nodes(conn, elem_new2old, degree):
    """new -> old node permutation: walk elements in the new order, append each
    element's unseen nodes sorted by (degree, local index)."""
    n_nodes = degree.size
    seen = np.zeros(n_nodes, bool)
    out = np.empty(n_nodes, np.int64)
    pos = 0
    deg = degree.tolist()
    for e in elem_new2old.tolist():
        fresh = [nd for nd in conn[e].tolist() if not seen[nd]]
        fresh.sort(key=lambda nd: deg[nd])                    # stable: local order on ties
        for nd in fresh:
            seen[nd] = True
            out[pos] = nd
            pos += 1
    assert pos == n_nodes
    return out


def reorder(kind: str, vxy, quads, conn, seed: int = 3, node_order: str = "first_touch"):
    """(elem_new2old, node_new2old) for one element order."""
    elem = element_order(kind, vxy, quads, seed)
    n_nodes = int(conn.max()) + 1
    if node_order == "original":
        return elem, np.arange(n_nodes, dtype=np.int64)
    deg = node_degree(conn, n_nodes)
    return elem, first_touch_nodes(conn, elem, deg)
