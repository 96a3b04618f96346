"""Node orderings: Morton (Z-order) and Reverse Cuthill-McKee.

Neither is part of the paper's method (the paper leaves node order to its node
generator); both only relabel nodes.  They are defined here bit for bit so that
the GPU library can be checked against them exactly.

Morton: the quantisation box is the cube [lo, lo + side)^d; per axis k,
q_k = min(floor((x_k - lo_k) * scale), 2^b - 1) with scale = 2^b / side (one
correctly rounded FP64 division), b = 32 bits in 2D and 21 in 3D; key bit
(d*i + k) is bit i of q_k (x lowest).  Nodes are sorted by (key, original
index).  ``morton_box`` gives the cube of a bounding box: side = the largest
extent.

RCM: graph = symmetrised stencil graph without self loops.  Start at the
unvisited node with the smallest (degree, original index); breadth-first,
appending each node's unvisited neighbours in increasing (degree, original
index); restart for every component; finally reverse the whole order.
"""
import numpy as np


def morton_bits(d):
    return 32 if d == 2 else 21


def morton_box(lo, hi):
    """(lo, side) of the quantisation cube of the bounding box [lo, hi]."""
    return tuple(float(v) for v in lo), max(float(hi[k]) - float(lo[k]) for k in range(len(lo)))


def morton_keys(xyz, lo, side):
    """uint64 Morton keys of the nodes (see module docstring)."""
    N, d = xyz.shape
    b = morton_bits(d)
    scale = float(2.0 ** b) / float(side)
    top = np.uint64((1 << b) - 1)
    key = np.zeros(N, dtype=np.uint64)
    for k in range(d):
        v = (xyz[:, k] - float(lo[k])) * scale
        q = np.floor(v)
        q = np.where(q < 0, 0.0, q)
        q = np.minimum(q.astype(np.uint64), top)
        for i in range(b):
            bit = (q >> np.uint64(i)) & np.uint64(1)
            key |= bit << np.uint64(d * i + k)
    return key


def morton_order(xyz, lo, side):
    """perm[p] = original index of the node at internal position p."""
    key = morton_keys(xyz, lo, side)
    return np.argsort(key, kind="stable").astype(np.int64)


def rcm_order(stencil):
    """RCM order from an [N, n] stencil index array (original labels)."""
    N = stencil.shape[0]
    nbr = [set() for _ in range(N)]
    for i in range(N):
        for j in stencil[i]:
            j = int(j)
            if j != i:
                nbr[i].add(j)
                nbr[j].add(i)
    deg = np.array([len(s) for s in nbr], dtype=np.int64)
    visited = np.zeros(N, dtype=bool)
    order = []
    by_deg = sorted(range(N), key=lambda v: (deg[v], v))
    for start in by_deg:
        if visited[start]:
            continue
        visited[start] = True
        queue = [start]
        head = 0
        while head < len(queue):
            v = queue[head]
            head += 1
            order.append(v)
            nxt = sorted((u for u in nbr[v] if not visited[u]), key=lambda u: (deg[u], u))
            for u in nxt:
                visited[u] = True
                queue.append(u)
    return np.array(order[::-1], dtype=np.int64)


def inverse(perm):
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size, dtype=perm.dtype)
    return inv
