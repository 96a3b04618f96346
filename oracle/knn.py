"""Brute-force stencils: the n nearest nodes of each centre (Section 4.1, eq. 11).

For centre c every candidate j is ranked by the key (d2_cj, j), where
d2 = (dx*dx) + (dy*dy) [+ (dz*dz)] is evaluated term by term, each product and
sum rounded separately (numpy never fuses them), and j is the candidate's
original index.  When the centre is itself a candidate it comes first (d2 = 0).
On a periodic box dx is the minimum image: dx -= L if dx > L/2, dx += L if
dx < -L/2.
"""
import math

import numpy as np


def _d2(src, c, period):
    acc = None
    for k in range(src.shape[1]):
        dk = src[:, k] - c[k]
        if period is not None and period[k] is not None:
            L = period[k]
            dk = np.where(dk > 0.5 * L, dk - L, dk)
            dk = np.where(dk < -0.5 * L, dk + L, dk)
        sq = dk * dk
        acc = sq if acc is None else acc + sq
    return acc


def knn(src, k, centres=None, period=None, src_ids=None):
    """Indices [C, k] into ``src`` of the k nearest sources of each centre.

    ``centres`` defaults to ``src`` itself.  ``src_ids`` (default: position)
    is the original index used to break ties.
    """
    if centres is None:
        centres = src
    ids = np.arange(src.shape[0], dtype=np.int64) if src_ids is None else np.asarray(src_ids)
    if k > src.shape[0]:
        raise ValueError("stencil larger than the node set")
    out = np.empty((centres.shape[0], k), dtype=np.int64)
    for c in range(centres.shape[0]):
        d2 = _d2(src, centres[c], period)
        # every j whose d2 does not exceed the k-th smallest is a candidate
        kth = np.partition(d2, k - 1)[k - 1]
        cand = np.nonzero(d2 <= kth)[0]
        order = np.lexsort((ids[cand], d2[cand]))
        out[c] = cand[order[:k]]
    return out


def min_image(v, period):
    """Apply the minimum-image rule to difference vectors v [..., d]."""
    if period is None:
        return v
    v = v.copy()
    for k, L in enumerate(period):
        if L is None:
            continue
        v[..., k] = np.where(v[..., k] > 0.5 * L, v[..., k] - L, v[..., k])
        v[..., k] = np.where(v[..., k] < -0.5 * L, v[..., k] + L, v[..., k])
    return v


def knn_cells(src, k, centres=None, period=None, src_ids=None):
    """The same stencils as ``knn`` (key (d2, original index), d2 evaluated
    term by term as there), found by searching grid cells instead of every
    node, for node sets of millions of nodes.

    Sources go into cells of side about the expected k-th neighbour
    distance.  For the centres of one cell the candidates are the sources of
    the block of (2L + 1)^d cells around it, ranked exactly as in ``knn``.
    A centre's list is accepted only when its k-th squared distance is below
    the squared distance from the centre to the nearest face of the searched
    block: every source outside the block is at least that far away, so it
    cannot belong to the list.  Centres that fail are searched again with
    L + 1; a block that covers the whole box along an axis has no face there
    (and on a periodic axis takes each cell once).
    """
    src = np.asarray(src, dtype=np.float64)
    centres = src if centres is None else np.asarray(centres, dtype=np.float64)
    ids = np.arange(src.shape[0], dtype=np.int64) if src_ids is None else np.asarray(src_ids, dtype=np.int64)
    Ns, d = src.shape
    if k > Ns:
        raise ValueError("stencil larger than the node set")
    per = [None] * d if period is None else [period[a] for a in range(d)]
    lo = np.minimum(src.min(axis=0), centres.min(axis=0))
    hi = np.maximum(src.max(axis=0), centres.max(axis=0))
    ext = np.array([per[a] if per[a] is not None else max(hi[a] - lo[a], 1e-300) for a in range(d)])
    vol = float(np.prod(ext))
    ball = math.pi if d == 2 else 4.0 * math.pi / 3.0
    side = (k / (Ns / vol) / ball) ** (1.0 / d)
    ncell = np.maximum(1, np.floor(ext / side)).astype(np.int64) if period is not None else \
        np.maximum(1, np.ceil(ext / side)).astype(np.int64)
    csz = ext / ncell

    def cell_of(x):
        c = np.floor((x - lo) / csz).astype(np.int64)
        for a in range(d):
            c[:, a] = np.mod(c[:, a], ncell[a]) if per[a] is not None else np.clip(c[:, a], 0, ncell[a] - 1)
        return c

    def linear(c):
        lin = c[:, d - 1].copy()
        for a in range(d - 2, -1, -1):
            lin = lin * ncell[a] + c[:, a]
        return lin

    scell = linear(cell_of(src))
    sorder = np.argsort(scell, kind="stable")
    bounds = np.searchsorted(scell[sorder], np.arange(ncell.prod() + 1))
    ccell = cell_of(centres)
    out = np.empty((centres.shape[0], k), dtype=np.int64)
    todo = np.arange(centres.shape[0])
    L = 1
    while todo.size:
        lin = linear(ccell[todo])
        grp = np.argsort(lin, kind="stable")
        starts = np.flatnonzero(np.r_[True, lin[grp][1:] != lin[grp][:-1]])
        failed = []
        for g0, g1 in zip(starts, np.r_[starts[1:], grp.size]):
            cen = todo[grp[g0:g1]]
            c0 = ccell[cen[0]]
            axes, full = [], []
            for a in range(d):
                if 2 * L + 1 >= ncell[a]:
                    axes.append(np.arange(ncell[a]))
                    full.append(True)
                else:
                    r = np.arange(c0[a] - L, c0[a] + L + 1)
                    if per[a] is not None:
                        axes.append(np.mod(r, ncell[a]))
                        full.append(False)
                    else:
                        axes.append(r[(r >= 0) & (r < ncell[a])])
                        full.append(c0[a] - L <= 0 and c0[a] + L >= ncell[a] - 1)
            mesh = np.meshgrid(*axes, indexing="ij")
            cells = linear(np.stack([m.reshape(-1) for m in mesh], axis=1))
            cand = np.concatenate([sorder[bounds[c]:bounds[c + 1]] for c in cells])
            if cand.size < k and not all(full):
                failed.append(cen)
                continue
            acc = None
            for a in range(d):
                dk = src[cand, a][None, :] - centres[cen, a][:, None]
                if per[a] is not None:
                    Lp = per[a]
                    dk = np.where(dk > 0.5 * Lp, dk - Lp, dk)
                    dk = np.where(dk < -0.5 * Lp, dk + Lp, dk)
                sq = dk * dk
                acc = sq if acc is None else acc + sq
            order = np.lexsort((np.broadcast_to(ids[cand], acc.shape), acc), axis=1)[:, :k]
            kth = np.take_along_axis(acc, order[:, k - 1:k], axis=1)[:, 0]
            # distance from each centre to the nearest face of the block
            face = np.full(cen.size, np.inf)
            for a in range(d):
                if full[a]:
                    continue
                x = centres[cen, a]
                if per[a] is not None:
                    # the block spans [start, start + (2L + 1) csz) around the
                    # centre's cell, measured on the unwrapped axis
                    base = lo[a] + (c0[a] - L) * csz[a]
                    t = np.mod(x - base, per[a])
                    face = np.minimum(face, np.minimum(t, (2 * L + 1) * csz[a] - t))
                else:
                    if c0[a] - L > 0:
                        face = np.minimum(face, x - (lo[a] + (c0[a] - L) * csz[a]))
                    if c0[a] + L < ncell[a] - 1:
                        face = np.minimum(face, (lo[a] + (c0[a] + L + 1) * csz[a]) - x)
            ok = kth < face * face * (1.0 - 1e-10)
            out[cen[ok]] = cand[order[ok]]
            if not ok.all():
                failed.append(cen[~ok])
        todo = np.concatenate(failed) if failed else np.empty(0, dtype=np.int64)
        L += 1
    return out
