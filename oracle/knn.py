"""Brute-force stencils: the n nearest nodes of each centre (Section 4.1, eq. 11).

For centre c every candidate j is ranked by the key (d2_cj, j), where
d2 = (dx*dx) + (dy*dy) [+ (dz*dz)] is evaluated term by term, each product and
sum rounded separately (numpy never fuses them), and j is the candidate's
original index.  When the centre is itself a candidate it comes first (d2 = 0).
On a periodic box dx is the minimum image: dx -= L if dx > L/2, dx += L if
dx < -L/2.
"""
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
