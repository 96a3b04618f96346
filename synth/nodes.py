"""Seeded synthetic node sets (scattered nodes with spacing about h).

The paper discretises its domains with a third-party advancing-front node
generator (Section 4) that is not available here; these generators stand in
for it with the same spacing and irregularity:

* ``jittered_grid``  -- a regular grid, each coordinate offset by a uniform
  draw in [-j*h, j*h] (j = 0.25 by default).  Nodes on a face of a bounded box
  move only tangentially to that face; corners stay put.  Periodic boxes jitter
  every node and wrap into [lo, hi).
* ``poisson_disk_2d`` -- a maximal-style Poisson-disk set on the unit square
  with boundary nodes seeded along the edges, built by phase-grouped parallel
  dart throwing (Wei, "Parallel Poisson disk sampling", SIGGRAPH 2008): cells of
  side r/sqrt(2) hold at most one point, and cells three apart in both
  directions are filled in the same phase.
* ``dual_grid_2d`` -- the jittered cell-centre grid used as the second node set
  of the two-set (staggered) variant.
* ``poisson_disk_periodic`` / ``line_seeded_periodic`` -- the same dart
  throwing on a periodic square around fixed seed points; with the seeds an
  equispaced line this is the node set of the dispersion study (Section 6),
  whose generator completes a discretised line y = L/2 into a scattered set.
* ``disk_nodes`` -- a curved PEC boundary: equispaced nodes on a circle
  (flagged as wall nodes) and Poisson-disk darts inside it.

Boundary flags (uint8 per node): bit 0/1 = x low/high face, bit 2/3 = y, bit
4/5 = z.  All random draws come from ``synth.rng`` keyed by (seed, stream,
node id), so every set is reproducible bit for bit.
"""
import math
import numpy as np

from . import rng

FACE_XLO, FACE_XHI, FACE_YLO, FACE_YHI, FACE_ZLO, FACE_ZHI = 1, 2, 4, 8, 16, 32


def jittered_grid(shape, lo=None, hi=None, jitter=0.25, seed=1, stream=0,
                  periodic=False):
    """Jittered grid with ``shape`` = (nx, ny) or (nx, ny, nz) nodes.

    Returns (xyz float64 [N, d], flags uint8 [N], h float) with h the grid
    spacing along x.
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    lo = np.zeros(d) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = np.ones(d) if hi is None else np.asarray(hi, dtype=np.float64)
    axes = []
    spacing = []
    for k in range(d):
        n = shape[k]
        if periodic:
            hk = (hi[k] - lo[k]) / n
        else:
            hk = (hi[k] - lo[k]) / (n - 1)
        spacing.append(hk)
        axes.append(np.arange(n))
    grids = np.meshgrid(*axes, indexing="ij")            # index [ix, iy(, iz)]
    # node id: x fastest
    idx = [g.transpose(tuple(reversed(range(d)))).reshape(-1) for g in grids]
    N = idx[0].size
    ids = np.arange(N, dtype=np.uint64)
    xyz = np.empty((N, d), dtype=np.float64)
    flags = np.zeros(N, dtype=np.uint8)
    for k in range(d):
        ik = idx[k]
        hk = spacing[k]
        base = lo[k] + ik * hk
        off = rng.uniform_range(seed, stream, ids * np.uint64(d) + np.uint64(k),
                                -jitter * hk, jitter * hk)
        if periodic:
            x = base + off
            L = hi[k] - lo[k]
            x = np.where(x < lo[k], x + L, x)
            x = np.where(x >= hi[k], x - L, x)
            xyz[:, k] = x
        else:
            on_lo = ik == 0
            on_hi = ik == shape[k] - 1
            x = np.where(on_lo | on_hi, base, base + off)
            x = np.where(on_lo, lo[k], x)
            x = np.where(on_hi, hi[k], x)
            xyz[:, k] = x
            flags |= np.where(on_lo, 1 << (2 * k), 0).astype(np.uint8)
            flags |= np.where(on_hi, 1 << (2 * k + 1), 0).astype(np.uint8)
    return xyz, flags, float(spacing[0])


def dual_grid_2d(n_cells, lo=(0.0, 0.0), hi=(1.0, 1.0), jitter=0.25, seed=1,
                 stream=3):
    """Jittered cell centres of an n_cells x n_cells grid (all interior)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    h = (hi - lo) / n_cells
    iy, ix = np.meshgrid(np.arange(n_cells), np.arange(n_cells), indexing="ij")
    ix = ix.reshape(-1)
    iy = iy.reshape(-1)
    ids = np.arange(ix.size, dtype=np.uint64)
    xyz = np.empty((ix.size, 2))
    for k, ik in enumerate((ix, iy)):
        off = rng.uniform_range(seed, stream, ids * np.uint64(2) + np.uint64(k),
                                -jitter * h[k], jitter * h[k])
        xyz[:, k] = lo[k] + (ik + 0.5) * h[k] + off
    return xyz, np.zeros(ix.size, dtype=np.uint8), float(h[0])


def poisson_disk_2d(r, seed=2, stream=0, rounds=12):
    """Poisson-disk-style nodes on the PEC unit square with minimum distance r.

    Boundary nodes are equispaced along the four edges (spacing 1/floor(1/r),
    corners included once) and fixed first; interior darts are accepted when
    they keep distance >= r from every accepted node.  Returns
    (xyz [N, 2], flags [N], h) with h = 1/sqrt(N), the mean spacing.
    """
    nb = int(math.floor(1.0 / r))
    t = np.arange(nb + 1) / nb
    bx, by, bf = [], [], []
    # bottom and top edges (including corners)
    bx += [t, t]
    by += [np.zeros_like(t), np.ones_like(t)]
    fb = np.full(t.size, FACE_YLO, np.uint8)
    ft = np.full(t.size, FACE_YHI, np.uint8)
    fb[0] |= FACE_XLO
    fb[-1] |= FACE_XHI
    ft[0] |= FACE_XLO
    ft[-1] |= FACE_XHI
    bf += [fb, ft]
    # left and right edges without corners
    ti = t[1:-1]
    bx += [np.zeros_like(ti), np.ones_like(ti)]
    by += [ti, ti]
    bf += [np.full(ti.size, FACE_XLO, np.uint8), np.full(ti.size, FACE_XHI, np.uint8)]
    px = np.concatenate(bx)
    py = np.concatenate(by)
    pf = np.concatenate(bf)

    cs = r / math.sqrt(2.0)
    nc = int(math.ceil(1.0 / cs))
    occ = np.full((nc + 4, nc + 4), -1, dtype=np.int64)   # 2-cell pad on each side

    def cell(v):
        return np.minimum((v / cs).astype(np.int64), nc - 1)

    cx = cell(px)
    cy = cell(py)
    occ[cy + 2, cx + 2] = np.arange(px.size)
    allx = px.copy()
    ally = py.copy()
    r2 = r * r
    gy, gx = np.meshgrid(np.arange(nc), np.arange(nc), indexing="ij")
    gx = gx.reshape(-1)
    gy = gy.reshape(-1)
    counter = 0
    for rnd in range(rounds):
        for ph in range(9):
            sel = ((gx % 3) == (ph % 3)) & ((gy % 3) == (ph // 3))
            cxs = gx[sel]
            cys = gy[sel]
            empty = occ[cys + 2, cxs + 2] < 0
            cxs = cxs[empty]
            cys = cys[empty]
            if cxs.size == 0:
                continue
            cid = (cys * nc + cxs).astype(np.uint64)
            key = cid * np.uint64(2) + np.uint64(2 * nc * nc) * np.uint64(counter)
            ux = rng.uniform(seed, stream, key)
            uy = rng.uniform(seed, stream, key + np.uint64(1))
            counter += 1
            qx = (cxs + ux) * cs
            qy = (cys + uy) * cs
            ok = (qx > 0.0) & (qx < 1.0) & (qy > 0.0) & (qy < 1.0)
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    j = occ[cys + 2 + dy, cxs + 2 + dx]
                    has = j >= 0
                    jj = np.where(has, j, 0)
                    ddx = qx - allx[jj]
                    ddy = qy - ally[jj]
                    ok &= ~(has & (ddx * ddx + ddy * ddy < r2))
            qx = qx[ok]
            qy = qy[ok]
            if qx.size == 0:
                continue
            start = allx.size
            occ[cys[ok] + 2, cxs[ok] + 2] = np.arange(start, start + qx.size)
            allx = np.concatenate([allx, qx])
            ally = np.concatenate([ally, qy])
    n_int = allx.size - px.size
    xyz = np.stack([allx, ally], axis=1)
    flags = np.concatenate([pf, np.zeros(n_int, np.uint8)])
    return xyz, flags, 1.0 / math.sqrt(xyz.shape[0])



def poisson_disk_periodic(L, r, seeds, seed=3, stream=0, rounds=12):
    """Poisson-disk-style nodes on the periodic square [0, L)^2 around seeds.

    seeds [S, 2] are kept first, in order (they must be r apart, minimum
    image); darts are accepted when they are at least r from every accepted
    point, measured across the periodic wrap.  The cell grid has a multiple of
    3 cells per side so that same-phase cells stay three apart across the wrap.
    Returns xyz [N, 2] in [0, L)^2.
    """
    nc = 3 * int(math.ceil(L / (r / math.sqrt(2.0)) / 3.0))
    cs = L / nc
    seeds = np.asarray(seeds, dtype=np.float64).reshape(-1, 2) % L
    occ = np.full((nc, nc), -1, dtype=np.int64)
    cx = np.minimum((seeds[:, 0] / cs).astype(np.int64), nc - 1)
    cy = np.minimum((seeds[:, 1] / cs).astype(np.int64), nc - 1)
    if np.unique(cy * nc + cx).size != cx.size:
        raise ValueError("two seeds share a cell: seeds must be at least r apart")
    occ[cy, cx] = np.arange(seeds.shape[0])
    allx = seeds[:, 0].copy()
    ally = seeds[:, 1].copy()
    r2 = r * r
    gy, gx = np.meshgrid(np.arange(nc), np.arange(nc), indexing="ij")
    gx = gx.reshape(-1)
    gy = gy.reshape(-1)
    counter = 0
    for rnd in range(rounds):
        for ph in range(9):
            sel = ((gx % 3) == (ph % 3)) & ((gy % 3) == (ph // 3))
            cxs = gx[sel]
            cys = gy[sel]
            empty = occ[cys, cxs] < 0
            cxs = cxs[empty]
            cys = cys[empty]
            if cxs.size == 0:
                continue
            cid = (cys * nc + cxs).astype(np.uint64)
            key = cid * np.uint64(2) + np.uint64(2 * nc * nc) * np.uint64(counter)
            ux = rng.uniform(seed, stream, key)
            uy = rng.uniform(seed, stream, key + np.uint64(1))
            counter += 1
            qx = np.minimum((cxs + ux) * cs, np.nextafter(L, 0.0))
            qy = np.minimum((cys + uy) * cs, np.nextafter(L, 0.0))
            ok = np.ones(qx.size, dtype=bool)
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    j = occ[(cys + dy) % nc, (cxs + dx) % nc]
                    has = j >= 0
                    jj = np.where(has, j, 0)
                    ddx = qx - allx[jj]
                    ddy = qy - ally[jj]
                    ddx -= L * np.round(ddx / L)
                    ddy -= L * np.round(ddy / L)
                    ok &= ~(has & (ddx * ddx + ddy * ddy < r2))
            qx = qx[ok]
            qy = qy[ok]
            if qx.size == 0:
                continue
            start = allx.size
            occ[cys[ok], cxs[ok]] = np.arange(start, start + qx.size)
            allx = np.concatenate([allx, qx])
            ally = np.concatenate([ally, qy])
    return np.stack([allx, ally], axis=1)


def line_seeded_periodic(L=200.0, h=1.0, r_factor=0.794, seed=3, stream=0, rounds=12):
    """Scattered periodic nodes on [0, L)^2 that contain the equispaced line
    y = L/2, x = 0, h, 2h, ... (Section 6): the L/h line nodes come first.

    r = r_factor * h gives about one node per h^2 (the same density relation
    as ``poisson_disk_2d``).  Returns (xyz [N, 2], flags zeros, h, line ids).
    """
    nl = int(round(L / h))
    line = np.stack([np.arange(nl) * h, np.full(nl, 0.5 * L)], axis=1)
    xyz = poisson_disk_periodic(L, r_factor * h, line, seed=seed, stream=stream, rounds=rounds)
    return xyz, np.zeros(xyz.shape[0], np.uint8), h, np.arange(nl)


def ball_nodes(R=1.0, h=0.1, jitter=0.25, seed=13, stream=0):
    """Nodes in the ball |x| <= R with a curved wall.

    Wall nodes: round(4 pi R^2 / h^2) points of the Fibonacci lattice on the
    sphere (flag FACE_XLO); inside, a cubic grid of spacing h centred on the
    origin with every coordinate moved by U(-jitter h, jitter h) (the node's
    counter-based stream), kept where |x| < R - h / 2.  Returns (xyz [N, 3],
    flags [N], h_mean) with h_mean = (4/3 pi R^3 / N)^(1/3).
    """
    ns = int(round(4.0 * math.pi * R * R / (h * h)))
    t = np.arange(ns, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * t / ns
    ph = t * math.pi * (3.0 - math.sqrt(5.0))
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    S = R * np.stack([rxy * np.cos(ph), rxy * np.sin(ph), z], axis=1)
    m = int(math.ceil(R / h))
    ax = np.arange(-m, m + 1, dtype=np.float64) * h
    gz, gy, gx = np.meshgrid(ax, ax, ax, indexing="ij")
    G = np.stack([gx.reshape(-1), gy.reshape(-1), gz.reshape(-1)], axis=1)
    ids = np.arange(G.shape[0], dtype=np.uint64)
    for k in range(3):
        G[:, k] += rng.uniform_range(seed, stream, ids * np.uint64(3) + np.uint64(k), -jitter * h, jitter * h)
    G = G[np.sqrt((G * G).sum(axis=1)) < R - 0.5 * h]
    xyz = np.concatenate([S, G])
    flags = np.zeros(xyz.shape[0], np.uint8)
    flags[:ns] = FACE_XLO
    return xyz, flags, (4.0 / 3.0 * math.pi * R ** 3 / xyz.shape[0]) ** (1.0 / 3.0)


def disk_nodes(R=1.0, h=0.02, centre=(0.0, 0.0), r_factor=0.794, seed=9, stream=0, rounds=12, R_in=0.0):
    """Scattered nodes in the disk |x - centre| <= R with a curved wall, or in
    the annulus R_in <= |x - centre| <= R (a conducting cylinder inside).

    The wall nodes are round(2 pi R / h) equispaced points on the circle (and
    round(2 pi R_in / h) on the inner one, after them; flag FACE_XLO: in 2D
    any wall flag marks a node on which Ez vanishes); darts between the
    circles are accepted at least r = r_factor h from every accepted node.
    Returns (xyz [N, 2], flags [N], h_mean) with h_mean = sqrt(area / N).
    """
    cx, cy = float(centre[0]), float(centre[1])
    nb = int(round(2.0 * math.pi * R / h))
    th = 2.0 * math.pi * np.arange(nb) / nb
    bx = cx + R * np.cos(th)
    by = cy + R * np.sin(th)
    if R_in > 0.0:
        ni = int(round(2.0 * math.pi * R_in / h))
        ti = 2.0 * math.pi * np.arange(ni) / ni
        bx = np.concatenate([bx, cx + R_in * np.cos(ti)])
        by = np.concatenate([by, cy + R_in * np.sin(ti)])
        nb += ni
    r = r_factor * h
    cs = r / math.sqrt(2.0)
    nc = int(math.ceil(2.0 * R / cs)) + 1
    x0, y0 = cx - R, cy - R
    occ = np.full((nc + 4, nc + 4), -1, dtype=np.int64)
    ix = np.minimum(((bx - x0) / cs).astype(np.int64), nc - 1)
    iy = np.minimum(((by - y0) / cs).astype(np.int64), nc - 1)
    occ[iy + 2, ix + 2] = np.arange(nb)
    allx, ally = bx.copy(), by.copy()
    r2 = r * r
    gy, gx = np.meshgrid(np.arange(nc), np.arange(nc), indexing="ij")
    gx = gx.reshape(-1)
    gy = gy.reshape(-1)
    counter = 0
    for rnd in range(rounds):
        for ph in range(9):
            sel = ((gx % 3) == (ph % 3)) & ((gy % 3) == (ph // 3))
            cxs, cys = gx[sel], gy[sel]
            empty = occ[cys + 2, cxs + 2] < 0
            cxs, cys = cxs[empty], cys[empty]
            if cxs.size == 0:
                continue
            cid = (cys * nc + cxs).astype(np.uint64)
            key = cid * np.uint64(2) + np.uint64(2 * nc * nc) * np.uint64(counter)
            ux = rng.uniform(seed, stream, key)
            uy = rng.uniform(seed, stream, key + np.uint64(1))
            counter += 1
            qx = x0 + (cxs + ux) * cs
            qy = y0 + (cys + uy) * cs
            d2 = (qx - cx) ** 2 + (qy - cy) ** 2
            ok = (d2 < R * R) & (d2 > R_in * R_in)
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    j = occ[cys + 2 + dy, cxs + 2 + dx]
                    has = j >= 0
                    jj = np.where(has, j, 0)
                    ddx = qx - allx[jj]
                    ddy = qy - ally[jj]
                    ok &= ~(has & (ddx * ddx + ddy * ddy < r2))
            qx, qy = qx[ok], qy[ok]
            if qx.size == 0:
                continue
            start = allx.size
            occ[cys[ok] + 2, cxs[ok] + 2] = np.arange(start, start + qx.size)
            allx = np.concatenate([allx, qx])
            ally = np.concatenate([ally, qy])
    xyz = np.stack([allx, ally], axis=1)
    flags = np.zeros(xyz.shape[0], np.uint8)
    flags[:nb] = FACE_XLO
    return xyz, flags, math.sqrt(math.pi * (R * R - R_in * R_in) / xyz.shape[0])
