"""Seeded input generators: determinism, bounds, boundary placement."""
import numpy as np

from synth import nodes, rng, fields, configs


def test_rng_is_counter_based_and_deterministic():
    a = rng.u64(7, 1, np.arange(10))
    b = rng.u64(7, 1, np.arange(10))
    assert (a == b).all()
    # each draw depends only on its own counter
    assert rng.u64(7, 1, np.array([5]))[0] == a[5]
    assert (rng.u64(8, 1, np.arange(10)) != a).all()
    assert (rng.u64(7, 2, np.arange(10)) != a).all()
    u = rng.uniform(3, 0, np.arange(100000))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01


def test_splitmix64_finaliser_published_value():
    # SplitMix64 seeded with 0: the first output is 0xE220A8397B1DCDAF
    # (state 0x9E3779B97F4A7C15 through the finaliser).
    from synth.rng import _mix, _GOLDEN
    assert int(_mix(np.uint64(0) + _GOLDEN)) == 0xE220A8397B1DCDAF


def test_jittered_grid_2d_bounds_and_flags():
    xyz, flags, h = nodes.jittered_grid((11, 9), seed=3)
    assert xyz.shape == (99, 2)
    assert abs(h - 0.1) < 1e-15
    ix = np.arange(99) % 11
    iy = np.arange(99) // 11
    assert np.all(np.abs(xyz[:, 0] - ix * 0.1) <= 0.25 * 0.1 + 1e-15)
    assert np.all(np.abs(xyz[:, 1] - iy * (1 / 8)) <= 0.25 / 8 + 1e-15)
    on_b = (ix == 0) | (ix == 10) | (iy == 0) | (iy == 8)
    assert ((flags != 0) == on_b).all()
    # boundary nodes stay on their face, corners fixed
    assert np.all(xyz[ix == 0, 0] == 0.0) and np.all(xyz[ix == 10, 0] == 1.0)
    assert np.all(xyz[iy == 0, 1] == 0.0) and np.all(xyz[iy == 8, 1] == 1.0)
    c = (ix == 0) & (iy == 0)
    assert np.all(xyz[c] == 0.0)
    x2, f2, _ = nodes.jittered_grid((11, 9), seed=3)
    assert (x2 == xyz).all() and (f2 == flags).all()


def test_jittered_grid_3d_and_periodic():
    xyz, flags, h = nodes.jittered_grid((5, 5, 5), seed=1)
    assert xyz.shape == (125, 3)
    assert (flags[62] == 0)           # centre node interior
    assert flags[0] == (1 | 4 | 16)
    xp, fp, hp = nodes.jittered_grid((10, 10), lo=(0, 0), hi=(10, 10), periodic=True, seed=2)
    assert hp == 1.0 and (fp == 0).all()
    assert xp.min() >= 0.0 and xp.max() < 10.0


def test_poisson_disk_min_distance_and_boundary():
    xyz, flags, h = nodes.poisson_disk_2d(0.03, seed=4, rounds=8)
    from scipy.spatial import cKDTree
    d, _ = cKDTree(xyz).query(xyz, 2)
    assert d[:, 1].min() >= 0.03 * (1 - 1e-12)
    b = flags != 0
    onb = (xyz[:, 0] == 0) | (xyz[:, 0] == 1) | (xyz[:, 1] == 0) | (xyz[:, 1] == 1)
    assert (b == onb).all()
    assert abs(h - 1 / np.sqrt(xyz.shape[0])) < 1e-15
    # near-maximal: no empty disk of radius 2r inside the square
    g = np.stack(np.meshgrid(np.linspace(0.1, 0.9, 30), np.linspace(0.1, 0.9, 30)), -1).reshape(-1, 2)
    dd, _ = cKDTree(xyz).query(g, 1)
    assert dd.max() < 2 * 0.03


def test_tm_mode_fields_vanish_on_walls():
    xyz, flags, h = nodes.jittered_grid((9, 9), seed=1)
    E, H, w = fields.tm_mode_2d(xyz, 0.3, 0.25)
    assert np.abs(E[flags != 0]).max() < 1e-15
    E3 = fields.tm111_cube(nodes.jittered_grid((5, 5, 5))[0], 0.0, 0.0)[0]
    assert E3.shape == (125, 3)


def test_workload_parameters():
    w = configs.tm_cavity_2d()
    assert w.N == 2601 and w.steps == 1000 and w.n == 12 and w.n_hv == 31
    assert abs(w.steps * w.dt - np.sqrt(2)) < 1e-12
    w3 = configs.tm111_3d(n_side=6)
    assert w3.n_hv == 71 and w3.n == 35


def test_line_seeded_periodic_nodes():
    # Section 6 node set: the equispaced line y = L/2 comes first and unchanged,
    # every pair of nodes is at least r apart across the periodic wrap, about
    # one node per h^2, reproducible bit for bit
    from synth import nodes as _n
    L, h = 40.0, 1.0
    xyz, flags, hh, line = _n.line_seeded_periodic(L, h, seed=7)
    assert hh == h and (flags == 0).all()
    assert np.array_equal(line, np.arange(40))
    assert np.array_equal(xyz[:40, 0], np.arange(40.0)) and (xyz[:40, 1] == 20.0).all()
    assert (xyz >= 0).all() and (xyz < L).all()
    d = xyz[:, None, :] - xyz[None, :, :]
    d -= L * np.round(d / L)
    r2 = (d ** 2).sum(-1)
    np.fill_diagonal(r2, np.inf)
    assert r2.min() >= (0.794 * h) ** 2 * (1 - 1e-12)
    assert 0.9 < xyz.shape[0] / (L * L) < 1.1
    xyz2, _, _, _ = _n.line_seeded_periodic(L, h, seed=7)
    assert np.array_equal(xyz, xyz2)


def test_curved_wall_node_sets():
    import math
    from synth import nodes
    # annulus: wall nodes exactly on both circles, the rest strictly between
    x, f, hm = nodes.disk_nodes(1.0, 0.05, R_in=0.5)
    r = np.hypot(x[:, 0], x[:, 1])
    wall = f != 0
    assert np.allclose(np.sort(r[wall])[[0, -1]], [0.5, 1.0])
    assert (np.isclose(r[wall], 0.5) | np.isclose(r[wall], 1.0)).all()
    assert ((r[~wall] > 0.5) & (r[~wall] < 1.0)).all()
    # the disk generator without an inner circle is unchanged by the option
    a, fa, _ = nodes.disk_nodes(1.0, 0.05)
    b, fb, _ = nodes.disk_nodes(1.0, 0.05, R_in=0.0)
    assert np.array_equal(a, b) and np.array_equal(fa, fb)
    # ball: Fibonacci wall nodes on the sphere, interior at least h/2 inside
    x3, f3, h3 = nodes.ball_nodes(1.0, 0.2)
    r3 = np.sqrt((x3 ** 2).sum(1))
    assert np.allclose(r3[f3 != 0], 1.0)
    assert (r3[f3 == 0] < 1.0 - 0.1 + 1e-12).all()
    assert (f3 != 0).sum() == round(4 * math.pi / 0.04)


def test_cavity_modes_satisfy_their_wall_conditions():
    from synth import fields
    th = np.linspace(0, 2 * np.pi, 37)[:-1]
    for R in (1.0, 0.5):
        pts = np.stack([R * np.cos(th), R * np.sin(th)], 1)
        # coaxial TM_01: Ez vanishes on both circles; TE_01: E is azimuthal and vanishes there
        E, H, _ = fields.coax_mode(pts, 0.3, 0.25, pol="TM")
        assert np.abs(E).max() < 1e-12
        E, Hz, _ = fields.coax_mode(pts, 0.3, 0.25, pol="TE")
        assert np.abs(E).max() < 1e-12
    ring = np.stack([np.cos(th), np.sin(th)], 1)
    E, Hz, _ = fields.te01_disk(ring, 0.3, 0.25)
    assert np.abs(E).max() < 1e-12
    # PEC sphere mode: E = 0 on the sphere, and E is tangential everywhere
    rs = np.random.default_rng(0)
    u = rs.standard_normal((50, 3))
    u /= np.sqrt((u ** 2).sum(1))[:, None]
    E, H, _ = fields.sphere_mode(u, 0.2, 0.15)
    assert np.abs(E).max() < 1e-12
    inner = 0.6 * u
    E, H, _ = fields.sphere_mode(inner, 0.2, 0.15)
    assert np.abs((E * inner).sum(1)).max() < 1e-12 and np.abs(E).max() > 1e-3
