"""Oracle pins for the local RBF weights (Section 4, eq. 9-15; Section 5.1).

Each check is independent of the closed-form right-hand sides the oracle uses:
polynomial reproduction, the cardinal property of the interpolant, minimal
(polynomial-only) stencils with textbook finite-difference weights, numerical
differentiation of the Lagrange functions, and the observed truncation order.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import knn, weights as W
from synth import nodes

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _stencils(shape, k, seed=11, periodic=False):
    xyz, flags, h = nodes.jittered_grid(shape, seed=seed, periodic=periodic)
    return xyz, flags, h, knn.knn(xyz, k)


def _mono_shift(xyz, c, e):
    v = np.ones(xyz.shape[0])
    for k, p in enumerate(e):
        v = v * (xyz[:, k] - c[k]) ** p
    return v


def _dmono_at_centre(e, axis):
    # d/dx_axis of prod (x_k - c_k)^e_k at the centre: nonzero only for e = unit(axis)
    return 1.0 if (e[axis] == 1 and sum(e) == 1) else 0.0


@pytest.mark.parametrize("dim,m,n", [(2, 2, 12), (2, 4, 25), (3, 2, 35)])
def test_fd_polynomial_reproduction(dim, m, n):
    shape = (9, 9) if dim == 2 else (6, 6, 6)
    xyz, _, h, idx = _stencils(shape, n)
    cw = W.curl_weights(xyz, xyz, idx, m)
    for e in W.monomial_exponents(dim, m):
        for c in range(0, xyz.shape[0], 7):
            vals = _mono_shift(xyz[idx[c]], xyz[c], e)
            for ax in range(dim):
                got = (cw[c, ax] * vals).sum()
                scale = np.abs(cw[c, ax] * vals).sum() + 1.0
                assert abs(got - _dmono_at_centre(e, ax)) <= 1e-9 * scale


@pytest.mark.parametrize("dim,alpha", [(2, 1), (2, 2), (2, 3), (3, 2)])
def test_hv_polynomial_reproduction_and_zero_sum(dim, alpha):
    nh = 2 * math.comb(2 * alpha + dim, dim) + 1          # Section 5.1 rule
    shape = (12, 12) if dim == 2 else (7, 7, 7)
    xyz, _, h, idx = _stencils(shape, nh)
    hw = W.hv_weights(xyz, xyz, idx, alpha)
    sel = range(0, xyz.shape[0], 11)
    for c in sel:
        assert abs(hw[c].sum()) <= 1e-9 * np.abs(hw[c]).sum()
    # Delta^alpha of (x - c)^(2 alpha) at the centre is (2 alpha)!; of
    # (x - c)^2 (y - c)^2 (alpha = 2) it is 8; lower degrees give 0.
    tests = [((2 * alpha,) + (0,) * (dim - 1), math.factorial(2 * alpha)), ((1,) + (0,) * (dim - 1), 0.0)]
    if alpha == 2:
        tests.append(((2, 2) + (0,) * (dim - 2), 8.0))
    for e, expect in tests:
        for c in sel:
            vals = _mono_shift(xyz[idx[c]], xyz[c], e)
            got = (hw[c] * vals).sum()
            scale = np.abs(hw[c] * vals).sum() + abs(expect)
            assert abs(got - expect) <= 1e-8 * scale


def test_vfd_cardinal_property_central_difference():
    # Regular grid, virtual points at distance delta = h land on nodes; the
    # interpolant reproduces node values there (psi_i(x_j) = delta_ij, eq. 10),
    # so the weights are exactly -1/(2h), +1/(2h) on x_c -+ h e_x.
    h = 0.1
    g = np.stack(np.meshgrid(np.arange(7) * h, np.arange(7) * h, indexing="xy"), -1).reshape(-1, 2)
    c = 24                                       # (3, 3)
    idx = knn.knn(g, 13, centres=g[c:c + 1])
    for ax, (lo_id, hi_id) in enumerate([(23, 25), (17, 31)]):
        cf, off = W.central_difference(2, ax)
        w = W.vfd_weights(g, g[c:c + 1], idx, 2, cf, off, np.array([h]), 1)[0]
        expect = np.zeros(13)
        expect[list(idx[0]).index(lo_id)] = -1 / (2 * h)
        expect[list(idx[0]).index(hi_id)] = 1 / (2 * h)
        assert np.abs(w - expect).max() <= 1e-9 / h


def test_vfd_cardinal_property_paper_laplacian():
    # The 5-point Laplacian printed in Section 4.2, used as a virtual stencil
    # with delta = h on a regular grid, gives back the printed coefficients / h^2.
    lap = GOLD["laplace_5pt"]
    h = 0.25
    g = np.stack(np.meshgrid(np.arange(7) * h, np.arange(7) * h, indexing="xy"), -1).reshape(-1, 2)
    c = 24
    idx = knn.knn(g, 21, centres=g[c:c + 1])
    w = W.vfd_weights(g, g[c:c + 1], idx, 4, lap["c"], lap["o"], np.array([h]), lap["order"])[0]
    expect = np.zeros(21)
    for coef, o in zip(lap["c"], lap["o"]):
        j = c + o[0] + 7 * o[1]
        expect[list(idx[0]).index(j)] = coef / h ** 2
    assert np.abs(w - expect).max() <= 1e-8 / h ** 2


def test_minimal_stencil_gives_polynomial_fd_weights():
    # n = M_m: P is square and invertible, the RBF part of the solution is
    # zero and the weights are those of the polynomial interpolant.
    h = 0.1
    tri = np.array([[0.0, 0.0], [h, 0.0], [0.0, h]])          # m = 1, M = 3
    cw = W.curl_weights(tri, tri[:1], np.array([[0, 1, 2]]), 1)[0]
    assert np.allclose(cw[0], [-1 / h, 1 / h, 0.0], atol=1e-10 / h)
    assert np.allclose(cw[1], [-1 / h, 0.0, 1 / h], atol=1e-10 / h)
    six = np.array([[0, 0], [h, 0], [-h, 0], [0, h], [0, -h], [h, h]])   # m = 2, M = 6
    cw = W.curl_weights(six, six[:1], np.array([[0, 1, 2, 3, 4, 5]]), 2)[0]
    assert np.allclose(cw[0], [0, 1 / (2 * h), -1 / (2 * h), 0, 0, 0], atol=1e-9 / h)
    assert np.allclose(cw[1], [0, 0, 0, 1 / (2 * h), -1 / (2 * h), 0], atol=1e-9 / h)


def test_fd_weights_are_derivatives_of_lagrange_functions():
    # eq. 13: w_j = d/dx psi_j(x_c).  Differentiate psi_j numerically (it only
    # needs phi itself, not the closed-form derivative of the RHS).
    xyz, _, h, idx = _stencils((9, 9), 12)
    for c in (40, 10, 0):
        cw = W.curl_weights(xyz, xyz[c:c + 1], idx[c:c + 1], 2)[0]
        for ax in range(2):
            e = np.zeros(2)
            e[ax] = 1e-5 * h
            ps = W.cardinal_values(xyz, xyz[c], idx[c], 2, 3, np.stack([xyz[c] + e, xyz[c] - e]))
            num = (ps[0] - ps[1]) / (2e-5 * h)
            assert np.abs(num - cw[ax]).max() <= 1e-6 * np.abs(cw[ax]).max()


def test_hv_weights_are_biharmonic_of_lagrange_functions():
    # Delta^2 psi_j(x_c) by the 13-point biharmonic difference of psi_j.  The
    # r^5 basis function centred on x_c itself is only C^4 there, which adds an
    # O(e) term to the difference; one Richardson step (2 f(e/2) - f(e))
    # removes it.
    xyz, _, h, idx = _stencils((12, 12), 31)
    offs = {(0, 0): 20.0, (1, 0): -8.0, (-1, 0): -8.0, (0, 1): -8.0, (0, -1): -8.0,
            (1, 1): 2.0, (1, -1): 2.0, (-1, 1): 2.0, (-1, -1): 2.0,
            (2, 0): 1.0, (-2, 0): 1.0, (0, 2): 1.0, (0, -2): 1.0}
    coef = np.array(list(offs.values()))[:, None]
    for c in (66, 13):
        hw = W.hv_weights(xyz, xyz[c:c + 1], idx[c:c + 1], 2)[0]
        nums = []
        for e in (0.01 * h, 0.005 * h):
            pts = np.array([xyz[c] + e * np.array(o) for o in offs])
            ps = W.cardinal_values(xyz, xyz[c], idx[c], 4, 5, pts)
            nums.append((coef * ps).sum(0) / e ** 4)
        num = 2 * nums[1] - nums[0]
        assert np.abs(num - hw).max() <= 1e-3 * np.abs(hw).max()


def test_radial_laplacian_constant_numerically():
    # Delta^alpha r^k = C r^(k - 2 alpha): check C by nested 5-point Laplacians
    for d, alpha, k in [(2, 1, 3), (2, 2, 5), (2, 3, 7)]:
        e = 1e-2
        x0 = np.array([0.7, 0.4])

        def f(p):
            return np.linalg.norm(p) ** k

        def lap(fun):
            return lambda p: (fun(p + [e, 0]) + fun(p - [e, 0]) + fun(p + [0, e]) + fun(p - [0, e]) - 4 * fun(p)) / e ** 2

        g = f
        for _ in range(alpha):
            g = lap(g)
        num = g(x0)
        C = W.laplacian_power_const(k, alpha, d)
        assert abs(num - C * np.linalg.norm(x0) ** (k - 2 * alpha)) <= 1e-3 * abs(num)


def _max_interior_err(ns, dim_m, op):
    xyz, flags, h = nodes.jittered_grid((ns, ns), seed=12)
    n, m = dim_m
    idx = knn.knn(xyz, n)
    f = np.sin(2 * xyz[:, 0] + 1) * np.sin(3 * xyz[:, 1] + 0.5)
    interior = (xyz.min(1) > 0.2) & (xyz.max(1) < 0.8)
    if op == "dx":
        w = W.curl_weights(xyz, xyz, idx, m)[:, 0]
        exact = 2 * np.cos(2 * xyz[:, 0] + 1) * np.sin(3 * xyz[:, 1] + 0.5)
    elif op == "vfd":
        w = W.curl_weights(xyz, xyz, idx, m, mode="VFD", h=h)[:, 0]
        exact = 2 * np.cos(2 * xyz[:, 0] + 1) * np.sin(3 * xyz[:, 1] + 0.5)
    else:
        w = W.hv_weights(xyz, xyz, idx, 2)
        exact = (2 ** 2 + 3 ** 2) ** 2 * f
    approx = (w * f[idx]).sum(1)
    return np.abs(approx - exact)[interior].max(), h


@pytest.mark.parametrize("op,nm,slope", [("dx", (12, 2), 1.6), ("vfd", (12, 2), 1.6), ("hv", (31, 4), 0.7)])
def test_truncation_order(op, nm, slope):
    # RBF-FD: O(h^(m+1-l)) (Section 4.2): m = 2, l = 1 -> 2; Delta^2 with m = 4 -> 1.
    # RBF-VFD: min(m + 1 - l, ord) = min(2, 2) = 2.  Maxima over scattered
    # nodes are noisy, so the observed slope is allowed to sit a little low.
    e1, h1 = _max_interior_err(41, nm, op)
    e2, h2 = _max_interior_err(81, nm, op)
    p = math.log(e1 / e2) / math.log(h1 / h2)
    assert p >= slope, p


def _rot(theta):
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s], [s, c]])


@pytest.mark.parametrize("mode", ["FD", "VFD"])
def test_rotated_frame_weights_are_rotation_covariant(mode):
    # Weights depend only on the geometry relative to the differentiation
    # direction: differentiating along u_1 = R(theta) e_x on nodes X equals
    # differentiating along e_x on the nodes R(-theta) X (PHS is radial, the
    # polynomial space is closed under rotation, the virtual points turn with u).
    xyz, _, h, idx = _stencils((9, 9), 13)
    theta = 0.7
    wr = W.curl_weights(xyz, xyz, idx, 2, mode=mode, h=h, frame_angle=theta)
    y = xyz @ _rot(-theta).T
    w0 = W.curl_weights(y, y, idx, 2, mode=mode, h=h)
    assert np.abs(wr - w0).max() <= 1e-9 * np.abs(w0).max()
    # and the frame is a genuine rotation of the unrotated weights for RBF-FD
    # only: the virtual points of RBF-VFD do not turn with the frame otherwise
    wx = W.curl_weights(xyz, xyz, idx, 2, mode=mode, h=h)
    lin = np.stack([math.cos(theta) * wx[:, 0] + math.sin(theta) * wx[:, 1],
                    -math.sin(theta) * wx[:, 0] + math.cos(theta) * wx[:, 1]], axis=1)
    dev = np.abs(wr - lin).max() / np.abs(w0).max()
    assert (dev <= 1e-9) if mode == "FD" else (dev > 1e-6)


@pytest.mark.parametrize("mode,deg", [("FD", 2), ("VFD", 2)])
def test_rotated_frame_directional_reproduction(mode, deg):
    # sum_j w_j p(x_j) = u . grad p (x_c) for every monomial of degree <= deg
    xyz, _, h, idx = _stencils((9, 9), 13)
    theta = -0.45
    wr = W.curl_weights(xyz, xyz, idx, 2, mode=mode, h=h, frame_angle=theta)
    u = np.array([[math.cos(theta), math.sin(theta)], [-math.sin(theta), math.cos(theta)]])
    for e in W.monomial_exponents(2, deg):
        for c in range(0, xyz.shape[0], 5):
            vals = _mono_shift(xyz[idx[c]], xyz[c], e)
            for ax in range(2):
                expect = sum(u[ax, k] * _dmono_at_centre(e, k) for k in range(2))
                got = (wr[c, ax] * vals).sum()
                scale = np.abs(wr[c, ax] * vals).sum() + 1.0
                assert abs(got - expect) <= 1e-9 * scale
