"""Pins of the oracle's large-set tools: the C leapfrog (oracle/cstep.c) and
the cell-bucket stencil search (oracle.knn.knn_cells).

* The C half updates reproduce the one-step closed forms on polynomial fields
  (curl and hyperviscosity parts, eps0 != mu0), the same pins the numpy step
  satisfies, and agree with the numpy step to rounding on scattered nodes
  with PEC walls and per-node eps_r; a TM_11 cavity run converges to the
  analytic mode as the numpy one does.  The same in 3D (full curl, PEC
  factors per component) on a jittered cube.
* knn_cells returns the brute-force stencils bit for bit: uniform, clustered
  and anisotropic sets, regular grids (distance ties everywhere), periodic
  boxes, centres drawn from another set, 2D and 3D.
"""
import math

import numpy as np
import pytest

from oracle import cstep, knn, setup, step, weights as W
from synth import configs, fields, nodes


def _op(xyz, n, m, nh, alpha):
    idx = knn.knn(xyz, max(n, nh))
    ci, hi = idx[:, :n], idx[:, :nh]
    cw = W.curl_weights(xyz, xyz, ci, m)
    hw = W.hv_weights(xyz, xyz, hi, alpha)
    return {"curl_idx": ci, "curl_w": cw, "hv_idx": hi, "hv_w": hw}


def test_c_step_polynomial_closed_forms():
    xyz, flags, h = nodes.jittered_grid((12, 12), seed=21)
    op = _op(xyz, 25, 4, 31, 2)
    cop = cstep.Operator(op)
    eps0, mu0, dt = 2.0, 0.5, 0.003
    a, kappa = dt / mu0, dt / eps0
    x, y = xyz[:, 0], xyz[:, 1]
    keep = step.pec_keep(flags, 2)[:, 0]
    # curl: E = x^2 y -> H = a (-x^2, 2 x y), then E + kappa * 2 a y off the wall
    E = (x * x * y)[:, None]
    H1 = cstep.h_update(E, np.zeros((xyz.shape[0], 2)), cop, a, 0.0)
    assert np.abs(H1[:, 0] - (-a * x * x)).max() < 1e-11
    assert np.abs(H1[:, 1] - (a * 2 * x * y)).max() < 1e-11
    E1 = cstep.e_update(E, H1, cop, kappa, 0.0, keep)
    assert np.abs(E1[:, 0] - np.where(flags == 0, x * x * y + kappa * 2 * a * y, 0.0)).max() < 1e-11
    # hyperviscosity: Delta^2 y^4 = 24, Delta^2 x^2 y^2 = 8, Delta^2 x^4 = 24
    gamma = -0.7
    xs, ys = x - 0.3, y - 0.6
    H = np.stack([ys ** 4, xs * xs * ys * ys], axis=1)
    H1 = cstep.h_update(np.zeros((xyz.shape[0], 1)), H, cop, a, gamma)
    assert np.abs(H1[:, 0] - (H[:, 0] + a * gamma * 24)).max() < 1e-9
    assert np.abs(H1[:, 1] - (H[:, 1] + a * gamma * 8)).max() < 1e-9
    E = (xs ** 4)[:, None]
    H1 = cstep.h_update(E, np.zeros((xyz.shape[0], 2)), cop, a, gamma)
    E1 = cstep.e_update(E, H1, cop, kappa, gamma, keep)
    assert np.abs(E1[:, 0] - np.where(flags == 0, xs ** 4 + kappa * (12 * a * xs * xs + 24 * gamma), 0.0)).max() \
        < 1e-9


def test_c_step_matches_numpy_step_with_eps_r_and_walls():
    w = configs.tm_cavity_2d(n_side=25, chat=1e-3, eps0=2.0, mu0=3.0)
    oh, _ = setup.operators(w)
    rng = np.random.default_rng(4)
    eps_r = 1.0 + rng.random(w.N)
    kappa = w.dt / (w.eps0 * eps_r)
    gamma = step.hv_gamma(w.hv_c, w.alpha, w.h)
    keep = step.pec_keep(w.flags, 2)
    E = rng.standard_normal((w.N, 1)) * keep
    H = rng.standard_normal((w.N, 2))
    cop = cstep.Operator(oh)
    Hn = step.h_update(E, H, oh, w.dt / w.mu0, gamma)
    Hc = cstep.h_update(E, H, cop, w.dt / w.mu0, gamma)
    assert np.abs(Hn - Hc).max() <= 1e-14 * np.abs(Hn).max()
    En = step.e_update(E, Hn, oh, kappa, gamma, keep)
    Ec = cstep.e_update(E, Hn, cop, kappa, gamma, keep[:, 0])
    assert np.abs(En - Ec).max() <= 1e-14 * np.abs(En).max()
    # a 300-step run with energy samples
    En_, Hn_, en, _ = step.run(w.E0, w.H0, oh, oh, w.dt, 300, gamma, w.dt / w.eps0, keep, mu0=w.mu0, eps0=w.eps0,
                               h_e=w.h, h_h=w.h, energy_every=50)
    Ec_, Hc_, ec = cstep.run(w.E0, w.H0, cop, w.dt, 300, gamma, w.dt / w.eps0, keep[:, 0], mu0=w.mu0, eps0=w.eps0,
                             h=w.h, energy_every=50)
    assert step.rel_l2(Ec_, En_) < 1e-13 and step.rel_l2(Hc_, Hn_) < 1e-13
    assert np.abs(ec - en).max() <= 1e-13 * en.max()


def test_c_step_tm11_cavity_converges():
    errs = []
    for ns in (17, 33):
        w = configs.tm_cavity_2d(n_side=ns, chat=1e-3, eps0=2.0, mu0=0.5)
        oh, _ = setup.operators(w)
        gamma = step.hv_gamma(w.hv_c, w.alpha, w.h)
        keep = step.pec_keep(w.flags, 2)[:, 0]
        E, H, _ = cstep.run(w.E0, w.H0, cstep.Operator(oh), w.dt, w.steps, gamma, w.dt / w.eps0, keep, mu0=w.mu0,
                            eps0=w.eps0, h=w.h)
        Ea, Ha, _ = fields.tm_mode_2d(w.xyz, w.steps * w.dt, (w.steps - 0.5) * w.dt, eps0=w.eps0, mu0=w.mu0)
        errs.append(step.linf_errors(E, H, Ea, Ha)[0])
    order = math.log(errs[0] / errs[1]) / math.log(2.0)
    assert errs[1] < errs[0] and order > 0.8, (errs, order)


def test_c_step_3d_polynomial_closed_forms():
    xyz, flags, h = nodes.jittered_grid((8, 8, 8), seed=22)
    N = xyz.shape[0]
    idx = knn.knn(xyz, 71)
    op = {"curl_idx": idx[:, :35], "curl_w": W.curl_weights(xyz, xyz, idx[:, :35], 2), "hv_idx": idx,
          "hv_w": W.hv_weights(xyz, xyz, idx, 2)}
    cop = cstep.Operator(op)
    assert cop.d == 3
    eps0, mu0, dt = 2.0, 0.5, 0.003
    a, kappa = dt / mu0, dt / eps0
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    keep = step.pec_keep(flags, 3)
    zero = np.zeros((N, 3))
    # curl: E = (0, 0, x y) -> curl E = (x, -y, 0), H = -a curl E
    E = np.stack([0 * x, 0 * x, x * y], axis=1)
    H1 = cstep.h_update(E, zero, cop, a, 0.0)
    assert np.abs(H1 - np.stack([-a * x, a * y, 0 * x], axis=1)).max() < 1e-11
    # H = (0, 0, x z) -> curl H = (0, -z, 0); E1 = keep * (E + kappa curl H)
    H = np.stack([0 * x, 0 * x, x * z], axis=1)
    E1 = cstep.e_update(zero, H, cop, kappa, 0.0, keep)
    assert np.abs(E1 - keep * np.stack([0 * x, -kappa * z, 0 * x], axis=1)).max() < 1e-11
    # hyperviscosity: Delta^2 x^4 = 24, Delta^2 y^2 z^2 = 8, Delta^2 x^2 y z = 0
    gamma = -0.7
    xs, ys, zs = x - 0.3, y - 0.6, z - 0.4
    H = np.stack([xs ** 4, ys * ys * zs * zs, xs * xs * ys * zs], axis=1)
    H1 = cstep.h_update(zero, H, cop, a, gamma)
    assert np.abs(H1 - (H + a * gamma * np.array([24.0, 8.0, 0.0]))).max() < 1e-8
    E1 = cstep.e_update(H, zero, cop, kappa, gamma, keep)
    assert np.abs(E1 - keep * (H + kappa * gamma * np.array([24.0, 8.0, 0.0]))).max() < 1e-8


def test_c_step_3d_matches_numpy_step():
    w = configs.tm111_3d(n_side=8, chat=1e-3)
    oh, _ = setup.operators(w)
    rng = np.random.default_rng(5)
    eps_r = 1.0 + rng.random(w.N)
    kappa = w.dt / (w.eps0 * eps_r)
    gamma = step.hv_gamma(w.hv_c, w.alpha, w.h)
    keep = step.pec_keep(w.flags, 3)
    E = rng.standard_normal((w.N, 3)) * keep
    H = rng.standard_normal((w.N, 3))
    cop = cstep.Operator(oh)
    Hn = step.h_update(E, H, oh, w.dt / w.mu0, gamma)
    Hc = cstep.h_update(E, H, cop, w.dt / w.mu0, gamma)
    assert np.abs(Hn - Hc).max() <= 1e-13 * np.abs(Hn).max()
    En = step.e_update(E, Hn, oh, kappa, gamma, keep)
    Ec = cstep.e_update(E, Hn, cop, kappa, gamma, keep)
    assert np.abs(En - Ec).max() <= 1e-13 * np.abs(En).max()
    # a 100-step run of the TM_111 mode with energy samples
    En_, Hn_, en, _ = step.run(w.E0, w.H0, oh, oh, w.dt, 100, gamma, w.dt / w.eps0, keep, mu0=w.mu0, eps0=w.eps0,
                               h_e=w.h, h_h=w.h, energy_every=25)
    Ec_, Hc_, ec = cstep.run(w.E0, w.H0, cop, w.dt, 100, gamma, w.dt / w.eps0, keep, mu0=w.mu0, eps0=w.eps0,
                             h=w.h, energy_every=25)
    assert step.rel_l2(Ec_, En_) < 1e-13 and step.rel_l2(Hc_, Hn_) < 1e-13
    assert np.abs(ec - en).max() <= 1e-13 * en.max()


def _knn_cases():
    rng = np.random.default_rng(1)
    yield "uniform 2D", rng.random((2500, 2)), None, None, 40
    yield "uniform 3D", rng.random((2000, 3)), None, None, 71
    xyz, _, _ = nodes.jittered_grid((40, 40), jitter=0.0)
    yield "regular grid (ties)", xyz, None, None, 57
    xyz, _, _ = nodes.jittered_grid((30, 30), jitter=0.0, periodic=True)
    yield "regular periodic (ties)", xyz, None, (1.0, 1.0), 31
    xyz, _, _ = nodes.jittered_grid((25, 20), lo=(0, 0), hi=(2.0, 1.0), periodic=True)
    yield "anisotropic periodic", xyz, None, (2.0, 1.0), 25
    xyz, _, _ = nodes.jittered_grid((9, 9, 9), jitter=0.0)
    yield "regular cube (ties)", xyz, None, None, 35
    cl = np.concatenate([rng.normal(0.5, 0.02, (1500, 2)), rng.random((500, 2))])
    yield "clustered", cl, None, None, 60
    xe, _, _ = nodes.jittered_grid((31, 31), seed=3)
    xh, _, _ = nodes.dual_grid_2d(30, seed=3)
    yield "centres from another set", xe, xh, None, 12
    yield "tiny set, k = N", rng.random((20, 2)), None, None, 20


@pytest.mark.parametrize("case", list(_knn_cases()), ids=lambda c: c[0])
def test_knn_cells_equals_brute_force(case):
    _, src, cen, per, k = case
    a = knn.knn(src, k, centres=cen, period=per)
    b = knn.knn_cells(src, k, centres=cen, period=per)
    assert (a == b).all()
