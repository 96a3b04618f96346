"""Oracle pins for the stabilised leapfrog (eq. 19), energy (eq. 20), errors (eq. 23).

* One step on polynomial fields: the weights reproduce polynomials, so one
  step has a closed form (curl part and hyperviscosity part separately, 2D and
  3D, with eps0 != mu0 so that misplaced constants show).
* Cavity modes (TM_11, TM_111, TE_11, and TM_01 of a circular cavity with a
  curved wall) and the paper's periodic pulse (eq. 21-23): errors against the
  analytic solutions fall as h falls.
* The TEz polarisation is the Maxwell dual of TMz with the update order
  swapped: checked exactly against the TMz functions.
* Energy (eq. 20) stays bounded with hyperviscosity and blows up without it
  on scattered nodes (Section 5, Appendix A).
* On a regular periodic grid one step maps a plane wave exactly as the
  amplification matrix of eq. A.6 says, and that matrix has lambda2 * lambda3 = 1
  (eq. A.9).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import knn, weights as W, step, setup
from synth import nodes, fields, configs, rng

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _op(xyz, n, m, nh, alpha, period=None, mode="FD", h=None):
    idx = knn.knn(xyz, max(n, nh), period=period)
    ci, hi = idx[:, :n], idx[:, :nh]
    cw = W.curl_weights(xyz, xyz, ci, m, mode=mode, h=h, period=period)
    hw = W.hv_weights(xyz, xyz, hi, alpha, period=period) if alpha else np.zeros(hi.shape)
    return {"curl_idx": ci, "curl_w": cw, "hv_idx": hi, "hv_w": hw}


def test_courant_number_matches_paper():
    assert abs(configs.SC - eval(GOLD["courant_meshless"]["value_expr"], {"sqrt": math.sqrt})) < 1e-16


def test_one_step_polynomial_curl_2d():
    xyz, flags, h = nodes.jittered_grid((12, 12), seed=21)
    op = _op(xyz, 25, 4, 31, 2)
    eps0, mu0, dt = 2.0, 0.5, 0.003
    a, kappa = dt / mu0, dt / eps0
    x, y = xyz[:, 0], xyz[:, 1]
    E = (x * x * y)[:, None]
    H = np.zeros((xyz.shape[0], 2))
    keep = step.pec_keep(flags, 2)
    H1 = step.h_update(E, H, op, a, 0.0)
    assert np.abs(H1[:, 0] - (-a * x * x)).max() < 1e-11
    assert np.abs(H1[:, 1] - (a * 2 * x * y)).max() < 1e-11
    E1 = step.e_update(E, H1, op, kappa, 0.0, keep)
    expect = np.where(flags == 0, x * x * y + kappa * 2 * a * y, 0.0)
    assert np.abs(E1[:, 0] - expect).max() < 1e-11


def test_one_step_polynomial_hyperviscosity_2d():
    xyz, flags, h = nodes.jittered_grid((12, 12), seed=22)
    op = _op(xyz, 25, 4, 31, 2)
    eps0, mu0, dt, gamma = 2.0, 0.5, 0.003, -0.7
    a, kappa = dt / mu0, dt / eps0
    x, y = xyz[:, 0] - 0.3, xyz[:, 1] - 0.6
    E = np.zeros((xyz.shape[0], 1))
    H = np.stack([y ** 4, x * x * y * y], axis=1)
    H1 = step.h_update(E, H, op, a, gamma)
    # Delta^2 y^4 = 24, Delta^2 x^2 y^2 = 8
    assert np.abs(H1[:, 0] - (H[:, 0] + a * gamma * 24)).max() < 1e-9
    assert np.abs(H1[:, 1] - (H[:, 1] + a * gamma * 8)).max() < 1e-9
    E = (x ** 4)[:, None]
    H = np.zeros((xyz.shape[0], 2))
    H1 = step.h_update(E, H, op, a, gamma)
    assert np.abs(H1[:, 1] - 4 * a * x ** 3).max() < 1e-10
    E1 = step.e_update(E, H1, op, kappa, gamma, step.pec_keep(flags, 2))
    expect = np.where(flags == 0, x ** 4 + kappa * (12 * a * x * x + 24 * gamma), 0.0)
    assert np.abs(E1[:, 0] - expect).max() < 1e-9


def test_one_step_polynomial_curl_3d_and_pec_faces():
    xyz, flags, h = nodes.jittered_grid((6, 6, 6), seed=23)
    op = _op(xyz, 35, 2, 35, 0)
    eps0, mu0, dt = 2.0, 0.5, 0.01
    a, kappa = dt / mu0, dt / eps0
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    E = np.stack([y * y, z * z, x * x], axis=1)
    H = np.zeros_like(E)
    H1 = step.h_update(E, H, op, a, 0.0)
    # curl (y^2, z^2, x^2) = (-2z, -2x, -2y)
    assert np.abs(H1 - a * np.stack([2 * z, 2 * x, 2 * y], 1)).max() < 1e-11
    keep = step.pec_keep(flags, 3)
    E1 = step.e_update(E, H1, op, kappa, 0.0, keep)
    # curl (2az, 2ax, 2ay) = (2a, 2a, 2a)
    assert np.abs(E1 - (E + 2 * a * kappa) * keep).max() < 1e-11
    # a node on the x-low face keeps only Ex; an edge node keeps nothing
    f0 = np.nonzero(flags == 1)[0][0]
    assert keep[f0].tolist() == [1.0, 0.0, 0.0]
    e0 = np.nonzero(flags == (1 | 4))[0][0]
    assert keep[e0].tolist() == [0.0, 0.0, 0.0]


def _cavity_err(ns, eps0=2.0, mu0=0.5):
    w = configs.tm_cavity_2d(n_side=ns, chat=1e-3, eps0=eps0, mu0=mu0)
    oh, oe = setup.operators(w)
    E, H, _, _ = setup.run_workload(w, oh, oe)
    Ea, Ha, _ = fields.tm_mode_2d(w.xyz, w.steps * w.dt, (w.steps - 0.5) * w.dt, eps0=eps0, mu0=mu0)
    return step.linf_errors(E, H, Ea, Ha), w.h


def test_tm11_cavity_converges():
    (e1, m1), h1 = _cavity_err(26)
    (e2, m2), h2 = _cavity_err(51)
    assert e2 < 5e-4 and m2 < 1e-3          # |H| ~ 1.4 here (mu0 = 0.5)
    assert math.log(e1 / e2) / math.log(h1 / h2) >= 0.8
    assert math.log(m1 / m2) / math.log(h1 / h2) >= 0.8


def test_tm111_cube_converges():
    errs = []
    for ns in (7, 11):
        w = configs.tm111_3d(n_side=ns, chat=1e-3, steps=0)
        w.steps = int(round(0.3 / w.dt))
        oh, oe = setup.operators(w)
        E, H, _, _ = setup.run_workload(w, oh, oe)
        Ea, Ha, _ = fields.tm111_cube(w.xyz, w.steps * w.dt, (w.steps - 0.5) * w.dt)
        errs.append((max(step.linf_errors(E, H, Ea, Ha)), w.h))
    (e1, h1), (e2, h2) = errs
    assert e2 < e1
    assert math.log(e1 / e2) / math.log(h1 / h2) >= 0.8


@pytest.mark.parametrize("mode", ["FD", "VFD"])
def test_periodic_pulse_paper_setup(mode):
    # eq. 21 on [0, 200] x [0, 20] periodic, sigma = 30, errors (eq. 23) at
    # c0 t = 5 sqrt 2 (Figure 7 caption), alpha = 2 and c = 1e-4 (Section 5.1).
    g = GOLD["pulse_test"]
    res = []
    for h in (2.0, 1.0):
        w = configs.periodic_pulse(h=h, Ly=20.0, sigma=g["sigma"], L=g["L"], chat=GOLD["hv_c"]["value"],
                                   mode=mode)
        oh, oe = setup.operators(w)
        E, H, en, _ = setup.run_workload(w, oh, oe, energy_every=5)
        Ea, Ha = fields.periodic_plane_pulse(w.xyz, w.steps * w.dt, (w.steps - 0.5) * w.dt,
                                             L=g["L"], sigma=g["sigma"])
        res.append((step.linf_errors(E, H, Ea, Ha), w.h, en / en[0]))
    (eE1, eH1), h1, _ = res[0]
    (eE2, eH2), h2, u = res[1]
    assert math.log(eE1 / eE2) / math.log(h1 / h2) >= 0.8
    assert math.log(eH1 / eH2) / math.log(h1 / h2) >= 0.8
    # energy: bounded, not increasing, not over-dissipated
    assert u.max() <= 1 + 1e-3 and u[-1] <= 1 + 1e-9 and u[-1] >= 0.9


def _periodic_noise_run(chat, steps):
    xyz, flags, h = nodes.jittered_grid((21, 21), periodic=True, seed=3)
    P = (1.0, 1.0)
    op = _op(xyz, 12, 2, 31, 2, period=P)
    dt = configs.SC * h
    N = xyz.shape[0]
    E = (np.sin(2 * math.pi * xyz[:, 0]) + 1e-6 * rng.uniform(1, 9, np.arange(N)))[:, None]
    g = step.hv_gamma(chat / dt, 2, h)
    _, _, en, _ = step.run(E, np.zeros((N, 2)), op, op, dt, steps, g, dt, np.ones((N, 1)),
                           h_e=h, h_h=h, energy_every=100)
    return en / en[0]


def test_no_hyperviscosity_is_unstable_on_scattered_nodes():
    # Section 5: without stabilisation the scheme blows up; with HV it does not.
    u0 = _periodic_noise_run(0.0, 2500)
    u1 = _periodic_noise_run(1e-3, 2500)
    assert u0[-1] > 100.0
    band = GOLD["narrow_pulse"]["u_band"]            # the paper's stability band
    assert 0.9 < u1.min() and u1.max() < band[1]


def test_plane_wave_amplification_matches_eq_A6():
    # Regular periodic grid: every node has the same stencil, so the plane wave
    # e^{ik(x+y)} is an eigenfunction of D^dx, D^dy and one step of eq. 16
    # multiplies its amplitudes by the matrix of eq. A.6.
    ns = 16
    g = np.stack(np.meshgrid(np.arange(ns) / ns, np.arange(ns) / ns, indexing="xy"), -1).reshape(-1, 2)
    P = (1.0, 1.0)
    op = _op(g, 13, 2, 13, 0, period=P)       # 13 = complete distance shells
    k = 2 * math.pi * 3
    ph = np.exp(1j * k * (g[:, 0] + g[:, 1]))
    c1, c2 = 0.02, 0.03
    i0 = 0
    d = g[op["curl_idx"][i0]] - g[i0]
    d = knn.min_image(d, P)
    wx = (op["curl_w"][i0, 0] * np.exp(1j * k * (d[:, 0] + d[:, 1]))).sum()
    wy = (op["curl_w"][i0, 1] * np.exp(1j * k * (d[:, 0] + d[:, 1]))).sum()
    G = np.array([[1, 0, -c1 * wy], [0, 1, c1 * wx],
                  [-c2 * wy, c2 * wx, 1 + c1 * c2 * (wx * wx + wy * wy)]])
    amp = np.array([0.3, -0.2, 1.0])
    E = (amp[2] * ph)[:, None]
    H = np.stack([amp[0] * ph, amp[1] * ph], 1)
    H1 = step.h_update(E, H, op, c1, 0.0)
    E1 = step.e_update(E, H1, op, c2, 0.0, np.ones((g.shape[0], 1)))
    new = G @ amp
    assert np.abs(H1[:, 0] - new[0] * ph).max() < 1e-12
    assert np.abs(H1[:, 1] - new[1] * ph).max() < 1e-12
    assert np.abs(E1[:, 0] - new[2] * ph).max() < 1e-12


def test_amplification_eigenvalue_product_eq_A9():
    xyz, _, h = nodes.jittered_grid((15, 15), periodic=True, seed=5)
    P = (1.0, 1.0)
    op = _op(xyz, 12, 2, 12, 0, period=P)
    c1 = c2 = configs.SC * h
    k = 2 * math.pi * 2
    grew = 0
    for i in range(0, xyz.shape[0], 9):
        d = knn.min_image(xyz[op["curl_idx"][i]] - xyz[i], P)
        e = np.exp(1j * k * (d[:, 0] + d[:, 1]))
        wx = (op["curl_w"][i, 0] * e).sum()
        wy = (op["curl_w"][i, 1] * e).sum()
        G = np.array([[1, 0, -c1 * wy], [0, 1, c1 * wx],
                      [-c2 * wy, c2 * wx, 1 + c1 * c2 * (wx * wx + wy * wy)]])
        lam = np.linalg.eigvals(G)
        j1 = np.argmin(np.abs(lam - 1))
        rest = np.delete(lam, j1)
        assert abs(rest[0] * rest[1] - GOLD["amplification_product"]["value"]) < 1e-12
        grew += np.abs(rest).max() > 1 + 1e-12
    assert grew > 0          # some scattered stencil amplifies (Appendix A)


def test_tm01_circular_cavity_converges():
    # a curved PEC wall: the TM_01 mode of a circular cavity (Ez = J0(j01 r / R)
    # cos(omega t), closed form) after one period; Ez = 0 on the wall nodes
    res = []
    for h in (0.05, 0.025):
        w = configs.tm01_disk(h=h)
        oh, oe = setup.operators(w)
        E, H, _, _ = setup.run_workload(w, oh, oe)
        Ea, Ha, _ = fields.tm01_disk(w.xyz, w.steps * w.dt, (w.steps - 0.5) * w.dt)
        assert np.abs(E[w.flags > 0]).max() == 0.0
        res.append(step.linf_errors(E, H, Ea, Ha) + (w.meta["h_mean"],))
    (eE1, eH1, h1), (eE2, eH2, h2) = res
    assert eE1 < 1e-3 and eH1 < 2e-3
    assert math.log(eE1 / eE2) / math.log(h1 / h2) >= 1.5
    assert math.log(eH1 / eH2) / math.log(h1 / h2) >= 1.5


def test_te_polarisation_is_the_dual_of_tm_with_the_update_order_swapped():
    # Maxwell duality on a periodic set: with Hx = Ex, Hy = Ey, Ez = -Hz the
    # TEz step (Hz from E, then E from the new Hz) is the TMz E update (with
    # kappa = dt/mu0) followed by the TMz H update (with a = dt/eps0); eps0 !=
    # mu0 so that exchanged constants show
    xyz, flags, h = nodes.jittered_grid((17, 17), periodic=True, seed=13)
    P = (1.0, 1.0)
    op = _op(xyz, 12, 2, 31, 2, period=P)
    N = xyz.shape[0]
    eps0, mu0, dt = 2.0, 0.5, 0.004
    g = step.hv_gamma(1e-3 / dt, 2, h)
    E = np.stack([np.sin(2 * math.pi * xyz[:, 1]), np.cos(2 * math.pi * (xyz[:, 0] + xyz[:, 1]))], 1)
    Hz = (np.cos(2 * math.pi * xyz[:, 0]) * np.sin(4 * math.pi * xyz[:, 1]))[:, None]
    Ete, Hte = E.copy(), Hz.copy()
    Htm, Etm = E.copy(), -Hz.copy()
    keep = np.ones((N, 2))
    for _ in range(40):
        Hte = step.te_h_update(Ete, Hte, op, dt / mu0, g)
        Ete = step.te_e_update(Ete, Hte, op, dt / eps0, g, keep)
        Etm = step.e_update(Etm, Htm, op, dt / mu0, g, np.ones((N, 1)))
        Htm = step.h_update(Etm, Htm, op, dt / eps0, g)
    assert np.abs(Ete - Htm).max() < 1e-13 * np.abs(Htm).max()
    assert np.abs(Hte + Etm).max() < 1e-13 * np.abs(Etm).max()


def _te_cavity_err(ns):
    w = configs.te_cavity_2d(n_side=ns, chat=1e-3, eps0=2.0, mu0=0.5)
    oh, oe = setup.operators(w)
    E, Hz, _, _ = setup.run_workload(w, oh, oe)
    Ea, Ha, _ = fields.te_mode_2d(w.xyz, w.steps * w.dt, (w.steps - 0.5) * w.dt, eps0=2.0, mu0=0.5)
    keep = step.pec_keep_te(w.flags)
    assert (E[keep == 0] == 0).all()          # tangential E vanishes on the walls
    return step.linf_errors(E, Hz, Ea, Ha), w.h


def test_te11_cavity_converges():
    (e1, m1), h1 = _te_cavity_err(26)
    (e2, m2), h2 = _te_cavity_err(51)
    assert e2 < 3e-4 and m2 < 3e-4
    assert math.log(e1 / e2) / math.log(h1 / h2) >= 1.5
    assert math.log(m1 / m2) / math.log(h1 / h2) >= 1.5


def test_te01_circular_cavity_converges():
    # a curved PEC wall in the TEz polarisation: only the normal component of
    # (Ex, Ey) survives on the wall nodes.  The TE_01 mode (Hz = J0(j11 r / R)
    # cos(omega t), E azimuthal, closed form) after 1 1/8 periods (E is not
    # near a zero of sin(omega t) there)
    res = []
    for h in (0.05, 0.025):
        w = configs.te01_disk(h=h, periods=1.125)
        oh, oe = setup.operators(w)
        E, Hz, _, _ = setup.run_workload(w, oh, oe)
        Ea, Ha, _ = fields.te01_disk(w.xyz, w.steps * w.dt, (w.steps - 0.5) * w.dt)
        wall = w.flags > 0
        # tangential E vanishes on the wall (to rounding)
        tang = -E[wall, 0] * w.normals[wall, 1] + E[wall, 1] * w.normals[wall, 0]
        assert np.abs(tang).max() < 1e-15
        res.append(step.linf_errors(E, Hz, Ea, Ha) + (w.meta["h_mean"],))
    (eE1, eH1, h1), (eE2, eH2, h2) = res
    assert eE1 < 3e-3 and eH1 < 3e-3
    assert math.log(eE1 / eE2) / math.log(h1 / h2) >= 1.5
    assert math.log(eH1 / eH2) / math.log(h1 / h2) >= 1.5


def test_wall_projection_on_axis_normals_is_the_axis_rule():
    # a unit normal along an axis keeps exactly the component the axis rule keeps
    rs = np.random.default_rng(3)
    E = rs.standard_normal((6, 2))
    flags = np.array([1, 2, 4, 8, 0, 0], dtype=np.uint8)
    nrm = np.array([[-1.0, 0], [1.0, 0], [0, -1.0], [0, 1.0], [0, 0], [0, 0]])
    keep = step.pec_keep_te(flags)
    assert np.array_equal(step.wall_project(E, keep, nrm), step.wall_project(E, keep))
    # a diagonal normal keeps the normal part only
    n = np.array([[0.6, 0.8]])
    out = step.wall_project(E[:1], np.ones((1, 2)), n)
    assert abs(out[0, 0] * 0.8 - out[0, 1] * 0.6) < 1e-15
    assert abs((out[0] * n[0]).sum() - (E[0] * n[0]).sum()) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_leapfrog_is_time_reversible_without_hyperviscosity(dim):
    # Time reversal of the interleaved leapfrog (eq. 19 with gamma = 0): if
    # (E^n, H^n) solve the scheme, so do E~^m = E^{T-m}, H~^m = -H^{T+1-m}.
    # Running T steps from (E^T, -H^{T+1}) must give back (E^0, -H^1); an E
    # update reading the old H, or a curl with a wrong sign in one half,
    # breaks the identity.  PEC masks are projections that commute with it.
    if dim == 2:
        xyz, flags, h = nodes.jittered_grid((15, 15), seed=21)
        op = _op(xyz, 12, 2, 31, 2)
        E0 = (np.sin(math.pi * xyz[:, 0]) * np.sin(2 * math.pi * xyz[:, 1]))[:, None]
        H0 = np.stack([np.cos(3 * xyz[:, 1]), np.sin(2 * xyz[:, 0] + xyz[:, 1])], 1)
    else:
        xyz, flags, h = nodes.jittered_grid((7, 7, 7), seed=22)
        op = _op(xyz, 35, 2, 71, 2)
        E0 = np.stack([np.sin(math.pi * xyz[:, 1]), np.cos(xyz[:, 2]), xyz[:, 0] * xyz[:, 1]], 1)
        H0 = np.stack([np.cos(2 * xyz[:, 2]), xyz[:, 0] ** 2, np.sin(xyz[:, 1] - xyz[:, 0])], 1)
    keep = step.pec_keep(flags, dim)
    E0 = E0 * keep
    dt = configs.SC * h
    T = 60
    E, H, _, _ = step.run(E0, H0, op, op, dt, T, 0.0, dt, keep)
    H_next = step.h_update(E, H, op, dt, 0.0)                       # H^{T+1}
    H1 = step.h_update(E0, H0, op, dt, 0.0)                         # H^1
    Eb, Hb, _, _ = step.run(E, -H_next, op, op, dt, T, 0.0, dt, keep)
    assert np.abs(Eb - E0).max() <= 1e-11 * np.abs(E0).max()
    assert np.abs(Hb + H1).max() <= 1e-11 * np.abs(H1).max()


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_coaxial_cavity_converges(pol):
    # an irregular PEC body: the annulus 0.5 <= r <= 1 between two conducting
    # cylinders, first circularly symmetric mode (TM_01: Ez = J0 Y0 - J0 Y0
    # cross product vanishing on both circles; TE_01: E azimuthal, vanishing
    # on both walls) after 1 1/8 periods, against its closed form
    res = []
    for h in (0.05, 0.025):
        w = configs.coax_2d(pol=pol, h=h, periods=1.125)
        oh, oe = setup.operators(w)
        E, H, _, _ = setup.run_workload(w, oh, oe)
        Ea, Ha, _ = fields.coax_mode(w.xyz, w.steps * w.dt, (w.steps - 0.5) * w.dt, pol=pol)
        wall = w.flags > 0
        if pol == "TM":
            assert np.abs(E[wall]).max() == 0.0
        else:
            tang = -E[wall, 0] * w.normals[wall, 1] + E[wall, 1] * w.normals[wall, 0]
            assert np.abs(tang).max() < 1e-15
        res.append(step.linf_errors(E, H, Ea, Ha) + (w.meta["h_mean"],))
    (eE1, eH1, h1), (eE2, eH2, h2) = res
    assert eE1 < 4e-3 and eH1 < 4e-3
    assert math.log(eE1 / eE2) / math.log(h1 / h2) >= 1.5
    assert math.log(eH1 / eH2) / math.log(h1 / h2) >= 1.5


def test_sphere_cavity_converges():
    # a curved 3D wall: the PEC sphere with its lowest azimuthal mode
    # (E = j1(kr)/r (-y, x, 0) cos(omega t), closed form), wall nodes keep the
    # normal component of E; 1 1/8 periods
    res = []
    for h in (0.2, 0.1):
        w = configs.sphere_3d(h=h, periods=1.125)
        oh, oe = setup.operators(w)
        E, H, _, _ = setup.run_workload(w, oh, oe)
        Ea, Ha, _ = fields.sphere_mode(w.xyz, w.steps * w.dt, (w.steps - 0.5) * w.dt)
        wall = w.flags > 0
        n = w.normals[wall]
        tang = E[wall] - (E[wall] * n).sum(axis=1)[:, None] * n
        assert np.abs(tang).max() < 1e-15
        res.append(step.linf_errors(E, H, Ea, Ha) + (w.meta["h_mean"],))
    (eE1, eH1, h1), (eE2, eH2, h2) = res
    assert eE2 < 2e-2 and eH2 < 3e-2
    assert math.log(eE1 / eE2) / math.log(h1 / h2) >= 1.5
    assert math.log(eH1 / eH2) / math.log(h1 / h2) >= 1.5
