"""Oracle pins for the discrete adjoint of the 2D update.

The forward map is linear in the source amplitudes, so the amplitude gradient
must equal the receiver traces of a unit source dotted with dJ/dtraces (a
dot-product test); the permittivity gradient must match central finite
differences of J along seeded directions.
"""
import math

import numpy as np

from oracle import knn, weights as W, step
from synth import nodes, fields, rng


def _problem(ns=13, steps=60):
    xyz, flags, h = nodes.jittered_grid((ns, ns), seed=31)
    idx = knn.knn(xyz, 31)
    op = {"curl_idx": idx[:, :12], "curl_w": W.curl_weights(xyz, xyz, idx[:, :12], 2),
          "hv_idx": idx, "hv_w": W.hv_weights(xyz, xyz, idx, 2)}
    dt = h / (10 * math.sqrt(2))
    gamma = step.hv_gamma(1e-3 / dt, 2, h)
    eps_r = fields.eps_r_smooth(xyz, seed=7)
    keep = step.pec_keep(flags, 2)
    N = xyz.shape[0]
    src_node = fields.nearest_node(xyz, np.array([[0.5, 0.5], [0.3, 0.6]]))
    src_amp = np.array([1.0, -0.5])
    t = (np.arange(steps) + 0.5) * dt
    tau = 6 * h
    wave = np.stack([fields.gaussian_wavelet(t, 3 * tau, tau), fields.gaussian_wavelet(t, 4 * tau, tau)], 1)
    rcv = fields.nearest_node(xyz, np.array([[0.2, 0.2], [0.7, 0.3], [0.6, 0.8]]))
    return dict(xyz=xyz, op=op, dt=dt, gamma=gamma, eps_r=eps_r, keep=keep, N=N, steps=steps,
                src=(src_node, src_amp, wave), rcv=rcv)


def _traces(p, eps_r, amp):
    N = p["N"]
    kappa = p["dt"] / eps_r
    _, _, _, tr = step.run(np.zeros((N, 1)), np.zeros((N, 2)), p["op"], p["op"], p["dt"], p["steps"],
                           p["gamma"], kappa, p["keep"], src=(p["src"][0], amp, p["src"][2]), rcv=p["rcv"])
    return tr


def test_amplitude_gradient_is_exact_dot_product():
    p = _problem()
    gt = rng.uniform_range(3, 0, np.arange(p["steps"] * 3), -1, 1).reshape(p["steps"], 3)
    g_eps, g_amp, _ = step.adjoint_2d(np.zeros((p["N"], 1)), np.zeros((p["N"], 2)), p["op"], p["dt"],
                                      p["steps"], p["gamma"], p["eps_r"], p["keep"], src=p["src"],
                                      rcv=p["rcv"], grad_traces=gt)
    for s in range(2):
        amp = np.zeros(2)
        amp[s] = 1.0
        tr = _traces(p, p["eps_r"], amp)
        assert abs(g_amp[s] - (tr * gt).sum()) <= 1e-12 * max(1.0, abs(g_amp[s]))


def test_permittivity_gradient_matches_central_differences():
    p = _problem()
    amp = p["src"][1]
    d = _traces(p, np.ones(p["N"]), amp)          # data from eps_r = 1

    def J(e):
        r = _traces(p, e, amp) - d
        return 0.5 * (r * r).sum()

    tr = _traces(p, p["eps_r"], amp)
    g_eps, _, tr_adj = step.adjoint_2d(np.zeros((p["N"], 1)), np.zeros((p["N"], 2)), p["op"], p["dt"],
                                       p["steps"], p["gamma"], p["eps_r"], p["keep"], src=p["src"],
                                       rcv=p["rcv"], grad_traces=tr - d)
    assert np.abs(tr_adj - tr).max() == 0.0
    for q in range(3):
        v = rng.uniform_range(11, q, np.arange(p["N"]), -1, 1)
        eps = 1e-5
        fd = (J(p["eps_r"] + eps * v) - J(p["eps_r"] - eps * v)) / (2 * eps)
        an = (g_eps * v).sum()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-14
