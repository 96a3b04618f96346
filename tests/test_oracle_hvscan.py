"""Oracle pins for the hyperviscosity parameter search (Section 5.1, Section 6).

* The search logic against closed forms: geometric candidates, K = 3 is
  plain bisection on log c, the bracket of a known threshold shrinks by K - 1
  per round around it, and the early stops.
* The physics against a different route: the spectral radius rho(c) of the
  one-step map of eq. 19 (eigenvalues of the dense one-step matrix of a small
  periodic scattered node set).  A candidate whose rho - 1 is large enough to
  grow the seeded perturbation past the band within T steps must be rejected;
  every accepted candidate has rho close to 1; the neutral ones that barely
  damp the smooth initial wave are accepted.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import hvscan, knn, step, weights as W
from synth import configs, nodes, rng

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_candidates_are_geometric_with_exact_endpoints():
    cs = hvscan.candidates(1e-3, 10.0, 5)
    assert cs[0] == 1e-3
    assert abs(cs[-1] / 10.0 - 1) < 1e-15
    assert np.allclose(cs[1:] / cs[:-1], 10.0, rtol=1e-14)


def test_three_candidates_is_bisection_on_log_c():
    cstar = 10 ** -2.345
    res = hvscan.k_section(lambda cs: cs >= cstar, 1e-4, 1.0, 3, 12)
    lo, hi = 1e-4, 1.0
    for _ in range(12):
        mid = math.sqrt(lo * hi)
        if mid >= cstar:
            hi = mid
        else:
            lo = mid
    assert res["status"] == "bracketed"
    assert abs(res["bracket"][0] / lo - 1) < 1e-12 and abs(res["bracket"][1] / hi - 1) < 1e-12
    assert res["bracket"][0] < cstar <= res["bracket"][1]


@pytest.mark.parametrize("K", [4, 8, 64])
def test_bracket_shrinks_by_k_minus_1_around_threshold(K):
    cstar = 3.3e-5
    rounds = 3
    res = hvscan.k_section(lambda cs: cs >= cstar, 1e-8, 1e-1, K, rounds)
    lo, hi = res["bracket"]
    assert lo < cstar <= hi
    assert abs(hi / lo / hvscan.bracket_width(1e-8, 1e-1, K, rounds) - 1) < 1e-9
    assert res["c_best"] == hi and len(res["history"]) == rounds


def test_lower_edge_of_an_interval_and_early_stops():
    a, b = 2e-4, 5e-3
    res = hvscan.k_section(lambda cs: (cs >= a) & (cs <= b), 1e-6, 1e-1, 16, 3)
    assert res["status"] == "bracketed" and res["bracket"][0] < a <= res["bracket"][1]
    none = hvscan.k_section(lambda cs: np.zeros(len(cs), bool), 1e-6, 1e-1, 8, 3)
    assert none["status"] == "none" and none["c_best"] is None and len(none["history"]) == 1
    below = hvscan.k_section(lambda cs: np.ones(len(cs), bool), 1e-6, 1e-1, 8, 3)
    assert below["status"] == "below" and below["c_best"] == 1e-6
    with pytest.raises(ValueError):
        hvscan.k_section(lambda cs: cs > 0, 1.0, 0.5, 8, 1)


def test_acceptance_band():
    band = GOLD["narrow_pulse"]["u_band"]
    assert hvscan.accepted([1.0, 0.995, 1.009], band)
    assert not hvscan.accepted([1.0, 1.02], band)
    assert not hvscan.accepted([1.0, 0.98], band)
    assert not hvscan.accepted([1.0, np.nan], band)
    assert not hvscan.accepted([1.0, np.inf], band)


def _strip():
    # periodic strip [0, 1) x [0, 1/8) of a 48 x 6 jittered grid: the smooth
    # wave sin(2 pi x) has 48 nodes per wavelength, so hyperviscosity barely
    # damps it while the scattered-node modes of eq. 19 can still grow
    nx, ny = 48, 6
    Ly = ny / nx
    xyz, _, h = nodes.jittered_grid((nx, ny), hi=(1.0, Ly), periodic=True, seed=5)
    P = (1.0, Ly)
    idx = knn.knn(xyz, 31, period=P)
    op = {"curl_idx": idx[:, :12], "curl_w": W.curl_weights(xyz, xyz, idx[:, :12], 2, period=P),
          "hv_idx": idx, "hv_w": W.hv_weights(xyz, xyz, idx, 2, period=P)}
    N = xyz.shape[0]
    noise = rng.uniform_range(5, 1, np.arange(N), -1.0, 1.0)
    E0 = (np.sin(2 * math.pi * xyz[:, 0]) + 1e-3 * noise)[:, None]
    return xyz, h, op, E0, np.zeros((N, 2))


def _rho(op, h, dt, c):
    N = op["curl_idx"].shape[0]
    g = step.hv_gamma(c, 2, h)
    keep = np.ones((N, 1))
    M = np.zeros((3 * N, 3 * N))
    for j in range(3 * N):
        s = np.zeros(3 * N)
        s[j] = 1.0
        Hn = step.h_update(s[:N, None], np.stack([s[N:2 * N], s[2 * N:]], 1), op, dt, g)
        En = step.e_update(s[:N, None], Hn, op, dt, g, keep)
        M[:N, j], M[N:2 * N, j], M[2 * N:, j] = En[:, 0], Hn[:, 0], Hn[:, 1]
    return float(np.abs(np.linalg.eigvals(M)).max())


def test_scan_agrees_with_spectral_radius():
    xyz, h, op, E0, H0 = _strip()
    N = xyz.shape[0]
    dt = configs.SC * h
    T, every = 3000, 50
    band = GOLD["narrow_pulse"]["u_band"]
    res = hvscan.hv_scan(E0, H0, op, op, dt, T, every, 2, h, dt, np.ones((N, 1)), 1e-5 / dt, 1e-2 / dt,
                         8, 2, band=band)
    assert res["status"] == "bracketed"
    neutral_accepted = 0
    for cs, ok in res["history"]:
        for c, o in zip(cs, ok):
            r = _rho(op, h, dt, c) - 1.0
            if r >= 30.0 / T:
                assert not o, (c * dt, r)
            if o:
                assert r < 15.0 / T, (c * dt, r)
            if abs(r) < 1e-12 and c * dt <= 1.5e-3:
                assert o, (c * dt, r)
                neutral_accepted += 1
    assert neutral_accepted >= 1
    # the explicit hyperviscosity term has its own limit: the largest candidate
    # (c dt = 1e-2) is unstable and rejected
    assert not res["history"][0][1][-1]
