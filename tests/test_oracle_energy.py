"""Pins of the oracle's energy (eq. 20) and error measures (eq. 23) against
closed forms.

On a regular periodic grid x_i = i h (i = 0 .. n - 1, L = n h) the node sums
of sin^2(2 pi q x / L) and cos^2(2 pi q x / L) are exactly n / 2 for any
integer q with 2 q not a multiple of n (the sum of cos(4 pi q i / n) over a
full period vanishes), and the sum of sin cos vanishes.  With E = A sin(.),
H_old = B cos(.), H_new = C cos(.) the energy of eq. 20,
U = h^d sum |E|^2 + eta0^2 h^d sum |(H_old + H_new) / 2|^2, eta0^2 = mu0 /
eps0, is therefore a closed form in A, B, C, h and N.  The constants are
chosen (eps0 != mu0, h != 1, B != C) so that each plausible slip -- eta0 in
place of eta0^2, the inverse ratio eps0 / mu0, a missing h^d, H_old or H_new
in place of their average, a sum of averaged squares -- moves U by far more
than the tolerance; each such variant is evaluated below and must miss.
"""
import math

import numpy as np
import pytest

from oracle import step as ostep
from synth import nodes

EPS0, MU0 = 2.0, 3.0
ETA2 = MU0 / EPS0


def _grid(shape, L):
    xyz, flags, h = nodes.jittered_grid(shape, lo=(0.0,) * len(shape), hi=(L,) * len(shape), jitter=0.0,
                                        periodic=True)
    return xyz, h


def _wave(x, q, L, kind):
    a = 2.0 * math.pi * q * x / L
    return np.sin(a) if kind == "s" else np.cos(a)


def _variants(E, Ho, Hn, h_e, h_h, d):
    """Plausible mistakes in eq. 20 (each must miss the closed form)."""
    Hb = 0.5 * (Ho + Hn)
    eta = math.sqrt(ETA2)
    e2 = (E * E).sum()
    return {
        "eta0 not squared": h_e ** d * e2 + eta * h_h ** d * (Hb * Hb).sum(),
        "eps0/mu0 inverted": h_e ** d * e2 + (EPS0 / MU0) * h_h ** d * (Hb * Hb).sum(),
        "no h^d": e2 + ETA2 * (Hb * Hb).sum(),
        "H_old only": h_e ** d * e2 + ETA2 * h_h ** d * (Ho * Ho).sum(),
        "H_new only": h_e ** d * e2 + ETA2 * h_h ** d * (Hn * Hn).sum(),
        "mean of squares": h_e ** d * e2 + ETA2 * h_h ** d * 0.5 * ((Ho * Ho).sum() + (Hn * Hn).sum()),
    }


def test_energy_closed_form_2d():
    L = 1.2
    xyz, h = _grid((24, 24), L)
    N = xyz.shape[0]
    x, y = xyz[:, 0], xyz[:, 1]
    A, B1, C1, B2, C2 = 0.7, 1.3, -0.4, 0.9, 2.1
    E = (A * _wave(x, 3, L, "s"))[:, None]
    Ho = np.stack([B1 * _wave(y, 2, L, "c"), B2 * _wave(x, 5, L, "c")], axis=1)
    Hn = np.stack([C1 * _wave(y, 2, L, "c"), C2 * _wave(x, 5, L, "c")], axis=1)
    U = ostep.energy(E, Ho, Hn, h, h, math.sqrt(ETA2), 2)
    closed = h ** 2 * (N / 2) * (A ** 2 + ETA2 * (((B1 + C1) / 2) ** 2 + ((B2 + C2) / 2) ** 2))
    assert abs(U - closed) <= 1e-13 * closed
    for name, v in _variants(E, Ho, Hn, h, h, 2).items():
        assert abs(v - closed) > 1e-2 * closed, name


def test_energy_closed_form_3d():
    L = 0.8
    xyz, h = _grid((10, 10, 10), L)
    N = xyz.shape[0]
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    A = np.array([0.5, -1.1, 0.3])
    B = np.array([1.7, 0.2, -0.6])
    C = np.array([-0.3, 1.4, 2.2])
    E = np.stack([A[0] * _wave(y, 1, L, "s"), A[1] * _wave(z, 2, L, "s"), A[2] * _wave(x, 3, L, "s")], axis=1)
    Ho = np.stack([B[0] * _wave(z, 4, L, "c"), B[1] * _wave(x, 1, L, "c"), B[2] * _wave(y, 2, L, "c")], axis=1)
    Hn = np.stack([C[0] * _wave(z, 4, L, "c"), C[1] * _wave(x, 1, L, "c"), C[2] * _wave(y, 2, L, "c")], axis=1)
    U = ostep.energy(E, Ho, Hn, h, h, math.sqrt(ETA2), 3)
    closed = h ** 3 * (N / 2) * ((A ** 2).sum() + ETA2 * (((B + C) / 2) ** 2).sum())
    assert abs(U - closed) <= 1e-13 * closed
    for name, v in _variants(E, Ho, Hn, h, h, 3).items():
        assert abs(v - closed) > 1e-2 * closed, name


def test_energy_two_sets_weights_each_set_by_its_spacing():
    # E on one grid, H on another with a different spacing (two-set variant)
    L = 1.0
    xe, he = _grid((20, 20), L)
    xh, hh = _grid((14, 14), L)
    A, B, C = 1.1, 0.6, -1.9
    E = (A * _wave(xe[:, 0], 3, L, "s"))[:, None]
    Ho = np.stack([B * _wave(xh[:, 1], 2, L, "c"), np.zeros(len(xh))], axis=1)
    Hn = np.stack([C * _wave(xh[:, 1], 2, L, "c"), np.zeros(len(xh))], axis=1)
    U = ostep.energy(E, Ho, Hn, he, hh, math.sqrt(ETA2), 2)
    closed = he ** 2 * (len(xe) / 2) * A ** 2 + ETA2 * hh ** 2 * (len(xh) / 2) * ((B + C) / 2) ** 2
    assert abs(U - closed) <= 1e-13 * closed
    swapped = hh ** 2 * (len(xe) / 2) * A ** 2 + ETA2 * he ** 2 * (len(xh) / 2) * ((B + C) / 2) ** 2
    assert abs(swapped - closed) > 1e-2 * closed


def _null_op(N, d):
    """An operator whose every weight is zero: the update leaves H and E as they are."""
    z = np.zeros((N, 1), dtype=np.int64)
    return {"curl_idx": z, "curl_w": np.zeros((N, d, 1)), "hv_idx": z, "hv_w": np.zeros((N, 1))}


@pytest.mark.parametrize("pol", ["TM", "TE"])
def test_run_samples_eq20_with_its_own_eta0(pol):
    # run()/run_te() form eta0 from eps0 and mu0 themselves; with null
    # operators H^1 = H^0, so the sample of step 0 is the closed form
    L = 1.2
    xyz, h = _grid((24, 24), L)
    N = xyz.shape[0]
    x, y = xyz[:, 0], xyz[:, 1]
    A, B1, B2 = 0.7, 1.3, -0.8
    op = _null_op(N, 2)
    dt = 0.01
    if pol == "TM":
        E0 = (A * _wave(x, 3, L, "s"))[:, None]
        H0 = np.stack([B1 * _wave(y, 2, L, "c"), B2 * _wave(x, 5, L, "c")], axis=1)
        _, _, en, _ = ostep.run(E0, H0, op, op, dt, 2, 0.0, dt / EPS0, np.ones((N, 1)), mu0=MU0, eps0=EPS0,
                                h_e=h, h_h=h, energy_every=1)
        closed = h ** 2 * (N / 2) * (A ** 2 + ETA2 * (B1 ** 2 + B2 ** 2))
    else:
        E0 = np.stack([A * _wave(x, 3, L, "s"), B2 * _wave(y, 1, L, "s")], axis=1)
        H0 = (B1 * _wave(y, 2, L, "c"))[:, None]
        _, _, en = ostep.run_te(E0, H0, op, dt, 2, 0.0, dt / EPS0, np.ones((N, 2)), mu0=MU0, eps0=EPS0, h=h,
                                energy_every=1)
        closed = h ** 2 * (N / 2) * (A ** 2 + B2 ** 2 + ETA2 * B1 ** 2)
    assert len(en) == 2
    assert abs(en[0] - closed) <= 1e-13 * closed
    assert abs(en[1] - closed) <= 1e-13 * closed


def test_linf_and_rel_l2_closed_forms():
    # eq. 23 (max-norm errors) and the relative L2 error on the same grid:
    # f = ref + delta cos, so max|f - ref| = delta (the grid holds x = 0),
    # ||f - ref|| / ||ref|| = delta sqrt(N/2) / (A sqrt(N/2)) = delta / A
    L = 1.0
    xyz, h = _grid((32, 32), L)
    x = xyz[:, 0]
    A, delta = 1.5, 1e-3
    ref = A * _wave(x, 3, L, "s")
    f = ref + delta * _wave(x, 3, L, "c")
    eE, eH = ostep.linf_errors(f, np.stack([f, f], 1), ref, np.stack([ref, f - 2 * delta], 1))
    assert abs(eE - delta) <= 1e-15
    assert abs(eH - 2 * delta) <= 1e-15
    assert abs(ostep.rel_l2(f, ref) - delta / A) <= 1e-13
