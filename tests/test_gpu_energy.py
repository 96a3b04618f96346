"""The GPU's FP64 reductions against closed forms: the energy of eq. 20
(rbffd_energy, and the samples rbffd_run takes), the error sums and maxima of
eq. 23 (rbffd_compare).

The field values are trigonometric in the grid INDEX of a periodic jittered
grid (node id = ix + nx iy (+ nx ny iz)): with x_i = i / n, the sums over the
grid of sin^2(2 pi q i / n) and cos^2(2 pi q i / n) are exactly n / 2 (2 q not
a multiple of n) and the sum of sin cos vanishes, so U = h^d (N / 2) (A^2 +
eta0^2 ((B + C) / 2)^2) and the compare sums are closed forms too.  eps0 = 2,
mu0 = 3 (eta0^2 = 3/2) and h != 1, so a wrong eta0 power, a missing h^d or an
unaveraged H misses them by far more than the tolerance.
"""
import ctypes as C
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_18205_amd import Solver, _abi  # noqa: E402
from synth import nodes  # noqa: E402

EPS0, MU0 = 2.0, 3.0
ETA2 = MU0 / EPS0


def _plan(dim, precision, pol="TM", n_side=None, L=1.3):
    ns = n_side or (24 if dim == 2 else 10)
    shape = (ns,) * dim
    xyz, flags, h = nodes.jittered_grid(shape, lo=(0.0,) * dim, hi=(L,) * dim, seed=21, periodic=True)
    if dim == 2:
        s = Solver(2, xyz, flags, h, 12, 2, 2, 1e-3, (0.0, 0.0), (L, L), n_hv=31, bc="PERIODIC", eps0=EPS0,
                   mu0=MU0, precision=precision, pol=pol)
    else:
        s = Solver(3, xyz, flags, h, 35, 2, 2, 1e-3, (0.0,) * 3, (L,) * 3, n_hv=71, bc="PERIODIC", eps0=EPS0,
                   mu0=MU0, precision=precision)
    ids = np.arange(xyz.shape[0])
    idx = [(ids // ns ** k) % ns for k in range(dim)]
    return s, h, ns, idx


def _w(i, q, n, kind):
    a = 2.0 * math.pi * q * i / n
    return np.sin(a) if kind == "s" else np.cos(a)


def _tm_fields(idx, n):
    A, B1, C1, B2, C2 = 0.7, 1.3, -0.4, 0.9, 2.1
    E = (A * _w(idx[0], 3, n, "s"))[:, None]
    Ho = np.stack([B1 * _w(idx[1], 2, n, "c"), B2 * _w(idx[0], 5, n, "c")], axis=1)
    Hn = np.stack([C1 * _w(idx[1], 2, n, "c"), C2 * _w(idx[0], 5, n, "c")], axis=1)
    return E, Ho, Hn, (A ** 2, ((B1 + C1) / 2) ** 2 + ((B2 + C2) / 2) ** 2, B1 ** 2 + B2 ** 2)


def _3d_fields(idx, n):
    A = np.array([0.5, -1.1, 0.3])
    B = np.array([1.7, 0.2, -0.6])
    Cc = np.array([-0.3, 1.4, 2.2])
    E = np.stack([A[0] * _w(idx[1], 1, n, "s"), A[1] * _w(idx[2], 2, n, "s"), A[2] * _w(idx[0], 3, n, "s")], 1)
    Ho = np.stack([B[0] * _w(idx[2], 4, n, "c"), B[1] * _w(idx[0], 1, n, "c"), B[2] * _w(idx[1], 2, n, "c")], 1)
    Hn = np.stack([Cc[0] * _w(idx[2], 4, n, "c"), Cc[1] * _w(idx[0], 1, n, "c"), Cc[2] * _w(idx[1], 2, n, "c")], 1)
    return E, Ho, Hn, ((A ** 2).sum(), (((B + Cc) / 2) ** 2).sum(), (B ** 2).sum())


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_rbffd_energy_closed_form(dim, precision):
    s, h, n, idx = _plan(dim, precision)
    E, Ho, Hn, (se, sh, sho) = (_tm_fields if dim == 2 else _3d_fields)(idx, n)
    closed = h ** dim * (s.N / 2) * (se + ETA2 * sh)
    print(f"energy closed form: dim={dim} {precision} N={s.N}", flush=True)
    U = s.energy(s.to_internal(E, s.FE), s.to_internal(Ho, s.FH), s.to_internal(Hn, s.FH))
    tol = 1e-12 if precision == "f64" else 1e-6
    print(f"  U = {U!r}, closed form {closed!r}", flush=True)
    assert abs(U - closed) <= tol * closed
    # the plausible slips all miss by more than 1 %: no h^d, eta0 unsquared,
    # eps0 / mu0 inverted, H_old in place of the average
    for wrong in (closed / h ** dim, h ** dim * (s.N / 2) * (se + math.sqrt(ETA2) * sh),
                  h ** dim * (s.N / 2) * (se + sh / ETA2), h ** dim * (s.N / 2) * (se + ETA2 * sho)):
        assert abs(U - wrong) > 1e-2 * closed


@pytest.mark.parametrize("which", [0, 1])
def test_rbffd_compare_closed_form(which):
    # f = ref + delta_c cos(.): sum (f - r)^2 = delta_c^2 N / 2, sum r^2 = A_c^2 N / 2,
    # max |f - r| = delta_c (index 0 is on the grid)
    s, h, n, idx = _plan(2, "f64")
    nc = 1 if which == 0 else 2
    A = np.array([0.8, -1.7])[:nc]
    delta = np.array([1e-3, 3e-4])[:nc]
    qs = (3, 5)
    ref = np.stack([A[c] * _w(idx[c], qs[c], n, "s") for c in range(nc)], 1)
    f = ref + np.stack([delta[c] * _w(idx[c], qs[c], n, "c") for c in range(nc)], 1)
    ft = s.to_internal(f, s.FE if which == 0 else s.FH)
    rt = s.to_internal(ref, nc, dtype=torch.float64)
    print(f"compare closed form: which={which} N={s.N}", flush=True)
    out = s.compare(which, ft, rt)
    for c in range(nc):
        assert abs(out[c, 0] - delta[c] ** 2 * s.N / 2) <= 1e-12 * delta[c] ** 2 * s.N / 2
        assert abs(out[c, 1] - A[c] ** 2 * s.N / 2) <= 1e-12 * A[c] ** 2 * s.N / 2
        assert abs(out[c, 2] - delta[c]) <= 1e-15


@pytest.mark.parametrize("case", ["tm", "te", "3d"])
def test_run_energy_samples_closed_form(case):
    # zero weights injected: every update leaves the fields as they are, so
    # each sample of the run's energy is the closed form with H_old = H_new
    dim = 3 if case == "3d" else 2
    s, h, n, idx = _plan(dim, "f64", pol="TE" if case == "te" else "TM")
    s.set_weights(_abi.OP_CURL_H, np.zeros((s.N, dim, 12 if dim == 2 else 35)))
    s.set_weights(_abi.OP_HV_H, np.zeros((s.N, 31 if dim == 2 else 71)))
    if case == "tm":
        E, Ho, _, (se, _, sho) = _tm_fields(idx, n)
        cs = se + ETA2 * sho
    elif case == "te":
        E = np.stack([0.7 * _w(idx[0], 3, n, "s"), -0.8 * _w(idx[1], 1, n, "s")], 1)
        Ho = (1.3 * _w(idx[1], 2, n, "c"))[:, None]
        cs = 0.7 ** 2 + 0.8 ** 2 + ETA2 * 1.3 ** 2
    else:
        E, Ho, _, (se, _, sho) = _3d_fields(idx, n)
        cs = se + ETA2 * sho
    closed = h ** dim * (s.N / 2) * cs
    print(f"run energy samples: {case} N={s.N}", flush=True)
    for graph in (False, True):
        st = s.state(E, Ho)
        r = s.run(st, 6, energy_every=2, use_graph=graph)
        en = r["energy"]
        assert en.shape == (3,)
        assert np.all(np.abs(en - closed) <= 1e-12 * closed), (en, closed)
