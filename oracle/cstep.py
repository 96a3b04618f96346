"""Loader of the oracle's plain C leapfrog (oracle/cstep.c) for large node sets.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The C file computes the
same 2D TMz and 3D half updates as ``oracle.step.h_update`` / ``e_update``
(eq. 19) with a loop over nodes (OpenMP over nodes, no fused multiply-adds);
this module only marshals arrays and runs the step loop.  ``build`` compiles it
with gcc; ``load`` builds it when it is missing.
"""
import ctypes as C
import math
import os
import subprocess

import numpy as np

from . import step as _step

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cstep.c")
LIB = os.path.join(HERE, "libostep.so")

_lib = None


def build():
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99", SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the C oracle failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = C.CDLL(LIB)
    P = C.c_void_p
    lib.oracle_h_update_tm.restype = None
    lib.oracle_h_update_tm.argtypes = [C.c_int64, P, P, P, C.c_int, P, P, C.c_int, P, P, C.c_double, C.c_double]
    lib.oracle_e_update_tm.restype = None
    lib.oracle_e_update_tm.argtypes = [C.c_int64, P, P, P, C.c_int, P, P, C.c_int, P, P, P, C.c_double, C.c_double,
                                       P]
    for nm in ("oracle_h_update_3d",):
        getattr(lib, nm).restype = None
        getattr(lib, nm).argtypes = lib.oracle_h_update_tm.argtypes
    lib.oracle_e_update_3d.restype = None
    lib.oracle_e_update_3d.argtypes = lib.oracle_e_update_tm.argtypes
    lib.oracle_threads.restype = C.c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_set_threads.restype = None
    lib.oracle_set_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


def threads():
    """OpenMP threads the C oracle runs on."""
    return int(load().oracle_threads())


def set_threads(t):
    """OpenMP threads of later calls."""
    load().oracle_set_threads(int(t))


class Operator:
    """Contiguous FP64 / int64 copies of an ``oracle.step`` operator dict
    (2D or 3D, from the curl weights' shape)."""

    def __init__(self, op):
        self.ci = np.ascontiguousarray(op["curl_idx"], dtype=np.int64)
        self.cw = np.ascontiguousarray(op["curl_w"], dtype=np.float64)
        self.hi = np.ascontiguousarray(op["hv_idx"], dtype=np.int64)
        self.hw = np.ascontiguousarray(op["hv_w"], dtype=np.float64)
        self.N, self.n = self.ci.shape
        self.nh = self.hi.shape[1] if self.hw.size else 0
        self.d = self.cw.shape[1]
        assert self.cw.shape == (self.N, self.d, self.n) and self.d in (2, 3)


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def h_update(E, H, op, a, gamma, out=None):
    """H^{n+1} from E^n and H^n: [N, 2] from [N, 1], [N, 2] in 2D TMz; [N, 3]
    from [N, 3], [N, 3] in 3D."""
    lib = load()
    E = np.ascontiguousarray(E, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.float64)
    out = np.empty_like(H) if out is None else out
    fn = lib.oracle_h_update_3d if op.d == 3 else lib.oracle_h_update_tm
    fn(op.N, _p(E), _p(H), _p(out), op.n, _p(op.ci), _p(op.cw), op.nh, _p(op.hi), _p(op.hw), float(a),
       float(gamma))
    return out


def e_update(E, Hn, op, kappa, gamma, keep, out=None):
    """E^{n+1} from E^n and H^{n+1} ([N, 1] in 2D TMz, [N, 3] in 3D); kappa
    scalar or [N]; keep shaped like E (or [N] in 2D)."""
    lib = load()
    E = np.ascontiguousarray(E, dtype=np.float64)
    Hn = np.ascontiguousarray(Hn, dtype=np.float64)
    keep = np.ascontiguousarray(np.asarray(keep, dtype=np.float64).reshape(-1))
    out = np.empty_like(E) if out is None else out
    karr = None
    k0 = 0.0
    if np.ndim(kappa) == 0:
        k0 = float(kappa)
    else:
        karr = np.ascontiguousarray(kappa, dtype=np.float64)
    assert keep.size == E.size
    fn = lib.oracle_e_update_3d if op.d == 3 else lib.oracle_e_update_tm
    fn(op.N, _p(E), _p(Hn), _p(out), op.n, _p(op.ci), _p(op.cw), op.nh, _p(op.hi), _p(op.hw), _p(karr), k0,
       float(gamma), _p(keep))
    return out


def run(E, H, op, dt, steps, gamma, kappa, keep, mu0=1.0, eps0=1.0, h=None, energy_every=0, callback=None):
    """``oracle.step.run`` for a collocated field without sources (2D TMz or
    3D): returns (E, H, energies).  callback(n, E, H), if given, sees the
    state after each step n = 1 .. steps."""
    a = dt / mu0
    eta0 = math.sqrt(mu0 / eps0)
    E = np.array(E, dtype=np.float64).reshape(op.N, -1)
    H = np.array(H, dtype=np.float64)
    E2, H2 = np.empty_like(E), np.empty_like(H)
    energies = []
    for n in range(steps):
        h_update(E, H, op, a, gamma, out=H2)
        if energy_every and n % energy_every == 0:
            energies.append(_step.energy(E, H, H2, h, h, eta0, op.d))
        e_update(E, H2, op, kappa, gamma, keep, out=E2)
        E, E2 = E2, E
        H, H2 = H2, H
        if callback is not None:
            callback(n + 1, E, H)
    return E, H, np.array(energies)
