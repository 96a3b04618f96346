"""The C-ABI library loads, exports every declared symbol, and validates plans
on the host (no GPU calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbffd.h")


def _lib():
    from paper_2508_18205_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("librbffd.so not built")
    return _abi, _abi.load()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbffd_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    _abi, lib = _lib()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
        assert n in _abi.PROTOTYPES, n


def test_struct_layouts_match_header_sizes():
    _abi, _ = _lib()
    # params: 14 int32 + 7 doubles + 6 doubles
    assert C.sizeof(_abi.Params) == 14 * 4 + 14 * 8
    assert C.sizeof(_abi.Fields) == 5 * 8 + 8
    # run args: 8 int32, 7 pointers, 1 double
    assert C.sizeof(_abi.RunArgs) == 8 * 4 + 7 * 8 + 8
    # scan args: 8 pointers, 7 doubles, 6 int32
    assert C.sizeof(_abi.HvScanArgs) == 8 * 8 + 7 * 8 + 6 * 4


def _params(_abi, **kw):
    p = _abi.Params()
    p.dim, p.mode, p.n, p.m, p.phs_k, p.hv_alpha = 2, 0, 12, 2, 3, 2
    p.bc, p.reorder, p.wdtype, p.fdtype, p.K = 0, 1, 0, 0, 1
    p.vfd_sigma, p.hv_c, p.h, p.eps0, p.mu0 = 0.5, 1.0, 0.1, 1.0, 1.0
    p.hi[0] = p.hi[1] = 1.0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_plan_validation_and_sizes_on_host():
    _abi, lib = _lib()
    from synth import nodes
    xyz, flags, h = nodes.jittered_grid((11, 11), seed=1)
    xyz = np.ascontiguousarray(xyz)
    plan = C.c_void_p()
    ok = _params(_abi)
    rc = lib.rbffd_plan_create(C.byref(ok), xyz.shape[0], xyz.ctypes.data, flags.ctypes.data, 0, None, None,
                               C.byref(plan))
    assert rc == 0
    s = _abi.Sizes()
    assert lib.rbffd_plan_sizes(plan, C.byref(s)) == 0
    assert s.N == 121 and s.n_stencil == 31 and s.n_hv == 31 and s.fe == 1 and s.fh == 2
    assert abs(s.dt - 0.1 / (10 * np.sqrt(2))) < 1e-18
    assert abs(s.gamma - (-1.0 * 0.1 ** 4)) < 1e-20          # c (-1)^(alpha-1) h^(2 alpha)
    assert s.arena_bytes > 0 and s.e_bytes == 121 * 8
    # out-of-order use is refused without touching the device
    assert lib.rbffd_get_perm(plan, 0, np.zeros(121, np.int32).ctypes.data, None) == _abi.ESTATE
    sa = _abi.HvScanArgs()
    assert lib.rbffd_hv_scan(plan, None, C.byref(sa), None, None) == _abi.ESTATE
    assert lib.rbffd_set_field_hv(plan, None, None) == _abi.ESTATE
    lib.rbffd_plan_destroy(plan)
    # n must exceed M_m; stencils must fit; BF16 needs F32 weights
    for bad in (dict(n=6), dict(n=200), dict(fdtype=2, wdtype=0), dict(dim=4), dict(phs_k=4)):
        p = _params(_abi, **bad)
        rc = lib.rbffd_plan_create(C.byref(p), xyz.shape[0], xyz.ctypes.data, flags.ctypes.data, 0, None, None,
                                   C.byref(plan))
        assert rc in (_abi.EINVAL, _abi.ESIZE, _abi.ENOTSUP), bad
    # empty node set
    p = _params(_abi)
    assert lib.rbffd_plan_create(C.byref(p), 0, xyz.ctypes.data, flags.ctypes.data, 0, None, None,
                                 C.byref(plan)) == _abi.ESIZE
    assert lib.rbffd_strerror(_abi.ESINGULAR) == b"singular local weight system"
    # TEz polarisation: (Ex, Ey) and Hz per node; collocated 2D, K = 1 only
    p = _params(_abi, pol=1)
    assert lib.rbffd_plan_create(C.byref(p), xyz.shape[0], xyz.ctypes.data, flags.ctypes.data, 0, None, None,
                                 C.byref(plan)) == 0
    assert lib.rbffd_plan_sizes(plan, C.byref(s)) == 0
    assert s.fe == 2 and s.fh == 1 and s.e_bytes == 121 * 2 * 8 and s.h_bytes == 121 * 8
    lib.rbffd_plan_destroy(plan)
    for bad, code in ((dict(pol=2), _abi.EINVAL), (dict(pol=1, K=4, fdtype=1, wdtype=1), _abi.ENOTSUP),
                      (dict(pol=1, adjoint=1), _abi.ENOTSUP), (dict(pol=1, mode=2), _abi.ENOTSUP),
                      # rotated frame: 2D only, finite, not with axis-aligned TEz walls
                      (dict(frame_angle=float("nan")), _abi.EINVAL),
                      (dict(pol=1, frame_angle=0.3), _abi.ENOTSUP),
                      # weight storage must match the fields; compressed (W22)
                      # weights: 2D collocated single-field FP32 only
                      (dict(wdtype=1, fdtype=0), _abi.EINVAL), (dict(wdtype=0, fdtype=1), _abi.EINVAL),
                      (dict(wdtype=3), _abi.ENOTSUP), (dict(wdtype=3, fdtype=1, K=4), _abi.ENOTSUP),
                      (dict(wdtype=3, fdtype=1, adjoint=1), _abi.ENOTSUP),
                      (dict(wdtype=3, fdtype=2), _abi.ENOTSUP), (dict(wdtype=4, fdtype=1), _abi.EINVAL)):
        p = _params(_abi, **bad)
        rc = lib.rbffd_plan_create(C.byref(p), xyz.shape[0], xyz.ctypes.data, flags.ctypes.data, 0, None, None,
                                   C.byref(plan))
        assert rc == code, bad
    nowall = np.zeros_like(flags)
    for good in (dict(frame_angle=0.3, mode=1), dict(frame_angle=-0.7, pol=1, bc=1), dict(wdtype=3, fdtype=1),
                 dict(wdtype=3, fdtype=1, pol=1, mode=1)):
        p = _params(_abi, **good)
        fl = nowall if good.get("bc") == 1 else flags
        if good.get("bc") == 1:
            p.hi[0] = p.hi[1] = 1.1                  # nodes in [lo, hi)
        rc = lib.rbffd_plan_create(C.byref(p), xyz.shape[0], xyz.ctypes.data, fl.ctypes.data, 0, None, None,
                                   C.byref(plan))
        assert rc == 0, (good, lib.rbffd_strerror(rc))
        lib.rbffd_plan_destroy(plan)


def test_wall_normals_validation_on_host():
    _abi, lib = _lib()
    from synth import nodes
    xyz, flags, h = nodes.jittered_grid((11, 11), seed=1)
    xyz = np.ascontiguousarray(xyz)
    N = xyz.shape[0]
    plan = C.c_void_p()

    def make(**kw):
        p = _params(_abi, **kw)
        assert lib.rbffd_plan_create(C.byref(p), N, xyz.ctypes.data, flags.ctypes.data, 0, None, None,
                                     C.byref(plan)) == 0
        return plan

    nrm = np.zeros((N, 2))
    wall = np.nonzero(flags)[0]
    nrm[wall, 0] = 1.0
    pl = make()                                              # TMz: Ez needs no normal
    assert lib.rbffd_set_wall_normals(pl, nrm.ctypes.data) == _abi.ENOTSUP
    lib.rbffd_plan_destroy(pl)
    pl = make(pol=1)
    assert lib.rbffd_set_wall_normals(pl, nrm.ctypes.data) == 0
    assert lib.rbffd_set_wall_normals(pl, None) == 0
    bad = nrm.copy()
    bad[wall[0]] = (0.6, 0.7)                                # not a unit vector
    assert lib.rbffd_set_wall_normals(pl, bad.ctypes.data) == _abi.EINVAL
    bad = nrm.copy()
    inner = np.nonzero(flags == 0)[0][0]
    bad[inner] = (0.0, 1.0)                                  # normal off the wall
    assert lib.rbffd_set_wall_normals(pl, bad.ctypes.data) == _abi.EINVAL
    lib.rbffd_plan_destroy(pl)
    # 3D plans take [N][3] normals
    x3, f3, h3 = nodes.jittered_grid((6, 6, 6), seed=2)
    x3 = np.ascontiguousarray(x3)
    p = _params(_abi, dim=3, n=35, n_hv=71)
    p.hi[2] = 1.0
    assert lib.rbffd_plan_create(C.byref(p), x3.shape[0], x3.ctypes.data, f3.ctypes.data, 0, None, None,
                                 C.byref(plan)) == 0
    n3 = np.zeros((x3.shape[0], 3))
    w3 = np.nonzero(f3)[0]
    n3[w3] = (0.0, 0.6, 0.8)
    assert lib.rbffd_set_wall_normals(plan, n3.ctypes.data) == 0
    n3[w3[0]] = (0.0, 0.6, 0.7)
    assert lib.rbffd_set_wall_normals(plan, n3.ctypes.data) == _abi.EINVAL
    lib.rbffd_plan_destroy(plan)


def test_missing_library_fails_loudly(monkeypatch):
    # the product path has no CPU fallback: without librbffd.so the binding
    # raises instead of computing anything
    from paper_2508_18205_amd import _abi
    monkeypatch.setattr(_abi, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "librbffd.so"))
    monkeypatch.setattr(_abi, "_lib", None)
    with pytest.raises(ImportError):
        _abi.load()
    from paper_2508_18205_amd import Solver
    from synth import configs
    w = configs.tm_cavity_2d(scale=0.3)
    with pytest.raises((ImportError, RuntimeError)):
        Solver.from_workload(w)
