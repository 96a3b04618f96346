"""rbffd_energy_static (no workspace, no allocation) against rbffd_energy.

Both entry points run the same reduction kernels, so their results must agree
bit for bit; the second call of each pair uses a smaller node set, so the
static scratch holds the previous call's partial sums when it starts.  FP64
and FP32 fields, 2D (TMz) and 3D plans.  The FP64 numpy sum of eq. 20 is a
sanity bound on both.
"""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_18205_amd import Solver, _abi  # noqa: E402
from synth import configs  # noqa: E402


def _fields(s, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    E = torch.rand((s.N, s.FE), generator=g, dtype=torch.float64) - 0.5
    Ha = torch.rand((s.N, s.FH), generator=g, dtype=torch.float64) - 0.5
    Hb = torch.rand((s.N, s.FH), generator=g, dtype=torch.float64) - 0.5
    if s.dim == 3:                      # the pad value of each 3-vector is unused
        E[:, 3] = 0
        Ha[:, 3] = 0
        Hb[:, 3] = 0
    return [t.to(device=s.device, dtype=s.dtype).contiguous() for t in (E, Ha, Hb)]


def _both(s, E, Ha, Hb):
    lib = _abi.load()
    out_ws = torch.full((1,), -1.0, dtype=torch.float64, device=s.device)
    out_st = torch.full((1,), -2.0, dtype=torch.float64, device=s.device)
    print(f"  energy_static N={s.N} {s.precision} dim={s.dim}", flush=True)
    _abi.check(lib.rbffd_energy(s.plan, E.data_ptr(), Ha.data_ptr(), Hb.data_ptr(), out_ws.data_ptr(),
                                s.ws.data_ptr(), s.stream()), s.plan, "rbffd_energy")
    _abi.check(lib.rbffd_energy_static(s.plan, C.c_void_p(E.data_ptr()), C.c_void_p(Ha.data_ptr()),
                                       C.c_void_p(Hb.data_ptr()), C.c_void_p(out_st.data_ptr()), s.stream()),
               s.plan, "rbffd_energy_static")
    torch.cuda.synchronize()
    return float(out_ws.cpu()[0]), float(out_st.cpu()[0])


def _numpy_energy(s, E, Ha, Hb, fe, fh):
    e = E.double().cpu().numpy()[:, :fe]
    hb = 0.5 * (Ha.double().cpu().numpy()[:, :fh] + Hb.double().cpu().numpy()[:, :fh])
    eta2 = s.params.mu0 / s.params.eps0
    return s.params.h ** s.dim * ((e * e).sum() + eta2 * (hb * hb).sum())


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_energy_static_equals_workspace_energy_two_calls(precision, dim):
    sizes = (41, 23) if dim == 2 else (11, 8)
    for k, ns in enumerate(sizes):
        if dim == 2:
            w = configs.tm_cavity_2d(n_side=ns, chat=1e-3, steps=10, eps0=2.0, mu0=3.0)
        else:
            w = configs.tm111_3d(n_side=ns, chat=1e-3, steps=10)
        s = Solver.from_workload(w, precision=precision)
        E, Ha, Hb = _fields(s, 100 + k)
        ws, st = _both(s, E, Ha, Hb)
        ref = _numpy_energy(s, E, Ha, Hb, 1 if dim == 2 else 3, 2 if dim == 2 else 3)
        print(f"  workspace {ws!r} static {st!r} numpy {ref!r}", flush=True)
        assert st == ws
        assert abs(st - ref) <= 1e-12 * abs(ref)


def test_energy_static_refuses_batch_and_unset_plans():
    lib = _abi.load()
    w = configs.batched_2d(n_side=20, K=4)
    s = Solver.from_workload(w, precision="f32", K=4)
    z = torch.zeros(16, dtype=torch.float64, device=s.device)
    rc = lib.rbffd_energy_static(s.plan, C.c_void_p(z.data_ptr()), C.c_void_p(z.data_ptr()),
                                 C.c_void_p(z.data_ptr()), C.c_void_p(z.data_ptr()), s.stream())
    assert rc == _abi.ENOTSUP
    assert lib.rbffd_energy_static(s.plan, None, None, None, None, s.stream()) == _abi.EINVAL
