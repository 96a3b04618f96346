"""Full-size workloads, checked on sampled nodes the oracle computes one by one.

* 1.0M-node Poisson-disk square (n = 25, m = 4, alpha = 3) and the 8.0M-node
  jittered cube (n = 35, m = 2, alpha = 2), in the FP32 launch configuration
  the benchmark times.
* Node order: bit-exact over all nodes.  Stencils: bit-exact on sampled
  centres (brute force over every node).  Weights: sampled centres, relative
  1e-9 of the node's weight scale (HV: cond(A) * 1e-15 when larger).
* One full step in FP32 from the workload's initial fields: sampled nodes
  against the FP64 oracle step built from oracle weights, within 1e-5 of the
  field scale.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_18205_amd import Solver, _abi  # noqa: E402
from oracle import reorder, knn, weights as OW, step as ostep  # noqa: E402
from synth import configs  # noqa: E402


def _sample(N, k, seed):
    rng = np.random.default_rng(seed)
    s = rng.choice(N, size=k, replace=False)
    return np.concatenate([s, [0, N - 1]])


def _oracle_rows(w, centres, k):
    return knn.knn(w.xyz, k, centres=w.xyz[centres])


def _check(w, nsamp, seed):
    print(f"{w.name}: N={w.N}", flush=True)
    s = Solver.from_workload(w, precision="f32")
    lo, side = reorder.morton_box(w.lo, w.hi)
    perm = reorder.morton_order(w.xyz, lo, side)
    assert (s.perm == perm).all()
    inv = s.inv
    ns = max(w.n, w.n_hv)
    smp = _sample(w.N, nsamp, seed)
    st_int = s.stencils()
    got = s.perm[st_int[inv[smp]]]
    ref = _oracle_rows(w, smp, ns)
    assert (got == ref).all()
    print("  order + sampled stencils bit-exact", flush=True)
    # weights on sampled centres (oracle stencils = the same rows)
    wc = s.weights(_abi.OP_CURL_H)[inv[smp]]
    wh = s.weights(_abi.OP_HV_H)[inv[smp]]
    oc = OW.curl_weights(w.xyz, w.xyz[smp], ref[:, :w.n], w.m)
    oh = OW.hv_weights(w.xyz, w.xyz[smp], ref[:, :w.n_hv], w.alpha)
    ec = (np.abs(wc - oc).reshape(len(smp), -1).max(1) / np.abs(oc).reshape(len(smp), -1).max(1))
    eh = np.abs(wh - oh).max(1) / np.abs(oh).max(1)
    cond = OW.system_condition(w.xyz, w.xyz[smp], ref[:, :w.n_hv], 2 * w.alpha, 2 * w.alpha + 1)
    print(f"  weights: curl {ec.max():.2e} hv {eh.max():.2e} (HV cond max {cond.max():.1e})", flush=True)
    assert ec.max() < 1e-9
    assert (eh <= np.maximum(1e-9, 1e-15 * cond)).all()
    # one FP32 step on the GPU vs the FP64 oracle at sampled nodes
    stt = s.state(w.E0, w.H0)
    s.step(stt, 1)
    E1 = s.E_original(stt)
    H1 = s.H_original(stt)
    # oracle: H^1 at the sampled nodes and at their stencil neighbours, then E^1
    nb = np.unique(ref[:, :w.n])
    need = np.unique(np.concatenate([smp, nb]))
    rows = _oracle_rows(w, need, ns)
    op = {"curl_idx": rows[:, :w.n], "curl_w": OW.curl_weights(w.xyz, w.xyz[need], rows[:, :w.n], w.m),
          "hv_idx": rows[:, :w.n_hv], "hv_w": OW.hv_weights(w.xyz, w.xyz[need], rows[:, :w.n_hv], w.alpha)}
    gamma = ostep.hv_gamma(w.hv_c, w.alpha, w.h)
    a = w.dt / w.mu0
    Hn = w.H0.copy()
    Hn[need] = ostep.h_update(w.E0, w.H0, op, a, gamma, rows=need)
    pos = np.searchsorted(need, smp)
    sub = {k: v[pos] for k, v in op.items()}
    keep = ostep.pec_keep(w.flags[smp], w.dim)
    E1o = ostep.e_update(w.E0, Hn, sub, w.dt / w.eps0, gamma, keep, rows=smp)
    escale = np.abs(w.E0).max()
    hscale = max(np.abs(Hn[need]).max(), 1e-300)
    dE = np.abs(E1[smp] - E1o).max() / escale
    dH = np.abs(H1[smp] - Hn[smp]).max() / hscale
    print(f"  one FP32 step vs FP64 oracle: E {dE:.2e} H {dH:.2e} (relative to field scale)", flush=True)
    assert dE < 1e-5 and dH < 1e-5


def test_pulse_2d_1M_sampled():
    _check(configs.pulse_2d(scale=1.0), 150, 1)


def test_cube_3d_8M_sampled():
    _check(configs.tm111_3d(scale=1.0), 60, 2)
