"""Oracle set-up for a workload: stencils and weights in original node order.

Collocated variants (RBF-FD, RBF-VFD; Section 5): one stencil per node, the
max(n, n_hv) nearest nodes of the node itself; the curl operators use its
first n entries and the hyperviscosity operator its first n_hv (both are
"the n nearest nodes", eq. 11, so the shorter list is a prefix of the longer).

Two-set variant (E and H on different node sets; not the paper's choice, which
keeps both fields on one set): the H update's curl stencil is the n nearest
E nodes of each H node, its hyperviscosity stencil the n_hv nearest H nodes,
and symmetrically for the E update.  All its weights are RBF-FD.
"""
import numpy as np

from . import knn as _knn
from . import weights as _w
from . import step as _step


def operators(w, mode=None):
    """Returns (op_h, op_e) dictionaries for ``oracle.step``."""
    mode = mode or w.mode
    period = w.period
    if mode in ("FD", "VFD"):
        ns = max(w.n, w.n_hv)
        idx = _knn.knn(w.xyz, ns, period=period)
        ci = idx[:, :w.n]
        hi = idx[:, :w.n_hv]
        cw = _w.curl_weights(w.xyz, w.xyz, ci, w.m, mode=mode, sigma=w.vfd_sigma, h=w.h,
                             period=period, frame_angle=w.frame_angle)
        hw = _w.hv_weights(w.xyz, w.xyz, hi, w.alpha, period=period)
        op = {"curl_idx": ci, "curl_w": cw, "hv_idx": hi, "hv_w": hw, "stencil": idx}
        return op, op
    if mode == "STAG2":
        XE, XH = w.xyz, w.xyz_h
        ci_h = _knn.knn(XE, w.n, centres=XH, period=period)
        hi_h = _knn.knn(XH, w.n_hv, period=period)
        ci_e = _knn.knn(XH, w.n, centres=XE, period=period)
        hi_e = _knn.knn(XE, w.n_hv, period=period)
        op_h = {"curl_idx": ci_h, "curl_w": _w.curl_weights(XE, XH, ci_h, w.m, period=period,
                                                           frame_angle=w.frame_angle),
                "hv_idx": hi_h, "hv_w": _w.hv_weights(XH, XH, hi_h, w.alpha, period=period)}
        op_e = {"curl_idx": ci_e, "curl_w": _w.curl_weights(XH, XE, ci_e, w.m, period=period,
                                                           frame_angle=w.frame_angle),
                "hv_idx": hi_e, "hv_w": _w.hv_weights(XE, XE, hi_e, w.alpha, period=period)}
        return op_h, op_e
    raise ValueError(mode)


def run_workload(w, op_h, op_e, steps=None, energy_every=0, use_eps=True, src=True,
                 rcv=True):
    """Run a workload's single-field forward problem with the oracle."""
    steps = w.steps if steps is None else steps
    gamma = _step.hv_gamma(w.hv_c, w.alpha, w.h) if w.alpha > 0 else 0.0
    if getattr(w, "pol", "TM") == "TE":
        keep = _step.pec_keep_te(w.flags) if w.bc == "PEC" else np.ones((w.N, 2))
        nrm = w.normals if w.bc == "PEC" else None
        E, Hz, en = _step.run_te(w.E0, w.H0, op_h, w.dt, steps, gamma, w.dt / w.eps0, keep, mu0=w.mu0,
                                 eps0=w.eps0, h=w.h, energy_every=energy_every, normals=nrm)
        return E, Hz, en, None
    keep = _step.pec_keep(w.flags, w.dim) if w.bc == "PEC" else np.ones((w.N, w.E0.shape[1]))
    kappa = w.dt / w.eps0
    if use_eps and w.eps_r is not None:
        kappa = w.dt / (w.eps0 * w.eps_r)
    s = None
    if src and w.src_node is not None:
        s = (w.src_node, w.src_amp, w.src_wave)
    r = w.rcv_node if (rcv and w.rcv_node is not None) else None
    h_h = w.h_h if w.h_h is not None else w.h
    nrm = w.normals if (w.bc == "PEC" and w.dim == 3) else None
    return _step.run(w.E0, w.H0, op_h, op_e, w.dt, steps, gamma, kappa, keep, mu0=w.mu0,
                     eps0=w.eps0, h_e=w.h, h_h=h_h, energy_every=energy_every, src=s, rcv=r, normals=nrm)


# ---------------------------------------------------------------------------
# Large node sets: the same weights, computed for slices of the centres in
# worker processes (fork start method; the inputs are inherited, each worker
# fills its rows of shared output arrays).  No arithmetic differs from the
# single-process calls: every row is one local system of weights.py.
# ---------------------------------------------------------------------------
_PW = {}


def _pw_rows(args):
    import numpy as _np
    b0, b1 = args
    g = _PW
    xyz, st = g["xyz"], g["st"]
    cw = _np.frombuffer(g["cw"], dtype=_np.float64).reshape(-1, xyz.shape[1], g["n"])
    cw[b0:b1] = _w.curl_weights(xyz, xyz[b0:b1], st[b0:b1, :g["n"]], g["m"])
    if g["alpha"] > 0:
        hw = _np.frombuffer(g["hw"], dtype=_np.float64).reshape(-1, g["n_hv"])
        hw[b0:b1] = _w.hv_weights(xyz, xyz[b0:b1], st[b0:b1, :g["n_hv"]], g["alpha"])
    return b1 - b0


def weights_parallel(xyz, stencils, n, m, n_hv, alpha, procs, chunk=16384):
    """(curl_w [N, d, n], hv_w [N, n_hv]) of the collocated RBF-FD operators
    for every node, from the stencil rows ``stencils`` (nearest first), with
    ``procs`` worker processes."""
    import multiprocessing as mp
    N, d = xyz.shape
    cw_buf = mp.RawArray("d", N * d * n)
    hw_buf = mp.RawArray("d", max(1, N * n_hv if alpha > 0 else 1))
    _PW.clear()
    _PW.update(xyz=xyz, st=stencils, cw=cw_buf, hw=hw_buf, n=n, m=m, n_hv=n_hv, alpha=alpha)
    jobs = [(b, min(N, b + chunk)) for b in range(0, N, chunk)]
    ctx = mp.get_context("fork")
    with ctx.Pool(max(1, int(procs))) as pool:
        done = sum(pool.map(_pw_rows, jobs))
    assert done == N
    cw = np.frombuffer(cw_buf, dtype=np.float64).reshape(N, d, n)
    hw = np.frombuffer(hw_buf, dtype=np.float64).reshape(N, n_hv) if alpha > 0 else None
    _PW.clear()
    return cw, hw
