"""GPU discrete adjoint vs the FP64 oracle adjoint, checkpointing, and finite
differences (2D TMz, soft sources, receivers, per-node eps_r)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_18205_amd import Solver, MaxwellFn, AdjointProblem, _abi  # noqa: E402
from oracle import setup as osetup, step as ostep  # noqa: E402
from synth import configs  # noqa: E402


def _problem(ns=21, steps=80):
    w = configs.adjoint_2d(n_side=ns, steps=steps, chat=1e-3, n=12, n_rcv=3)
    w.src_node = np.concatenate([w.src_node, configs._fields.nearest_node(w.xyz, np.array([[0.3, 0.6]]))])
    w.src_amp = np.array([1.0, -0.5])
    w.src_wave = np.concatenate([w.src_wave, 0.7 * w.src_wave[::-1]], axis=1)
    return w


def _solver(w, prec="f64"):
    s = Solver.from_workload(w, precision=prec, adjoint=True)
    oh, oe = osetup.operators(w)
    p = s.perm
    s.set_weights(_abi.OP_CURL_H, oh["curl_w"][p])
    s.set_weights(_abi.OP_HV_H, oh["hv_w"][p])
    return s, oh


def _forward(s, w, eps_r, amp, ckpt_every):
    st = s.state(np.zeros((w.N, 1)), np.zeros((w.N, 2)), eps_r=eps_r)
    out = s.run(st, w.steps, src=(w.src_node, amp, w.src_wave), rcv=w.rcv_node, ckpt_every=ckpt_every)
    return st, out


def test_adjoint_matches_oracle_and_checkpointing_is_exact():
    print("adjoint vs oracle", flush=True)
    w = _problem()
    s, oh = _solver(w)
    T = w.steps
    # data from eps_r = 1, misfit at the seeded eps_r
    _, d = _forward(s, w, np.ones(w.N), w.src_amp, T)
    d = d["traces"].cpu().numpy()
    C = math.ceil(math.sqrt(T))
    st, out = _forward(s, w, w.eps_r, w.src_amp, C)
    tr = out["traces"].cpu().numpy()
    gt = tr - d
    g_eps, g_amp = s.adjoint(st, T, out["ckpt"], C, torch.tensor(gt), src=(w.src_node, w.src_amp, w.src_wave),
                             rcv=w.rcv_node)
    # store-all schedule (one segment) gives the same bits
    st2, out2 = _forward(s, w, w.eps_r, w.src_amp, T)
    g2, a2 = s.adjoint(st2, T, out2["ckpt"], T, torch.tensor(gt), src=(w.src_node, w.src_amp, w.src_wave),
                       rcv=w.rcv_node)
    assert (g2 == g_eps).all() and (a2 == g_amp).all()
    # oracle adjoint on the same weights
    keep = ostep.pec_keep(w.flags, 2)
    gamma = ostep.hv_gamma(w.hv_c, w.alpha, w.h)
    og, oa, otr = ostep.adjoint_2d(np.zeros((w.N, 1)), np.zeros((w.N, 2)), oh, w.dt, T, gamma, w.eps_r, keep,
                                   src=(w.src_node, w.src_amp, w.src_wave), rcv=w.rcv_node, grad_traces=gt)
    assert np.abs(tr - otr).max() <= 1e-12 * np.abs(otr).max()
    eg = np.abs(g_eps - og).max() / np.abs(og).max()
    ea = np.abs(g_amp - oa).max() / np.abs(oa).max()
    print(f"  grad eps rel {eg:.2e}  grad amp rel {ea:.2e}", flush=True)
    assert eg < 1e-10 and ea < 1e-10


def test_adjoint_matches_central_differences():
    print("adjoint vs central differences (GPU forward)", flush=True)
    w = _problem()
    s, _ = _solver(w)
    T = w.steps
    _, d = _forward(s, w, np.ones(w.N), w.src_amp, T)
    d = d["traces"].cpu().numpy()

    def J(e, a):
        _, o = _forward(s, w, e, a, T)
        r = o["traces"].cpu().numpy() - d
        return 0.5 * float((r * r).sum())

    st, out = _forward(s, w, w.eps_r, w.src_amp, 9)
    gt = out["traces"].cpu().numpy() - d
    g_eps, g_amp = s.adjoint(st, T, out["ckpt"], 9, torch.tensor(gt), src=(w.src_node, w.src_amp, w.src_wave),
                             rcv=w.rcv_node)
    rng = np.random.default_rng(3)
    for q in range(2):
        v = rng.uniform(-1, 1, w.N)
        h = 1e-5
        fd = (J(w.eps_r + h * v, w.src_amp) - J(w.eps_r - h * v, w.src_amp)) / (2 * h)
        an = float((g_eps * v).sum())
        print(f"  eps dir {q}: fd {fd:.10e} adjoint {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-6 * abs(an)
    h = 1e-3
    e0 = np.array([1.0, 0.0])
    fd = (J(w.eps_r, w.src_amp + h * e0) - J(w.eps_r, w.src_amp - h * e0)) / (2 * h)
    assert abs(fd - g_amp[0]) <= 1e-8 * abs(g_amp[0])


def test_autograd_function_and_fp32_adjoint():
    print("torch.autograd bridge, FP32 adjoint vs FP64", flush=True)
    w = _problem()
    grads = {}
    for prec in ("f64", "f32"):
        s, _ = _solver(w, prec)
        prob = AdjointProblem(s, w.steps, w.src_node, w.src_wave, w.rcv_node)
        eps = torch.tensor(w.eps_r, dtype=torch.float64, requires_grad=True)
        amp = torch.tensor(w.src_amp, dtype=torch.float64, requires_grad=True)
        tr = MaxwellFn.apply(eps, amp, prob)
        loss = 0.5 * (tr.double() ** 2).sum()
        loss.backward()
        grads[prec] = (eps.grad.numpy().copy(), amp.grad.numpy().copy())
    ge = np.abs(grads["f32"][0] - grads["f64"][0]).max() / np.abs(grads["f64"][0]).max()
    ga = np.abs(grads["f32"][1] - grads["f64"][1]).max() / np.abs(grads["f64"][1]).max()
    print(f"  fp32 vs fp64 gradient rel: eps {ge:.2e} amp {ga:.2e}", flush=True)
    assert ge < 1e-3 and ga < 1e-4
