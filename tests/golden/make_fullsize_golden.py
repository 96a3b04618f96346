"""Writes the FP64 oracle's results for full-size runs of the 1M-node pulse.

Calls only ``oracle`` (stencils, weights, the C leapfrog, the energy) and
``synth`` (the seeded node set and initial field); nothing here touches the
GPU library.  Output: one ``.npz`` per run in this directory, read by
tests/test_gpu_fullsize_parity.py and by the benchmark:

  pulse2d_1M_a3.npz   the workload as configured: ~1.0M Poisson-disk nodes on
                      the PEC unit square, n = 25, m = 4, hyperviscosity
                      alpha = 3 (n_hv = 57), chat = 1e-4, Gaussian pulse
                      sigma = 20 h at the centre, 2000 steps (the pulse has not
                      reached a wall; the FP64 energy of this configuration
                      first leaves [0, 1.01] near step 7000)
  pulse2d_1M_a2.npz   the same nodes and curl stencils with alpha = 2
                      (n_hv = 31), chat = 3e-3, 10^4 steps (energy-stable)
  tm111_3d_8M.npz     the 3D cube: 200^3 jittered nodes on the PEC unit cube,
                      n = 35, m = 2, alpha = 2 (n_hv = 71), chat = 1e-3, the
                      TM_111 mode, 2000 steps
  batch64_250k.npz    the K-field batch workload: 500^2 jittered nodes on the
                      PEC unit square, n = 25, m = 2, alpha = 2 (n_hv = 31),
                      chat = 1e-4, 64 seeded Gaussian pulses (sigma = 20 h),
                      the configured 5000 steps; fields 0, 21, 42 and 63 are
                      run (each is a single-field run of its pulse) and stored
                      with a leading field axis

Each file holds: the sampled node ids (original order) and the oracle's E
[S, 1], H [S, 2] there after the last step; the energy U^n of eq. 20 every
``energy_every`` steps; random projections P[c, j] = sum_i g_j,i F_i,c of
each full field component on 8 seeded standard normal vectors g_j (numpy
default_rng(seed 2508) drawn as [8, N]), which turn any widespread
difference into a global relative L2 estimate; and the run's parameters.

Usage:  python tests/golden/make_fullsize_golden.py [a3] [a2] [c3] [b4]
(about 15, 40, 75 and 5 minutes on 8 cores; c3 needs ~30 GB of memory).
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import cstep, knn, step as ostep, weights as OW  # noqa: E402
from synth import configs  # noqa: E402

PROJ_SEED = 2508
N_PROJ = 8


def projections(F, g):
    """[comp, N_PROJ] sums of each component against the seeded vectors."""
    return np.stack([g @ F[:, c] for c in range(F.shape[1])])


def sample_nodes(w, seed, n_uniform, n_centre, r_centre):
    rng = np.random.default_rng(seed)
    a = rng.choice(w.N, size=n_uniform, replace=False)
    near = np.flatnonzero(np.linalg.norm(w.xyz - 0.5, axis=1) < r_centre)
    b = rng.choice(near, size=min(n_centre, near.size), replace=False) if n_centre else np.empty(0, np.int64)
    return np.unique(np.concatenate([a, b, [0, w.N - 1]])).astype(np.int64)


def log(*a):
    print(*a, flush=True)


def run_one(tag, w, alpha, n_hv, chat, steps, energy_every, stencils, curl_w, smp):
    t0 = time.time()
    hw = OW.hv_weights(w.xyz, w.xyz, stencils[:, :n_hv], alpha)
    log(f"[{tag}] hv weights (alpha={alpha}, n_hv={n_hv}) {time.time() - t0:.0f} s")
    op = cstep.Operator({"curl_idx": stencils[:, :w.n], "curl_w": curl_w, "hv_idx": stencils[:, :n_hv],
                         "hv_w": hw})
    del hw
    gamma = ostep.hv_gamma(chat / w.dt, alpha, w.h)
    keep = ostep.pec_keep(w.flags, 2)[:, 0]
    t0 = time.time()

    def progress(n, E, H):
        if n % 500 == 0:
            log(f"[{tag}] step {n}/{steps} ({time.time() - t0:.0f} s)")

    E, H, en = cstep.run(w.E0, w.H0, op, w.dt, steps, gamma, w.dt / w.eps0, keep, mu0=w.mu0, eps0=w.eps0, h=w.h,
                         energy_every=energy_every, callback=progress)
    g = np.random.default_rng(PROJ_SEED).standard_normal((N_PROJ, w.N))
    out = os.path.join(HERE, f"pulse2d_1M_{tag}.npz")
    np.savez_compressed(out, nodes=smp, E=E[smp], H=H[smp], energy=en, energy_every=energy_every,
                        projE=projections(E, g), projH=projections(H, g), N=w.N, steps=steps, alpha=alpha,
                        n_hv=n_hv, chat=chat, n=w.n, m=w.m, proj_seed=PROJ_SEED,
                        threads=cstep.threads(), run_s=time.time() - t0)
    log(f"[{tag}] wrote {out}: {steps} steps in {time.time() - t0:.0f} s; u range "
        f"[{(en / en[0]).min():.6f}, {(en / en[0]).max():.6f}]")


def run_cube(procs=8):
    """The 8M-node 3D cube (tm111_3d as the benchmark runs it), 2000 steps."""
    from oracle import setup as osetup
    t0 = time.time()
    w = configs.tm111_3d(scale=1.0, chat=1e-3)
    log(f"[c3] nodes: N={w.N} h={w.h:.4e} ({time.time() - t0:.0f} s)")
    t0 = time.time()
    stencils = knn.knn_cells(w.xyz, max(w.n, w.n_hv))
    log(f"[c3] stencils (n_s = {stencils.shape[1]}) {time.time() - t0:.0f} s")
    t0 = time.time()
    curl_w, hv_w = osetup.weights_parallel(w.xyz, stencils, w.n, w.m, w.n_hv, w.alpha, procs)
    log(f"[c3] weights {time.time() - t0:.0f} s")
    op = cstep.Operator({"curl_idx": stencils[:, :w.n], "curl_w": curl_w, "hv_idx": stencils[:, :w.n_hv],
                         "hv_w": hv_w})
    del curl_w, hv_w
    gamma = ostep.hv_gamma(w.hv_c, w.alpha, w.h)
    keep = ostep.pec_keep(w.flags, 3)
    steps, every = w.steps, 100
    t0 = time.time()

    def progress(n, E, H):
        if n % 100 == 0:
            log(f"[c3] step {n}/{steps} ({time.time() - t0:.0f} s)")

    E, H, en = cstep.run(w.E0, w.H0, op, w.dt, steps, gamma, w.dt / w.eps0, keep, mu0=w.mu0, eps0=w.eps0, h=w.h,
                         energy_every=every, callback=progress)
    smp = sample_nodes(w, 33, 4000, 0, 0.0)
    g = np.random.default_rng(PROJ_SEED).standard_normal((N_PROJ, w.N))
    out = os.path.join(HERE, "tm111_3d_8M.npz")
    np.savez_compressed(out, nodes=smp, E=E[smp], H=H[smp], energy=en, energy_every=every,
                        projE=projections(E, g), projH=projections(H, g), N=w.N, steps=steps, alpha=w.alpha,
                        n_hv=w.n_hv, chat=w.chat, n=w.n, m=w.m, proj_seed=PROJ_SEED,
                        threads=cstep.threads(), run_s=time.time() - t0)
    log(f"[c3] wrote {out}: {steps} steps in {time.time() - t0:.0f} s; u range "
        f"[{(en / en[0]).min():.6f}, {(en / en[0]).max():.6f}]")


BATCH_FIELDS = (0, 21, 42, 63)


def run_batch(procs=8):
    """Fields of the K = 64 batch workload (batched_2d as the benchmark runs
    it), each run alone for the configured 5000 steps."""
    from oracle import setup as osetup
    t0 = time.time()
    w = configs.batched_2d(scale=1.0)
    stencils = knn.knn_cells(w.xyz, max(w.n, w.n_hv))
    curl_w, hv_w = osetup.weights_parallel(w.xyz, stencils, w.n, w.m, w.n_hv, w.alpha, procs)
    log(f"[b4] N={w.N} K={w.K}: stencils and weights {time.time() - t0:.0f} s")
    op = cstep.Operator({"curl_idx": stencils[:, :w.n], "curl_w": curl_w, "hv_idx": stencils[:, :w.n_hv],
                         "hv_w": hv_w})
    del curl_w, hv_w
    gamma = ostep.hv_gamma(w.hv_c, w.alpha, w.h)
    keep = ostep.pec_keep(w.flags, 2)[:, 0]
    steps, every = w.steps, 100
    smp = sample_nodes(w, 34, 2000, 0, 0.0)
    g = np.random.default_rng(PROJ_SEED).standard_normal((N_PROJ, w.N))
    Es, Hs, ens, pE, pH = [], [], [], [], []
    for k in BATCH_FIELDS:
        t0 = time.time()
        E, H, en = cstep.run(w.E0_batch[k], np.zeros((w.N, 2)), op, w.dt, steps, gamma, w.dt / w.eps0, keep,
                             mu0=w.mu0, eps0=w.eps0, h=w.h, energy_every=every)
        Es.append(E[smp]); Hs.append(H[smp]); ens.append(en)
        pE.append(projections(E, g)); pH.append(projections(H, g))
        log(f"[b4] field {k}: {steps} steps in {time.time() - t0:.0f} s; u range "
            f"[{(en / en[0]).min():.6f}, {(en / en[0]).max():.6f}]")
    out = os.path.join(HERE, "batch64_250k.npz")
    np.savez_compressed(out, nodes=smp, fields=np.array(BATCH_FIELDS), E=np.stack(Es), H=np.stack(Hs),
                        energy=np.stack(ens), energy_every=every, projE=np.stack(pE), projH=np.stack(pH), N=w.N,
                        K=w.K, steps=steps, alpha=w.alpha, n_hv=w.n_hv, chat=w.chat, n=w.n, m=w.m,
                        proj_seed=PROJ_SEED, threads=cstep.threads())
    log(f"[b4] wrote {out}")


def main(which):
    if "b4" in which:
        run_batch()
        which = [x for x in which if x != "b4"]
        if not which:
            return
    if "c3" in which:
        run_cube()
        which = [x for x in which if x != "c3"]
        if not which:
            return
    t0 = time.time()
    w = configs.pulse_2d(scale=1.0)
    log(f"nodes: N={w.N} h={w.h:.4e} ({time.time() - t0:.0f} s)")
    t0 = time.time()
    stencils = knn.knn_cells(w.xyz, max(w.n, w.n_hv))
    log(f"stencils (n_s = {stencils.shape[1]}) {time.time() - t0:.0f} s")
    t0 = time.time()
    curl_w = OW.curl_weights(w.xyz, w.xyz, stencils[:, :w.n], w.m)
    log(f"curl weights {time.time() - t0:.0f} s")
    if "a3" in which:
        smp = sample_nodes(w, 31, 2000, 2000, 0.15)
        run_one("a3", w, w.alpha, w.n_hv, w.chat, 2000, 100, stencils, curl_w, smp)
    if "a2" in which:
        smp = sample_nodes(w, 32, 4000, 0, 0.0)
        run_one("a2", w, 2, 31, 3e-3, 10000, 100, stencils, curl_w, smp)


if __name__ == "__main__":
    main(sys.argv[1:] or ["a3", "a2"])
