"""Benchmark of the meshless FDTD hot path on one MI355X.

Default workload: the 2D TMz PEC unit-square cavity on ~1.0M Poisson-disk
nodes (h ~ 1e-3), RBF-FD curl weights with n = 25, m = 4, hyperviscosity
Delta^3 (n_hv = 57), Gaussian pulse (sigma = 20 h) at the centre, FP32 fields
and weights.  A step is one full leapfrog step (H update + E update, eq. 19)
over all nodes; inputs are resident in HBM before timing starts.

Prints ONE JSON line.  Besides the headline FP32 node-steps/s it reports the
FP64 rate on the same nodes, the FP32-vs-FP64 relative L2 difference after the
workload's 10^4 steps, the K = 64 batched rate (250k-node jittered grid), the
roofline of the dominant kernel (the H update) and the FP64 CPU oracle timed on
a bounded sample of the same workload.
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-steps/s (all field comps) + % HBM peak; FP32/batched vs FP64 at L2 err"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes_half(n, nh, d, sw, sf, fe, fh, which):
    """Algorithmic bytes per node of one half update (int32 union ELL).

    Index list (n_hv entries) + curl (d n) and HV (n_hv) weights + fields:
    the H update reads E and H and writes H, the E update reads E and H and
    writes E.  Both halves sum to the per-node-step figure
    2 n_hv s_i + 2 (d n + n_hv) s_w + 3 (F_E + F_H) s_f.
    """
    ns = max(n, nh)
    fields = (fe + 2 * fh) if which == 0 else (2 * fe + fh)
    return ns * 4 + (d * n + nh) * sw + fields * sf


def time_halves(s, st, reps, torch):
    """Average duration of each half-update kernel: reps back-to-back launches
    between one HIP event pair on the library's stream.  The field structs are
    built once and the ABI call is made directly, so the host enqueues far
    faster than the kernels run and no gaps enter the average; consecutive
    launches alternate the two buffers of each pair, as the step loop does,
    so that no launch rewrites the buffer its predecessor has just written."""
    stream = torch.cuda.current_stream()
    fa = st.struct()
    fb = st.struct()
    fb.cur = 1 - fa.cur
    sp = s.stream()
    out = []
    for which in (0, 1):
        s.half(st, which)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        rc = 0
        e0.record(stream)
        for r in range(reps):
            rc |= s.lib.rbffd_half(s.plan, ctypes.byref(fa if r % 2 == 0 else fb), which, sp)
        e1.record(stream)
        e1.synchronize()
        if rc:
            raise RuntimeError(f"rbffd_half failed ({rc})")
        out.append(e0.elapsed_time(e1) / reps * 1e-3)
    return out


def dispersion_l1(samples, every, jmax=45):
    """||err||_1 of the propagation speed (Section 6, eq. 24-26) from line
    samples [N_t, N_x]: Hann window in time, transform pairing e^{-ikx} with
    e^{+i omega t}, peak wavenumber per frequency, |omega/k - S_c| summed over
    j = 1..jmax."""
    import numpy as np
    e = np.asarray(samples, dtype=np.float64)
    nt, nx = e.shape
    spec = np.abs(np.fft.ifft(np.fft.fft(e * np.hanning(nt)[:, None], axis=1), axis=0))
    i = np.argmax(spec[1:jmax + 1], axis=1)
    om = 2 * math.pi * np.arange(1, jmax + 1) / (every * nt)
    with np.errstate(divide="ignore"):
        c = om / (2 * math.pi * i / nx)
    return float(np.abs(c - 1.0 / (10 * math.sqrt(2.0))).sum())


def counted_traffic(kernel):
    """HBM bytes per launch of ``kernel`` (e.g. "k_h2l<float,float>") from the
    committed counter summary: FETCH_SIZE and WRITE_SIZE, each scaled by what
    the same counter reads for the 2 GiB copy probe (the per-size request
    counts give the same bytes to 0.01 %).  None unless the step-kernel
    sources are the ones the counters were taken on (hash in the summary)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_pulse2d_1M.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ("step.hip", "common.h", "fields.h", "wpack.h"):
        h.update(open(os.path.join(ROOT, "paper_2508_18205_amd", "csrc", f), "rb").read())
    text = open(path).read()
    if f"(step.hip, common.h, fields.h, wpack.h): {h.hexdigest()[:16]}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(f"traffic_bytes_per_launch {kernel}:"):
            return float(line.split(":")[1])
    return None


def host_info():
    """nproc, usable cores, CPU model and OMP_NUM_THREADS of this host."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": model,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(w, seconds=15.0):
    """The FP64 CPU oracle on the headline workload itself (every node, the
    walls, n, m, alpha): its plain C leapfrog (oracle/cstep.c, OpenMP over
    nodes) timed over whole steps on all host threads, then on one thread.
    The oracle's set-up (cell-bucket stencils, numpy FP64 local solves split
    over a process pool of at most 16 workers) is not timed."""
    import numpy as np
    from oracle import cstep, knn, setup as osetup, step as ostep
    info = host_info()
    procs = max(1, min(16, info["usable_cores"] or 1))
    t0 = time.time()
    log(f"cpu oracle: set-up on {procs} worker processes")
    st = knn.knn_cells(w.xyz, max(w.n, w.n_hv))
    log(f"cpu oracle: stencils in {time.time() - t0:.0f} s")
    cw, hw = osetup.weights_parallel(w.xyz, st, w.n, w.m, w.n_hv, w.alpha, procs)
    log(f"cpu oracle: weights, set-up {time.time() - t0:.0f} s")
    op = cstep.Operator({"curl_idx": st[:, :w.n], "curl_w": cw, "hv_idx": st[:, :w.n_hv], "hv_w": hw})
    del st, cw, hw
    t_setup = time.time() - t0
    gamma = ostep.hv_gamma(w.hv_c, w.alpha, w.h)
    keep = ostep.pec_keep(w.flags, 2)[:, 0]
    threads = cstep.threads()

    def timed(T):
        t = time.time()
        cstep.run(w.E0, w.H0, op, w.dt, T, gamma, w.dt / w.eps0, keep, mu0=w.mu0, eps0=w.eps0)
        return time.time() - t

    per = timed(2) / 2
    T = max(3, int(seconds / per))
    dt_all = timed(T)
    cstep.set_threads(1)
    T1 = max(2, int(seconds / 3 / (per * threads)))
    dt_one = timed(T1)
    cstep.set_threads(threads)
    log(f"cpu oracle: {threads} threads {w.N * T / dt_all:.3e} node-steps/s, one thread {w.N * T1 / dt_one:.3e}")
    return {"value": w.N * T / dt_all, "unit": "node-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole headline workload ({w.N} nodes with walls, n={w.n}, m={w.m}, alpha={w.alpha}, "
                      f"n_hv={w.n_hv}, FP64): the C oracle step (oracle/cstep.c, OpenMP over nodes) for {T} steps "
                      f"in {dt_all:.1f} s on {threads} threads; set-up {t_setup:.0f} s untimed",
            "one_core": {"value": w.N * T1 / dt_one, "steps": T1, "seconds": round(dt_one, 2)},
            "host": info}


def golden(tag):
    """The FP64 oracle's stored results of a full-size run (tests/golden):
    tag a3 / a2 (the 1M-node pulse), "tm111_3d_8M" (the 3D cube) or
    "batch64_250k" (four fields of the K = 64 batch workload)."""
    import numpy as np
    name = tag if tag.startswith(("tm111", "batch64")) else f"pulse2d_1M_{tag}"
    path = os.path.join(ROOT, "tests", "golden", f"{name}.npz")
    return np.load(path) if os.path.exists(path) else None


def vs_oracle(s, st, energy, g, whole_vector=False):
    """Relative differences of a GPU run from the oracle's stored run: E and H
    at the sampled nodes (relative L2 over the sample, worst component, or
    over all components together with ``whole_vector``), the energy series,
    and the random projections of the whole fields."""
    import numpy as np
    E, H = s.E_original(st), s.H_original(st)
    nodes = g["nodes"]

    def rel(x, ref):
        if whole_vector:
            return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
        return max(float(np.linalg.norm(x[:, c] - ref[:, c]) / np.linalg.norm(ref[:, c])) for c in range(ref.shape[1]))

    gv = np.random.default_rng(int(g["proj_seed"])).standard_normal((g["projE"].shape[1], E.shape[0]))
    pE = np.stack([gv @ E[:, c] for c in range(E.shape[1])])
    pH = np.stack([gv @ H[:, c] for c in range(H.shape[1])])

    def prel(p, ref):
        if whole_vector:
            return float(np.linalg.norm(p - ref) / np.linalg.norm(ref))
        return max(float(np.sqrt(((p[c] - ref[c]) ** 2).mean() / (ref[c] ** 2).mean())) for c in range(ref.shape[0]))

    return {"sampled_rel_l2_E": rel(E[nodes], g["E"]), "sampled_rel_l2_H": rel(H[nodes], g["H"]),
            "energy_rel_max": float(np.abs(np.asarray(energy) / g["energy"] - 1.0).max()),
            "whole_field_rel_l2_E_est": prel(pE, g["projE"]), "whole_field_rel_l2_H_est": prel(pH, g["projH"])}


def kernels_only(args):
    """Average duration of each half-update kernel of the named plans, with
    the same autotuned variant the benchmark uses, from rbffd_half launches
    alone (no graph replay): the process runs only the set-up, the tuner and
    these launches, for per-kernel profiler counters."""
    import numpy as np
    import torch
    from synth import configs
    from paper_2508_18205_amd import Solver
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    out = {}
    for name in args.kernels.split(","):
        if name == "copy":
            # the streaming copy probe: 10 copies of 2 GiB
            import ctypes as _ct
            from paper_2508_18205_amd import _abi as _ab
            lib = _ab.load()
            ca = torch.ones(1 << 29, dtype=torch.float32, device="cuda:0")
            cb = torch.empty_like(ca)
            sp = _ct.c_void_p(torch.cuda.current_stream().cuda_stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                _ab.check(lib.rbffd_stream_copy(_ct.c_void_p(ca.data_ptr()), _ct.c_void_p(cb.data_ptr()),
                                                ca.numel() * 4, sp))
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / 10
            out[name] = {"bytes_each_way": ca.numel() * 4, "avg_us": round(us, 2),
                         "GBs": round(2 * ca.numel() * 4 / (us * 1e-6) / 1e9, 1)}
            log(f"copy: {out[name]}")
            del ca, cb
            torch.cuda.empty_cache()
            continue
        if name == "batch64":
            # the K = 64 batch on the 250k-node set: whole steps (H and E
            # updates), launched one by one
            wb = configs.batched_2d(scale=args.scale, K=64)
            sb = Solver.from_workload(wb, precision="f32", K=64)
            stb = sb.state_batched(wb.E0_batch, np.zeros((64, wb.N, 2)))
            if not args.no_tune:
                sb.autotune(stb, reps=3)
                stb = sb.state_batched(wb.E0_batch, np.zeros((64, wb.N, 2)))
            sb.step(stb, 1)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            sb.step(stb, args.kernel_reps)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / args.kernel_reps
            out[name] = {"N": wb.N, "K": 64, "step_us": round(us, 2),
                         "field_node_steps_per_s": wb.N * 64 / (us * 1e-6), "variant": sb.variant()}
            log(f"{name}: {out[name]}")
            del sb, stb
            torch.cuda.empty_cache()
            continue
        wl, _, prec = name.partition("_")
        w = configs.pulse_2d(scale=args.scale) if wl == "pulse2d" else configs.tm111_3d(scale=args.scale, chat=1e-3)
        kw = {"weights": "w22"} if prec == "w22" else {}
        s = Solver.from_workload(w, precision="f32" if prec == "w22" else prec, **kw)
        st = s.state(w.E0, w.H0)
        if not args.no_tune:
            s.autotune(st, reps=3)
            st = s.state(w.E0, w.H0)
        th, te = time_halves(s, st, args.kernel_reps, torch)
        out[name] = {"N": w.N, "h_update_us": round(th * 1e6, 2), "e_update_us": round(te * 1e6, 2),
                     "variant": s.variant()}
        log(f"{name}: {out[name]}")
        del s, st
        torch.cuda.empty_cache()
    print(json.dumps({"kernels": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "bf16"])
    ap.add_argument("--scale", type=float, default=1.0, help="node-count scale of the workload (1 = 1M)")
    ap.add_argument("--accuracy-steps", type=int, default=10000)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip every leg after the headline one")
    ap.add_argument("--legs", default="fp64,accuracy,alpha2,w22,cavity,batched,bf16,adjoint,stag2,hv_scan,dispersion,disk,te,3d",
                    help="comma-separated extra legs to run after the headline measurement")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--kernels", default=None,
                    help="profiling mode: only time the half-step kernels, launched one by one (no graph replay), "
                         "for a comma-separated list of pulse2d_f32, pulse2d_f64, pulse2d_w22, cube3d_f32, "
                         "cube3d_f64 (and copy: the 2 GiB streaming copy probe; batch64: whole steps of the K = 64 "
                         "batch); prints one JSON line of average launch times")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library has no multi-GPU path "
              f"(one process drives one GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from synth import configs
    from paper_2508_18205_amd import Solver

    if args.kernels:
        return kernels_only(args)
    t0 = time.time()
    w = configs.pulse_2d(scale=args.scale)
    t_gen = time.time() - t0
    log(f"workload: N={w.N} h={w.h:.3e} n={w.n} m={w.m} alpha={w.alpha} n_hv={w.n_hv} (generated in {t_gen:.1f} s)")
    # the CPU oracle first, before anything initialises the GPU (its set-up
    # forks worker processes)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w)
        log(f"cpu baseline: {cpu}")
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")

    def setup_w(wl, prec):
        torch.cuda.synchronize()
        t = time.time()
        s = Solver.from_workload(wl, precision=prec)
        torch.cuda.synchronize()
        return s, time.time() - t

    def setup(prec):
        return setup_w(w, prec)

    def finite_or_null(o):
        # strict JSON has no NaN/Infinity: a diverged run reports null
        if isinstance(o, dict):
            return {k: finite_or_null(v) for k, v in o.items()}
        if isinstance(o, (list, tuple)):
            return [finite_or_null(v) for v in o]
        if isinstance(o, float) and not math.isfinite(o):
            return None
        return o

    def rl2(x, y):
        ny = np.linalg.norm(y)
        return float(np.linalg.norm(x - y) / ny) if ny > 0 and np.isfinite(ny) else float("nan")

    s, t_setup = setup(args.precision)
    st = s.state(w.E0, w.H0)
    log(f"setup ({args.precision}): {t_setup:.2f} s")
    variant = None
    if not args.no_tune:
        variant = s.autotune(st, reps=10)
        st = s.state(w.E0, w.H0)
        log(f"tuned variant: {variant}")
    s.run(st, args.warmup, use_graph=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.time()
    e0.record(stream)
    s.run(st, args.steps, use_graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.time() - t_wall
    elapsed = e0.elapsed_time(e1) * 1e-3
    value = w.N * args.steps / elapsed
    log(f"timed {args.steps} steps: {elapsed * 1e3:.2f} ms ({value:.4e} node-steps/s; wall {t_wall * 1e3:.1f} ms)")
    # five more timed runs of the same K steps: their median, for context
    reps = []
    for _ in range(5):
        e0.record(stream)
        s.run(st, args.steps, use_graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(w.N * args.steps / (e0.elapsed_time(e1) * 1e-3))
    repeat_median = float(np.median(reps))

    # roofline of the dominant kernel (H update) from HIP events on the same stream
    th, te = time_halves(s, st, args.kernel_reps, torch)
    sw = 8 if args.precision == "f64" else 4
    sf = {"f64": 8, "f32": 4, "bf16": 2}[args.precision]
    bh = alg_bytes_half(w.n, w.n_hv, w.dim, sw, sf, 1, 2, 0) * w.N
    be = alg_bytes_half(w.n, w.n_hv, w.dim, sw, sf, 1, 2, 1) * w.N
    gbs_h = bh / th / 1e9
    gbs_e = be / te / 1e9
    log(f"H update {th * 1e6:.1f} us -> {gbs_h:.0f} GB/s ; E update {te * 1e6:.1f} us -> {gbs_e:.0f} GB/s")
    dominant = "H" if th >= te else "E"
    ach = gbs_h if dominant == "H" else gbs_e
    staged = bool(s.variant()["lds"]) and s.sizes.N == w.N
    kname = ("k_h2l" if dominant == "H" else "k_e2l") if staged else ("k_h2" if dominant == "H" else "k_e2")
    traffic = None
    if staged and args.precision == "f32" and args.scale == 1.0:
        traffic = counted_traffic(kname + "<float,float>")
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by the same counter read for the 2 GiB stream copy; profiles/traffic_pulse2d_1M.md)",
            "kernel": f"{kname}<float,float> ({'H' if dominant == 'H' else 'E'} update)",
            "alg_bytes_per_launch": int(bh if dominant == "H" else be),
            "avg_launch_us": round((th if dominant == "H" else te) * 1e6, 2),
            "other_half": {"achieved": round(gbs_e if dominant == "H" else gbs_h, 1),
                           "avg_launch_us": round((te if dominant == "H" else th) * 1e6, 2)}}
    if traffic:
        # the staged kernels read 16-bit halo positions instead of the int32
        # indices the algorithmic count assumes: the counted rate is lower
        cgbs = traffic / (th if dominant == "H" else te) / 1e9
        roof["counted_GBs"] = round(cgbs, 1)
        roof["counted_frac"] = round(cgbs / HBM_PEAK_GBS, 4)
    # measured streaming ceiling: the library's 16-byte copy kernel over 2 GiB
    # (read + write bytes / time)
    from paper_2508_18205_amd import _abi as _ab
    lib = _ab.load()
    ca = torch.empty(1 << 29, dtype=torch.float32, device=dev)
    cb = torch.empty_like(ca)
    ca.fill_(1.0)
    nb_ = ca.numel() * 4
    sp = ctypes.c_void_p(stream.cuda_stream)
    for _ in range(3):
        _ab.check(lib.rbffd_stream_copy(ctypes.c_void_p(ca.data_ptr()), ctypes.c_void_p(cb.data_ptr()), nb_, sp))
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(10):
        lib.rbffd_stream_copy(ctypes.c_void_p(ca.data_ptr()), ctypes.c_void_p(cb.data_ptr()), nb_, sp)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * nb_ * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    assert bool((cb == 1.0).all())
    roof["copy_ceiling_GBs"] = round(copy_gbs, 1)
    if "counted_GBs" in roof:
        roof["counted_frac_of_copy_ceiling"] = round(roof["counted_GBs"] / copy_gbs, 4)
    del ca, cb
    torch.cuda.empty_cache()
    log(f"device copy ceiling: {copy_gbs:.0f} GB/s")

    extras = {}
    legs = set() if args.no_extras else set(x for x in args.legs.split(",") if x)
    def timed_rate(sv, wl, steps, tune):
        stv = sv.state(wl.E0, wl.H0)
        if tune and not args.no_tune:
            sv.autotune(stv, reps=5)
            stv = sv.state(wl.E0, wl.H0)
        sv.run(stv, min(args.warmup, 100), use_graph=True)
        torch.cuda.synchronize()
        e0.record(stream)
        sv.run(stv, steps, use_graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        return wl.N * steps / (e0.elapsed_time(e1) * 1e-3)

    def oracle_run(sv, wl, g):
        stv = sv.state(wl.E0, wl.H0)
        r = sv.run(stv, int(g["steps"]), energy_every=int(g["energy_every"]), use_graph=True)
        return vs_oracle(sv, stv, r["energy"], g)

    if legs & {"fp64", "accuracy"}:
        # FP64 rate on the same nodes; both precisions against the FP64
        # oracle's own full-size run of this configuration (2000 steps: the
        # pulse has not reached a wall, and the FP64 energy of this
        # configuration first leaves [0, 1.01] near step 7000)
        s64, t64 = setup("f64")
        v64 = timed_rate(s64, w, args.steps, True)
        extras["fp64"] = {"value": v64, "unit": "node-steps/s", "setup_s": round(t64, 2),
                          "fp32_over_fp64": round(value / v64, 3)}
        log(f"fp64: {extras['fp64']}")
        g3 = golden("a3")
        if "accuracy" in legs and g3 is not None:
            acc = {"steps": int(g3["steps"]), "reference": "FP64 CPU oracle run of this configuration "
                   "(tests/golden/pulse2d_1M_a3.npz)", "sampled_nodes": int(g3["nodes"].size)}
            acc["f32"] = oracle_run(s, w, g3)
            acc["f64"] = oracle_run(s64, w, g3)
            # over the configured 10^4 steps the energy of this configuration
            # grows without bound: say where it leaves [0, 1.01]
            T = args.accuracy_steps
            a64 = s64.state(w.E0, w.H0)
            r64 = s64.run(a64, T, energy_every=100, use_graph=True)
            u64 = r64["energy"] / r64["energy"][0]
            grown = np.nonzero(~(u64 <= 1.01))[0]
            acc["configured_steps"] = T
            acc["fp64_energy_above_1.01_at_step"] = int(grown[0]) * 100 if grown.size else None
            extras["accuracy_vs_oracle"] = acc
            log(f"accuracy vs oracle (configured, alpha = {w.alpha}): {acc}")
        del s64
        torch.cuda.empty_cache()
    if "alpha2" in legs:
        # the same nodes and curl stencils with alpha = 2 (n_hv = 31, chat =
        # 3e-3), energy-stable over the configured 10^4 steps: FP32 and FP64
        # rates and their errors against the oracle's 10^4-step run
        g2 = golden("a2")
        ws = configs.Workload(w.name, w.dim, w.xyz, w.flags, w.h, w.n, w.m, 2, 31, 3e-3, args.accuracy_steps)
        ws.E0, ws.H0 = w.E0, w.H0
        a2 = {"alpha": 2, "n_hv": 31, "chat": 3e-3}
        for prec in ("f32", "f64", "bf16"):
            sv = Solver.from_workload(ws, precision=prec)
            a2[f"value_{prec}"] = timed_rate(sv, ws, args.steps, True)
            if g2 is not None:
                a2[f"vs_oracle_{prec}"] = oracle_run(sv, ws, g2)
            del sv
            torch.cuda.empty_cache()
        a2["fp32_over_fp64"] = round(a2["value_f32"] / a2["value_f64"], 3)
        if g2 is not None:
            a2["steps"] = int(g2["steps"])
            a2["oracle_energy_ratio_range"] = [float((g2["energy"] / g2["energy"][0]).min()),
                                               float((g2["energy"] / g2["energy"][0]).max())]
        extras["alpha2"] = a2
        log(f"alpha = 2 variant: {a2}")
    if "w22" in legs:
        # compressed weights: four 22-bit mantissas and one shared exponent per
        # 4-slot chunk (12 bytes instead of 16), FP32 fields and arithmetic, on
        # the headline workload; the per-kernel roofline counts 3 bytes per
        # weight; accuracy against both oracle runs
        sw = Solver.from_workload(w, precision="f32", weights="w22")
        v22 = timed_rate(sw, w, args.steps, True)
        stw = sw.state(w.E0, w.H0)
        th22, te22 = time_halves(sw, stw, args.kernel_reps, torch)
        bh22 = alg_bytes_half(w.n, w.n_hv, w.dim, 3, 4, 1, 2, 0) * w.N
        be22 = alg_bytes_half(w.n, w.n_hv, w.dim, 3, 4, 1, 2, 1) * w.N
        leg = {"value": v22, "unit": "node-steps/s", "over_fp32_weights": round(v22 / value, 3),
               "variant": sw.variant(), "alg_bytes_per_node_h": alg_bytes_half(w.n, w.n_hv, w.dim, 3, 4, 1, 2, 0),
               "h_update_us": round(th22 * 1e6, 2), "e_update_us": round(te22 * 1e6, 2),
               "h_update_GBs": round(bh22 / th22 / 1e9, 1), "e_update_GBs": round(be22 / te22 / 1e9, 1),
               "h_update_frac": round(bh22 / th22 / 1e9 / HBM_PEAK_GBS, 4)}
        t22 = counted_traffic("k_h2l<float,w22>")
        if t22:
            leg["h_update_traffic"] = t22
            leg["h_update_counted_GBs"] = round(t22 / th22 / 1e9, 1)
        g3 = golden("a3")
        if g3 is not None:
            leg["vs_oracle_configured"] = oracle_run(sw, w, g3)
        del sw, stw
        torch.cuda.empty_cache()
        g2 = golden("a2")
        if g2 is not None:
            ws = configs.Workload(w.name, w.dim, w.xyz, w.flags, w.h, w.n, w.m, 2, 31, 3e-3, int(g2["steps"]))
            ws.E0, ws.H0 = w.E0, w.H0
            sw = Solver.from_workload(ws, precision="f32", weights="w22")
            leg["vs_oracle_alpha2"] = oracle_run(sw, ws, g2)
            del sw
            torch.cuda.empty_cache()
        extras["w22_weights"] = leg
        log(f"w22 weights: {leg}")
    if "cavity" in legs:
        # the 2D cavity at its configured size: 51^2 jittered nodes, n = 12,
        # m = 2, alpha = 2, TM_11 for one period (1000 steps), FP64; collocated
        # RBF-FD and two node sets (50^2 H nodes); error against the mode
        from synth import fields as _fields
        cav = {}
        for mode in ("FD", "STAG2"):
            wc = configs.tm_cavity_2d(mode=mode)
            sc, _ = setup_w(wc, "f64")
            stc = sc.state(wc.E0, wc.H0)
            if not args.no_tune:
                sc.autotune(stc, reps=20)
                stc = sc.state(wc.E0, wc.H0)
            sc.run(stc, 20, use_graph=True)
            stc = sc.state(wc.E0, wc.H0)
            torch.cuda.synchronize()
            e0.record(stream)
            sc.run(stc, wc.steps, use_graph=True)
            e1.record(stream)
            torch.cuda.synchronize()
            tc = e0.elapsed_time(e1) * 1e-3
            Ea, Ha, _ = _fields.tm_mode_2d(wc.xyz, wc.steps * wc.dt, (wc.steps - 0.5) * wc.dt)
            Ec = sc.E_original(stc)
            cav[mode] = {"N_E": wc.N, "N_H": int(wc.xyz_h.shape[0]) if wc.xyz_h is not None else wc.N,
                         "steps": wc.steps, "us_per_step": round(tc / wc.steps * 1e6, 2),
                         "node_steps_per_s": wc.N * wc.steps / tc, "linf_E_vs_TM11": float(np.abs(Ec - Ea).max()),
                         "variant": sc.variant()}
            if mode == "FD":
                cav[mode]["linf_H_vs_TM11"] = float(np.abs(sc.H_original(stc) - Ha).max())
            del sc, stc
        extras["cavity_2d"] = cav
        log(f"cavity: {cav}")
    if "batched" in legs:
        # K = 64 fields sharing one weight set (250k-node jittered grid)
        wb = configs.batched_2d(scale=1.0, K=64)
        sb = Solver.from_workload(wb, precision="f32", K=64)
        stb = sb.state_batched(wb.E0_batch, np.zeros((64, wb.N, 2)))
        vb = sb.autotune(stb, reps=5) if not args.no_tune else sb.variant()
        stb = sb.state_batched(wb.E0_batch, np.zeros((64, wb.N, 2)))
        sb.run(stb, 20, use_graph=True)
        torch.cuda.synchronize()
        kb = 200
        e0.record(stream)
        sb.run(stb, kb, use_graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        tb = e0.elapsed_time(e1) * 1e-3
        # the configured steps from the initial fields, four fields against
        # the oracle's single-field runs of their pulses
        gb = golden("batch64_250k")
        acc_b = None
        if gb is not None and int(gb["steps"]) == wb.steps:
            stb = sb.state_batched(wb.E0_batch, np.zeros((64, wb.N, 2)))
            rb = sb.run(stb, wb.steps, energy_every=int(gb["energy_every"]), use_graph=True)
            Eb, Hb = sb.to_original(stb.E)[:, 0, :], sb.to_original(stb.H)
            enb = np.asarray(rb["energy"])
            nb = gb["nodes"]
            gvb = np.random.default_rng(int(gb["proj_seed"])).standard_normal((gb["projE"].shape[-1], wb.N))
            acc_b = {"steps": wb.steps, "fields": [int(k) for k in gb["fields"]]}
            worst = dict(sampled_rel_l2_E=0.0, sampled_rel_l2_H=0.0, energy_rel_max=0.0,
                         whole_field_rel_l2_E_est=0.0, whole_field_rel_l2_H_est=0.0)
            for j, k in enumerate(gb["fields"]):
                refE, refH = gb["E"][j], gb["H"][j]
                pE = gvb @ Eb[:, k]
                pH = np.stack([gvb @ Hb[:, c, k] for c in range(2)])
                vals = dict(
                    sampled_rel_l2_E=float(np.linalg.norm(Eb[nb, k] - refE[:, 0]) / np.linalg.norm(refE[:, 0])),
                    sampled_rel_l2_H=max(float(np.linalg.norm(Hb[nb, c, k] - refH[:, c]) / np.linalg.norm(refH[:, c]))
                                         for c in range(2)),
                    energy_rel_max=float(np.abs(enb[:, k] / gb["energy"][j] - 1.0).max()),
                    whole_field_rel_l2_E_est=float(np.sqrt(((pE - gb["projE"][j][0]) ** 2).mean()
                                                           / (gb["projE"][j][0] ** 2).mean())),
                    whole_field_rel_l2_H_est=max(float(np.sqrt(((pH[c] - gb["projH"][j][c]) ** 2).mean()
                                                               / (gb["projH"][j][c] ** 2).mean())) for c in range(2)))
                worst = {key: max(worst[key], vals[key]) for key in worst}
            acc_b.update(worst)
            acc_b["oracle_reference"] = ("FP64 CPU oracle single-field runs of these pulses "
                                         "(tests/golden/batch64_250k.npz); worst of the four fields")
        del sb, stb
        torch.cuda.empty_cache()
        # one field on the same nodes and weights: 64 such runs are the alternative
        s1 = Solver.from_workload(wb, precision="f32")
        st1 = s1.state(wb.E0_batch[0], np.zeros((wb.N, 2)))
        if not args.no_tune:
            s1.autotune(st1, reps=5)
            st1 = s1.state(wb.E0_batch[0], np.zeros((wb.N, 2)))
        s1.run(st1, 20, use_graph=True)
        torch.cuda.synchronize()
        e0.record(stream)
        s1.run(st1, kb, use_graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        t1 = e0.elapsed_time(e1) * 1e-3
        del s1, st1
        extras["batched"] = {"value": wb.N * 64 * kb / tb, "unit": "field-node-steps/s", "K": 64, "N": wb.N,
                             "single_field_node_steps_per_s": wb.N * kb / t1,
                             "speedup_vs_64_single_runs": round(64 * t1 / tb, 2),
                             "variant": vb,
                             "steps": kb, "node_steps_per_s": wb.N * kb / tb,
                             "alg_bytes_per_field_node_step": 50.0,
                             "hbm_frac_at_50B": round(wb.N * 64 * kb / tb * 50.0 / (HBM_PEAK_GBS * 1e9), 4),
                             "vs_oracle": acc_b}
        log(f"batched: {extras['batched']}")
        torch.cuda.empty_cache()
    if "bf16" in legs:
        # BF16 field storage (FP32 weights and arithmetic) on the headline workload
        sbf, tbf = setup("bf16")
        abf = sbf.state(w.E0, w.H0)
        sbf.run(abf, args.warmup, use_graph=True)
        torch.cuda.synchronize()
        e0.record(stream)
        sbf.run(abf, args.steps, use_graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        extras["bf16_storage"] = {"value": w.N * args.steps / (e0.elapsed_time(e1) * 1e-3), "unit": "node-steps/s",
                                  "note": "accuracy in accuracy_alpha2 (BF16 updates below the BF16 ulp stagnate)"}
        log(f"bf16: {extras['bf16_storage']}")
        del sbf, abf
        torch.cuda.empty_cache()
    if "adjoint" in legs:
        # 250k-node adjoint workload: FP32 forward with sqrt(T) checkpoints and
        # the discrete adjoint; FP64 gradient checked by central differences
        wa = configs.adjoint_2d(scale=1.0, chat=1e-3)
        d_res = {}
        for prec in ("f32", "f64"):
            sa = Solver.from_workload(wa, precision=prec, adjoint=True)
            src = (wa.src_node, wa.src_amp, wa.src_wave)
            C = int(math.ceil(math.sqrt(wa.steps)))
            st0 = sa.state(np.zeros((wa.N, 1)), np.zeros((wa.N, 2)), eps_r=np.ones(wa.N))
            dat = sa.run(st0, wa.steps, src=src, rcv=wa.rcv_node)["traces"].clone()
            stf = sa.state(np.zeros((wa.N, 1)), np.zeros((wa.N, 2)), eps_r=wa.eps_r)
            torch.cuda.synchronize()
            e0.record(stream)
            out = sa.run(stf, wa.steps, src=src, rcv=wa.rcv_node, ckpt_every=C)
            e1.record(stream)
            torch.cuda.synchronize()
            t_fwd = e0.elapsed_time(e1) * 1e-3
            gt = out["traces"] - dat
            e0.record(stream)
            g_eps, g_amp = sa.adjoint(stf, wa.steps, out["ckpt"], C, gt, src=src, rcv=wa.rcv_node)
            e1.record(stream)
            torch.cuda.synchronize()
            t_adj = e0.elapsed_time(e1) * 1e-3
            d_res[prec] = dict(t_fwd=t_fwd, t_adj=t_adj, g=g_eps, a=g_amp)
            if prec == "f64":
                rng = np.random.default_rng(7)
                v = rng.uniform(-1, 1, wa.N)
                hh = 1e-6

                def J(e):
                    stj = sa.state(np.zeros((wa.N, 1)), np.zeros((wa.N, 2)), eps_r=e)
                    r = sa.run(stj, wa.steps, src=src, rcv=wa.rcv_node)["traces"] - dat
                    return 0.5 * float((r * r).sum())

                fd = (J(wa.eps_r + hh * v) - J(wa.eps_r - hh * v)) / (2 * hh)
                an = float((g_eps * v).sum())
                d_res["fd"] = (fd, an)
            del sa, st0, stf, out
            torch.cuda.empty_cache()
        fd, an = d_res["fd"]
        g32, g64 = d_res["f32"]["g"], d_res["f64"]["g"]
        extras["adjoint"] = {
            "N": wa.N, "steps": wa.steps, "receivers": len(wa.rcv_node), "ckpt_every": int(math.ceil(math.sqrt(wa.steps))),
            "forward_ms_f32": round(d_res["f32"]["t_fwd"] * 1e3, 2), "adjoint_ms_f32": round(d_res["f32"]["t_adj"] * 1e3, 2),
            "gradient_node_steps_per_s_f32": wa.N * wa.steps / (d_res["f32"]["t_fwd"] + d_res["f32"]["t_adj"]),
            "forward_ms_f64": round(d_res["f64"]["t_fwd"] * 1e3, 2), "adjoint_ms_f64": round(d_res["f64"]["t_adj"] * 1e3, 2),
            "fd_check_f64": {"central_difference": fd, "adjoint": an, "rel_diff": abs(fd - an) / abs(an)},
            "grad_eps_f32_vs_f64_rel": float(np.abs(g32 - g64).max() / np.abs(g64).max()),
            "grad_amp_f32_vs_f64_rel": float(np.abs(d_res["f32"]["a"] - d_res["f64"]["a"]).max()
                                             / np.abs(d_res["f64"]["a"]).max())}
        log(f"adjoint: {extras['adjoint']}")
    if "stag2" in legs:
        # two node sets (E on a 1000^2 jittered grid, H on its 999^2 cell centres)
        from synth import nodes as _nodes
        xe, fe_, he = _nodes.jittered_grid((1000, 1000), seed=8)
        xh, fh_, hh_ = _nodes.dual_grid_2d(999, seed=8)
        w2 = configs.Workload("stag2", 2, xe, fe_, he, 12, 2, 2, 31, 1e-3, 100, mode="STAG2")
        w2.xyz_h, w2.flags_h, w2.h_h = xh, fh_, hh_
        w2.E0 = np.zeros((w2.N, 1))
        w2.H0 = np.zeros((xh.shape[0], 2))
        s2 = Solver.from_workload(w2, precision="f32")
        a2 = s2.state(w2.E0, w2.H0)
        s2.run(a2, 10, use_graph=True)
        torch.cuda.synchronize()
        e0.record(stream)
        s2.run(a2, 200, use_graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        t2 = e0.elapsed_time(e1) * 1e-3
        extras["two_set"] = {"N_E": w2.N, "N_H": int(xh.shape[0]), "n": 12, "n_hv": 31,
                             "node_steps_per_s": (w2.N + xh.shape[0]) / 2 * 200 / t2,
                             "ms_per_step": t2 / 200 * 1e3}
        log(f"two-set: {extras['two_set']}")
        del s2, a2
        torch.cuda.empty_cache()
    if "hv_scan" in legs:
        # hyperviscosity parameter search on the 1M-node set: K = 64 values of
        # c per round advanced together (per-field gamma, per-field energy)
        scans = {}
        Ts = w.steps
        # the node-sum energy of the PEC cavity swings by about 1% as the pulse
        # meets the walls, so the alpha = 2 search also runs with a 2% band
        for alpha, nhv, lo, hi, rounds, band in ((w.alpha, w.n_hv, 1e-8, 1e-1, 1, (0.99, 1.01)),
                                                 (2, 31, 1e-7, 1e-1, 1, (0.99, 1.01)),
                                                 (2, 31, 1e-7, 1e-1, 2, (0.98, 1.02))):
            ws_ = configs.Workload(w.name, w.dim, w.xyz, w.flags, w.h, w.n, w.m, alpha, nhv, 1e-3, Ts)
            sk = Solver.from_workload(ws_, precision="f32", K=64)
            # the scan fills the buffers from (E0, H0) itself
            from paper_2508_18205_amd.solver import State
            zE = torch.zeros((w.N, 1, 64), dtype=torch.float32, device=dev)
            zH = torch.zeros((w.N, 2, 64), dtype=torch.float32, device=dev)
            stk = State([zE, torch.zeros_like(zE)], [zH, torch.zeros_like(zH)], 0, None)
            torch.cuda.synchronize()
            t0 = time.time()
            r = sk.hv_scan(stk, w.E0, w.H0, lo / w.dt, hi / w.dt, rounds, Ts, 100, band)
            tsc = time.time() - t0
            acc = [float(c * w.dt) for c, o in zip(r["c"].ravel(), r["ok"].ravel()) if o]
            scans[f"alpha{alpha}_band{round((band[1] - 1) * 100)}pct"] = {
                "n_hv": nhv, "chat_range": [lo, hi], "K": 64, "rounds_done": int(len(r["c"])), "steps": Ts,
                "band": list(band), "status": r["status"],
                "chat_best": (r["c_best"] * w.dt) if r["c_best"] else None,
                "chat_bracket": [r["bracket"][0] * w.dt, r["bracket"][1] * w.dt],
                "accepted_chat_round1": [float(c * w.dt) for c, o in zip(r["c"][0], r["ok"][0]) if o],
                "accepted_total": len(acc),
                "umax_min_round1": float(np.min(r["umax"][0])),
                "chat_at_umax_min_round1": float(r["c"][0][int(np.argmin(r["umax"][0]))] * w.dt),
                "umin_there": float(r["umin"][0][int(np.argmin(r["umax"][0]))]),
                "scan_s": round(tsc, 2),
                "field_node_steps_per_s": w.N * 64 * Ts * len(r["c"]) / tsc}
            del sk, stk
            torch.cuda.empty_cache()
        extras["hv_scan"] = scans
        log(f"hv scan: {scans}")
    if "dispersion" in legs:
        # Section 6: line-seeded periodic [0, 200)^2 (40.7k nodes), sigma = 2
        # pulse, 2820 steps, E on the 200 line nodes every 15 steps; the
        # paper's hyperviscosity constants; FP32
        disp = {}
        for mode in ("FD", "VFD"):
            for nn in (13, 20, 30, 60):
                wd = configs.dispersion_2d(n=nn, mode=mode)
                sd = Solver.from_workload(wd, precision="f32")
                sdt = sd.state(wd.E0, wd.H0)
                if not args.no_tune:
                    sd.autotune(sdt, reps=10)
                    sdt = sd.state(wd.E0, wd.H0)
                sd.run(sdt, 20, use_graph=True)
                sdt = sd.state(wd.E0, wd.H0)
                torch.cuda.synchronize()
                e0.record(stream)
                rd = sd.run(sdt, wd.steps, energy_every=20, rcv=wd.rcv_node, use_graph=True)
                e1.record(stream)
                torch.cuda.synchronize()
                td = e0.elapsed_time(e1) * 1e-3
                tr = rd["traces"].double().cpu().numpy()[wd.meta["save_every"] - 1::wd.meta["save_every"]]
                u = rd["energy"] / rd["energy"][0]
                disp[f"{mode}_n{nn}"] = {"err_l1": dispersion_l1(tr, wd.meta["save_every"]),
                                         "u_min": float(np.nanmin(u)), "u_max": float(np.nanmax(u)),
                                         "node_steps_per_s": wd.N * wd.steps / td}
                del sd, sdt
        # angle study (eq. 27, Figure 12): the curl in the frame turned by
        # -phi, n = 60, phi from 0 to pi/4
        for mode in ("FD", "VFD"):
            row = {}
            for q in range(5):
                phi = q * math.pi / 16
                wd = configs.dispersion_2d(n=60, mode=mode, phi=phi)
                sd = Solver.from_workload(wd, precision="f32")
                sdt = sd.state(wd.E0, wd.H0)
                rd = sd.run(sdt, wd.steps, energy_every=20, rcv=wd.rcv_node, use_graph=True)
                tr = rd["traces"].double().cpu().numpy()[wd.meta["save_every"] - 1::wd.meta["save_every"]]
                u = rd["energy"] / rd["energy"][0]
                row[f"{q}pi/16"] = {"err_l1": dispersion_l1(tr, wd.meta["save_every"]),
                                    "u_min": float(np.nanmin(u)), "u_max": float(np.nanmax(u))}
                del sd, sdt
            disp[f"angle_{mode}_n60"] = row
        wd = configs.dispersion_2d(n=60, mode="FD")
        disp["N"] = wd.N
        disp["chat"] = {"FD": 10 ** -4.76, "VFD": 10 ** -5.02}
        # the hyperviscosity search on the same node sets (K = 64 candidates per
        # round, 10^4 steps as in Section 6, band 5 %: with the paper's 1 % band
        # no c qualifies on these nodes)
        for mode in ("FD", "VFD"):
            wd = configs.dispersion_2d(n=60, mode=mode)
            sk = Solver.from_workload(wd, precision="f32", K=64)
            from paper_2508_18205_amd.solver import State
            zE = torch.zeros((wd.N, 1, 64), dtype=torch.float32, device=dev)
            zH = torch.zeros((wd.N, 2, 64), dtype=torch.float32, device=dev)
            stk = State([zE, torch.zeros_like(zE)], [zH, torch.zeros_like(zH)], 0, None)
            r = sk.hv_scan(stk, wd.E0, wd.H0, 1e-8 / wd.dt, 1e-2 / wd.dt, 2, 10000, 50, (0.95, 1.05))
            disp[f"hv_scan_{mode}_n60"] = {
                "band": [0.95, 1.05], "steps": 10000, "status": r["status"],
                "chat_best": (r["c_best"] * wd.dt) if r["c_best"] else None,
                "chat_bracket": [r["bracket"][0] * wd.dt, r["bracket"][1] * wd.dt]}
            del sk, stk
        extras["dispersion"] = disp
        log(f"dispersion: {disp}")
    if "disk" in legs:
        # curved PEC wall: circular cavity with ~0.5M nodes, one period, FP32,
        # error against the Bessel solution: TM_01 (TMz) and TE_01 (TEz, wall
        # nodes keep the normal component of E)
        from synth import fields as _fields
        # and the coaxial cavity 0.5 <= r <= 1 (a conducting cylinder inside)
        coax = {pol: (lambda h, pol=pol: configs.coax_2d(pol=pol, h=h),
                      lambda x, te, th, pol=pol: _fields.coax_mode(x, te, th, pol=pol)) for pol in ("TM", "TE")}
        for key, make, exact in (("tm01_disk", configs.tm01_disk, _fields.tm01_disk),
                                 ("te01_disk", configs.te01_disk, _fields.te01_disk),
                                 ("coax_tm01", coax["TM"][0], coax["TM"][1]),
                                 ("coax_te01", coax["TE"][0], coax["TE"][1]),
                                 ("sphere_3d", configs.sphere_3d, _fields.sphere_mode)):
            # the 3D sphere (curved 3D wall) at h = 0.02: ~0.55M nodes
            wk = make(h=0.02) if key == "sphere_3d" else make(h=0.0025)
            sk, tk = setup_w(wk, "f32")
            ak = sk.state(wk.E0, wk.H0)
            if not args.no_tune:
                sk.autotune(ak, reps=5)
                ak = sk.state(wk.E0, wk.H0)
            torch.cuda.synchronize()
            e0.record(stream)
            sk.run(ak, wk.steps, use_graph=True)
            e1.record(stream)
            torch.cuda.synchronize()
            tk2 = e0.elapsed_time(e1) * 1e-3
            Ea, Ha, _ = exact(wk.xyz, wk.steps * wk.dt, (wk.steps - 0.5) * wk.dt)
            Ek, Hk = sk.E_original(ak), sk.H_original(ak)
            extras[key] = {"N": wk.N, "steps": wk.steps, "node_steps_per_s": wk.N * wk.steps / tk2,
                           "linf_E_vs_bessel": float(np.abs(Ek - Ea).max()),
                           "linf_H_vs_bessel": float(np.abs(Hk - Ha).max()), "setup_s": round(tk, 2)}
            log(f"disk: {key} {extras[key]}")
            del sk, ak
            torch.cuda.empty_cache()
    if "te" in legs:
        # TEz polarisation: TE_11 mode of the PEC square on a 1001^2 jittered
        # grid (1.0M nodes, n = 12, n_hv = 31), one period, FP32
        from synth import fields as _fields
        wt = configs.te_cavity_2d(n_side=1001, chat=1e-3)
        st_, tt = setup_w(wt, "f32")
        at = st_.state(wt.E0, wt.H0)
        if not args.no_tune:
            st_.autotune(at, reps=5)
            at = st_.state(wt.E0, wt.H0)
        torch.cuda.synchronize()
        e0.record(stream)
        st_.run(at, wt.steps, use_graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        tte = e0.elapsed_time(e1) * 1e-3
        Ea, Ha, _ = _fields.te_mode_2d(wt.xyz, wt.steps * wt.dt, (wt.steps - 0.5) * wt.dt)
        extras["te_cavity"] = {"N": wt.N, "steps": wt.steps, "node_steps_per_s": wt.N * wt.steps / tte,
                               "linf_E_vs_TE11": float(np.abs(st_.E_original(at) - Ea).max()),
                               "linf_Hz_vs_TE11": float(np.abs(st_.H_original(at) - Ha).max()),
                               "variant": st_.variant()}
        log(f"te: {extras['te_cavity']}")
        del st_, at
        torch.cuda.empty_cache()
    if "3d" in legs:
        # 3D cube, 8.0M nodes, FP32 rate and FP32 vs FP64 over the workload's 2000 steps
        w3 = configs.tm111_3d(scale=1.0, chat=1e-3)
        r3 = {}
        for prec in ("f32", "f64"):
            s3, t3 = setup_w(w3, prec)
            a3 = s3.state(w3.E0, w3.H0)
            if not args.no_tune:
                s3.autotune(a3, reps=3)
                a3 = s3.state(w3.E0, w3.H0)
            s3.run(a3, 10, use_graph=True)
            torch.cuda.synchronize()
            e0.record(stream)
            s3.run(a3, 200, use_graph=True)
            e1.record(stream)
            torch.cuda.synchronize()
            rate = w3.N * 200 / (e0.elapsed_time(e1) * 1e-3)
            th3, te3 = time_halves(s3, a3, 10, torch)
            a3 = s3.state(w3.E0, w3.H0)
            g3 = golden("tm111_3d_8M")
            ev3 = int(g3["energy_every"]) if g3 is not None else 0
            rr3 = s3.run(a3, w3.steps, energy_every=ev3, use_graph=True)
            r3[prec] = dict(rate=rate, setup=t3, th=th3, te=te3, E=s3.E_original(a3), H=s3.H_original(a3),
                            variant=s3.variant(),
                            vs_oracle=(vs_oracle(s3, a3, rr3["energy"], g3, whole_vector=True)
                                       if g3 is not None and int(g3["steps"]) == w3.steps else None))
            del s3, a3
            torch.cuda.empty_cache()
        sw3 = 4
        bh3 = alg_bytes_half(w3.n, w3.n_hv, 3, sw3, 4, 3, 3, 0) * w3.N
        bh3d = alg_bytes_half(w3.n, w3.n_hv, 3, 8, 8, 3, 3, 0) * w3.N
        extras["tm111_3d"] = {
            "N": w3.N, "n": w3.n, "n_hv": w3.n_hv, "value_f32": r3["f32"]["rate"], "value_f64": r3["f64"]["rate"],
            "unit": "node-steps/s", "fp32_over_fp64": round(r3["f32"]["rate"] / r3["f64"]["rate"], 3),
            "setup_s_f32": round(r3["f32"]["setup"], 2),
            "h_update_us": round(r3["f32"]["th"] * 1e6, 1), "e_update_us": round(r3["f32"]["te"] * 1e6, 1),
            "h_update_GBs": round(bh3 / r3["f32"]["th"] / 1e9, 1),
            "h_update_frac": round(bh3 / r3["f32"]["th"] / 1e9 / HBM_PEAK_GBS, 4),
            "variant_f32": r3["f32"]["variant"], "variant_f64": r3["f64"]["variant"],
            "h_update_us_f64": round(r3["f64"]["th"] * 1e6, 1), "e_update_us_f64": round(r3["f64"]["te"] * 1e6, 1),
            "h_update_GBs_f64": round(bh3d / r3["f64"]["th"] / 1e9, 1),
            "h_update_frac_f64": round(bh3d / r3["f64"]["th"] / 1e9 / HBM_PEAK_GBS, 4),
            "steps_accuracy": w3.steps,
            "fp32_vs_fp64_rel_l2_E": rl2(r3["f32"]["E"], r3["f64"]["E"]),
            "fp32_vs_fp64_rel_l2_H": rl2(r3["f32"]["H"], r3["f64"]["H"]),
            "vs_oracle_f32": r3["f32"]["vs_oracle"], "vs_oracle_f64": r3["f64"]["vs_oracle"],
            "oracle_reference": "FP64 CPU oracle run of this configuration (tests/golden/tm111_3d_8M.npz); "
                                "relative L2 over all three components"}
        log(f"3D: {extras['tm111_3d']}")

    line = {
        "metric": METRIC, "value": value, "unit": "node-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"pulse_2d: 2D TMz PEC unit square, {w.N} Poisson-disk nodes (h={w.h:.3e}), "
                               f"RBF-FD n={w.n} m={w.m}, hyperviscosity alpha={w.alpha} n_hv={w.n_hv}, "
                               f"Gaussian pulse sigma=20h, {args.precision} fields and weights",
                   "N": w.N, "n": w.n, "m": w.m, "alpha": w.alpha, "n_hv": w.n_hv, "setup_s": round(t_setup, 2),
                   "variant": variant},
        "repeat_median_value": repeat_median,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    line.update(extras)
    print(json.dumps(finite_or_null(line)), flush=True)


if __name__ == "__main__":
    main()
