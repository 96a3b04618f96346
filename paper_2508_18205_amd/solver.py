"""Thin Python front end of librbffd (argument marshalling only).

PyTorch provides device memory and the stream; every step of the method runs
in the library's HIP kernels.  Arrays handed in by the caller are in the
caller's (original) node order; the library keeps state in its internal
(reordered) order and ``to_internal`` / ``to_original`` convert with the
library's own permutation kernel.
"""
import ctypes as C
import math
import os

import numpy as np
import torch

from . import _abi
from ._abi import check

_TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class State:
    """Ping-pong field buffers; E[cur], H[cur] hold the current (E^n, H^n)."""

    def __init__(self, E, H, cur=0, eps_r=None):
        self.Eb = E          # list of two tensors
        self.Hb = H
        self.cur = cur
        self.eps_r = eps_r

    @property
    def E(self):
        return self.Eb[self.cur]

    @property
    def H(self):
        return self.Hb[self.cur]

    def struct(self):
        f = _abi.Fields()
        f.E[0], f.E[1] = self.Eb[0].data_ptr(), self.Eb[1].data_ptr()
        f.H[0], f.H[1] = self.Hb[0].data_ptr(), self.Hb[1].data_ptr()
        f.cur = self.cur
        f.eps_r = self.eps_r.data_ptr() if self.eps_r is not None else None
        return f


class Solver:
    """One plan: node set, parameters, weights resident on the GPU."""

    def __init__(self, dim, xyz, flags, h, n, m, alpha, hv_c, lo, hi, *, n_hv=0, dt=0.0, mode="FD",
                 bc="PEC", eps0=1.0, mu0=1.0, vfd_sigma=0.5, phs_k=3, precision="f64", K=1,
                 adjoint=False, reorder="MORTON", xyz_h=None, flags_h=None, h_h=0.0, pol="TM", frame_angle=0.0,
                 normals=None, weights=None, device="cuda:0"):
        self.lib = _abi.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the rbffd library needs a GPU (no CPU path)")
        self.device = torch.device(device)
        self.precision = precision
        self.dtype = _TORCH[precision]
        self.cdtype = torch.float64 if precision == "f64" else torch.float32
        p = _abi.Params()
        p.dim, p.mode, p.n, p.m, p.phs_k = dim, _abi.MODE[mode], n, m, phs_k
        p.hv_alpha, p.n_hv, p.bc, p.reorder = alpha, n_hv, _abi.BC[bc], _abi.ORDER[reorder]
        # weight storage: FP64 with FP64 fields, else FP32, or "w22" (compressed
        # FP32 weights: 22-bit mantissas, one exponent per 4-slot chunk)
        p.wdtype = 0 if precision == "f64" else (_abi.W22 if weights == "w22" else 1)
        p.fdtype = _abi.DTYPE[precision]
        p.K, p.adjoint = K, int(bool(adjoint))
        p.pol = {"TM": 0, "TE": 1}[pol]
        p.frame_angle = frame_angle
        p.vfd_sigma, p.hv_c, p.h, p.h_h, p.dt, p.eps0, p.mu0 = vfd_sigma, hv_c, h, h_h, dt, eps0, mu0
        for k in range(dim):
            p.lo[k], p.hi[k] = lo[k], hi[k]
        self.params = p
        self.dim = dim
        self.K = K
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.flags = np.ascontiguousarray(flags, dtype=np.uint8)
        plan = C.c_void_p()
        xh = fh = None
        NH = 0
        if mode == "STAG2":
            xh = np.ascontiguousarray(xyz_h, dtype=np.float64)
            fh = np.ascontiguousarray(flags_h, dtype=np.uint8) if flags_h is not None else np.zeros(len(xh), np.uint8)
            NH = xh.shape[0]
        self._keep = (self.xyz, self.flags, xh, fh)
        rc = self.lib.rbffd_plan_create(C.byref(p), self.xyz.shape[0], self.xyz.ctypes.data,
                                        self.flags.ctypes.data, NH,
                                        xh.ctypes.data if xh is not None else None,
                                        fh.ctypes.data if fh is not None else None, C.byref(plan))
        check(rc, None, "rbffd_plan_create")
        self.plan = plan
        if normals is not None:
            nrm = np.ascontiguousarray(normals, dtype=np.float64)
            assert nrm.shape == (self.xyz.shape[0], dim)
            check(self.lib.rbffd_set_wall_normals(plan, nrm.ctypes.data), plan, "set_wall_normals")
        s = _abi.Sizes()
        check(self.lib.rbffd_plan_sizes(plan, C.byref(s)), plan, "plan_sizes")
        self.sizes = s
        self.N, self.NH = s.N, s.N_h
        self.FE, self.FH = s.fe, s.fh
        self.pol = pol
        self.fe = (2 if pol == "TE" else 1) if dim == 2 else 3
        self.fh = (1 if pol == "TE" else 2) if dim == 2 else 3
        self.dt, self.gamma = s.dt, s.gamma
        with torch.cuda.device(self.device):
            self.arena = torch.empty(max(s.arena_bytes, 256), dtype=torch.uint8, device=self.device)
            self.ws = torch.empty(max(s.workspace_bytes, 256), dtype=torch.uint8, device=self.device)
            check(self.lib.rbffd_weights(plan, _ptr(self.arena), _ptr(self.ws), self.stream()), plan, "rbffd_weights")
        self.perm = self.get_perm(0)
        self.inv = np.empty_like(self.perm)
        self.inv[self.perm] = np.arange(self.perm.size, dtype=self.perm.dtype)
        if mode == "STAG2":
            self.perm_h = self.get_perm(1)

    @classmethod
    def from_workload(cls, w, precision="f64", **kw):
        args = dict(n_hv=w.n_hv, mode=w.mode, bc=w.bc, eps0=w.eps0, mu0=w.mu0, vfd_sigma=w.vfd_sigma,
                    precision=precision, xyz_h=w.xyz_h, flags_h=w.flags_h, h_h=w.h_h or 0.0,
                    pol=getattr(w, "pol", "TM"), frame_angle=getattr(w, "frame_angle", 0.0),
                    normals=getattr(w, "normals", None) if w.bc == "PEC" else None)
        args.update(kw)
        return cls(w.dim, w.xyz, w.flags, w.h, w.n, w.m, w.alpha, w.hv_c, w.lo, w.hi, **args)

    def __del__(self):
        try:
            if getattr(self, "plan", None):
                self.lib.rbffd_plan_destroy(self.plan)
                self.plan = None
        except Exception:
            pass

    # ---- plumbing --------------------------------------------------------------
    def stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def sync(self):
        torch.cuda.synchronize(self.device)

    def get_perm(self, set_=0):
        n = self.N if set_ == 0 else self.NH
        out = np.empty(n, dtype=np.int32)
        check(self.lib.rbffd_get_perm(self.plan, set_, out.ctypes.data, self.stream()), self.plan, "get_perm")
        return out

    def stencils(self, which=_abi.ST_UNION):
        s = self.sizes
        shape = {0: (s.N, s.n_stencil), 1: (s.N_h, self.params.n), 2: (s.N_h, s.n_hv),
                 3: (s.N, self.params.n), 4: (s.N, s.n_hv)}[which]
        out = np.empty(shape, dtype=np.int32)
        check(self.lib.rbffd_get_stencils(self.plan, which, out.ctypes.data, self.stream()), self.plan,
              "get_stencils")
        return out

    def _wshape(self, op):
        s = self.sizes
        nt = s.N_h if op in (_abi.OP_CURL_H, _abi.OP_HV_H) and self.params.mode == 2 else s.N
        if op in (_abi.OP_CURL_H, _abi.OP_CURL_E):
            return (nt, self.dim, self.params.n)
        return (nt, s.n_hv)

    def weights(self, op):
        out = np.empty(self._wshape(op), dtype=np.float64)
        check(self.lib.rbffd_get_weights(self.plan, op, out.ctypes.data, self.stream()), self.plan, "get_weights")
        return out

    def set_weights(self, op, w):
        w = np.ascontiguousarray(w, dtype=np.float64)
        assert w.shape == self._wshape(op)
        check(self.lib.rbffd_set_weights(self.plan, op, w.ctypes.data, self.stream()), self.plan, "set_weights")

    def permute(self, t, set_=0, to_internal=True):
        out = torch.empty_like(t)
        n = self.N if set_ == 0 else self.NH
        eb = t.numel() * t.element_size() // n
        check(self.lib.rbffd_permute(self.plan, set_, int(to_internal), eb, _ptr(t), _ptr(out), self.stream()),
              self.plan, "permute")
        return out

    def to_internal(self, arr, width, set_=0, dtype=None):
        """[N, c] original-order values -> device tensor [N, width] in internal order."""
        a = np.asarray(arr, dtype=np.float64)
        if a.ndim == 1:
            a = a[:, None]
        n = a.shape[0]
        pad = np.zeros((n, width), dtype=np.float64)
        pad[:, :a.shape[1]] = a
        t = torch.tensor(pad, dtype=dtype or self.dtype, device=self.device)
        return self.permute(t, set_, True)

    def to_original(self, t, set_=0):
        """Device tensor in internal order -> numpy float64 in original order."""
        o = self.permute(t.contiguous(), set_, False)
        return o.to(torch.float64).cpu().numpy()

    # ---- state -------------------------------------------------------------------
    def state(self, E0, H0, eps_r=None):
        """Single-field state from original-order E0 [N, fe], H0 [N_h, fh]."""
        hset = 1 if self.params.mode == 2 else 0
        E = self.to_internal(E0, self.FE)
        H = self.to_internal(H0, self.FH, set_=hset)
        er = None
        if eps_r is not None:
            er = self.to_internal(np.asarray(eps_r)[:, None], 1, dtype=self.cdtype).reshape(-1).contiguous()
        return State([E, torch.zeros_like(E)], [H, torch.zeros_like(H)], 0, er)

    def state_batched(self, E0b, H0b):
        """K-field state from original-order E0b [K, N, 1], H0b [K, N, 2] -> [N, F, K]."""
        K = E0b.shape[0]
        assert K == self.K
        Et = torch.tensor(np.ascontiguousarray(np.transpose(E0b, (1, 2, 0))), dtype=self.dtype, device=self.device)
        Ht = torch.tensor(np.ascontiguousarray(np.transpose(H0b, (1, 2, 0))), dtype=self.dtype, device=self.device)
        E = self.permute(Et)
        H = self.permute(Ht)
        return State([E, torch.zeros_like(E)], [H, torch.zeros_like(H)], 0, None)

    def E_original(self, st):
        return self.to_original(st.E)[:, :self.fe]

    def H_original(self, st):
        return self.to_original(st.H, 1 if self.params.mode == 2 else 0)[:, :self.fh]

    # ---- the hot path ----------------------------------------------------------------
    def step(self, st, nsteps):
        f = st.struct()
        check(self.lib.rbffd_step(self.plan, C.byref(f), int(nsteps), self.stream()), self.plan, "rbffd_step")
        st.cur = f.cur
        return st

    def half(self, st, which):
        """One half update (0 = H, 1 = E) into the spare buffer; cur unchanged."""
        f = st.struct()
        check(self.lib.rbffd_half(self.plan, C.byref(f), int(which), self.stream()), self.plan, "rbffd_half")

    def run(self, st, T, energy_every=0, src=None, rcv=None, ckpt_every=0, use_graph=False,
            unstable_threshold=0.0):
        """Forward run.  src = (nodes [S] original ids, amps [S], wave [T, S]); rcv = nodes [R].

        Returns dict with 'energy' (numpy), 'traces' (tensor [T, R]) and
        'ckpt' (tensor of checkpoint slots) when requested.
        """
        a = _abi.RunArgs()
        a.T = int(T)
        out = {}
        keep = []
        if energy_every:
            ne = (T - 1) // energy_every + 1
            en = torch.zeros((ne, self.K) if self.K > 1 else ne, dtype=torch.float64, device=self.device)
            a.energy_every, a.energy_out = energy_every, en.data_ptr()
            out["energy_t"] = en
        if src is not None:
            nodes = torch.tensor(self.inv[np.asarray(src[0])].astype(np.int32), device=self.device)
            amp = torch.tensor(np.asarray(src[1], dtype=np.float64), dtype=self.cdtype, device=self.device)
            wave = torch.tensor(np.asarray(src[2], dtype=np.float64), dtype=self.cdtype, device=self.device)
            keep += [nodes, amp, wave]
            a.n_src, a.src_node, a.src_amp, a.src_wave = len(src[0]), nodes.data_ptr(), amp.data_ptr(), wave.data_ptr()
            out["src_dev"] = (nodes, amp, wave)
        if rcv is not None:
            rn = torch.tensor(self.inv[np.asarray(rcv)].astype(np.int32), device=self.device)
            tr = torch.zeros((T, len(rcv)), dtype=self.cdtype, device=self.device)
            keep += [rn]
            a.n_rcv, a.rcv_node, a.traces = len(rcv), rn.data_ptr(), tr.data_ptr()
            out["traces"] = tr
            out["rcv_dev"] = rn
        if ckpt_every:
            nslot = (T + ckpt_every - 1) // ckpt_every
            slot = self.sizes.e_bytes + self.sizes.h_bytes
            ck = torch.empty(nslot * slot, dtype=torch.uint8, device=self.device)
            a.ckpt, a.ckpt_every = ck.data_ptr(), ckpt_every
            out["ckpt"] = ck
        a.use_graph = int(bool(use_graph))
        a.unstable_threshold = unstable_threshold
        f = st.struct()
        check(self.lib.rbffd_run(self.plan, C.byref(f), C.byref(a), _ptr(self.ws), self.stream()), self.plan,
              "rbffd_run")
        st.cur = f.cur
        if energy_every:
            out["energy"] = out["energy_t"].cpu().numpy()
        return out

    def set_field_hv(self, c=None):
        """K-field batch: field k uses the hyperviscosity constant c[k] (None: the plan's c)."""
        ct = None
        if c is not None:
            ct = torch.tensor(np.asarray(c, dtype=np.float64).reshape(self.K), device=self.device)
        check(self.lib.rbffd_set_field_hv(self.plan, _ptr(ct) if ct is not None else None, self.stream()),
              self.plan, "rbffd_set_field_hv")
        self.sync()

    def hv_scan(self, st, E0, H0, c_lo, c_hi, rounds, T, energy_every, band=(0.99, 1.01)):
        """Search of the smallest accepted hyperviscosity constant (rbffd_hv_scan).

        st: a K-field state whose buffers are overwritten; E0 [N, fe], H0 [N, fh]
        one original-order initial state shared by every field.  Returns a dict
        with status ("bracketed", "below", "none"), c_best, bracket and per-round
        arrays c, ok, umin, umax [rounds_done, K].
        """
        K = self.K
        E0t = self.to_internal(E0, self.FE)
        H0t = self.to_internal(H0, self.FH)
        ne = (int(T) - 1) // int(energy_every) + 1
        cdev = torch.zeros(K, dtype=torch.float64, device=self.device)
        edev = torch.zeros(ne * K, dtype=torch.float64, device=self.device)
        ch = np.zeros((rounds, K))
        umin = np.zeros((rounds, K))
        umax = np.zeros((rounds, K))
        ok = np.zeros((rounds, K), dtype=np.int32)
        a = _abi.HvScanArgs()
        a.E0, a.H0, a.c_lo, a.c_hi = _ptr(E0t), _ptr(H0t), float(c_lo), float(c_hi)
        a.rounds, a.T, a.energy_every = int(rounds), int(T), int(energy_every)
        a.u_lo, a.u_hi = float(band[0]), float(band[1])
        a.c_dev, a.energy_dev = _ptr(cdev), _ptr(edev)
        a.c_host, a.umin_host, a.umax_host, a.ok_host = (ch.ctypes.data, umin.ctypes.data, umax.ctypes.data,
                                                         ok.ctypes.data)
        f = st.struct()
        check(self.lib.rbffd_hv_scan(self.plan, C.byref(f), C.byref(a), _ptr(self.ws), self.stream()), self.plan,
              "rbffd_hv_scan")
        st.cur = f.cur
        r = a.rounds_done
        return {"status": ("bracketed", "below", "none")[a.status], "c_best": a.c_best if a.c_best > 0 else None,
                "bracket": (a.bracket[0], a.bracket[1]), "c": ch[:r], "ok": ok[:r].astype(bool),
                "umin": umin[:r], "umax": umax[:r]}

    def adjoint(self, st_eps, T, ckpt, ckpt_every, grad_traces, src=None, rcv=None):
        """Gradients (grad_eps [N] original order, grad_amp [S]) of J(traces)."""
        a = _abi.AdjointArgs()
        a.T, a.ckpt_every, a.ckpt = int(T), int(ckpt_every), ckpt.data_ptr()
        keep = []
        gamp = None
        if src is not None:
            nodes = torch.tensor(self.inv[np.asarray(src[0])].astype(np.int32), device=self.device)
            amp = torch.tensor(np.asarray(src[1], dtype=np.float64), dtype=self.cdtype, device=self.device)
            wave = torch.tensor(np.asarray(src[2], dtype=np.float64), dtype=self.cdtype, device=self.device)
            gamp = torch.zeros(len(src[0]), dtype=torch.float64, device=self.device)
            keep += [nodes, amp, wave]
            a.n_src, a.src_node, a.src_amp, a.src_wave = len(src[0]), nodes.data_ptr(), amp.data_ptr(), wave.data_ptr()
            a.grad_amp = gamp.data_ptr()
        gtr = None
        if rcv is not None:
            rn = torch.tensor(self.inv[np.asarray(rcv)].astype(np.int32), device=self.device)
            gtr = torch.as_tensor(grad_traces).to(device=self.device, dtype=self.cdtype).contiguous()
            keep += [rn, gtr]
            a.n_rcv, a.rcv_node, a.grad_traces = len(rcv), rn.data_ptr(), gtr.data_ptr()
        geps = torch.zeros(self.N, dtype=torch.float64, device=self.device)
        seg = torch.empty((ckpt_every + 1) * self.sizes.e_bytes, dtype=torch.uint8, device=self.device)
        aws = torch.empty(self.sizes.adjoint_ws_bytes, dtype=torch.uint8, device=self.device)
        a.grad_eps, a.seg_buf, a.workspace = geps.data_ptr(), seg.data_ptr(), aws.data_ptr()
        f = st_eps.struct()
        check(self.lib.rbffd_adjoint(self.plan, C.byref(f), C.byref(a), self.stream()), self.plan, "rbffd_adjoint")
        g = self.permute(geps.reshape(-1, 1), 0, False).reshape(-1)
        return g.cpu().numpy(), (gamp.cpu().numpy() if gamp is not None else None)

    # ---- diagnostics -------------------------------------------------------------------
    def energy(self, E, Ha, Hb):
        out = torch.zeros(1, dtype=torch.float64, device=self.device)
        check(self.lib.rbffd_energy(self.plan, _ptr(E), _ptr(Ha), _ptr(Hb), _ptr(out), _ptr(self.ws), self.stream()),
              self.plan, "rbffd_energy")
        return float(out.cpu()[0])

    def compare(self, which, field, ref_internal):
        nc = 1 if self.K > 1 else (self.fe if which == 0 else self.fh)
        out = torch.zeros(3 * nc, dtype=torch.float64, device=self.device)
        r = ref_internal.to(device=self.device, dtype=torch.float64).contiguous()
        check(self.lib.rbffd_compare(self.plan, which, _ptr(field), _ptr(r), _ptr(out), _ptr(self.ws), self.stream()),
              self.plan, "rbffd_compare")
        return out.cpu().numpy().reshape(nc, 3)

    def autotune(self, st, reps=20, cache=None):
        """Tune the launch variant (rbffd_autotune), or with ``cache`` (a file
        path) look it up there first (rbffd_autotune_cached); the attribute
        ``tune_hit`` tells whether the cache held it."""
        f = st.struct()
        if cache is None:
            check(self.lib.rbffd_autotune(self.plan, C.byref(f), int(reps), self.stream()), self.plan, "autotune")
            self.tune_hit = False
        else:
            hit = C.c_int32(0)
            check(self.lib.rbffd_autotune_cached(self.plan, C.byref(f), int(reps), os.fsencode(cache), C.byref(hit),
                                                 self.stream()), self.plan, "autotune_cached")
            self.tune_hit = bool(hit.value)
        st.cur = f.cur
        return self.variant()

    def set_variant(self, block=256, xcd=1, lds=1, persist=8):
        check(self.lib.rbffd_set_variant(self.plan, block, xcd, lds, persist), self.plan, "set_variant")

    def variant(self):
        v = C.c_int32()
        self.lib.rbffd_get_variant(self.plan, C.byref(v))
        return {"block": v.value & 0xFFFF, "xcd": (v.value >> 16) & 1, "lds": (v.value >> 17) & 7,
                "persist": (v.value >> 20) & 0xFF}
