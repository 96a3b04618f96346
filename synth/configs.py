"""Named synthetic workloads (node sets, parameters, initial data).

Each workload bundles what both the GPU path and the oracle consume: nodes,
boundary flags, method parameters and initial fields.  Everything is seeded
and regenerated on demand; nothing is read from disk.

Parameters follow the paper where it fixes them: S_c = c0 dt / h = 1/(10
sqrt 2) (Section 5, footnote 7), phi = r^3 (Section 4.3), hyperviscosity
alpha = 2 unless stated (Section 5.1) with n_hv = 2 M_{2 alpha} + 1.  The
hyperviscosity constant c is given through the per-step dimensionless value
chat = c * dt (the paper quotes c = 1e-4 in units where h = dt = 1).

Workloads (sizes at scale = 1):
  tm_cavity_2d   51 x 51 jittered grid on the PEC unit square, n = 12, m = 2,
                 alpha = 2, TM_11 mode, 1000 steps (one period), FP64.
  pulse_2d       ~1.0M Poisson-disk nodes, PEC unit square, n = 25, m = 4,
                 alpha = 3, Gaussian pulse (sigma = 20 h) at the centre,
                 10^4 steps.
  tm111_3d       200^3 jittered grid, PEC unit cube, n = 35, m = 2, alpha = 2,
                 TM_111 mode, 2000 steps.
  batched_2d     500 x 500 jittered grid, n = 25, m = 2, alpha = 2, K = 64
                 Gaussian pulses at seeded centres in [0.2, 0.8]^2, 5000 steps.
  adjoint_2d     500 x 500 jittered grid, n = 25, m = 2, alpha = 2, smooth
                 seeded eps_r, 16 receivers, one soft source, 2000 steps.
  periodic_pulse the paper's periodic test: [0, 200] x [0, Ly] jittered grid,
                 h = 1, sigma = 30, c0 t = 5 sqrt 2 (eq. 21-23).
"""
import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import nodes as _nodes
from . import fields as _fields

SC = 1.0 / (10.0 * math.sqrt(2.0))


def n_monomials(d, m):
    return math.comb(m + d, d)


@dataclass
class Workload:
    name: str
    dim: int
    xyz: np.ndarray
    flags: np.ndarray
    h: float
    n: int
    m: int
    alpha: int
    n_hv: int
    chat: float
    steps: int
    mode: str = "FD"          # FD | VFD | STAG2
    bc: str = "PEC"           # PEC | PERIODIC
    lo: tuple = (0.0, 0.0)
    hi: tuple = (1.0, 1.0)
    eps0: float = 1.0
    mu0: float = 1.0
    vfd_sigma: float = 0.5
    E0: Optional[np.ndarray] = None
    H0: Optional[np.ndarray] = None
    # two-set variant: the H node set
    xyz_h: Optional[np.ndarray] = None
    flags_h: Optional[np.ndarray] = None
    h_h: Optional[float] = None
    # extras
    pol: str = "TM"           # 2D polarisation: TM (Ez, Hx, Hy) | TE (Ex, Ey, Hz)
    frame_angle: float = 0.0  # 2D: angle of the frame the curl is discretised in
    normals: Optional[np.ndarray] = None       # [N, d] unit wall normals (curved TEz / 3D walls), 0 elsewhere
    K: int = 1
    E0_batch: Optional[np.ndarray] = None      # [K, N, FE]
    eps_r: Optional[np.ndarray] = None
    src_node: Optional[np.ndarray] = None
    src_amp: Optional[np.ndarray] = None
    src_wave: Optional[np.ndarray] = None      # [steps, S]
    rcv_node: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.xyz.shape[0]

    @property
    def c0(self):
        return 1.0 / math.sqrt(self.eps0 * self.mu0)

    @property
    def dt(self):
        return SC * self.h / self.c0

    @property
    def hv_c(self):
        return self.chat / self.dt

    @property
    def period(self):
        if self.bc == "PERIODIC":
            return tuple(self.hi[k] - self.lo[k] for k in range(self.dim))
        return None


def _hv_default(d, alpha):
    return 2 * n_monomials(d, 2 * alpha) + 1


def tm_cavity_2d(scale=1.0, n_side=None, seed=1, mode="FD", chat=1e-4, steps=None,
                 eps0=1.0, mu0=1.0, n=12, m=2, alpha=2):
    ns = n_side or max(8, int(round(50 * scale)) + 1)
    xyz, flags, h = _nodes.jittered_grid((ns, ns), seed=seed)
    w = Workload("tm_cavity_2d", 2, xyz, flags, h, n, m, alpha, _hv_default(2, alpha),
                 chat, 0, mode=mode, eps0=eps0, mu0=mu0)
    # one period of TM_11: T = 2 pi / omega = sqrt(2) / c0
    w.steps = steps if steps is not None else int(round(math.sqrt(2.0) / w.c0 / w.dt))
    E, H, omega = _fields.tm_mode_2d(xyz, 0.0, -0.5 * w.dt, eps0=eps0, mu0=mu0)
    w.E0, w.H0 = E, H
    w.meta["omega"] = omega
    if mode == "STAG2":
        xh, fh, hh = _nodes.dual_grid_2d(ns - 1, seed=seed)
        w.xyz_h, w.flags_h, w.h_h = xh, fh, hh
        _, H, _ = _fields.tm_mode_2d(xh, 0.0, -0.5 * w.dt, eps0=eps0, mu0=mu0)
        w.H0 = H
    return w


def te_cavity_2d(scale=1.0, n_side=None, seed=1, mode="FD", chat=1e-3, steps=None, eps0=1.0, mu0=1.0,
                 n=12, m=2, alpha=2, periods=1.0):
    """TEz polarisation on the PEC unit square with its TE_11 mode (Hz at
    half steps, E at whole steps) for ``periods`` periods."""
    ns = n_side or max(8, int(round(50 * scale)) + 1)
    xyz, flags, h = _nodes.jittered_grid((ns, ns), seed=seed)
    w = Workload("te_cavity_2d", 2, xyz, flags, h, n, m, alpha, _hv_default(2, alpha),
                 chat, 0, mode=mode, eps0=eps0, mu0=mu0, pol="TE")
    w.steps = steps if steps is not None else int(round(periods * math.sqrt(2.0) / w.c0 / w.dt))
    E, Hz, omega = _fields.te_mode_2d(xyz, 0.0, -0.5 * w.dt, eps0=eps0, mu0=mu0)
    w.E0, w.H0 = E, Hz
    w.meta["omega"] = omega
    return w


def pulse_2d(scale=1.0, r=None, seed=2, chat=1e-4, steps=10000, n=25, m=4, alpha=3):
    rr = r if r is not None else 0.00079 / math.sqrt(scale)
    xyz, flags, h = _nodes.poisson_disk_2d(rr, seed=seed, rounds=8)
    w = Workload("pulse_2d", 2, xyz, flags, h, n, m, alpha, _hv_default(2, alpha), chat, steps)
    w.E0, w.H0 = _fields.gaussian_pulse(xyz, (0.5, 0.5), 20.0 * h)
    return w


def tm111_3d(scale=1.0, n_side=None, seed=3, chat=1e-4, steps=2000, n=35, m=2, alpha=2):
    ns = n_side or max(6, int(round(200 * scale)))
    xyz, flags, h = _nodes.jittered_grid((ns, ns, ns), seed=seed)
    w = Workload("tm111_3d", 3, xyz, flags, h, n, m, alpha, _hv_default(3, alpha), chat,
                 steps, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0))
    E, H, omega = _fields.tm111_cube(xyz, 0.0, -0.5 * w.dt)
    w.E0, w.H0 = E, H
    w.meta["omega"] = omega
    return w


def batched_2d(scale=1.0, n_side=None, K=64, seed=4, chat=1e-4, steps=5000, n=25, m=2, alpha=2):
    ns = n_side or max(8, int(round(500 * scale)))
    xyz, flags, h = _nodes.jittered_grid((ns, ns), seed=seed)
    w = Workload("batched_2d", 2, xyz, flags, h, n, m, alpha, _hv_default(2, alpha), chat, steps)
    centres = _fields.seeded_points(K, 0.2, 0.8, seed, stream=1)
    Eb = np.stack([_fields.gaussian_pulse(xyz, c, 20.0 * h)[0] for c in centres])
    w.K = K
    w.E0_batch = Eb
    w.E0, w.H0 = Eb[0], np.zeros((xyz.shape[0], 2))
    w.meta["centres"] = centres
    return w


def adjoint_2d(scale=1.0, n_side=None, seed=5, chat=1e-4, steps=2000, n=25, m=2, alpha=2,
               n_rcv=16):
    ns = n_side or max(8, int(round(500 * scale)))
    xyz, flags, h = _nodes.jittered_grid((ns, ns), seed=seed)
    w = Workload("adjoint_2d", 2, xyz, flags, h, n, m, alpha, _hv_default(2, alpha), chat, steps)
    w.eps_r = _fields.eps_r_smooth(xyz, seed=seed)
    w.E0 = np.zeros((xyz.shape[0], 1))
    w.H0 = np.zeros((xyz.shape[0], 2))
    w.src_node = _fields.nearest_node(xyz, np.array([[0.5, 0.5]]))
    w.src_amp = np.array([1.0])
    tau = 10.0 * h / w.c0
    t_half = (np.arange(steps) + 0.5) * w.dt
    w.src_wave = _fields.gaussian_wavelet(t_half, 4.0 * tau, tau)[:, None]
    pts = _fields.seeded_points(n_rcv, 0.1, 0.9, seed, stream=1)
    w.rcv_node = _fields.nearest_node(xyz, pts)
    return w


def periodic_pulse(h=1.0, Ly=None, sigma=30.0, seed=6, chat=1e-4, mode="FD", n=12, m=2,
                   alpha=2, L=200.0, phi=0.0, t_end=5.0 * math.sqrt(2.0)):
    Ly = Ly if Ly is not None else L
    nx = int(round(L / h))
    ny = int(round(Ly / h))
    xyz, flags, hh = _nodes.jittered_grid((nx, ny), lo=(0.0, 0.0), hi=(L, Ly), seed=seed,
                                          periodic=True)
    w = Workload("periodic_pulse", 2, xyz, flags, hh, n, m, alpha, _hv_default(2, alpha),
                 chat, 0, mode=mode, bc="PERIODIC", lo=(0.0, 0.0), hi=(L, Ly))
    w.steps = int(round(t_end / w.dt))
    w.E0, w.H0 = _fields.periodic_plane_pulse(xyz, 0.0, -0.5 * w.dt, L=L, sigma=sigma, phi=phi)
    w.meta.update(sigma=sigma, L=L, phi=phi)
    return w


def dispersion_2d(n=60, mode="FD", L=200.0, h=1.0, sigma=2.0, chat=None, steps=2820, save_every=15,
                  seed=3, m=2, alpha=2, phi=0.0):
    """The dispersion study of Section 6: periodic [0, L)^2 with a scattered
    node set that contains the equispaced line y = L/2 (node ids 0..L/h-1),
    the narrow pulse of eq. 21 (sigma = 2), 2820 steps (one passage across the
    domain), E sampled on the line every ``save_every`` steps.

    phi: propagation angle of the angle study (eq. 27).  The domain and the
    seeded line are those of phi = 0 seen from coordinates rotated by -phi:
    the pulse runs along the line, and the curl is discretised in the frame
    at angle -phi to the domain (the x and y axes of eq. 27), where H has the
    components (sin phi, -cos phi) g / eta0.

    chat defaults to the paper's hyperviscosity constants for this setup,
    c = 10^-4.76 (RBF-FD) and 10^-5.02 (RBF-VFD) in units h = dt = 1, i.e.
    chat = c * dt with dt = 1.
    """
    if chat is None:
        chat = 10.0 ** (-4.76 if mode == "FD" else -5.02)
    xyz, flags, hh, line = _nodes.line_seeded_periodic(L, h, seed=seed)
    w = Workload("dispersion_2d", 2, xyz, flags, hh, n, m, alpha, _hv_default(2, alpha), chat, steps,
                 mode=mode, bc="PERIODIC", lo=(0.0, 0.0), hi=(L, L), frame_angle=-phi)
    E0, H0 = _fields.periodic_plane_pulse(xyz, 0.0, -0.5 * w.dt, L=L, sigma=sigma)
    w.E0, w.H0 = E0, (_fields.in_frame(H0, -phi) if phi != 0.0 else H0)
    w.rcv_node = line
    w.meta.update(sigma=sigma, L=L, save_every=save_every, line=line, phi=phi)
    return w


def tm01_disk(h=0.02, R=1.0, n=12, m=2, alpha=2, chat=1e-3, periods=1.0, seed=9):
    """Circular PEC cavity (curved wall) with its TM_01 mode for ``periods``
    periods; nodes from ``disk_nodes`` (equispaced on the circle, Poisson-disk
    inside)."""
    xyz, flags, hm = _nodes.disk_nodes(R, h, seed=seed)
    w = Workload("tm01_disk", 2, xyz, flags, h, n, m, alpha, _hv_default(2, alpha), chat, 0,
                 lo=(-R, -R), hi=(R, R))
    E0, H0, om = _fields.tm01_disk(xyz, 0.0, -0.5 * w.dt, R=R)
    w.E0, w.H0 = E0, H0
    w.steps = int(round(periods * 2 * math.pi / om / w.dt))
    w.meta.update(R=R, omega=om, h_mean=hm)
    return w


def te01_disk(h=0.02, R=1.0, n=12, m=2, alpha=2, chat=1e-3, periods=1.0, seed=9):
    """Circular PEC cavity in the TEz polarisation with its TE_01 mode for
    ``periods`` periods; the same nodes as ``tm01_disk``, with the outward
    unit normal of the circle on every wall node."""
    xyz, flags, hm = _nodes.disk_nodes(R, h, seed=seed)
    w = Workload("te01_disk", 2, xyz, flags, h, n, m, alpha, _hv_default(2, alpha), chat, 0,
                 lo=(-R, -R), hi=(R, R), pol="TE")
    wall = flags != 0
    nrm = np.zeros((w.N, 2))
    nrm[wall] = xyz[wall] / np.hypot(xyz[wall, 0], xyz[wall, 1])[:, None]
    w.normals = nrm
    E0, H0, om = _fields.te01_disk(xyz, 0.0, -0.5 * w.dt, R=R)
    w.E0, w.H0 = E0, H0
    w.steps = int(round(periods * 2 * math.pi / om / w.dt))
    w.meta.update(R=R, omega=om, h_mean=hm)
    return w


def coax_2d(pol="TM", h=0.02, a=0.5, b=1.0, n=12, m=2, alpha=2, chat=1e-3, periods=1.0, seed=11):
    """Coaxial PEC cavity a <= r <= b (a conducting cylinder inside the
    domain) with its first circularly symmetric mode (TM_01 in TMz, TE_01 in
    TEz) for ``periods`` periods; in TEz every wall node carries the radial
    unit normal."""
    xyz, flags, hm = _nodes.disk_nodes(b, h, seed=seed, R_in=a)
    w = Workload(f"coax_{pol.lower()}", 2, xyz, flags, h, n, m, alpha, _hv_default(2, alpha), chat, 0,
                 lo=(-b, -b), hi=(b, b), pol=pol)
    if pol == "TE":
        wall = flags != 0
        nrm = np.zeros((w.N, 2))
        nrm[wall] = xyz[wall] / np.hypot(xyz[wall, 0], xyz[wall, 1])[:, None]
        w.normals = nrm
    E0, H0, om = _fields.coax_mode(xyz, 0.0, -0.5 * w.dt, pol=pol, a=a, b=b)
    w.E0, w.H0 = E0, H0
    w.steps = int(round(periods * 2 * math.pi / om / w.dt))
    w.meta.update(a=a, b=b, omega=om, h_mean=hm)
    return w


def sphere_3d(h=0.1, R=1.0, n=35, m=2, alpha=2, chat=1e-4, periods=1.0, seed=13):
    """PEC sphere (curved 3D wall) with its lowest azimuthal mode for
    ``periods`` periods; every wall node carries the outward unit normal."""
    xyz, flags, hm = _nodes.ball_nodes(R, h, seed=seed)
    w = Workload("sphere_3d", 3, xyz, flags, h, n, m, alpha, _hv_default(3, alpha), chat, 0,
                 lo=(-R, -R, -R), hi=(R, R, R))
    wall = flags != 0
    nrm = np.zeros((w.N, 3))
    nrm[wall] = xyz[wall] / np.sqrt((xyz[wall] ** 2).sum(axis=1))[:, None]
    w.normals = nrm
    E0, H0, om = _fields.sphere_mode(xyz, 0.0, -0.5 * w.dt, R=R)
    w.E0, w.H0 = E0, H0
    w.steps = int(round(periods * 2 * math.pi / om / w.dt))
    w.meta.update(R=R, omega=om, h_mean=hm)
    return w


REGISTRY = {
    "tm_cavity_2d": tm_cavity_2d,
    "pulse_2d": pulse_2d,
    "tm111_3d": tm111_3d,
    "batched_2d": batched_2d,
    "adjoint_2d": adjoint_2d,
    "periodic_pulse": periodic_pulse,
    "dispersion_2d": dispersion_2d,
    "tm01_disk": tm01_disk,
    "te_cavity_2d": te_cavity_2d,
    "te01_disk": te01_disk,
    "coax_2d": coax_2d,
    "sphere_3d": sphere_3d,
}


def make(name, **kw):
    return REGISTRY[name](**kw)
