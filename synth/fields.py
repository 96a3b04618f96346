"""Seeded synthetic initial fields, permittivity maps, sources and receivers.

Initial conditions follow the leapfrog convention of the paper's scheme
(Section 5, eq. 19 and eq. 21): E is given at t = 0 and H at t = -dt/2.
Field layouts returned here are plain numpy arrays in the caller's (original)
node order: 2D TMz -> E [N, 1] (Ez), H [N, 2] (Hx, Hy); 3D -> E [N, 3],
H [N, 3].

The closed-form cavity modes are standard solutions of the vacuum curl
equations (eq. 2) with perfectly conducting walls; with them the same
functions also give the exact field at any later time, which tests use as the
analytic reference.
"""
import math
import numpy as np

from . import rng


def consts(eps0=1.0, mu0=1.0):
    c0 = 1.0 / math.sqrt(eps0 * mu0)
    eta0 = math.sqrt(mu0 / eps0)
    return c0, eta0


def tm_mode_2d(xyz, t_e, t_h, m=1, n=1, eps0=1.0, mu0=1.0):
    """TM_mn mode of the PEC unit square: Ez at time t_e, (Hx, Hy) at t_h."""
    c0, _ = consts(eps0, mu0)
    w = c0 * math.pi * math.hypot(m, n)
    x, y = xyz[:, 0], xyz[:, 1]
    sx, cx = np.sin(m * math.pi * x), np.cos(m * math.pi * x)
    sy, cy = np.sin(n * math.pi * y), np.cos(n * math.pi * y)
    E = (sx * sy * math.cos(w * t_e))[:, None]
    Hx = -(n * math.pi / (mu0 * w)) * sx * cy * math.sin(w * t_h)
    Hy = (m * math.pi / (mu0 * w)) * cx * sy * math.sin(w * t_h)
    return E, np.stack([Hx, Hy], axis=1), w


def te_mode_2d(xyz, t_e, t_h, m=1, n=1, eps0=1.0, mu0=1.0):
    """TE_mn mode of the PEC unit square: (Ex, Ey) at time t_e, Hz at t_h.

    Hz = cos(m pi x) cos(n pi y) cos(omega t); Ampere's law gives
    Ex = -(n pi / (eps0 omega)) cos(m pi x) sin(n pi y) sin(omega t) and
    Ey = (m pi / (eps0 omega)) sin(m pi x) cos(n pi y) sin(omega t), which vanish
    on the walls they are tangential to.
    """
    c0, _ = consts(eps0, mu0)
    w = c0 * math.pi * math.hypot(m, n)
    x, y = xyz[:, 0], xyz[:, 1]
    sx, cx = np.sin(m * math.pi * x), np.cos(m * math.pi * x)
    sy, cy = np.sin(n * math.pi * y), np.cos(n * math.pi * y)
    Hz = (cx * cy * math.cos(w * t_h))[:, None]
    Ex = -(n * math.pi / (eps0 * w)) * cx * sy * math.sin(w * t_e)
    Ey = (m * math.pi / (eps0 * w)) * sx * cy * math.sin(w * t_e)
    return np.stack([Ex, Ey], axis=1), Hz, w


def tm111_cube(xyz, t_e, t_h, eps0=1.0, mu0=1.0):
    """TM_111 mode of the PEC unit cube: E at t_e, H at t_h."""
    c0, _ = consts(eps0, mu0)
    w = c0 * math.pi * math.sqrt(3.0)
    p = math.pi
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    sx, cx = np.sin(p * x), np.cos(p * x)
    sy, cy = np.sin(p * y), np.cos(p * y)
    sz, cz = np.sin(p * z), np.cos(p * z)
    ce = math.cos(w * t_e)
    sh = math.sin(w * t_h)
    E = np.stack([-0.5 * cx * sy * sz * ce, -0.5 * sx * cy * sz * ce, sx * sy * cz * ce], axis=1)
    a = 3.0 * p / (2.0 * mu0 * w)
    H = np.stack([-a * sx * cy * cz * sh, a * cx * sy * cz * sh, np.zeros_like(x)], axis=1)
    return E, H, w


def gaussian_pulse(xyz, centre, sigma):
    """Ez = exp(-|x - centre|^2 / (2 sigma^2)), H = 0 (2D TMz)."""
    d2 = ((xyz - np.asarray(centre)[None, :]) ** 2).sum(axis=1)
    E = np.exp(-d2 / (2.0 * sigma * sigma))[:, None]
    return E, np.zeros((xyz.shape[0], 2))


def _wrap(u, L):
    """Signed distance along a periodic axis into [-L/2, L/2)."""
    return u - L * np.floor(u / L + 0.5)


def periodic_plane_pulse(xyz, t_e, t_h, L=200.0, sigma=30.0, phi=0.0, eps0=1.0,
                         mu0=1.0, images=2):
    """Plane Gaussian pulse on the periodic square [0, L]^2 (eq. 21, eq. 27).

    Travels along (cos phi, sin phi) at c0, centred on the line
    cos(phi) x + sin(phi) y = L/2 at t = 0.  H = (sin phi, -cos phi) E / eta0,
    which is the d'Alembert solution (eq. 22) for phi = 0.  The field is the
    sum over ``images`` periodic copies on each side along the propagation
    direction (one period L along x for phi = 0).
    """
    c0, eta0 = consts(eps0, mu0)
    cp, sp = math.cos(phi), math.sin(phi)
    s = cp * xyz[:, 0] + sp * xyz[:, 1]

    def prof(t):
        acc = np.zeros_like(s)
        for k in range(-images, images + 1):
            u = s - 0.5 * L - c0 * t + k * L
            acc += np.exp(-u * u / (2.0 * sigma * sigma))
        return acc

    E = prof(t_e)[:, None]
    g = prof(t_h)
    H = np.stack([sp * g / eta0, -cp * g / eta0], axis=1)
    return E, H


def te01_disk(xyz, t_e, t_h, R=1.0, centre=(0.0, 0.0), eps0=1.0, mu0=1.0):
    """TE_01 mode of the circular PEC cavity of radius R (2D TEz).

    Hz = J0(k r) cos(omega t), k = j_11 / R (first zero of J1, where the
    tangential E vanishes), omega = c0 k; Ampere's law gives
    E = eta0 J1(k r) (-sin theta, cos theta) sin(omega t).  Returns
    (E [N, 2] at t_e, Hz [N, 1] at t_h, omega).
    """
    from scipy import special
    c0, eta0 = consts(eps0, mu0)
    k = special.jn_zeros(1, 1)[0] / R
    om = c0 * k
    dx = xyz[:, 0] - centre[0]
    dy = xyz[:, 1] - centre[1]
    r = np.hypot(dx, dy)
    with np.errstate(invalid="ignore", divide="ignore"):
        st = np.where(r > 0, dy / np.where(r > 0, r, 1.0), 0.0)
        ct = np.where(r > 0, dx / np.where(r > 0, r, 1.0), 0.0)
    amp = eta0 * special.j1(k * r) * math.sin(om * t_e)
    E = np.stack([-amp * st, amp * ct], axis=1)
    Hz = (special.j0(k * r) * math.cos(om * t_h))[:, None]
    return E, Hz, om


def coax_wavenumber(a, b, pol):
    """Smallest k > 0 of the first circularly symmetric mode of the coaxial
    cavity a <= r <= b: TM_01 needs Z(kb) = 0 for Z(r) = J0(kr) Y0(ka) -
    J0(ka) Y0(kr); TE_01 needs Z'(b) = 0 for Z(r) = J0(kr) Y1(ka) - J1(ka)
    Y0(kr), i.e. J1(kb) Y1(ka) - J1(ka) Y1(kb) = 0."""
    from scipy import optimize, special
    if pol == "TM":
        f = lambda k: special.j0(k * b) * special.y0(k * a) - special.j0(k * a) * special.y0(k * b)
    else:
        f = lambda k: special.j1(k * b) * special.y1(k * a) - special.j1(k * a) * special.y1(k * b)
    ks = np.linspace(0.05, 10.0 * math.pi / (b - a), 4000)
    v = f(ks)
    i = int(np.nonzero(np.sign(v[1:]) != np.sign(v[:-1]))[0][0])
    return optimize.brentq(f, ks[i], ks[i + 1], xtol=1e-15, rtol=1e-15, maxiter=200)


def coax_mode(xyz, t_e, t_h, pol="TM", a=0.5, b=1.0, eps0=1.0, mu0=1.0):
    """First circularly symmetric mode of the coaxial PEC cavity a <= r <= b.

    TM_01 (TMz): Ez = Z(r) cos(omega t), Z as in ``coax_wavenumber``;
    Faraday's law gives H = (Z'(r) / (mu0 omega)) (-sin theta, cos theta)
    sin(omega t).  TE_01 (TEz): Hz = Z(r) cos(omega t); Ampere's law gives
    E = (Z'(r) / (eps0 omega)) (sin theta, -cos theta) sin(omega t), which
    vanishes on both walls.  Returns (E at t_e, H at t_h, omega) in the
    polarisation's layout (TM: [N, 1], [N, 2]; TE: [N, 2], [N, 1]).
    """
    from scipy import special
    c0, _ = consts(eps0, mu0)
    k = coax_wavenumber(a, b, pol)
    om = c0 * k
    x, y = xyz[:, 0], xyz[:, 1]
    r = np.hypot(x, y)
    st, ct = y / r, x / r
    if pol == "TM":
        Z = special.j0(k * r) * special.y0(k * a) - special.j0(k * a) * special.y0(k * r)
        dZ = k * (-special.j1(k * r) * special.y0(k * a) + special.j0(k * a) * special.y1(k * r))
        E = (Z * math.cos(om * t_e))[:, None]
        amp = dZ / (mu0 * om) * math.sin(om * t_h)
        return E, np.stack([-amp * st, amp * ct], axis=1), om
    Z = special.j0(k * r) * special.y1(k * a) - special.j1(k * a) * special.y0(k * r)
    dZ = k * (-special.j1(k * r) * special.y1(k * a) + special.j1(k * a) * special.y1(k * r))
    amp = dZ / (eps0 * om) * math.sin(om * t_e)
    return np.stack([amp * st, -amp * ct], axis=1), (Z * math.cos(om * t_h))[:, None], om


def sphere_mode(xyz, t_e, t_h, R=1.0, eps0=1.0, mu0=1.0):
    """Lowest azimuthal mode of the PEC sphere |x| <= R (3D).

    E = g(r) (-y, x, 0) cos(omega t) with g(r) = j1(k r) / r, k R the first
    zero of the spherical Bessel function j1 (E is tangential and vanishes on
    the wall); Faraday's law gives H = -(curl E) sin(omega t) / (mu0 omega),
    curl of g (-y, x, 0) = (-x z g'/r, -y z g'/r, 2 g + (x^2 + y^2) g'/r).
    Returns (E [N, 3] at t_e, H [N, 3] at t_h, omega).
    """
    from scipy import optimize, special
    c0, _ = consts(eps0, mu0)
    x0 = optimize.brentq(lambda s: special.spherical_jn(1, s), 4.0, 5.0, xtol=1e-15, rtol=1e-15)
    k = x0 / R
    om = c0 * k
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    r = np.sqrt(x * x + y * y + z * z)
    rs = np.where(r > 0, r, 1.0)
    j1 = special.spherical_jn(1, k * rs)
    dj1 = special.spherical_jn(1, k * rs, derivative=True)
    g = np.where(r > 0, j1 / rs, k / 3.0)
    gr = np.where(r > 0, (k * dj1 * rs - j1) / (rs ** 3), -k ** 3 / 15.0)     # g'(r) / r
    E = np.stack([-y * g, x * g, np.zeros_like(x)], axis=1) * math.cos(om * t_e)
    curl = np.stack([-x * z * gr, -y * z * gr, 2.0 * g + (x * x + y * y) * gr], axis=1)
    return E, -curl * math.sin(om * t_h) / (mu0 * om), om


def in_frame(H, theta):
    """Components of the 2D vectors H [N, 2] in the frame with axes
    u_1 = (cos theta, sin theta), u_2 = (-sin theta, cos theta)."""
    c, s = math.cos(theta), math.sin(theta)
    return np.stack([c * H[:, 0] + s * H[:, 1], -s * H[:, 0] + c * H[:, 1]], axis=1)


def eps_r_smooth(xyz, seed=5, stream=2, n_modes=16, kmax=4, amp=0.5):
    """eps_r = 1 + amp * s(x) / max|s|, s = sum of 16 seeded cosine modes.

    s(x) = sum_q a_q cos(2 pi k_q . x + phi_q), k_q integer with |k_q|_inf <= kmax
    (not both zero), a_q ~ U(-1, 1), phi_q ~ U(0, 2 pi).
    """
    d = xyz.shape[1]
    q = np.arange(n_modes, dtype=np.uint64)
    per = np.uint64(d + 2)
    ks = []
    for k in range(d):
        u = rng.uniform(seed, stream, q * per + np.uint64(k))
        ks.append(np.floor(u * (2 * kmax + 1)).astype(np.int64) - kmax)
    K = np.stack(ks, axis=1)
    zero = (K == 0).all(axis=1)
    K[zero, 0] = 1
    a = rng.uniform_range(seed, stream, q * per + np.uint64(d), -1.0, 1.0)
    ph = rng.uniform_range(seed, stream, q * per + np.uint64(d + 1), 0.0, 2 * math.pi)
    s = np.zeros(xyz.shape[0])
    for j in range(n_modes):
        s += a[j] * np.cos(2 * math.pi * (xyz @ K[j].astype(np.float64)) + ph[j])
    return 1.0 + amp * s / np.abs(s).max()


def seeded_points(n, lo, hi, seed, stream=1, d=2):
    """n points uniform in the box [lo, hi]^d (source / receiver positions)."""
    c = np.arange(n * d, dtype=np.uint64)
    return rng.uniform_range(seed, stream, c, lo, hi).reshape(n, d)


def nearest_node(xyz, pts):
    """Index of the node closest to each point (lowest index on ties)."""
    out = np.empty(pts.shape[0], dtype=np.int64)
    for k, p in enumerate(pts):
        d2 = ((xyz - p[None, :]) ** 2).sum(axis=1)
        out[k] = int(np.argmin(d2))
    return out


def gaussian_wavelet(t, t0, tau):
    """Time profile of the soft source: exp(-(t - t0)^2 / (2 tau^2))."""
    return np.exp(-((np.asarray(t) - t0) ** 2) / (2.0 * tau * tau))


def tm01_disk(xyz, t_e, t_h, R=1.0, centre=(0.0, 0.0), eps0=1.0, mu0=1.0):
    """TM_01 mode of the circular PEC cavity of radius R (2D TMz).

    Ez = J0(k r) cos(omega t), k = j_01 / R (first zero of J0), omega = c0 k;
    Faraday's law gives H = (k / (mu0 omega)) J1(k r) (sin theta, -cos theta)
    sin(omega t).  Returns (E [N, 1] at t_e, H [N, 2] at t_h, omega).
    """
    from scipy import special
    c0, _ = consts(eps0, mu0)
    k = special.jn_zeros(0, 1)[0] / R
    om = c0 * k
    dx = xyz[:, 0] - centre[0]
    dy = xyz[:, 1] - centre[1]
    r = np.hypot(dx, dy)
    E = (special.j0(k * r) * math.cos(om * t_e))[:, None]
    with np.errstate(invalid="ignore", divide="ignore"):
        st = np.where(r > 0, dy / np.where(r > 0, r, 1.0), 0.0)
        ct = np.where(r > 0, dx / np.where(r > 0, r, 1.0), 0.0)
    amp = k / (mu0 * om) * special.j1(k * r) * math.sin(om * t_h)
    H = np.stack([amp * st, -amp * ct], axis=1)
    return E, H, om
