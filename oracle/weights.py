"""Local RBF differentiation weights (Section 4, eq. 8-15; Section 5.1).

For a centre x_c with stencil nodes x_j (j = 1..n):

* Scaled local coordinates xi_j = (x_j - x_c) / s_c, s_c = max_j |x_j - x_c|.
  Polyharmonic splines with monomials are scale covariant, so scaling changes
  only the conditioning, not the weights.
* Interpolation matrix (eq. 9): A_jk = phi(|xi_j - xi_k|) with phi(r) = r^k_phi,
  P_jq = p_q(xi_j) for the M_m = C(m + d, d) monomials of total degree <= m
  (footnote 4), in graded lexicographic order (1, x, y, x^2, xy, y^2, ...; z
  last in 3D), and A~ = [[A, P], [P^T, 0]].
* Weights: the first n entries of A~^{-1} b where b collects the operator
  applied to every basis function at the evaluation point:
  - RBF-FD (eq. 13): b = [L phi(|xi - xi_j|), L p_q(xi)] at xi = 0;
  - RBF-VFD (eq. 14-15) with the central difference: the virtual points are
    xi = +-delta' e_x, delta' = sigma h / s_c, and
    b = ([phi, p](+delta') - [phi, p](-delta')) / (2 delta').  The worked
    example of Section 4.2 prints the central-difference coefficients without
    the factor 1/2; the 1/2 is the only reading that reproduces d/dx x = 1 and
    is used here.
  - Rotated frame (the angle study of Section 6, eq. 27): with a frame angle
    theta the two derivatives are taken along u_1 = (cos theta, sin theta)
    and u_2 = (-sin theta, cos theta) instead of e_x and e_y: RBF-FD
    differentiates along u (b = u . grad of every basis function at 0) and
    RBF-VFD places its virtual points at +-delta' u.
  - Hyperviscosity (Section 5.1): RBF-FD of the iterated Laplacian Delta^alpha
    with phi = r^(2 alpha + 1) and m = 2 alpha.
* Unscaling: w = w_xi / s_c^l with l = 1 for first derivatives and 2 alpha for
  Delta^alpha.

Closed forms used in the right-hand sides:
  d/dx r^k at 0 for a centre xi_j   -> -k r_j^(k-2) xi_{j,x}
  Delta r^k = k (k + d - 2) r^(k-2)   (radial Laplacian), iterated alpha times
  Delta^alpha (x^a y^b z^c), a+b+c = 2 alpha, at 0 -> alpha!/(i! j! l!) a! b! c!
  with a = 2i, b = 2j, c = 2l (zero if any exponent is odd).
The local systems are solved with numpy's LAPACK solver (LU with partial
pivoting), one system per centre.
"""
import math
import numpy as np

from .knn import min_image


def n_monomials(d, m):
    return math.comb(m + d, d)


def monomial_exponents(d, m):
    """Exponent tuples of all monomials of total degree <= m, graded lex."""
    out = []
    for g in range(m + 1):
        if d == 2:
            for a in range(g, -1, -1):
                out.append((a, g - a))
        else:
            for a in range(g, -1, -1):
                for b in range(g - a, -1, -1):
                    out.append((a, b, g - a - b))
    return out


def _monomials(xi, exps):
    """[..., M] monomial values at points xi [..., d]."""
    cols = []
    for e in exps:
        v = np.ones(xi.shape[:-1])
        for k, p in enumerate(e):
            if p:
                v = v * xi[..., k] ** p
        cols.append(v)
    return np.stack(cols, axis=-1)


def _dmonomials_dx(xi, exps, axis):
    cols = []
    for e in exps:
        p = e[axis]
        if p == 0:
            cols.append(np.zeros(xi.shape[:-1]))
            continue
        v = np.full(xi.shape[:-1], float(p))
        for k, q in enumerate(e):
            qq = q - 1 if k == axis else q
            if qq:
                v = v * xi[..., k] ** qq
        cols.append(v)
    return np.stack(cols, axis=-1)


def laplacian_power_const(k, alpha, d):
    """C with Delta^alpha r^k = C r^(k - 2 alpha) (radial Laplacian iterated)."""
    c = 1.0
    kk = k
    for _ in range(alpha):
        c *= kk * (kk + d - 2)
        kk -= 2
    return c


def laplacian_power_of_monomial_at_0(e, alpha):
    """Delta^alpha of prod x_k^e_k evaluated at the origin."""
    if sum(e) != 2 * alpha or any(p % 2 for p in e):
        return 0.0
    half = [p // 2 for p in e]
    multinom = math.factorial(alpha)
    for q in half:
        multinom //= math.factorial(q)
    val = float(multinom)
    for p in e:
        val *= math.factorial(p)
    return val


def local_frames(src, centres, idx, period=None):
    """Scaled stencil offsets xi [C, n, d] and scales s_c [C]."""
    X = src[idx] - centres[:, None, :]
    X = min_image(X, period)
    s = np.sqrt((X * X).sum(axis=2)).max(axis=1)
    return X / s[:, None, None], s


def _system(xi, phs_k, exps):
    n = xi.shape[1]
    diff = xi[:, :, None, :] - xi[:, None, :, :]
    r = np.sqrt((diff * diff).sum(axis=3))
    A = r ** phs_k
    P = _monomials(xi, exps)
    M = P.shape[2]
    C = xi.shape[0]
    At = np.zeros((C, n + M, n + M))
    At[:, :n, :n] = A
    At[:, :n, n:] = P
    At[:, n:, :n] = np.transpose(P, (0, 2, 1))
    return At


def fd_rhs_derivative(xi, phs_k, exps, axis):
    """b for L = d/dx_axis at xi = 0 (RBF-FD, eq. 13)."""
    r = np.sqrt((xi * xi).sum(axis=2))
    # d/dx |x - xi_j|^k at x = 0  =  -k r_j^(k-2) xi_{j,axis}
    bphi = -phs_k * r ** (phs_k - 2) * xi[:, :, axis]
    bp = _dmonomials_dx(np.zeros((xi.shape[0], xi.shape[2])), exps, axis)
    return np.concatenate([bphi, bp], axis=1)


def vfd_rhs(xi, phs_k, exps, coeffs, offsets, delta, order):
    """b for a virtual finite-difference stencil (eq. 14-15).

    The operator is approximated by delta^-l sum_i c_i s(x_c + delta o_i); with
    s the local interpolant this is b = delta^-l sum_i c_i [phi, p](delta o_i).
    ``delta`` [C] is the virtual spacing in scaled units, ``order`` = l.
    """
    C, n, d = xi.shape
    b = None
    for c_i, o_i in zip(coeffs, offsets):
        if c_i == 0.0:
            continue
        xv = delta[:, None] * np.asarray(o_i, dtype=np.float64)[None, :]   # [C, d]
        diff = xv[:, None, :] - xi
        r = np.sqrt((diff * diff).sum(axis=2))
        term = c_i * np.concatenate([r ** phs_k, _monomials(xv, exps)], axis=1)
        b = term if b is None else b + term
    return b / delta[:, None] ** order


def central_difference(d, axis):
    """Central first difference along ``axis``: c = (-1/2, 1/2), o = (-e, +e)."""
    e = np.zeros(d)
    e[axis] = 1.0
    return (-0.5, 0.5), (-e, e)


def frame_axes(d, theta):
    """Unit vectors u_1, u_2 (rows) of the 2D frame at angle theta; the
    identity for theta = 0 or in 3D (no rotated frame there)."""
    if theta == 0.0 or d != 2:
        return np.eye(d)
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, s], [-s, c]])


def fd_rhs_directional(xi, phs_k, exps, u):
    """b for L = u . grad at xi = 0 (RBF-FD along the unit vector u)."""
    b = None
    for ax in range(xi.shape[2]):
        if u[ax] == 0.0:
            continue
        t = u[ax] * fd_rhs_derivative(xi, phs_k, exps, ax)
        b = t if b is None else b + t
    return b


def hv_rhs(xi, alpha, exps):
    """b for L = Delta^alpha with phi = r^(2 alpha + 1) at xi = 0."""
    d = xi.shape[2]
    k = 2 * alpha + 1
    r = np.sqrt((xi * xi).sum(axis=2))
    bphi = laplacian_power_const(k, alpha, d) * r ** (k - 2 * alpha)
    bp = np.array([laplacian_power_of_monomial_at_0(e, alpha) for e in exps])
    return np.concatenate([bphi, np.broadcast_to(bp, (xi.shape[0], bp.size))], axis=1)


def curl_weights(src, centres, idx, m, phs_k=3, mode="FD", sigma=0.5, h=None,
                 period=None, batch=4096, frame_angle=0.0):
    """First-derivative weights [C, d, n] (axis-major) for every centre.

    mode "FD" = RBF-FD (eq. 13); "VFD" = RBF-VFD (eq. 15) with delta = sigma h.
    frame_angle (2D): derivatives along the axes of the frame rotated by that
    angle (axis 0 along u_1, axis 1 along u_2).
    """
    d = src.shape[1]
    exps = monomial_exponents(d, m)
    C, n = idx.shape
    U = frame_axes(d, frame_angle)
    W = np.empty((C, d, n))
    for b0 in range(0, C, batch):
        sl = slice(b0, min(C, b0 + batch))
        xi, s = local_frames(src, centres[sl], idx[sl], period)
        At = _system(xi, phs_k, exps)
        cols = []
        for ax in range(d):
            if mode == "FD":
                cols.append(fd_rhs_directional(xi, phs_k, exps, U[ax]))
            elif mode == "VFD":
                cols.append(vfd_rhs(xi, phs_k, exps, (-0.5, 0.5), (-U[ax], U[ax]), sigma * h / s, 1))
            else:
                raise ValueError(mode)
        B = np.stack(cols, axis=2)
        sol = np.linalg.solve(At, B)
        W[sl] = np.transpose(sol[:, :n, :], (0, 2, 1)) / s[:, None, None]
    return W


def vfd_weights(src, centres, idx, m, coeffs, offsets, delta, order, phs_k=3, period=None):
    """General RBF-VFD weights [C, n] for one virtual stencil (eq. 15)."""
    d = src.shape[1]
    exps = monomial_exponents(d, m)
    xi, s = local_frames(src, centres, idx, period)
    At = _system(xi, phs_k, exps)
    b = vfd_rhs(xi, phs_k, exps, coeffs, offsets, delta / s, order)
    sol = np.linalg.solve(At, b[:, :, None])[:, :, 0]
    return sol[:, :idx.shape[1]] / s[:, None] ** order


def hv_weights(src, centres, idx, alpha, period=None, batch=4096):
    """Delta^alpha weights [C, n_hv] (RBF-FD, phi = r^(2a+1), m = 2a)."""
    d = src.shape[1]
    exps = monomial_exponents(d, 2 * alpha)
    C, n = idx.shape
    W = np.empty((C, n))
    for b0 in range(0, C, batch):
        sl = slice(b0, min(C, b0 + batch))
        xi, s = local_frames(src, centres[sl], idx[sl], period)
        At = _system(xi, 2 * alpha + 1, exps)
        b = hv_rhs(xi, alpha, exps)
        sol = np.linalg.solve(At, b[:, :, None])[:, :, 0]
        W[sl] = sol[:, :n] / s[:, None] ** (2 * alpha)
    return W


def system_condition(src, centres, idx, m, phs_k, period=None):
    """2-norm condition numbers of the scaled local systems (diagnostic)."""
    d = src.shape[1]
    xi, _ = local_frames(src, centres, idx, period)
    return np.linalg.cond(_system(xi, phs_k, monomial_exponents(d, m)))


def cardinal_values(src, centre, idx, m, phs_k, points, period=None):
    """psi_j(points) for one centre: the Lagrange functions of eq. 10-11.

    Returns [P, n].  Used by tests to differentiate the interpolant
    numerically, independently of the closed-form right-hand sides.
    """
    d = src.shape[1]
    exps = monomial_exponents(d, m)
    xi, s = local_frames(src, centre[None, :], idx[None, :], period)
    At = _system(xi, phs_k, exps)[0]
    n = idx.size
    q = (np.asarray(points) - centre[None, :]) / s[0]
    diff = q[:, None, :] - xi[0][None, :, :]
    r = np.sqrt((diff * diff).sum(axis=2))
    rhs = np.concatenate([r ** phs_k, _monomials(q, exps)], axis=1)   # [P, n+M]
    sol = np.linalg.solve(At, rhs.T)                                  # [n+M, P]
    return sol[:n, :].T
