"""The stabilised meshless leapfrog (Section 5, eq. 16-19) and its diagnostics.

Notation of the paper: D^L f (x_i) = sum_{j in S(x_i)} w_j^L f(x_j) (eq. 16).
With a = dt / mu0, kappa_i = dt / (eps0 * eps_r,i) and the hyperviscosity
strength gamma = c (-1)^(alpha-1) h^(2 alpha) (Section 5.1), one step is

  Hx <- Hx - a (D^dy Ez - gamma D^hv Hx)                        (eq. 19)
  Hy <- Hy + a (D^dx Ez + gamma D^hv Hy)
  Ez <- Ez + kappa (D^dx Hy_new - D^dy Hx_new + gamma D^hv Ez) + source

with every operator acting on old values except the curl in the E update,
which uses the new H.  In 3D the same scheme with the full discrete curl:
H <- H - a (curl_D E - gamma D^hv H), E <- E + kappa (curl_D H_new +
gamma D^hv E).  Readings where the paper is silent (all stated in the design
notes): eps_r replaces eps0 in the whole E bracket; a perfectly conducting
wall zeroes the E components tangential to it after every E update (Ez on every
wall in 2D TMz); a soft source adds a_s g_s(t_{n+1/2}) at its node after the
bracket, unscaled by eps_r.

Field layout (one node set): E [N, FE], H [N, FH] with (FE, FH) = (1, 2) for
2D TMz and (3, 3) in 3D.  H^n holds H(t_{n-1/2}).

Operators are dictionaries {"curl_idx" [N, n], "curl_w" [N, d, n],
"hv_idx" [N, nh], "hv_w" [N, nh]}; the collocated variants use the same one
for both half steps, the two-set variant passes one per half step (curl
stencils drawn from the other set, hyperviscosity from the own set).
"""
import math
import numpy as np


def D(w, idx, f):
    """D^L f at every centre: sum_j w_j f(x_j) (eq. 12/16)."""
    return (w * f[idx]).sum(axis=1)


def hv_gamma(c, alpha, h):
    """gamma = c (-1)^(alpha - 1) h^(2 alpha) (Section 5.1)."""
    return c * (-1.0) ** (alpha - 1) * h ** (2 * alpha)


def pec_keep(flags, dim):
    """[N, FE] 0/1 factors: which E components a PEC wall leaves free."""
    flags = np.asarray(flags)
    if dim == 2:
        return (flags == 0).astype(np.float64)[:, None]
    keep = np.ones((flags.size, 3))
    for k in range(3):
        on = (flags & (3 << (2 * k))) != 0
        for c in range(3):
            if c != k:                       # components tangential to the face
                keep[on, c] = 0.0
    return keep


def h_update(E, H, op, a, gamma, rows=None):
    """H^{n+1} from E^n and H^n (first lines of eq. 19).

    ``rows`` (default: every node) names the centres the operator rows belong
    to, so that a subset of nodes can be updated on its own.
    """
    cw, ci = op["curl_w"], op["curl_idx"]
    hw, hi = op["hv_w"], op["hv_idx"]
    Hc = H if rows is None else H[rows]
    if H.shape[1] == 2:
        Ez = E[:, 0]
        Hx = Hc[:, 0] - a * (D(cw[:, 1], ci, Ez) - gamma * D(hw, hi, H[:, 0]))
        Hy = Hc[:, 1] + a * (D(cw[:, 0], ci, Ez) + gamma * D(hw, hi, H[:, 1]))
        return np.stack([Hx, Hy], axis=1)
    dx = lambda f: D(cw[:, 0], ci, f)
    dy = lambda f: D(cw[:, 1], ci, f)
    dz = lambda f: D(cw[:, 2], ci, f)
    Ex, Ey, Ez = E[:, 0], E[:, 1], E[:, 2]
    curl = [dy(Ez) - dz(Ey), dz(Ex) - dx(Ez), dx(Ey) - dy(Ex)]
    return np.stack([Hc[:, c] - a * (curl[c] - gamma * D(hw, hi, H[:, c])) for c in range(3)], axis=1)


def e_update(E, Hn, op, kappa, gamma, keep, src=None, rows=None, normals=None):
    """E^{n+1} from E^n and H^{n+1} (last line of eq. 19), then PEC.

    src = (nodes [S], values [S]) adds values at nodes after the bracket.
    ``rows`` as in h_update (keep and an array kappa are then per row).
    normals (3D) [N, 3]: unit normals of curved-wall nodes (see wall_project).
    """
    cw, ci = op["curl_w"], op["curl_idx"]
    hw, hi = op["hv_w"], op["hv_idx"]
    Ec = E if rows is None else E[rows]
    if Hn.shape[1] == 2:
        br = D(cw[:, 0], ci, Hn[:, 1]) - D(cw[:, 1], ci, Hn[:, 0]) + gamma * D(hw, hi, E[:, 0])
        out = (Ec[:, 0] + kappa * br)[:, None]
    else:
        dx = lambda f: D(cw[:, 0], ci, f)
        dy = lambda f: D(cw[:, 1], ci, f)
        dz = lambda f: D(cw[:, 2], ci, f)
        Hx, Hy, Hz = Hn[:, 0], Hn[:, 1], Hn[:, 2]
        curl = [dy(Hz) - dz(Hy), dz(Hx) - dx(Hz), dx(Hy) - dy(Hx)]
        out = np.stack([Ec[:, c] + kappa * (curl[c] + gamma * D(hw, hi, E[:, c])) for c in range(3)], axis=1)
    if src is not None:
        nodes, vals = src
        for s in range(len(nodes)):
            out[nodes[s], 0 if out.shape[1] == 1 else 2] += vals[s]
    return wall_project(out, keep, normals)


# ---------------------------------------------------------------------------
# 2D TEz polarisation (Hz, Ex, Ey): the same leapfrog and hyperviscosity with
# the roles of the fields exchanged.  From the curl equations with the fields
# (Ex, Ey, 0) and (0, 0, Hz):
#   mu0 dHz/dt = -(dEy/dx - dEx/dy),  eps0 dEx/dt = dHz/dy,  eps0 dEy/dt = -dHz/dx,
# so one step is
#   Hz <- Hz - a (D^dx Ey - D^dy Ex - gamma D^hv Hz)
#   Ex <- Ex + kappa (D^dy Hz_new + gamma D^hv Ex)
#   Ey <- Ey + kappa (-D^dx Hz_new + gamma D^hv Ey)
# with Hz^n = Hz(t_{n-1/2}) and a perfectly conducting wall zeroing the E
# component tangential to it (Ey on x = const walls, Ex on y = const walls).
# ---------------------------------------------------------------------------
def te_h_update(E, Hz, op, a, gamma, rows=None):
    """Hz^{n+1} [N, 1] from E^n = (Ex, Ey) [N, 2] and Hz^n [N, 1]."""
    cw, ci = op["curl_w"], op["curl_idx"]
    hw, hi = op["hv_w"], op["hv_idx"]
    Hc = Hz if rows is None else Hz[rows]
    curl = D(cw[:, 0], ci, E[:, 1]) - D(cw[:, 1], ci, E[:, 0])
    return (Hc[:, 0] - a * (curl - gamma * D(hw, hi, Hz[:, 0])))[:, None]


def te_e_update(E, Hz_new, op, kappa, gamma, keep, rows=None, normals=None):
    """E^{n+1} [N, 2] from E^n and Hz^{n+1}, then the PEC rule of
    ``wall_project`` (factors ``keep``, curved-wall ``normals``)."""
    cw, ci = op["curl_w"], op["curl_idx"]
    hw, hi = op["hv_w"], op["hv_idx"]
    Ec = E if rows is None else E[rows]
    h = Hz_new[:, 0]
    Ex = Ec[:, 0] + kappa * (D(cw[:, 1], ci, h) + gamma * D(hw, hi, E[:, 0]))
    Ey = Ec[:, 1] + kappa * (-D(cw[:, 0], ci, h) + gamma * D(hw, hi, E[:, 1]))
    return wall_project(np.stack([Ex, Ey], axis=1), keep, normals)


def wall_project(E, keep, normals=None):
    """PEC on the vector E [N, 2] (TEz) or [N, 3] (3D): the tangential part
    vanishes on the wall.

    Component c survives where keep[:, c] = 1 (walls normal to an axis); at a
    node with a unit normal n (a curved wall) only the normal component
    survives, E <- (E . n) n.  ``normals`` [N, 2 or 3] is zero off the wall."""
    out = E * keep
    if normals is not None:
        sel = np.abs(normals).sum(axis=1) > 0
        en = (E[sel] * normals[sel]).sum(axis=1)
        out[sel] = en[:, None] * normals[sel]
    return out


def pec_keep_te(flags):
    """[N, 2] factors: a wall normal to x keeps only Ex, one normal to y only Ey."""
    flags = np.asarray(flags)
    keep = np.ones((flags.size, 2))
    keep[(flags & 3) != 0, 1] = 0.0
    keep[(flags & 12) != 0, 0] = 0.0
    return keep


def run_te(E, Hz, op, dt, steps, gamma, kappa, keep, mu0=1.0, eps0=1.0, h=None, energy_every=0,
           normals=None):
    """TEz counterpart of ``run``: returns (E, Hz, energies)."""
    a = dt / mu0
    eta0 = math.sqrt(mu0 / eps0)
    E = np.array(E, dtype=np.float64)
    Hz = np.array(Hz, dtype=np.float64)
    energies = []
    for n in range(steps):
        Hn = te_h_update(E, Hz, op, a, gamma)
        if energy_every and n % energy_every == 0:
            energies.append(energy(E, Hz, Hn, h, h, eta0, 2))
        E = te_e_update(E, Hn, op, kappa, gamma, keep, normals=normals)
        Hz = Hn
    return E, Hz, np.array(energies)


def energy(E, H_old, H_new, h_e, h_h, eta0, dim):
    """U = h^d sum (|E|^2 + eta0^2 |(H_old + H_new)/2|^2) (eq. 20).

    For the two-set variant h_e and h_h are the spacings of the E and H sets.
    """
    Hb = 0.5 * (H_old + H_new)
    return h_e ** dim * (E * E).sum() + eta0 ** 2 * h_h ** dim * (Hb * Hb).sum()


def linf_errors(E, H, Ea, Ha):
    """(||e||_inf^E, ||e||_inf^H) of eq. 23."""
    return float(np.abs(E - Ea).max()), float(np.abs(H - Ha).max())


def rel_l2(x, ref):
    """Relative L2 error, maximum over components."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64).T).T
    ref = np.atleast_2d(np.asarray(ref, dtype=np.float64).T).T
    errs = []
    for c in range(ref.shape[1]):
        nr = np.linalg.norm(ref[:, c])
        if nr == 0.0:
            continue
        errs.append(np.linalg.norm(x[:, c] - ref[:, c]) / nr)
    return max(errs) if errs else 0.0


def run(E, H, op_h, op_e, dt, steps, gamma, kappa, keep, mu0=1.0, eps0=1.0,
        h_e=None, h_h=None, energy_every=0, src=None, rcv=None, normals=None):
    """Advance ``steps`` full leapfrog steps.

    kappa: scalar or [N_E] array (dt / (eps0 eps_r)).
    src = (nodes [S], amps [S], wave [steps, S]) -> soft sources.
    rcv = nodes [R] -> traces [steps, R] of E (last component) after each step.
    Returns (E, H, energies, traces); energies[k] = U^{k * energy_every}.
    """
    a = dt / mu0
    eta0 = math.sqrt(mu0 / eps0)
    dim = 2 if H.shape[1] == 2 else 3
    energies = []
    traces = [] if rcv is not None else None
    E = np.array(E, dtype=np.float64)
    H = np.array(H, dtype=np.float64)
    for n in range(steps):
        Hn = h_update(E, H, op_h, a, gamma)
        if energy_every and n % energy_every == 0:
            energies.append(energy(E, H, Hn, h_e, h_h, eta0, dim))
        s = None
        if src is not None:
            s = (src[0], src[1] * src[2][n])
        E = e_update(E, Hn, op_e, kappa, gamma, keep, s, normals=normals)
        H = Hn
        if rcv is not None:
            traces.append(E[rcv, -1].copy())
    return E, H, np.array(energies), (np.array(traces) if traces is not None else None)


def run_batched(Es, Hs, op, dt, steps, gamma, kappa, keep, mu0=1.0):
    """K independent runs sharing one operator set (a loop over the fields)."""
    outE, outH = [], []
    for k in range(len(Es)):
        E, H, _, _ = run(Es[k], Hs[k], op, op, dt, steps, gamma, kappa, keep, mu0=mu0)
        outE.append(E)
        outH.append(H)
    return np.stack(outE), np.stack(outH)


# ---------------------------------------------------------------------------
# Discrete adjoint of the 2D TMz update (collocated operators)
# ---------------------------------------------------------------------------

def DT(w, idx, v, N):
    """(D^L)^T v: scatter sum_i w_ij v_i into every source node j."""
    out = np.zeros(N)
    np.add.at(out, idx.reshape(-1), (w * v[:, None]).reshape(-1))
    return out


def adjoint_2d(E0, H0, op, dt, steps, gamma, eps_r, keep, eps0=1.0, mu0=1.0,
               src=None, rcv=None, grad_traces=None):
    """Gradient of J(traces) w.r.t. eps_r [N] and the source amplitudes [S].

    Forward (state after step n: H^n = H(t_{n-1/2}), E^n):
      H^{n+1} = (I + B) H^n + A E^n,          A = a [-D^dy; D^dx], B = a gamma D^hv
      E^{n+1} = P[(I + K G) E^n + K C H^{n+1} + s^{n+1}],
      C = [-D^dy, D^dx], G = gamma D^hv, K = diag(kappa), P = PEC projector.
    traces[n-1, r] = E^n at receiver r (n = 1..T); grad_traces = dJ/dtraces.
    Reverse (n = T-1 .. 0, mu = P lambda_E^{n+1}):
      lamH_hat = lambda_H^{n+1} + C^T K mu
      lambda_E^n = mu + G^T K mu + A^T lamH_hat + r^n
      lambda_H^n = (I + B^T) lamH_hat
      dJ/deps_r,i += -(mu_i / eps_r,i) (E^{n+1}_i - E^n_i - s^{n+1}_i)
      dJ/da_s     += g_s^n mu_{node_s}
    where r^n is the receiver residual of E^n (n >= 1).
    """
    N = E0.shape[0]
    a = dt / mu0
    kappa = dt / (eps0 * eps_r)
    P = keep[:, 0]
    cw, ci = op["curl_w"], op["curl_idx"]
    hw, hi = op["hv_w"], op["hv_idx"]
    # forward sweep, storing every E^n (and E^T)
    Es = [np.array(E0[:, 0], dtype=np.float64)]
    svals = []
    E = np.array(E0, dtype=np.float64)
    H = np.array(H0, dtype=np.float64)
    for n in range(steps):
        Hn = h_update(E, H, op, a, gamma)
        s = None
        sv = np.zeros(N)
        if src is not None:
            vals = src[1] * src[2][n]
            s = (src[0], vals)
            np.add.at(sv, src[0], vals)
        E = e_update(E, Hn, op, kappa, gamma, keep, s)
        H = Hn
        Es.append(E[:, 0].copy())
        svals.append(sv)
    lamE = np.zeros(N)
    lamH = np.zeros((N, 2))
    if rcv is not None:
        np.add.at(lamE, rcv, grad_traces[steps - 1])
    g_eps = np.zeros(N)
    g_amp = np.zeros(len(src[0])) if src is not None else None
    for n in range(steps - 1, -1, -1):
        mu = P * lamE
        Kmu = kappa * mu
        lhx = lamH[:, 0] - DT(cw[:, 1], ci, Kmu, N)
        lhy = lamH[:, 1] + DT(cw[:, 0], ci, Kmu, N)
        newE = mu + gamma * DT(hw, hi, Kmu, N) + a * (-DT(cw[:, 1], ci, lhx, N) + DT(cw[:, 0], ci, lhy, N))
        if rcv is not None and n >= 1:
            np.add.at(newE, rcv, grad_traces[n - 1])
        lamH = np.stack([lhx + a * gamma * DT(hw, hi, lhx, N),
                         lhy + a * gamma * DT(hw, hi, lhy, N)], axis=1)
        g_eps += -(mu / eps_r) * (Es[n + 1] - Es[n] - svals[n]) * (P > 0)
        if src is not None:
            g_amp += src[2][n] * mu[src[0]]
        lamE = newE
    return g_eps, g_amp, np.stack(Es[1:])[:, rcv] if rcv is not None else None
