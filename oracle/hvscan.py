"""Hyperviscosity parameter search (Section 5.1 with Figures 5-6; Section 6).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

The paper fixes the hyperviscosity exponent alpha and constant c by running
the problem for several c and watching the relative energy u(t) = U(t)/U(0) of
eq. 20: inside an interval of c the solution stays bounded, outside it
diverges, and a bisection on c (the approach of the paper's ref. [20]) is used
where a fine sweep would be slow.  Section 6 accepts a value when u(t) stays
inside [0.99, 1.01] over the whole run.

Reading used here (the paper gives no more detail): a candidate c is accepted
when every energy sample is finite and inside the band [u_lo, u_hi].  The
search narrows a bracket [c_lo, c_hi] of the lower edge of the accepted
interval (the least dissipative stable value).  Each round tries K candidates
spaced geometrically over the bracket, endpoints included:
    c_k = c_lo * (c_hi / c_lo) ** (k / (K - 1)),   k = 0 .. K-1,
and the next bracket is [c_{k*-1}, c_{k*}] with k* the smallest accepted index.
K = 3 is bisection on log c; larger K shrinks the bracket by K - 1 per round.
The search stops early when nothing is accepted ("none") or when c_lo itself
is accepted ("below": the edge lies under the bracket).
"""
import math

import numpy as np

from . import step as _step


def candidates(c_lo, c_hi, K):
    """The K geometric candidates of one round, endpoints included."""
    k = np.arange(K, dtype=np.float64)
    return c_lo * (c_hi / c_lo) ** (k / (K - 1))


def accepted(u, band):
    """True when every sample of u is finite and inside [band[0], band[1]]."""
    u = np.asarray(u, dtype=np.float64)
    return bool(np.all(np.isfinite(u)) and np.all(u >= band[0]) and np.all(u <= band[1]))


def k_section(classify, c_lo, c_hi, K, rounds):
    """Narrow the bracket of the lower edge of the accepted interval.

    classify(cs [K]) -> bool [K].  Returns {"status", "c_best", "bracket",
    "history": [(cs, ok), ...]}; status is "bracketed", "below" or "none".
    """
    if not (0 < c_lo < c_hi) or K < 3 or rounds < 1:
        raise ValueError("need 0 < c_lo < c_hi, K >= 3, rounds >= 1")
    hist = []
    lo, hi = c_lo, c_hi
    best = None
    status = "bracketed"
    for _ in range(rounds):
        cs = candidates(lo, hi, K)
        ok = np.asarray(classify(cs), dtype=bool)
        hist.append((cs, ok))
        if not ok.any():
            status = "none" if best is None else status
            break
        ks = int(np.argmax(ok))
        best = float(cs[ks])
        if ks == 0:
            status = "below"
            break
        lo, hi = float(cs[ks - 1]), float(cs[ks])
    return {"status": status, "c_best": best, "bracket": (lo, hi), "history": hist}


def energy_ratios(E0, H0, op_h, op_e, dt, steps, every, cs, alpha, h, kappa, keep, mu0=1.0,
                  eps0=1.0):
    """u_k = U(t)/U(0) sampled every ``every`` steps, one run per constant c_k.

    Every run starts from the same (E0, H0); only gamma = c_k (-1)^(alpha-1)
    h^(2 alpha) differs (Section 5.1).  Returns [K, samples].
    """
    out = []
    for c in cs:
        g = _step.hv_gamma(float(c), alpha, h)
        # a rejected c may overflow: its samples become inf or nan
        with np.errstate(all="ignore"):
            _, _, en, _ = _step.run(E0, H0, op_h, op_e, dt, steps, g, kappa, keep, mu0=mu0,
                                    eps0=eps0, h_e=h, h_h=h, energy_every=every)
            out.append(en / en[0])
    return np.array(out)


def hv_scan(E0, H0, op_h, op_e, dt, steps, every, alpha, h, kappa, keep, c_lo, c_hi, K, rounds,
            band=(0.99, 1.01), mu0=1.0, eps0=1.0):
    """The search of ``k_section`` with runs of the stabilised leapfrog (eq. 19).

    Adds "u" (the energy ratios of every round, [K, samples] each) to the
    result.
    """
    us = []

    def classify(cs):
        u = energy_ratios(E0, H0, op_h, op_e, dt, steps, every, cs, alpha, h, kappa, keep, mu0,
                          eps0)
        us.append(u)
        return [accepted(row, band) for row in u]

    res = k_section(classify, c_lo, c_hi, K, rounds)
    res["u"] = us
    return res


def bracket_width(c_lo, c_hi, K, rounds):
    """Ratio hi/lo of the bracket after ``rounds`` full rounds."""
    return math.exp(math.log(c_hi / c_lo) / (K - 1) ** rounds)
