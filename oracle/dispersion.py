"""Numerical dispersion of a run, measured as in Section 6 (eq. 24-26).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

Input: E on the N_x equispaced nodes of the line y = L/2 (spacing h), saved
every ``save_every`` steps: samples [N_t, N_x].  The field is transformed to
(k, omega) with k_i = 2 pi i / N_x (per h) and omega_j = 2 pi j /
(save_every N_t) (per step), after a Hann window along time.  For each
frequency the wavenumber of largest magnitude gives a propagation speed
c(omega_j) = omega_j / k_i(j) (eq. 24), its error against the exact speed
S_c = c0 dt / h = 1/(10 sqrt 2) in these units is err(omega_j) (eq. 25), and
the sum of err over j = 1..45 is the scalar summary ||err||_1 (eq. 26).

Readings (the paper does not spell them out):
* sign convention: the transform pairs e^{-i k x} with e^{+i omega t}, so a
  pulse moving towards +x puts its energy at omega = c k with both indices
  in the lower half (a wave moving towards -x lands at i > N_x / 2);
* the window is the symmetric Hann window of length N_t;
* j = 0 is left out of the sum: omega_0 = 0 gives c = 0 / k, undefined at the
  DC peak (k_0 = 0).
"""
import math

import numpy as np


def exact_speed():
    """Propagation speed of the continuous waves in units h per step: S_c."""
    return 1.0 / (10.0 * math.sqrt(2.0))


def spectrum(samples):
    """|E(k_i, omega_j)| for samples [N_t, N_x] -> [N_t (j), N_x (i)]."""
    e = np.asarray(samples, dtype=np.float64)
    nt = e.shape[0]
    w = np.hanning(nt)[:, None]
    a = np.fft.fft(e * w, axis=1)              # sum_x e^{-i k x}
    b = np.fft.ifft(a, axis=0) * nt            # sum_t e^{+i omega t}
    return np.abs(b)


def wavenumbers(nx):
    return 2.0 * math.pi * np.arange(nx) / nx


def frequencies(nt, save_every):
    return 2.0 * math.pi * np.arange(nt) / (save_every * nt)


def phase_speed(samples, save_every):
    """(i(j), c(omega_j)) of eq. 24 for every frequency index j (c[0] = nan)."""
    s = spectrum(samples)
    nt, nx = s.shape
    idx = np.argmax(s, axis=1)
    k = wavenumbers(nx)[idx]
    om = frequencies(nt, save_every)
    with np.errstate(divide="ignore", invalid="ignore"):
        c = om / k
    c[0] = np.nan
    return idx, c


def err_l1(samples, save_every, jmax=45):
    """||err||_1 of eq. 26 summed over j = 1..jmax, with err of eq. 25."""
    _, c = phase_speed(samples, save_every)
    err = np.abs(c[1:jmax + 1] - exact_speed())
    return float(err.sum()), err


def line_samples(traces, save_every):
    """Every save_every-th row of per-step traces [T, N_x] (after steps
    save_every, 2 save_every, ..., T)."""
    tr = np.asarray(traces)
    return tr[save_every - 1::save_every]
