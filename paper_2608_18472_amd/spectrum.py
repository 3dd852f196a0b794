"""High-harmonic spectra of observable series and the plateau-band error.

Section IV.A: the harmonic spectrum is the squared modulus of the windowed
Fourier transform of the dipole acceleration, or omega^4 times that of the
dipole itself, with an apodisation window W(t) against edge artefacts; the
paper names a Kaiser window as an example and gives no shape parameter.
Reading taken here: a Kaiser window with beta = 8 over the whole record
(numpy's `kaiser` convention), the transform zero-padded to
2^ceil(log2(4 (n+1))) points, X(w) = sum_n W_n f_n exp(i w t_n) dt.

The plateau-band error compares two spectra at the odd harmonics
q = 3 .. floor(q_cut) + 6 of the carrier w0: S at harmonic q is the largest
value of S on the bins within [q - 1/4, q + 1/4] w0 (the harmonic peak), and
the error is max_q |log10 S_test(q) - log10 S_ref(q)| in decades ("dex").
q_cut = (I_p + 3.17 U_p) / w0 with U_p = E0^2 / (4 w0^2) is the
semiclassical cutoff law used for the molecular spectra of section VII.C.

Analysis of series only: nothing here takes part in the propagation.
"""
import math

import numpy as np

KAISER_BETA = 8.0


def spectrum(series, dt, kind="dipole", beta=KAISER_BETA, pad=4):
    """(w, S): angular frequencies of the one-sided DFT grid and the spectrum
    S(w) = w^4 |X_d(w)|^2 (kind "dipole") or |X_a(w)|^2 (kind "accel")."""
    f = np.asarray(series, dtype=np.float64)
    n1 = f.shape[-1]
    nfft = 1 << int(math.ceil(math.log2(pad * n1)))
    X = np.fft.rfft(f * np.kaiser(n1, beta), n=nfft) * dt
    w = 2.0 * math.pi * np.fft.rfftfreq(nfft, d=dt)
    S = np.abs(X) ** 2
    if kind == "dipole":
        S = S * w ** 4
    elif kind != "accel":
        raise ValueError("kind must be 'dipole' or 'accel'")
    return w, S


def harmonic_peaks(w, S, omega, qs, halfwidth=0.25):
    """Largest S on the bins within [q - halfwidth, q + halfwidth] omega,
    for every order q in qs."""
    out = np.empty(len(qs))
    for i, q in enumerate(qs):
        sel = (w >= (q - halfwidth) * omega) & (w <= (q + halfwidth) * omega)
        if not np.any(sel):
            raise ValueError("no DFT bin near harmonic %g" % q)
        out[i] = S[sel].max()
    return out


def cutoff_order(ip, e0, omega):
    """Semiclassical cutoff order (I_p + 3.17 U_p) / omega, U_p = E0^2/(4 w^2)."""
    up = e0 * e0 / (4.0 * omega * omega)
    return (ip + 3.17 * up) / omega


def plateau_orders(q_cut, extra=6):
    """Odd harmonic orders 3 .. floor(q_cut) + extra."""
    return [q for q in range(3, int(math.floor(q_cut)) + extra + 1) if q % 2 == 1]


def plateau_error(test, ref, dt, omega, q_cut, kind="dipole", beta=KAISER_BETA):
    """max over the plateau-band odd harmonics of |log10 S_test - log10 S_ref|."""
    qs = plateau_orders(q_cut)
    w, st = spectrum(test, dt, kind, beta)
    _, sr = spectrum(ref, dt, kind, beta)
    pt = harmonic_peaks(w, st, omega, qs)
    pr = harmonic_peaks(w, sr, omega, qs)
    return float(np.max(np.abs(np.log10(pt) - np.log10(pr))))
