"""Satellite-peak finder for comparing spectral functions (test and report helper).

The paper's criterion for the lowest satellite is in its supporting
information, which is not available.  Reading used here: the quasiparticle
line Z eta / (pi ((w - E_QP)^2 + eta^2)) is subtracted from A; satellites are
the local maxima of the remainder more than 0.5 eV below E_QP whose height is
at least 5 % of the remainder's largest value there, refined by a parabola
through the maximum and its two neighbours.
"""
import numpy as np

EV_PER_HA = 27.211386245988


def satellite_peaks(w, A, e_qp, Z, eta, min_sep_ev=0.5, rel_height=0.05):
    w = np.asarray(w)
    A = np.asarray(A) - Z * (eta / np.pi) / ((np.asarray(w) - e_qp) ** 2 + eta * eta)
    region = w < e_qp - min_sep_ev / EV_PER_HA
    if not np.any(region):
        return []
    top = np.max(A[region])
    idx = np.where((A[1:-1] > A[:-2]) & (A[1:-1] >= A[2:]))[0] + 1
    out = []
    for i in idx:
        if not region[i] or A[i] < rel_height * top:
            continue
        y0, y1, y2 = A[i - 1], A[i], A[i + 1]
        den = y0 - 2 * y1 + y2
        dx = 0.5 * (y0 - y2) / den if den != 0 else 0.0
        out.append(w[i] + dx * (w[i + 1] - w[i]))
    return out
