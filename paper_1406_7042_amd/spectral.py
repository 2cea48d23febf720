"""Reading resonances and transmission coefficients from probe spectra.

The spectra come from the library's probe_dft kernel (yeerom.probe_dft);
what is here is the small host-side read-out of its [nf, nprb] result, as
Sec. V reports it: the resonant frequencies of a cavity (Sec. V-A) and the
ratio of the spectra of two probes, S21 of a guide (Sec. V-B, V-D).
"""
from __future__ import annotations

import numpy as np


def resonances(freqs, Y, count: int, record: float, lobes: float = 4.0,
               floor: float = 1e-4) -> np.ndarray:
    """The first ``count`` resonant frequencies (ascending) in Hann-tapered
    spectra Y [nf, nprb] of records ``record`` seconds long, sampled on the
    ascending, uniform grid ``freqs``.  A resonance is a sample whose power
    (summed over probes) is the largest within +-lobes / record (the taper's
    main lobe spans +-2 / record; its side lobes fall below 1e-4 of the peak
    beyond +-4 / record) and above ``floor`` times the largest power; it is
    refined by the vertex of the parabola through the log power at the three
    samples around it.  Fewer are returned if fewer peaks exist."""
    f = np.asarray(freqs, dtype=np.float64).ravel()
    Y = np.asarray(Y)
    if Y.ndim == 1:
        Y = Y[:, None]
    if f.size < 3 or Y.shape[0] != f.size:
        raise ValueError("need at least 3 frequencies, one spectrum row per frequency")
    step = f[1] - f[0]
    if step <= 0 or not np.allclose(np.diff(f), step, rtol=1e-6, atol=0):
        raise ValueError("frequencies must be ascending and uniformly spaced")
    if not record > 0:
        raise ValueError("record length must be positive")
    p = np.sum(np.abs(Y) ** 2, axis=1)
    top = p.max()
    if not top > 0:
        return np.zeros(0)
    w = max(1, int(round(lobes / record / step)))
    out = []
    for k in range(1, f.size - 1):
        lo, hi = max(0, k - w), min(f.size, k + w + 1)
        if p[k] > floor * top and p[k] >= p[lo:hi].max() and p[k] > p[k + 1]:
            a, b, c = np.log(p[k - 1:k + 2])
            den = a - 2 * b + c
            off = 0.5 * (a - c) / den if den < 0 else 0.0
            out.append(f[k] + off * step)
            if len(out) == count:
                break
    return np.array(out)


def transmission(Y_out, Y_in) -> np.ndarray:
    """S21-type ratio of two probe spectra (same frequencies): the wave that
    reaches the output probe over the wave that passed the input probe."""
    Y_out = np.asarray(Y_out)
    Y_in = np.asarray(Y_in)
    return Y_out / Y_in
