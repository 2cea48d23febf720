"""Frequency-domain read-out of probe records (Sec. V).  FP64, test
infrastructure only.

Sec. V measures accuracy in the frequency domain: the first six resonant
frequencies of the PEC cavities against analytical values (Sec. V-A), and the
transmission coefficient S21 of the waveguide (Sec. V-B) and S11, S21 of the
microstrip (Sec. V-D), all read from spectra of time-domain probe records.

* ``dtft``: the discrete-time Fourier transform of a sampled record at
  arbitrary frequencies, written out as its defining sum.
* ``box_resonances``: the resonant frequencies of the Yee leapfrog in an
  empty PEC box.  A mode of wavenumbers m_d pi / (n_d Delta_d) has the
  singular value sigma = 2 c sqrt(sum_d sin^2(m_d pi / 2 n_d) / Delta_d^2) of
  D_eps^-1/2 K D_mu^-1/2, and the leapfrog rotates it by theta per step with
  sin(theta / 2) = dt sigma / 2 (Sec. II-B), i.e. f = asin(dt sigma / 2) / (pi dt).
  Its limit dt, Delta -> 0 is the analytical cavity resonance
  c/2 sqrt(sum (m_d / a_d)^2) that Sec. V-A compares against.
* ``guide_wavenumber``: the axial wavenumber of the lowest mode of a
  parallel-plate guide on the same grid, from the same relation with the
  transverse index fixed at 1 (Sec. V-B guide, filled with eps_r).
"""
from __future__ import annotations

import math

import numpy as np

C0 = 299792458.0


def dtft(y: np.ndarray, dt: float, freqs, t0: float = 0.0, hann: bool = False) -> np.ndarray:
    """Y[k, p] = dt sum_n w_n y[n, p] exp(-j 2 pi f_k (t0 + n dt)), w_n = 1 or
    the Hann taper sin^2(pi (n + 1/2) / N)."""
    y = np.asarray(y, dtype=np.float64)
    if y.ndim == 1:
        y = y[:, None]
    n = np.arange(y.shape[0])
    w = np.sin(np.pi * (n + 0.5) / y.shape[0]) ** 2 if hann else np.ones(y.shape[0])
    t = t0 + n * dt
    f = np.asarray(freqs, dtype=np.float64).ravel()
    E = np.exp(-2j * np.pi * np.outer(f, t))
    return dt * (E @ (w[:, None] * y))


def distinct(f, rel: float = 1e-9) -> np.ndarray:
    """Ascending values with those within rel of the previous kept one merged."""
    out = []
    for v in np.sort(np.asarray(f, dtype=np.float64).ravel()):
        if not out or v > out[-1] * (1 + rel):
            out.append(v)
    return np.array(out)


def box_resonances(ncells, spacings, dt: float, eps_r: float = 1.0, fmax=None,
                   ez_pol_2d: bool = False) -> np.ndarray:
    """Distinct resonant frequencies (ascending) of the Yee leapfrog at time
    step dt in an empty PEC box of ncells = (nx, ny[, nz]) uniform cells of
    spacings (dx, dy[, dz]) filled with eps_r.  2-D Ez-polarisation: indices
    m, n >= 1.  3-D: index triples with at most one zero (TE and TM modes)."""
    c = C0 / math.sqrt(eps_r)
    dims = len(ncells)
    ranges = []
    for a in range(dims):
        lo = 1 if ez_pol_2d else 0
        ranges.append(np.arange(lo, ncells[a]))
    grids = np.meshgrid(*ranges, indexing="ij")
    nz = sum((g > 0).astype(int) for g in grids)
    keep = nz >= (dims - 1 if dims == 3 else dims)
    s2 = sum(np.sin(g * np.pi / (2 * ncells[a])) ** 2 / spacings[a] ** 2
             for a, g in enumerate(grids))
    sig = 2 * c * np.sqrt(s2[keep])
    arg = dt * sig / 2
    f = distinct(np.arcsin(arg[arg < 1]) / (np.pi * dt))  # degenerate modes: one frequency
    if fmax is not None:
        f = f[f <= fmax]
    return f


def analytic_box_resonances(sides, eps_r: float = 1.0, count: int = 6, ez_pol_2d=False):
    """Continuum PEC-box resonances c/2 sqrt(sum (m_d / a_d)^2), distinct,
    ascending (the analytical values Sec. V-A compares against)."""
    c = C0 / math.sqrt(eps_r)
    dims = len(sides)
    out = set()
    top = 12
    for idx in np.ndindex(*([top] * dims)):
        nzc = sum(1 for v in idx if v > 0)
        if ez_pol_2d and nzc < dims:
            continue
        if not ez_pol_2d and nzc < dims - 1:
            continue
        out.add(round(c / 2 * math.sqrt(sum((v / a) ** 2 for v, a in zip(idx, sides))), 3))
    return np.array(sorted(out)[:count])


def guide_wavenumber(f, dx: float, dy: float, ny: int, dt: float, eps_r: float) -> np.ndarray:
    """Axial wavenumber beta(f) [rad/m] of the lowest mode (transverse index 1)
    of a 2-D Ez-polarised parallel-plate guide of ny cells between PEC plates:
    (sin(pi f dt) / (c dt))^2 = (sin(beta dx / 2) / dx)^2 + (sin(pi / 2 ny) / dy)^2.
    NaN below cutoff."""
    c = C0 / math.sqrt(eps_r)
    f = np.asarray(f, dtype=np.float64)
    lhs = (np.sin(np.pi * f * dt) / (c * dt)) ** 2 - (math.sin(math.pi / (2 * ny)) / dy) ** 2
    with np.errstate(invalid="ignore"):
        return 2.0 / dx * np.arcsin(dx * np.sqrt(lhs))
