"""Pins of the oracle's frequency-domain read-out (Sec. V) against facts fixed
by the mathematics: the FFT at its bins, the closed-form sum of a damped
sinusoid, the singular values of the assembled Yee operator, the modes of a
closed guide, and the paper's cube resonances (Sec. III-B).  Also the host
peak read-out of the package on oracle spectra."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import spectrum as S
from oracle import yee


def _golden(name):
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


def test_dtft_equals_fft_at_its_bins():
    rng = np.random.default_rng(11)
    y = rng.standard_normal((257, 3))
    dt = 1.3e-12
    k = np.arange(0, 257)
    f = k / (257 * dt)
    Y = S.dtft(y, dt, f)
    ref = dt * np.fft.fft(y, axis=0)
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_dtft_of_a_damped_sinusoid_is_a_geometric_sum():
    """y_n = a^n cos(w0 n dt): sum_n r^n = (1 - r^N) / (1 - r) for each of the
    two exponentials, r = a exp(+-j w0 dt - j w dt); with t0 the whole sum
    turns by exp(-j w t0)."""
    N, dt, a, f0, t0 = 3001, 2e-12, 0.999, 31e9, 5e-12
    n = np.arange(N)
    y = a ** n * np.cos(2 * np.pi * f0 * n * dt)
    f = np.array([0.0, 7e9, 30.5e9, 31e9, 44e9, -12e9])
    Y = S.dtft(y, dt, f, t0=t0)[:, 0]
    ref = np.zeros(f.size, complex)
    for sgn in (1, -1):
        r = a * np.exp(1j * 2 * np.pi * (sgn * f0 - f) * dt)
        ref += 0.5 * (1 - r ** N) / (1 - r)
    ref *= dt * np.exp(-2j * np.pi * f * t0)
    assert np.max(np.abs(Y - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_hann_taper_is_the_sine_squared_window():
    """With the taper, the DTFT of a constant record at f = 0 is dt times the
    window's sum, which is N / 2 for sin^2(pi (n + 1/2) / N)."""
    N, dt = 1000, 1e-12
    Y = S.dtft(np.ones(N), dt, [0.0], hann=True)
    assert Y[0, 0].real == pytest.approx(dt * N / 2, rel=1e-12)


@pytest.mark.parametrize("shape", [(6, 5), (4, 3, 5)])
def test_box_resonances_are_the_leapfrog_rotations_of_the_operator(shape):
    """f = asin(dt s / 2) / (pi dt) over the singular values s of
    De^-1/2 K Dm^-1/2 of the assembled box (Sec. II-B: the leapfrog turns a
    mode by theta per step, sin(theta/2) = dt s / 2)."""
    d = 1e-3
    if len(shape) == 2:
        wl = W.cavity2d(nx=shape[0], ny=shape[1], d=d, seed=0)
    else:
        wl = W.cavity3d(n=shape[0], ny=shape[1], nz=shape[2], d=d, seed=0, block=100,
                        eps_range=(1, 1), sigma_range=(0, 0), nports=1, margin=1)
    op = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    A = (op.K.toarray() / np.sqrt(op.De)[:, None]) / np.sqrt(op.Dm)[None, :]
    s = np.linalg.svd(A, compute_uv=False)
    s = s[s > 1e-6 * s.max()]
    fref = S.distinct(np.arcsin(dt * s / 2) / (np.pi * dt), rel=1e-8)
    f = S.box_resonances(shape, (d,) * len(shape), dt, ez_pol_2d=len(shape) == 2)
    assert f.shape == fref.shape
    assert np.allclose(f, fref, rtol=1e-9)


def test_guide_wavenumber_fits_the_modes_of_a_closed_guide():
    """A guide of nx cells closed by PEC walls resonates where the axial
    wavenumber of its lowest transverse mode is m pi / (nx dx)."""
    nx, ny, dx, dy, eps_r = 30, 8, 1e-3, 0.7e-3, 2.5
    dt = 0.99 / (C := S.C0) / math.sqrt(1 / dx ** 2 + 1 / dy ** 2)
    c = C / math.sqrt(eps_r)
    m = np.arange(1, nx)
    s = 2 * c * np.sqrt(np.sin(m * np.pi / (2 * nx)) ** 2 / dx ** 2
                        + math.sin(math.pi / (2 * ny)) ** 2 / dy ** 2)
    f = np.arcsin(dt * s / 2) / (np.pi * dt)
    beta = S.guide_wavenumber(f, dx, dy, ny, dt, eps_r)
    assert np.allclose(beta, m * np.pi / (nx * dx), rtol=1e-9)
    # the same frequencies are Yee box resonances of the filled guide
    fb = S.box_resonances((nx, ny), (dx, dy), dt, eps_r=eps_r, ez_pol_2d=True)
    assert np.all(np.min(np.abs(fb[None, :] - f[:, None]), axis=1) <= 1e-6 * f)


def test_analytic_resonances_of_the_section_IIIB_cube():
    g = _golden("cube_resonances.txt")
    f = S.analytic_box_resonances((1.0, 1.0, 1.0), count=2)
    assert f[0] / 1e9 == pytest.approx(g["f110_GHz"], abs=1e-5)
    assert f[1] / 1e9 == pytest.approx(g["f111_GHz"], abs=1e-5)


def test_box_resonances_converge_to_the_analytic_ones():
    """Sec. V-A compares against analytical cavity resonances: the Yee values
    approach them at second order in the spacing (dt at 0.99 of the CFL
    limit)."""
    errs = []
    for n in (20, 40):
        d = 1.0 / n
        dt = 0.99 * d / (S.C0 * math.sqrt(3))
        f = S.box_resonances((n, n, n), (d, d, d), dt)[:6]
        a = S.analytic_box_resonances((1.0, 1.0, 1.0), count=6)
        errs.append(np.max(np.abs(f - a) / a))
    assert errs[0] < 5e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_peak_readout_finds_the_first_six_resonances():
    """The package's host read-out (Hann spectrum on a fine grid, peak within
    +-4 bins, parabolic vertex) on the oracle's leapfrog record of a 2-D
    cavity: the first six resonances within 1e-3 of a frequency bin."""
    from paper_1406_7042_amd import spectral
    nx, ny, d = 24, 17, 1e-3
    wl = W.cavity2d(nx=nx, ny=ny, d=d, seed=3, f0=25e9, bw=40e9)
    op = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    B = yee.port_matrix(op, wl.sources, True)
    Lp = yee.port_matrix(op, wl.probes, False)
    nsteps = 8000
    y, _ = yee.leapfrog(op, dt, B, W.drive(wl, dt, nsteps), Lp)
    rec = nsteps * dt
    f = np.arange(1e9, 40e9, 1 / rec / 16)
    pk = spectral.resonances(f, S.dtft(y, dt, f, t0=dt, hann=True), 6, rec)
    ref = S.box_resonances((nx, ny), (d, d), dt, ez_pol_2d=True)[:6]
    assert pk.shape == (6,)
    assert np.max(np.abs(pk - ref)) * rec <= 1e-3
