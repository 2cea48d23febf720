"""Matched absorber and line ports (the open-structure terminations of the
guide, microstrip and metascreen structures of Sec. V-B to V-D): pins of the
oracle's lossy leapfrog with graded electric and magnetic losses, eq.
(MNAform) with D_sigma_m != 0.

The paper fixes only the absorber's order (4) and thickness (5 cells); the
peak conductivity follows the continuum design rule for a reflection of
exp(-8) (a reading).  The pins check what the physics fixes: the profile
and the matching condition, the design rule against quadrature, energy
conservation with PEC ends, and that the matched layer absorbs far better
than an electric-only layer of the same sigma_e.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import yee


def test_graded_profile_and_matching_condition():
    ncell, order, smax = 5, 4, 10.0
    prof = W.graded_absorber(ncell, order, smax)
    depth = np.array([4.5, 3.5, 2.5, 1.5, 0.5]) / 5
    assert np.allclose(prof, smax * depth ** 4, rtol=0, atol=1e-15)
    assert np.all(np.diff(prof) < 0)  # outermost cell most lossy
    wl = W.waveguide2d(nx=40, ny=8, src_x=15, probe_x=(25,))
    eps0 = 1.0 / (yee.MU0 * yee.C0 ** 2)
    m = wl.sigma_e > 0
    assert m[:, :5].all() and m[:, -5:].all() and not m[:, 5:-5].any()
    # sigma_m / mu = sigma_e / eps in every absorber cell
    assert np.allclose(wl.sigma_m[m] / yee.MU0, wl.sigma_e[m] / (eps0 * wl.eps_r[m]), rtol=1e-9)
    # left and right layers mirror each other
    assert np.array_equal(wl.sigma_e[:, :5], wl.sigma_e[:, -5:][:, ::-1])


def test_design_rule_against_quadrature():
    """round trip exp(-2 eta int sigma dx) through the continuous graded layer
    equals the requested reflection"""
    ncell, order, d, eps_r, refl = 5, 4, 1e-3, 2.5, math.exp(-8)
    smax = W.absorber_sigma_max(ncell, order, d, eps_r, refl)
    delta = ncell * d
    eta = yee.MU0 * yee.C0 / math.sqrt(eps_r)
    integral, _ = integrate.quad(lambda x: smax * (x / delta) ** order, 0.0, delta)
    assert math.exp(-2 * eta * integral) == pytest.approx(refl, rel=1e-12)


def _energy_after(wl, nsteps, at):
    op = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    B = yee.port_matrix(op, wl.sources, True)
    L = yee.port_matrix(op, wl.probes, False)
    R, _ = yee.R_F(op, dt)
    u = W.drive(wl, dt, nsteps)
    _, st = yee.leapfrog(op, dt, B, u, L, return_states=True)
    return [yee.energy(R, st[k]) for k in at], u


def test_matched_layer_absorbs_and_pec_ends_conserve():
    """A mode-shaped pulse (8-16 GHz, cutoff 5.9 GHz) launched from a line
    source crosses the guide about four times by step 1500.  PEC ends keep all
    the injected energy (the lossless energy of condition (Dstability2) is
    constant once the source is off); the matched layer leaves under 2 % of
    it and under a quarter of what an electric-only layer leaves."""
    at = (400, 1500, 2000)
    (p4, p15, p20), u = _energy_after(W.waveguide2d(absorber=0), 2001, at)
    assert np.abs(u[400:]).max() < 1e-12 * np.abs(u).max()
    assert abs(p15 - p4) <= 1e-9 * p4 and abs(p20 - p4) <= 1e-9 * p4
    (_, m15, _), _ = _energy_after(W.waveguide2d(), 2001, at)
    (_, e15, _), _ = _energy_after(W.waveguide2d(matched=False), 2001, at)
    assert m15 < 0.02 * p4
    assert m15 < 0.25 * e15
