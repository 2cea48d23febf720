"""Pins of the oracle's per-cell -> per-sample material averaging (Sec. II-A:
materials are given "for each cell"; the edge and face values are dual-area
and dual-length weighted means of the touching cells).

A layered medium separates: with eps_r and mu_r constant along x and a
uniform x spacing, every x-sine mode of a 2-D Ez-polarised PEC box obeys its
own 1-D generalised eigenproblem along y, written here directly from the
integral (finite-integration) form of Ampere's and Faraday's laws on the
dual and primal cells.  The union of those 1-D spectra over the x modes must
equal the spectrum of the oracle's assembled matrices, the singular values
of D_eps^-1/2 K D_mu^-1/2 (squared: the eigenvalues omega^2 of
D_eps^-1 K D_mu^-1 K^T).  A wrong orientation of the averages (the cells of
row j instead of rows j-1 and j), wrong weights (plain instead of
spacing-weighted means on a graded axis) or a swap of the electric and
magnetic rules changes those eigenvalues.

In 3-D the same families exist: fields that do not vary along one axis a,
with only the electric component along a, reduce to the 2-D Ez-polarised
problem in the plane normal to a, so the 3-D spectrum contains the 1-D
unions for the Ex, Ey and Ez families of a medium layered along another
axis.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import yee


def _union_1d(mu_xy_cell, eps_cell, mu_cell, dx, dy_nodes):
    """omega^2 of every x-sine mode m of an Ez-polarised layered box.

    eps_cell[j], mu_cell[j]: per-row cell values (j = 0..ny-1), graded
    spacings dy_nodes[j] of row j, uniform dx with nx cells.  Unknowns along
    y: Ez at nodes j = 1..ny-1.

    Ampere over the dual cell of node j (area dx * dual dy_j):
        eps_n(j) dx dyd_j dEz/dt = dyd_j (Hy(i+1/2) - Hy(i-1/2)) - dx (Hx(j+1/2) - Hx(j-1/2))
    with eps_n(j) the area-weighted mean of the rows j-1, j.
    Faraday on the primal edges: mu_x(j) dy_j dHx(j+1/2)/dt = -(Ez(j+1) - Ez(j)) (cells i-1, i
    of row j: mean mu of row j), mu_y(j) dx dHy(i+1/2, j)/dt = Ez(i+1) - Ez(i) (cells rows j-1, j
    weighted by dy: length-weighted mean).
    With Ez = sin(m pi i / nx) f_j, the x second difference gives -4 sin^2(m pi / 2 nx):
        omega^2 eps_n dyd f = [4 s_m^2 dyd / (mu_y dx^2)] f + (f_j - f_{j+1}) / (mu_x(j) dy_j)
                                                            + (f_j - f_{j-1}) / (mu_x(j-1) dy_{j-1})
    """
    nx = mu_xy_cell
    dy = np.asarray(dy_nodes, float)
    ny = len(dy)
    eps_cell = np.asarray(eps_cell, float) * yee.EPS0
    mu_cell = np.asarray(mu_cell, float) * yee.MU0
    js = np.arange(1, ny)
    dyd = 0.5 * (dy[js - 1] + dy[js])
    eps_n = (eps_cell[js - 1] * dy[js - 1] + eps_cell[js] * dy[js]) / (dy[js - 1] + dy[js])
    mu_y = (mu_cell[js - 1] * dy[js - 1] + mu_cell[js] * dy[js]) / (dy[js - 1] + dy[js])
    # stiffness along y (Ez vanishes at j = 0 and j = ny)
    T = np.zeros((ny - 1, ny - 1))
    for r, j in enumerate(js):
        gu = 1.0 / (mu_cell[j] * dy[j])  # edge j -> j+1 (row j)
        gd = 1.0 / (mu_cell[j - 1] * dy[j - 1])  # edge j-1 -> j (row j-1)
        T[r, r] = gu + gd
        if r + 1 < ny - 1:
            T[r, r + 1] = -gu
        if r > 0:
            T[r, r - 1] = -gd
    Mmat = np.diag(eps_n * dyd)
    out = []
    for m in range(1, nx):
        s2 = 4.0 * math.sin(m * math.pi / (2 * nx)) ** 2
        A = T + np.diag(s2 * dyd / (mu_y * dx * dx))
        out.append(sla.eigh(A, Mmat, eigvals_only=True))
    return np.sort(np.concatenate(out))


def _oracle_omega2(op):
    A = (op.K.toarray() / np.sqrt(op.De)[:, None]) / np.sqrt(op.Dm)[None, :]
    s = np.linalg.svd(A, compute_uv=False)
    return np.sort(s ** 2)


def _layered_2d(nx, ny, eps_rows, mu_rows, dy, dx=1e-3):
    wl = W.cavity2d(nx=nx, ny=ny, d=dx, seed=0)
    wl.dy = np.asarray(dy, float)
    wl.eps_r = np.repeat(np.asarray(eps_rows, float)[:, None], nx, axis=1)
    wl.mu_r = np.repeat(np.asarray(mu_rows, float)[:, None], nx, axis=1)
    wl.sigma_e = np.zeros((ny, nx))
    return wl


def test_layered_2d_spectrum_uniform_spacing():
    """eps_r varying from row to row (uniform grid): eigenvalues equal the union
    of the 1-D problems to 1e-12."""
    rng = np.random.default_rng(11)
    nx, ny = 7, 9
    eps_rows = rng.uniform(1.0, 6.0, ny)
    mu_rows = np.ones(ny)
    wl = _layered_2d(nx, ny, eps_rows, mu_rows, np.full(ny, 1e-3))
    op = yee.assemble(wl)
    ref = _union_1d(nx, eps_rows, mu_rows, 1e-3, np.full(ny, 1e-3))
    got = _oracle_omega2(op)
    assert len(got) == len(ref) == op.Ne
    assert np.allclose(got, ref, rtol=1e-12)


def test_layered_2d_spectrum_graded_eps_and_mu():
    """Graded y spacing with eps_r and mu_r varying by row: pins the
    dual-area (electric) and dual-length (magnetic) weights of the means."""
    rng = np.random.default_rng(12)
    nx, ny = 6, 8
    eps_rows = rng.uniform(1.0, 5.0, ny)
    mu_rows = rng.uniform(1.0, 3.0, ny)
    dy = rng.uniform(0.4e-3, 2.0e-3, ny)
    wl = _layered_2d(nx, ny, eps_rows, mu_rows, dy)
    op = yee.assemble(wl)
    ref = _union_1d(nx, eps_rows, mu_rows, 1e-3, dy)
    got = _oracle_omega2(op)
    assert np.allclose(got, ref, rtol=1e-12)


def test_layered_2d_spectrum_detects_a_shifted_average():
    """Control: the same 1-D construction with the electric mean taken over the
    wrong pair of rows (j, j+1) misses the oracle's spectrum."""
    rng = np.random.default_rng(11)
    nx, ny = 7, 9
    eps_rows = rng.uniform(1.0, 6.0, ny)
    wl = _layered_2d(nx, ny, eps_rows, np.ones(ny), np.full(ny, 1e-3))
    got = _oracle_omega2(yee.assemble(wl))
    shifted = np.concatenate([eps_rows[1:], eps_rows[-1:]])
    wrong = _union_1d(nx, shifted, np.ones(ny), 1e-3, np.full(ny, 1e-3))
    assert not np.allclose(got, wrong, rtol=1e-6)


def _contains(spectrum, values, rtol):
    """Every value has a partner in the spectrum within rtol."""
    idx = np.searchsorted(spectrum, values)
    for v, i in zip(values, idx):
        cands = spectrum[max(i - 1, 0):i + 1]
        if np.min(np.abs(cands - v)) > rtol * abs(v):
            return False
    return True


@pytest.mark.parametrize("layer_axis,family", [("y", "z"), ("y", "x"), ("z", "y")])
def test_layered_3d_spectrum_contains_2d_families(layer_axis, family):
    """3-D box with eps_r and mu_r layered along one axis on a graded spacing:
    the spectrum contains the omega^2 of the fields with only the electric
    component along `family` and no variation along it (they reduce to the
    Ez-polarised problem in the normal plane), which pins the edge means of
    Ex, Ey and Ez and the face means of the magnetic samples in 3-D."""
    rng = np.random.default_rng({"y": 21, "z": 22}[layer_axis] + ord(family))
    n = {"x": 5, "y": 6, "z": 4}
    nlay = n[layer_axis]
    eps_l = rng.uniform(1.0, 5.0, nlay)
    mu_l = rng.uniform(1.0, 2.5, nlay)
    dl = rng.uniform(0.5e-3, 2.0e-3, nlay)
    d = 1e-3
    wl = W.cavity3d(n=n["x"], ny=n["y"], nz=n["z"], d=d, seed=0, block=100, eps_range=(1, 1),
                    sigma_range=(0, 0), nports=1, margin=1)
    shape = (n["z"], n["y"], n["x"])
    ax = {"z": 0, "y": 1, "x": 2}[layer_axis]
    bshape = [1, 1, 1]
    bshape[ax] = nlay
    wl.eps_r = np.broadcast_to(eps_l.reshape(bshape), shape).copy()
    wl.mu_r = np.broadcast_to(mu_l.reshape(bshape), shape).copy()
    setattr(wl, "d" + layer_axis, dl)
    op = yee.assemble(wl)
    got = _oracle_omega2(op)
    # the in-plane axis that is neither the family axis nor the layer axis
    (other,) = [a for a in "xyz" if a not in (family, layer_axis)]
    ref = _union_1d(n[other], eps_l, mu_l, d, dl)
    assert _contains(got, ref, 1e-11)
