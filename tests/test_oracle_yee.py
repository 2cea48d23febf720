"""Pins of the oracle's Yee matrices and leapfrog against facts fixed by the
paper and by the mathematics (no comparison of the oracle with itself)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import yee

C0 = yee.C0


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


def vacuum2d(nx, ny, d=1e-3):
    return W.cavity2d(nx=nx, ny=ny, d=d, seed=0)


def vacuum3d(nx, ny, nz, d):
    wl = W.cavity3d(n=nx, ny=ny, nz=nz, d=d, seed=0, block=100, eps_range=(1, 1),
                    sigma_range=(0, 0), nports=1, margin=1)
    return wl


def test_unknown_counts_match_table_I():
    """Table I / Sec. V-B: N = 30,200 (101x101) and 48,440 (41x401), Ez-pol."""
    g = _golden("unknown_counts.txt")
    assert yee.count_unknowns_2d(101, 101) == g["cavity2d_101x101"]
    assert yee.count_unknowns_2d(41, 401) == g["waveguide2d_41x401"]
    # the oracle's numbering enumerates exactly these unknowns
    op = yee.assemble(vacuum2d(9, 7))
    assert op.N == yee.count_unknowns_2d(9, 7)
    # 3-D: interior edges / faces of a PEC box
    wl = vacuum3d(5, 4, 3, 1e-3)
    op3 = yee.assemble(wl)
    nx, ny, nz = 5, 4, 3
    ne = nx * (ny - 1) * (nz - 1) + (nx - 1) * ny * (nz - 1) + (nx - 1) * (ny - 1) * nz
    nh = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    assert (op3.Ne, op3.Nh) == (ne, nh)


def _faraday_reference(g, E_of, c, i, j, k):
    """-curl E at a magnetic sample, written directly from Faraday's law."""
    dx, dy, dz = g.dx, g.dy, g.dz
    if g.dim == 2:
        if c == 3:  # mu dHx/dt = -dEz/dy
            return -(E_of(2, i, j + 1, 0) - E_of(2, i, j, 0)) / dy[j]
        return (E_of(2, i + 1, j, 0) - E_of(2, i, j, 0)) / dx[i]  # mu dHy/dt = dEz/dx
    if c == 3:  # dEy/dz - dEz/dy
        return ((E_of(1, i, j, k + 1) - E_of(1, i, j, k)) / dz[k]
                - (E_of(2, i, j + 1, k) - E_of(2, i, j, k)) / dy[j])
    if c == 4:  # dEz/dx - dEx/dz
        return ((E_of(2, i + 1, j, k) - E_of(2, i, j, k)) / dx[i]
                - (E_of(0, i, j, k + 1) - E_of(0, i, j, k)) / dz[k])
    return ((E_of(0, i, j + 1, k) - E_of(0, i, j, k)) / dy[j]  # dEx/dy - dEy/dx
            - (E_of(1, i + 1, j, k) - E_of(1, i, j, k)) / dx[i])


@pytest.mark.parametrize("dim", [2, 3])
def test_KT_is_faraday_curl_on_graded_grid(dim):
    """eq. (matrix) uses K in Ampere's rows and K^T in Faraday's rows; K is
    built from Ampere's law only, so K^T E must reproduce the primal curl of
    Faraday's law written independently (times the magnetic row weights)."""
    rng = np.random.default_rng(5)
    if dim == 2:
        wl = vacuum2d(6, 5)
        wl.dx = rng.uniform(0.5e-3, 2e-3, 6)
        wl.dy = rng.uniform(0.5e-3, 2e-3, 5)
    else:
        wl = vacuum3d(4, 5, 3, 1e-3)
        wl.dx = rng.uniform(0.5e-3, 2e-3, 4)
        wl.dy = rng.uniform(0.5e-3, 2e-3, 5)
        wl.dz = rng.uniform(0.5e-3, 2e-3, 3)
    op = yee.assemble(wl)
    E = rng.standard_normal(op.Ne)
    vals = {key: E[r] for r, key in enumerate(op.ne.keys)}
    E_of = lambda c, i, j, k: vals.get((c, i, j, k), 0.0)
    KTE = op.K.T @ E
    for r, (c, i, j, k) in enumerate(op.nh.keys):
        ref = _faraday_reference(op.grid, E_of, c, i, j, k) * op.Wh[r]
        assert KTE[r] == pytest.approx(ref, rel=1e-12, abs=1e-9 * np.abs(KTE).max())


def test_uniform_grid_is_papers_form():
    """Sec. II-A: on a uniform grid D_eps holds eps per sample and K holds +-1/Delta."""
    wl = vacuum3d(4, 4, 4, 2e-3)
    op = yee.assemble(wl)
    assert np.allclose(op.De, yee.EPS0, rtol=1e-15)
    assert np.allclose(op.Dm, yee.MU0, rtol=1e-15)
    assert np.allclose(np.abs(op.K.data), 1 / 2e-3, rtol=1e-13)
    # every electric row of K has 4 entries (two differences), interior rows
    # 2 per difference; rows next to a wall lose the normal-H entries only
    assert op.K.getnnz(axis=1).max() == 4


def _closed_form_sigmas_2d(nx, ny, dx, dy):
    m = np.arange(1, nx)[:, None]
    n = np.arange(1, ny)[None, :]
    s = 2 * C0 * np.sqrt(np.sin(m * np.pi / (2 * nx)) ** 2 / dx ** 2
                         + np.sin(n * np.pi / (2 * ny)) ** 2 / dy ** 2)
    return np.sort(s.ravel())


def _closed_form_sigmas_3d(nx, ny, nz, d):
    out = []
    for a in range(nx):
        for b in range(ny):
            for c in range(nz):
                nonzero = (a > 0) + (b > 0) + (c > 0)
                mult = {3: 2, 2: 1}.get(nonzero, 0)
                s = 2 * C0 * math.sqrt((math.sin(a * math.pi / (2 * nx)) ** 2
                                        + math.sin(b * math.pi / (2 * ny)) ** 2
                                        + math.sin(c * math.pi / (2 * nz)) ** 2)) / d
                out += [s] * mult
    return np.sort(out)


def test_spectrum_2d_matches_discrete_dispersion():
    """Uniform vacuum PEC box: singular values of De^-1/2 K Dm^-1/2 are
    2 c sqrt(sin^2(m pi/2nx)/dx^2 + sin^2(n pi/2ny)/dy^2) (Yee dispersion)."""
    nx, ny, dx = 7, 5, 1e-3
    wl = vacuum2d(nx, ny, dx)
    op = yee.assemble(wl)
    A = (op.K.toarray() / np.sqrt(op.De)[:, None]) / np.sqrt(op.Dm)[None, :]
    s = np.sort(np.linalg.svd(A, compute_uv=False))
    ref = _closed_form_sigmas_2d(nx, ny, dx, dx)
    assert np.allclose(s, ref, rtol=1e-12)


def test_spectrum_3d_matches_discrete_dispersion():
    nx, ny, nz, d = 4, 3, 5, 1e-2
    op = yee.assemble(vacuum3d(nx, ny, nz, d))
    A = (op.K.toarray() / np.sqrt(op.De)[:, None]) / np.sqrt(op.Dm)[None, :]
    s = np.sort(np.linalg.svd(A, compute_uv=False))
    ref = _closed_form_sigmas_3d(nx, ny, nz, d)
    # the remaining singular values are zero: static (gradient) E modes
    assert len(s) == op.Ne
    nzero = op.Ne - len(ref)
    assert nzero == (nx - 1) * (ny - 1) * (nz - 1)
    assert np.all(s[:nzero] < 1e-6 * s[-1])
    assert np.allclose(s[nzero:], ref, rtol=1e-12)


def test_leapfrog_eigenvalues_match_dispersion():
    """One-step map of eq. (MNAform), lossless: eigenvalues e^{+-j theta},
    sin(theta/2) = dt sigma / 2, plus N_h - N_e eigenvalues equal to 1."""
    nx, ny, d = 5, 4, 1e-3
    op = yee.assemble(vacuum2d(nx, ny, d))
    dt = 0.9 * yee.cfl_dt_max(op.grid)
    R, F = yee.R_F(op, dt)
    G = np.linalg.solve((R + F).toarray(), (R - F).toarray())
    lam = np.linalg.eigvals(G)
    assert np.allclose(np.abs(lam), 1.0, atol=1e-10)
    theta = np.sort(np.abs(np.angle(lam)))
    sig = _closed_form_sigmas_2d(nx, ny, d, d)
    ref = np.sort(np.concatenate([np.zeros(op.Nh - op.Ne), 2 * np.arcsin(dt * sig / 2),
                                  2 * np.arcsin(dt * sig / 2)]))
    assert np.allclose(theta, ref, atol=1e-9)


def test_cfl_limit_is_the_stability_edge():
    """eq. (CFL) is the limit of condition (Dstability2): R > 0 just below it
    on a fine grid, and R indefinite just above it on any grid."""
    op = yee.assemble(vacuum2d(24, 24))
    dtm = yee.cfl_dt_max(op.grid)
    R, _ = yee.R_F(op, 0.999 * dtm)
    assert spla.eigsh(R, k=1, which="SA", return_eigenvectors=False)[0] > 0
    R, _ = yee.R_F(op, 1.02 * dtm)
    assert spla.eigsh(R, k=1, which="SA", return_eigenvectors=False)[0] < 0
    # closed form: dt_max = 1/(c sqrt(1/dx^2 + 1/dy^2))
    assert dtm == pytest.approx(1e-3 / (C0 * math.sqrt(2)), rel=1e-15)


def test_energy_identity_lossy_with_source():
    """W = x^T R x obeys W^{n+1} - W^n = (x^{n+1}+x^n)^T B u^{n+1}
    - 1/2 (x^{n+1}+x^n)^T diag(Dse, Dsm) (x^{n+1}+x^n) (from eq. (MNAform))."""
    wl = W.cavity2d(nx=10, ny=8, d=1e-3, seed=3, eps_block=3, eps_range=(1, 4),
                    sigma_range=(0.0, 5.0))
    op = yee.assemble(wl)
    dt = 0.95 * yee.cfl_dt_max(op.grid)
    B = yee.port_matrix(op, wl.sources, True)
    L = yee.port_matrix(op, wl.probes, False)
    u = W.drive(wl, dt, 60) * 1e3
    _, X = yee.leapfrog(op, dt, B, u, L, return_states=True)
    R, F = yee.R_F(op, dt)
    S = np.concatenate([op.Dse, op.Dsm])
    X = np.vstack([np.zeros(op.N), X])
    Ws = np.array([yee.energy(R, x) for x in X])
    for n in range(u.shape[0]):
        s = X[n + 1] + X[n]
        rhs = s @ (B @ u[n]) - 0.5 * s @ (S * s)
        assert Ws[n + 1] - Ws[n] == pytest.approx(rhs, rel=1e-9, abs=1e-12 * Ws.max())


def test_lossless_energy_conserved():
    wl = W.cavity3d(n=6, d=1e-3, seed=2, block=2, eps_range=(1, 4), sigma_range=(0, 0),
                    nports=1, margin=2)
    op = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    B = yee.port_matrix(op, wl.sources, True)
    L = yee.port_matrix(op, wl.probes, False)
    u = np.zeros((200, 1))
    x0 = W.random_vectors(4, op.N)
    R, _ = yee.R_F(op, dt)
    W0 = yee.energy(R, x0)
    _, x = yee.leapfrog(op, dt, B, u, L, x0=x0)
    assert yee.energy(R, x) == pytest.approx(W0, rel=1e-12)


def test_leapfrog_is_block_substitution_of_MNAform():
    """The E-then-H update equals solving (R+F) x^{n+1} = (R-F) x^n + B u^{n+1}."""
    wl = W.cavity2d(nx=8, ny=9, d=1e-3, seed=1, eps_block=2, eps_range=(1, 3),
                    sigma_range=(0, 2.0))
    op = yee.assemble(wl)
    dt = 0.9 * yee.cfl_dt_max(op.grid)
    B = yee.port_matrix(op, wl.sources, True)
    L = yee.port_matrix(op, wl.probes, False)
    u = W.drive(wl, dt, 25)
    _, X = yee.leapfrog(op, dt, B, u, L, return_states=True)
    R, F = yee.R_F(op, dt)
    x = np.zeros(op.N)
    for n in range(u.shape[0]):
        x = spla.spsolve((R + F).tocsc(), (R - F) @ x + B @ u[n])
        assert np.allclose(x, X[n], rtol=1e-11, atol=1e-13 * np.abs(X[n]).max())


def test_probe_spectrum_peaks_at_discrete_resonances():
    """A lossless cavity rings at the discrete resonances
    f = asin(c dt sqrt(sum sin^2(m pi/2n)/d^2)) / (pi dt)."""
    nx = ny = 6
    d = 1e-3
    wl = vacuum2d(nx, ny, d)
    op = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    B = yee.port_matrix(op, [[(2, 2, 3, 0, 1.0)]], True)
    L = yee.port_matrix(op, [[(2, 4, 2, 0, 1.0)]], False)
    nsteps = 8192
    u = np.zeros((nsteps, 1))
    u[0, 0] = 1.0  # impulse
    y, _ = yee.leapfrog(op, dt, B, u, L)
    spec = np.abs(np.fft.rfft(y[:, 0] * np.hanning(nsteps)))
    f = np.fft.rfftfreq(nsteps, dt)
    sig = _closed_form_sigmas_2d(nx, ny, d, d)
    fres = np.arcsin(dt * sig / 2) / (np.pi * dt)
    # the strongest spectral peak lies on one of the discrete resonances
    fpk = f[np.argmax(spec)]
    assert np.min(np.abs(fres - fpk)) < 1.5 / (nsteps * dt)


def test_cube_resonances_of_section_IIIB():
    """Sec. III-B: the 1 m PEC cube resonates at 0.21199 and 0.25963 GHz in the
    pulse band.  The 9^3 Yee grid (Delta = 1/9 m) approaches these modes
    (1,1,0) and (1,1,1) from below and converges as the grid is refined."""
    g = _golden("cube_resonances.txt")
    ref = np.array([g["f110_GHz"], g["f111_GHz"]]) * 1e9
    cont = C0 / 2 * np.sqrt([2.0, 3.0])
    assert np.allclose(cont, ref, rtol=3e-5)  # printed to 5 digits
    errs = []
    for n in (9, 18):
        op = yee.assemble(vacuum3d(n, n, n, 1.0 / n))
        KK = (op.K / np.sqrt(op.De)[:, None]).tocsr()
        M = (KK @ sp.diags(1 / op.Dm) @ KK.T).tocsc()
        w2 = spla.eigsh(M, k=10, sigma=0.5 * (2 * np.pi * 0.2e9) ** 2, return_eigenvectors=False)
        f = np.sort(np.sqrt(np.abs(w2)) / (2 * np.pi))
        f110 = f[np.argmin(np.abs(f - ref[0]))]
        f111 = f[np.argmin(np.abs(f - ref[1]))]
        errs.append([abs(f110 - ref[0]) / ref[0], abs(f111 - ref[1]) / ref[1]])
        assert f110 < ref[0] and f111 < ref[1]
    errs = np.array(errs)
    assert np.all(errs[0] < 0.01)
    assert np.all(errs[1] < errs[0] / 3.5)  # second-order convergence
