"""Pins of the oracle's reduction, perturbation and adjoint against facts the
paper proves or the mathematics fixes."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import adjoint, mor, perturb, yee


def small_case(seed=0, nx=12, ny=10, lossy=True, nsrc=1):
    wl = W.cavity2d(nx=nx, ny=ny, d=1e-3, seed=seed, eps_block=3, eps_range=(1, 4),
                    sigma_range=(0.0, 2.0) if lossy else (0.0, 0.0), nsrc=nsrc)
    op = yee.assemble(wl)
    B = yee.port_matrix(op, wl.sources, True)
    L = yee.port_matrix(op, wl.probes, False)
    return wl, op, B, L


def test_shifted_matrix_reading_static_point():
    """Sec. IV-A: z = 1 corresponds to static conditions.  With the reading
    z (R+F) - (R-F) the shifted matrix at z = 1 is 2F (no 1/dt terms)."""
    _, op, _, _ = small_case()
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    R, F = yee.R_F(op, dt)
    A1 = mor.shifted_matrix(op, dt, 1.0)
    assert abs(A1 - 2 * F).max() < 1e-9 * abs(F).max()


def test_schur_solve_equals_direct_solve():
    """eqs. (reduced_linear_system_solution1/2) solve eq. (linear_system_solution)."""
    _, op, B, _ = small_case()
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    z = mor.expansion_points(1.1, 2, 125e9, dt)[2]
    b = W.random_vectors(1, op.N) + 1j * W.random_vectors(2, op.N)
    x_direct = spla.spsolve(mor.shifted_matrix(op, dt, z), b)
    x_schur = mor.schur_solve(op, dt, z, b)
    assert np.allclose(x_schur, x_direct, rtol=1e-10, atol=1e-12 * np.abs(x_direct).max())


def test_expansion_points_distribution():
    """eq. (distrib): 2L+1 points on an arc of radius M; z_0 = M near z = 1."""
    dt = 1e-12
    z = mor.expansion_points(1.1, 2, 125e9, dt)
    assert len(z) == 3
    assert np.allclose(np.abs(z), 1.1)
    assert z[0] == pytest.approx(1.1)
    assert np.angle(z[2]) == pytest.approx(2 * math.pi * 125e9 * dt)
    assert np.angle(z[1]) == pytest.approx(0.5 * 2 * math.pi * 125e9 * dt)


@pytest.fixture(scope="module")
def reduced_small():
    wl, op, B, L = small_case(seed=4)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    rom = mor.mor_reduce(op, B, L, q=20, dt_ref=dt, fmax=125e9, M=1.1, npts_half=2)
    return wl, op, B, L, dt, rom


def test_basis_orthonormal_and_block_diagonal(reduced_small):
    """eq. (V): V1 and V2 orthonormal, N_e x N~ and N_h x N~."""
    _, op, _, _, _, rom = reduced_small
    assert rom.V1.shape == (op.Ne, 20) and rom.V2.shape == (op.Nh, 20)
    assert np.allclose(rom.V1.T @ rom.V1, np.eye(20), atol=1e-12)
    assert np.allclose(rom.V2.T @ rom.V2, np.eye(20), atol=1e-12)


def test_moment_matching_at_all_points(reduced_small):
    """Sec. II-C/IV-A: the projected model matches H(z) = L^T (zP-Q)^{-1} B and
    its first z-derivatives at every expansion point and its conjugate."""
    _, op, B, L, dt, rom = reduced_small
    P, Q = mor.system_pq(op, dt)
    Rr, Fr = mor.reduced_R_F(rom, dt)
    Pr, Qr = Rr + Fr, Rr - Fr
    Br = np.vstack([rom.B1, rom.B2])
    Lr = np.vstack([rom.L1, rom.L2])
    for z in list(rom.points) + list(np.conj(rom.points[1:])):
        Hf = mor.transfer(P, Q, B, L, z)
        Hr = mor.transfer(Pr, Qr, Br, Lr, z)
        assert np.allclose(Hr, Hf, rtol=1e-9), z
        # first derivative: -L^T A^{-1} P A^{-1} B
        Af = (z * P - Q).tocsc().astype(complex)
        lu = spla.splu(Af)
        dHf = -L.T @ lu.solve(P @ lu.solve(B.astype(complex)))
        Ar = z * Pr - Qr
        dHr = -Lr.T @ np.linalg.solve(Ar, Pr @ np.linalg.solve(Ar, Br))
        assert np.allclose(dHr, dHf, rtol=1e-7), z


def test_moments_not_matched_away_from_points(reduced_small):
    """Control for the previous test: far from the points the ROM is approximate."""
    _, op, B, L, dt, rom = reduced_small
    P, Q = mor.system_pq(op, dt)
    z = 1.05 * np.exp(1j * 2.5)
    Hf = mor.transfer(P, Q, B, L, z)
    Hr = mor.rom_transfer(rom, dt, z)
    assert not np.allclose(Hr, Hf, rtol=1e-6)


def test_full_basis_reproduces_fom_exactly():
    """With V spanning every reachable direction the reduced leapfrog is the
    full leapfrog seen through a congruence: identical probe waveforms."""
    wl = W.cavity2d(nx=5, ny=4, d=1e-3, seed=0, eps_block=2, eps_range=(1, 3),
                    sigma_range=(0, 1.0))
    op = yee.assemble(wl)
    B = yee.port_matrix(op, wl.sources, True)
    L = yee.port_matrix(op, wl.probes, False)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    rom = mor.mor_reduce(op, B, L, q=30, dt_ref=dt, fmax=150e9, rank_tol=1e-10)
    assert rom.q1 == op.Ne  # every electric direction reached
    u = W.drive(wl, dt, 300)
    y_full, _ = yee.leapfrog(op, dt, B, u, L)
    y_rom = mor.rom_leapfrog(rom, dt, u)
    assert np.linalg.norm(y_rom - y_full) <= 1e-10 * np.linalg.norm(y_full)


def test_basis_invariance(reduced_small):
    """The reduced model depends on span(V1), span(V2) only (output invariance
    under V_i -> V_i Q_i with Q_i orthogonal)."""
    _, op, B, L, dt, rom = reduced_small
    Q1 = np.linalg.qr(W.random_vectors(8, (20, 20)))[0]
    Q2 = np.linalg.qr(W.random_vectors(9, (20, 20)))[0]
    pr = mor.project(op, rom.V1 @ Q1, rom.V2 @ Q2, B, L)
    rom2 = mor.Reduced(V1=rom.V1 @ Q1, V2=rom.V2 @ Q2, **pr)
    u = W.drive(W.cavity2d(), dt, 200)
    assert np.allclose(mor.rom_leapfrog(rom2, dt, u), mor.rom_leapfrog(rom, dt, u), rtol=1e-9,
                       atol=1e-12)


def test_reduced_energy_is_full_energy_of_lifted_state(reduced_small):
    """x~^T R~ x~ = (V x~)^T R (V x~) (congruence, Sec. II-D)."""
    _, op, _, _, dt, rom = reduced_small
    R, _ = yee.R_F(op, dt)
    Rr, _ = mor.reduced_R_F(rom, dt)
    xr = W.random_vectors(3, rom.q1 + rom.q2)
    x = np.concatenate([rom.V1 @ xr[:rom.q1], rom.V2 @ xr[rom.q1:]])
    assert xr @ Rr @ xr == pytest.approx(x @ (R @ x), rel=1e-10)


def _max_abs_eig(Rr, Fr):
    return np.abs(np.linalg.eigvals(np.linalg.solve(Rr + Fr, Rr - Fr))).max()


def test_reduced_model_stable_below_cfl_by_construction(reduced_small):
    """Sec. II-D: R~ > 0 and F~^T + F~ >= 0, hence all poles in the unit disk."""
    _, op, _, _, dt, rom = reduced_small
    Rr, Fr = mor.reduced_R_F(rom, dt)
    assert np.linalg.eigvalsh(Rr).min() > 0
    assert np.linalg.eigvalsh(Fr + Fr.T).min() > -1e-12 * np.abs(Fr).max()
    assert _max_abs_eig(Rr, Fr) <= 1 + 1e-12


def test_reduced_model_unstable_above_cfl_then_perturbed(reduced_small):
    """Sec. III-A: at s = 4.95 the unperturbed reduced model is unstable; the
    clamp of the singular values of De~^-1/2 K~ Dm~^-1/2 at gamma 2/dt makes
    it stable, and sigma_max(after) = min(sigma_max, gamma 2/dt)."""
    _, op, _, _, dt0, rom = reduced_small
    dt = 5 * dt0  # s = 4.95
    Rr, Fr = mor.reduced_R_F(rom, dt)
    assert _max_abs_eig(Rr, Fr) > 1.01
    Kp, n, s, s2 = perturb.perturb(rom.De, rom.Dm, rom.K, dt, 0.9999)
    assert n > 0
    s_after = perturb.scaled_singular_values(rom.De, rom.Dm, Kp)
    assert s_after.max() == pytest.approx(min(s.max(), 0.9999 * 2 / dt), rel=1e-12)
    # unchanged singular values below the threshold
    below = np.sort(s[s < 0.9999 * 2 / dt])
    assert np.allclose(np.sort(s_after)[:len(below)], below, rtol=1e-10)
    Rp, Fp = mor.reduced_R_F(rom, dt, K=Kp)
    assert np.linalg.eigvalsh(Rp).min() > 0
    assert _max_abs_eig(Rp, Fp) <= 1 + 1e-10


def test_perturbation_noop_below_cfl(reduced_small):
    """Reduced singular values never exceed the full model's, so at s <= 0.99
    nothing is clamped."""
    _, op, _, _, dt, rom = reduced_small
    Kp, n, _, _ = perturb.perturb(rom.De, rom.Dm, rom.K, dt)
    assert n == 0
    assert np.allclose(Kp, rom.K, rtol=1e-12, atol=1e-12 * np.abs(rom.K).max())


def test_perturbation_cholesky_route_equals_symmetric_sqrt(reduced_small):
    """K~' does not depend on which square root of De~, Dm~ is used."""
    _, _, _, _, dt0, rom = reduced_small
    dt = 5 * dt0
    Kp, _, _, _ = perturb.perturb(rom.De, rom.Dm, rom.K, dt)
    Le = np.linalg.cholesky(rom.De)
    Lm = np.linalg.cholesky(rom.Dm)
    A = np.linalg.solve(Le, np.linalg.solve(Lm, rom.K.T).T)
    U, s, Wt = np.linalg.svd(A)
    s2 = np.minimum(s, 0.9999 * 2 / dt)
    Kc = Le @ (U * s2) @ Wt @ Lm.T
    assert np.allclose(Kc, Kp, rtol=1e-10, atol=1e-12 * np.abs(Kp).max())


def test_lossless_perturbed_model_on_unit_circle():
    """Sec. III-B (E1 demo, on a small grid): a lossless model perturbed at
    s = 1.98 has all its eigenvalues on the unit circle; at s = 0.99 the
    unperturbed one is stable and at s = 1.98 unstable."""
    wl = W.cavity3d(n=5, ny=4, nz=4, d=1.0 / 9, seed=0, block=100, eps_range=(1, 1),
                    sigma_range=(0, 0), nports=1, margin=1)
    op = yee.assemble(wl)
    dtm = yee.cfl_dt_max(op.grid)

    def max_eig(dt, K):
        import scipy.sparse as sp
        R = np.block([[np.diag(op.De / dt), -0.5 * K], [-0.5 * K.T, np.diag(op.Dm / dt)]])
        F = np.block([[np.zeros((op.Ne, op.Ne)), 0.5 * K], [-0.5 * K.T, np.zeros((op.Nh, op.Nh))]])
        return np.abs(np.linalg.eigvals(np.linalg.solve(R + F, R - F)))

    K = op.K.toarray()
    assert max_eig(0.99 * dtm, K).max() <= 1 + 1e-10
    lam = max_eig(1.98 * dtm, K)
    assert lam.max() > 1.5
    Kp, n, _, _ = perturb.perturb(np.diag(op.De), np.diag(op.Dm), K, 1.98 * dtm)
    assert n > 0
    lam = max_eig(1.98 * dtm, Kp)
    assert np.allclose(lam, 1.0, atol=1e-9)


# --------------------------------------------------------------------------- adjoint


def _fd_objective(wl, dt, u, eps=None, sig=None):
    import copy
    w2 = copy.deepcopy(wl)
    if eps is not None:
        w2.eps_r = eps
    if sig is not None:
        w2.sigma_e = sig
    op = yee.assemble(w2)
    B = yee.port_matrix(op, w2.sources, True)
    L = yee.port_matrix(op, w2.probes, False)
    y, _ = yee.leapfrog(op, dt, B, u, L)
    return adjoint.objective(y, dt)


def test_full_adjoint_matches_central_differences():
    """dJ/d eps_r and dJ/d sigma_e per cell vs FP64 central differences."""
    wl = W.cavity2d(nx=9, ny=8, d=1e-3, seed=2, eps_block=2, eps_range=(1, 4),
                    sigma_range=(0.0, 3.0))
    op = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    B = yee.port_matrix(op, wl.sources, True)
    L = yee.port_matrix(op, wl.probes, False)
    u = W.drive(wl, dt, 120)
    J, gDe, gDse = adjoint.full_adjoint(op, dt, B, u, L)
    ge, gs = adjoint.cell_gradients(op, wl, gDe, gDse)
    rng = np.random.default_rng(0)
    for _ in range(6):
        j, i = int(rng.integers(0, 8)), int(rng.integers(0, 9))
        h = 1e-4
        ep, em = wl.eps_r.copy(), wl.eps_r.copy()
        ep[j, i] += h
        em[j, i] -= h
        fd = (_fd_objective(wl, dt, u, eps=ep) - _fd_objective(wl, dt, u, eps=em)) / (2 * h)
        assert ge[j, i] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(J))
        sp_, sm = wl.sigma_e.copy(), wl.sigma_e.copy()
        sp_[j, i] += h
        sm[j, i] -= h
        fd = (_fd_objective(wl, dt, u, sig=sp_) - _fd_objective(wl, dt, u, sig=sm)) / (2 * h)
        assert gs[j, i] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(J))


def test_reduced_adjoint_matches_central_differences(reduced_small):
    """Reduced leapfrog: dJ/dDe~ (trace pairing with a random symmetric
    direction) and dJ/dK~ vs central differences."""
    _, op, _, _, dt, rom = reduced_small
    u = W.drive(W.cavity2d(), dt, 150)
    J, gDe, gDse, gK = adjoint.reduced_adjoint(rom, dt, u)
    D = W.random_vectors(11, (rom.q1, rom.q1))
    D = 0.5 * (D + D.T) * np.abs(rom.De).max() * 1e-3
    import copy

    def Jof(De=None, Dse=None, K=None):
        r = copy.copy(rom)
        if De is not None:
            r.De = De
        if Dse is not None:
            r.Dse = Dse
        y = mor.rom_leapfrog(r, dt, u, K=K)
        return adjoint.objective(y, dt)

    h = 1e-3
    fd = (Jof(De=rom.De + h * D) - Jof(De=rom.De - h * D)) / (2 * h)
    assert np.sum(gDe * D) == pytest.approx(fd, rel=1e-6)
    Dk = W.random_vectors(12, rom.K.shape) * np.abs(rom.K).max() * 1e-3
    fd = (Jof(K=rom.K + h * Dk) - Jof(K=rom.K - h * Dk)) / (2 * h)
    assert np.sum(gK * Dk) == pytest.approx(fd, rel=1e-6)
    Ds = 0.5 * (D + D.T) / np.abs(rom.De).max() * np.abs(rom.Dse).max()
    fd = (Jof(Dse=rom.Dse + h * Ds) - Jof(Dse=rom.Dse - h * Ds)) / (2 * h)
    assert np.sum(gDse * Ds) == pytest.approx(fd, rel=1e-6)


def test_reduced_theta_gradient_through_clamp_matches_central_differences(reduced_small):
    """dJ/dtheta through the reduced leapfrog *and* the singular-value clamp
    (s = 4.95, several values clamped) equals FP64 central differences of the
    whole chain: perturb(De~ + theta dDe) then step."""
    _, op, _, _, dt0, rom = reduced_small
    dt = 5 * dt0
    u = W.drive(W.cavity2d(f0=10e9, bw=10e9), dt, 300)
    V = W.random_vectors(21, (rom.q1, rom.q1))
    dDe = 0.5 * (V + V.T) * np.abs(rom.De).max() * 1e-2
    J, dJ, *_ = adjoint.reduced_theta_gradient(rom, dt, u, dDe)
    import copy

    def Jof(theta):
        r = copy.copy(rom)
        r.De = rom.De + theta * dDe
        Kp, n, _, _ = perturb.perturb(r.De, r.Dm, r.K, dt, 0.9999)
        return adjoint.objective(mor.rom_leapfrog(r, dt, u, K=Kp), dt), n

    h = 1e-5
    (jp, n1), (jm, n2) = Jof(h), Jof(-h)
    assert n1 == n2 > 0
    fd = (jp - jm) / (2 * h)
    assert dJ == pytest.approx(fd, rel=1e-6)
    # holding the clamp fixed gives a different (wrong for this chain) number
    _, dJ_frozen, *_ = adjoint.reduced_theta_gradient(rom, dt, u, dDe, through_clamp=False)
    assert abs(dJ_frozen - fd) > 1e-3 * abs(fd)


# --------------------------------------------------------------- several ports


def _multiport_case(ports):
    """12 x 10 lossy cavity with the given source columns (B built here as
    weighted sums of point sources at seeded interior nodes) and two probes."""
    wl = W.cavity2d(nx=12, ny=10, d=1e-3, seed=6, eps_block=3, eps_range=(1, 4),
                    sigma_range=(0.0, 2.0), nsrc=3, nprobe=2)
    op = yee.assemble(wl)
    Bp = yee.port_matrix(op, wl.sources, True)
    B = np.column_stack([Bp @ np.asarray(w, float) for w in ports])
    L = yee.port_matrix(op, wl.probes, False)
    return op, B, L


def _derivs(lu, P, B, L, order):
    """H(z), H'(z), H''(z) of L^T (zP-Q)^{-1} B from one factorisation:
    d^k/dz^k A^{-1} = (-1)^k k! (A^{-1} P)^k A^{-1}."""
    X = lu(B)
    out = [L.T @ X]
    fact = 1.0
    for kk in range(1, order + 1):
        X = lu(P @ X)
        fact *= kk
        out.append((-1) ** kk * fact * (L.T @ X))
    return out


@pytest.mark.parametrize("ports,expect_deflation", [
    ([(1, 0, 0), (0, 1, 0)], False),                 # b = 2
    ([(1, 0, 0), (0, 1, 0), (0, 0, 1)], False),      # b = 3
    ([(1, 0, 0), (0, 1, 0), (1, 0, 0)], True),       # b = 3, a duplicated port
    ([(1, 0, 0), (0, 1, 0), (0.5, -2.0, 0)], True),  # b = 3, a dependent port
])
def test_block_arnoldi_moment_matching_several_ports(ports, expect_deflation):
    """Sec. II-C / IV-A with B holding several ports: per expansion point the
    block Krylov basis of (zP-Q)^{-1}P started at (zP-Q)^{-1}B (three block
    moments each, L = 2) makes the projected model match H(z), H'(z) and
    H''(z) of every port pair at all 2L+1 points and the conjugates.  A port
    that lies in the span of the others deflates in every block, and the
    moments of all ports (the dependent one included) are still matched."""
    op, B, L = _multiport_case(ports)
    b = B.shape[1]
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    q = 5 * 3 * b  # three block moments per point
    rom = mor.mor_reduce(op, B, L, q=q, dt_ref=dt, fmax=125e9, M=1.1, npts_half=2)
    assert (rom.deflated > 0) == expect_deflation
    if expect_deflation:
        # one column of every block: 3 blocks at z_0, 2 x 3 (Re, Im) per complex point
        assert rom.deflated == 3 + 2 * 2 * 3
    P, Q = mor.system_pq(op, dt)
    Rr, Fr = mor.reduced_R_F(rom, dt)
    Pr, Qr = Rr + Fr, Rr - Fr
    Br = np.vstack([rom.B1, rom.B2])
    Lr = np.vstack([rom.L1, rom.L2])
    for z in list(rom.points) + list(np.conj(rom.points[1:])):
        luf = spla.splu((z * P - Q).tocsc().astype(complex)).solve
        Ar = z * Pr - Qr
        lur = lambda X, Ar=Ar: np.linalg.solve(Ar, X)
        full = _derivs(luf, P, B.astype(complex), L, 2)
        red = _derivs(lur, Pr, Br.astype(complex), Lr, 2)
        for kk, (hf, hr) in enumerate(zip(full, red)):
            scale = np.abs(hf).max()
            assert np.abs(hr - hf).max() <= 1e-9 * scale, (z, kk)


def test_block_arnoldi_several_ports_not_matched_beyond_the_moments():
    """Control: the third derivative, the first moment beyond the three block
    moments per point, is not matched (at z_0 and at the outer point)."""
    op, B, L = _multiport_case([(1, 0, 0), (0, 1, 0)])
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    rom = mor.mor_reduce(op, B, L, q=30, dt_ref=dt, fmax=125e9, M=1.1, npts_half=2)
    P, Q = mor.system_pq(op, dt)
    Rr, Fr = mor.reduced_R_F(rom, dt)
    for z in (rom.points[0], rom.points[2]):
        full = _derivs(spla.splu((z * P - Q).tocsc().astype(complex)).solve, P,
                       B.astype(complex), L, 3)
        Ar = z * (Rr + Fr) - (Rr - Fr)
        red = _derivs(lambda X: np.linalg.solve(Ar, X), Rr + Fr,
                      np.vstack([rom.B1, rom.B2]).astype(complex), np.vstack([rom.L1, rom.L2]), 3)
        assert np.abs(red[2] - full[2]).max() <= 1e-9 * np.abs(full[2]).max()
        assert np.abs(red[3] - full[3]).max() > 1e-4 * np.abs(full[3]).max()


# ------------------------------------------------- sensitivity to inexact solves


class _InexactLU:
    """An exact sparse LU whose solves return x + A^-1 r for a random residual
    r of norm tol |b|: what an iterative solve stopped at a normalised
    residual tol leaves (Sec. IV-B stops at 1e-4)."""

    def __init__(self, splu, A, tol, rng):
        self.lu = splu(A)
        self.U = self.lu.U
        self.tol, self.rng = tol, rng

    def solve(self, b):
        x = self.lu.solve(b)
        b2 = b.reshape(b.shape[0], -1)
        r = self.rng.standard_normal(b2.shape)
        if np.iscomplexobj(b):
            r = r + 1j * self.rng.standard_normal(b2.shape)
        r *= self.tol * np.linalg.norm(b2, axis=0) / np.linalg.norm(r, axis=0)
        return x + self.lu.solve(r.astype(b.dtype)).reshape(x.shape)


def test_inexact_solves_move_the_subspaces_not_the_moments(monkeypatch):
    """3-D lossy 11 x 10 x 9 cavity, 2 ports, q = 20: solves to a residual of
    1e-6 (random residual directions) move span(V1), span(V2) by angles of a
    few 1e-3 and the reduced waveform by ~1e-4, yet the reduced transfer
    function still matches the full one at every point to ~1e-12 (the
    projection error is quadratic in the basis error).  This fixes how
    closely any reduction with iterative solves at that tolerance can agree
    with the exact-solve oracle in subspace and waveform terms."""
    import scipy.linalg as sla
    wl = W.cavity3d(n=11, ny=10, nz=9, d=1e-3, seed=4, block=3, nports=2, margin=2,
                    f0=20e9, bw=20e9)
    op = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    B = yee.port_matrix(op, wl.sources, True)
    L = yee.port_matrix(op, wl.probes, False)
    fmax = wl.f0 + wl.bw
    ref = mor.mor_reduce(op, B, L, q=20, dt_ref=dt, fmax=fmax)
    u = W.drive(wl, dt, 600)
    y_ref = mor.rom_leapfrog(ref, dt, u)
    exact = spla.splu
    rng = np.random.default_rng(0)
    monkeypatch.setattr(mor.spla, "splu", lambda A: _InexactLU(exact, A, 1e-6, rng))
    r = mor.mor_reduce(op, B, L, q=20, dt_ref=dt, fmax=fmax)
    monkeypatch.setattr(mor.spla, "splu", exact)

    def angle(U, V):
        s = np.linalg.svd(sla.orth(U).T @ sla.orth(V), compute_uv=False)
        return float(np.sqrt(max(0.0, 1 - s.min() ** 2)))

    ang = max(angle(r.V1, ref.V1), angle(r.V2, ref.V2))
    ew = np.linalg.norm(mor.rom_leapfrog(r, dt, u) - y_ref) / np.linalg.norm(y_ref)
    P, Q = mor.system_pq(op, dt)
    et = max(np.linalg.norm(mor.rom_transfer(r, dt, z) - mor.transfer(P, Q, B, L, z))
             / np.linalg.norm(mor.transfer(P, Q, B, L, z))
             for z in list(ref.points) + list(np.conj(ref.points[1:])))
    assert 1e-3 < ang < 1e-2
    assert 2e-5 < ew < 1e-3
    assert et < 1e-10


def test_conjugate_pair_points_match_moments_at_the_pair_only():
    """Sec. V-C: a single conjugate pair z_1,2 = M exp(+-j 2 pi f_max dt), no
    real point.  The reduced model matches H and dH/dz at z and at conj(z), and
    at the real point M (not an expansion point any more) it does not; its
    q/2 complex vectors fill V1 and V2 (q columns each)."""
    wl, op, B, L = small_case(seed=9)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    fmax = 60e9
    rom = mor.mor_reduce(op, B, L, q=16, dt_ref=dt, fmax=fmax, M=1.1, pair_only=True)
    z = 1.1 * np.exp(2j * math.pi * fmax * dt)
    assert rom.points.shape == (1,) and rom.points[0] == pytest.approx(z)
    assert rom.V1.shape[1] == 16 and rom.V2.shape[1] == 16
    P, Q = mor.system_pq(op, dt)
    Rr, Fr = mor.reduced_R_F(rom, dt)
    Pr, Qr = Rr + Fr, Rr - Fr
    Br = np.vstack([rom.B1, rom.B2])
    Lr = np.vstack([rom.L1, rom.L2])
    for zz in (z, np.conj(z)):
        Hf = mor.transfer(P, Q, B, L, zz)
        Hr = mor.transfer(Pr, Qr, Br, Lr, zz)
        assert np.allclose(Hr, Hf, rtol=1e-9)
        lu = spla.splu((zz * P - Q).tocsc().astype(complex))
        dHf = -L.T @ lu.solve(P @ lu.solve(B.astype(complex)))
        Ar = zz * Pr - Qr
        dHr = -Lr.T @ np.linalg.solve(Ar, Pr @ np.linalg.solve(Ar, Br))
        assert np.allclose(dHr, dHf, rtol=1e-7)
    Hf = mor.transfer(P, Q, B, L, 1.1)
    Hr = mor.transfer(Pr, Qr, Br, Lr, 1.1)
    assert not np.allclose(Hr, Hf, rtol=1e-6)
