"""mor_reduce, rom_perturb, rom_step (HIP) against the FP64 oracle.

The projection basis is not unique (any orthonormal basis of the same
subspaces), so the reduction is compared through basis-invariant
quantities: principal angles between the subspaces, the reduced model's
transfer function and its output waveform.  FP64 steps given identical
inputs: 1e-10 relative; FP32 stepping: 1e-4 relative L2.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import mor, perturb, yee
from tests.gpuutil import log, rel_l2, require_gpu, slots_of, state_to_oracle

pytestmark = pytest.mark.gpu


def _oracle_case(wl, q, s=0.99, L=2, fmax=None):
    oop = yee.assemble(wl)
    dt = s * yee.cfl_dt_max(oop.grid)
    B = yee.port_matrix(oop, wl.sources, True)
    Lp = yee.port_matrix(oop, wl.probes, False)
    fmax = fmax if fmax is not None else wl.f0 + wl.bw
    rom = mor.mor_reduce(oop, B, Lp, q=q, dt_ref=dt, fmax=fmax, M=1.1, npts_half=L)
    return oop, dt, B, Lp, fmax, rom


def _max_angle(U, V):
    """Largest principal angle (sin) between the column spaces of U and V."""
    Qu = sla.orth(U)
    Qv = sla.orth(V)
    s = np.linalg.svd(Qu.T @ Qv, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2)))


def _gpu_basis(gop, oop, grom):
    V1, V2 = grom.basis(gop)
    V1 = V1.cpu().numpy().T
    V2 = V2.cpu().numpy().T
    e_rows = slots_of(gop, oop.ne.keys)
    h_rows = slots_of(gop, oop.nh.keys) - gop.ne_slots * gop.len
    # everything off the unknowns must be exactly zero
    mask_e = np.ones(V1.shape[0], bool)
    mask_e[e_rows] = False
    mask_h = np.ones(V2.shape[0], bool)
    mask_h[h_rows] = False
    assert np.all(V1[mask_e] == 0) and np.all(V2[mask_h] == 0)
    return V1[e_rows], V2[h_rows]


def _as_oracle_rom(grom):
    m = grom.matrices()
    return mor.Reduced(V1=np.zeros((1, m["De"].shape[0])), V2=np.zeros((1, m["Dm"].shape[0])),
                       De=m["De"], Dse=m["Dse"], Dm=m["Dm"], Dsm=m["Dsm"], K=m["K"],
                       B1=m["B1"], B2=m["B2"], L1=m["L1"], L2=m["L2"])


@pytest.mark.parametrize("case", ["2d", "3d"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_schur_apply_matches_oracle(case, prec):
    """The Schur complement of eq. (reduced_linear_system_solution1) applied
    by two stencil sweeps equals the oracle's assembled sparse matrix."""
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    log(f"schur {case} {prec}")
    if case == "2d":
        wl = W.cavity2d(nx=23, ny=17, seed=2, eps_block=3, eps_range=(1, 4), sigma_range=(0, 3.0))
        wl.pec = [(2, 11, j, 0) for j in range(3, 9)]
    else:
        wl = W.board3d(nx=9, ny=8, nz_fine=2, nz_coarse=3, d=1e-3, dz_fine=0.3e-3,
                       strip=(2, 7, 3, 5))
        wl.sigma_e = np.random.default_rng(1).uniform(0, 2, size=wl.eps_r.shape)
    oop = yee.assemble(wl)
    gop = P.Operator.from_workload(wl)
    dt = 0.99 * yee.cfl_dt_max(oop.grid)
    z = 1.1 * np.exp(1j * 0.37)
    S = mor.schur_complement(oop, dt, z)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, oop.Ne)) + 1j * rng.standard_normal((2, oop.Ne))
    y_ref = (S @ x.T).T
    rows = slots_of(gop, oop.ne.keys)
    xg = np.zeros((2, gop.ne_slots * gop.len), complex)
    xg[:, rows] = x
    ct = torch.complex128 if prec == "f64" else torch.complex64
    y = P.schur_apply(gop, dt, z, torch.tensor(xg, dtype=ct, device="cuda"), prec).cpu().numpy()
    tol = 1e-12 if prec == "f64" else 2e-6
    assert rel_l2(y[:, rows], y_ref) <= tol
    mask = np.ones(y.shape[1], bool)
    mask[rows] = False
    assert np.all(y[:, mask] == 0)


def _collected_condition(oop, dt, B, fmax, q, L=2):
    """Smallest relative singular value of the electric / magnetic rows of the
    oracle's collected real Krylov vectors (how well span(V1), span(V2) are
    determined by the data: perturbations of size eps move them by ~eps/c)."""
    import scipy.sparse.linalg as spla
    P_, Q_ = mor.system_pq(oop, dt)
    pts = mor.expansion_points(1.1, L, fmax, dt)
    k, b = q // (2 * L + 1), B.shape[1]
    cols = []
    for l, z in enumerate(pts):
        lu = spla.splu((z * P_ - Q_).tocsc() if l else (z.real * P_ - Q_).tocsc())
        for v in mor.arnoldi_point(lu, P_, B.astype(complex) if l else B, k // b,
                                   mor._balance(oop), 1e-10):
            cols += [v.real] + ([v.imag] if l else [])
    Vh = np.array(cols).T
    se = np.linalg.svd(Vh[:oop.Ne], compute_uv=False)
    sh = np.linalg.svd(Vh[oop.Ne:], compute_uv=False)
    return min(se[-1] / se[0], sh[-1] / sh[0])


@pytest.mark.parametrize("q", [20, 40])
def test_mor_reduce_config0_fp64(q):
    """2-D 20x20 cavity, 1 port, 5 points (q = 40 is the benchmark order):
    same subspaces and the same reduced model as the oracle (exact LU solves
    vs FP64 COCG at 1e-13).  The tolerances scale with how well the data
    determine the subspaces (q = 40 on 361 electric unknowns leaves one
    direction at 1e-11 relative singular value)."""
    require_gpu()
    import paper_1406_7042_amd as P
    log(f"mor config0 fp64 q={q}")
    wl = W.cavity2d()
    oop, dt, B, Lp, fmax, orom = _oracle_case(wl, q=q)
    c = _collected_condition(oop, dt, B, fmax, q)
    gop = P.Operator.from_workload(wl)
    grom = P.mor_reduce(gop, wl.sources, wl.probes, q, dt_ref=dt, fmax=fmax, precision="f64",
                        tol=1e-13)
    info = grom.info()
    assert (info["q1"], info["q2"]) == (orom.q1, orom.q2) == (q, q)
    assert info["relres_max"] <= 1e-13
    V1, V2 = _gpu_basis(gop, oop, grom)
    assert np.allclose(V1.T @ V1, np.eye(q), atol=1e-12)
    assert np.allclose(V2.T @ V2, np.eye(q), atol=1e-12)
    ang = max(_max_angle(V1, orom.V1), _max_angle(V2, orom.V2))
    g = _as_oracle_rom(grom)
    errs = []
    for z in list(orom.points) + [1.05 * np.exp(0.7j), 1.2 * np.exp(2.0j)]:
        errs.append(rel_l2(mor.rom_transfer(g, dt, z), mor.rom_transfer(orom, dt, z)))
    u = W.drive(wl, dt, 2000)
    ew = rel_l2(mor.rom_leapfrog(g, dt, u), mor.rom_leapfrog(orom, dt, u))
    log(f"  condition {c:.2e} max angle {ang:.2e} transfer {max(errs):.2e} waveform {ew:.2e}")
    # a solve residual of 1e-13 leaves errors of ~kappa(S) 1e-13 ~ 1e-10 in each
    # Krylov vector; a direction determined to relative singular value c moves
    # by that over c.  The reduced model's outputs are far less sensitive.
    assert ang <= 1e-9 / c
    tol = max(1e-9, 1e-13 / c)
    assert max(errs) <= tol
    assert ew <= tol


@pytest.mark.parametrize("precision,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_mor_reduce_conjugate_pair_only(precision, tol):
    """Sec. V-C: expansion at the conjugate pair z = M exp(+-j 2 pi f_max dt)
    alone, under a single-frequency drive (a sinusoid at f_max switched on by
    a smooth ramp).  The reduced model matches the full transfer function at z
    and conj(z) and agrees with the oracle's pair-only reduction (transfer
    function at the pair, steady-state waveform) to the solve accuracy."""
    require_gpu()
    import paper_1406_7042_amd as P
    log(f"mor conjugate pair {precision}")
    wl = W.cavity2d(nx=20, ny=16, seed=12, eps_block=4, eps_range=(1, 3), sigma_range=(0, 0.5))
    oop = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(oop.grid)
    B = yee.port_matrix(oop, wl.sources, True)
    Lp = yee.port_matrix(oop, wl.probes, False)
    fmax = 40e9
    orom = mor.mor_reduce(oop, B, Lp, q=16, dt_ref=dt, fmax=fmax, M=1.1, pair_only=True)
    gop = P.Operator.from_workload(wl)
    grom = P.mor_reduce(gop, wl.sources, wl.probes, 16, dt_ref=dt, fmax=fmax, precision=precision,
                        tol=tol, pair_only=True)
    info = grom.info()
    assert (info["q1"], info["q2"]) == (orom.q1, orom.q2) == (16, 16)
    g = _as_oracle_rom(grom)
    Pf, Qf = mor.system_pq(oop, dt)
    z = orom.points[0]
    for zz in (z, np.conj(z)):
        ef = rel_l2(mor.rom_transfer(g, dt, zz), mor.transfer(Pf, Qf, B, Lp, zz))
        eo = rel_l2(mor.rom_transfer(g, dt, zz), mor.rom_transfer(orom, dt, zz))
        log(f"  at {zz:.4f}: vs full {ef:.2e}, vs oracle ROM {eo:.2e}")
        assert ef <= 1e3 * tol and eo <= 1e3 * tol
    n = np.arange(3000)
    ramp = 1 - np.exp(-(n / 300.0) ** 2)
    u = (ramp * np.sin(2 * np.pi * fmax * (n + 0.5) * dt))[:, None]
    ew = rel_l2(mor.rom_leapfrog(g, dt, u), mor.rom_leapfrog(orom, dt, u))
    log(f"  sinusoidal drive waveform vs oracle ROM {ew:.2e}")
    assert ew <= 1e3 * tol


@pytest.mark.parametrize("defl", [1e-10, 1e-6])
def test_mor_reduce_3d_lossy_fp32_solves_moment_matching(defl):
    """3-D lossy blocks, 2 ports, FP32 COCG at 1e-6: the GPU reduced model
    matches the full model's transfer function at every expansion point
    (Sec. II-C) to the solve accuracy, and agrees with the oracle's ROM.
    defl = 1e-10 orthonormalises V1, V2 block by block (CGS2 + CholQR2);
    defl = 1e-6 takes one deflating CholQR2 of all raw columns at the end."""
    require_gpu()
    import paper_1406_7042_amd as P
    log(f"mor 3d fp32 defl {defl}")
    wl = W.cavity3d(n=11, ny=10, nz=9, d=1e-3, seed=4, block=3, nports=2, margin=2,
                    f0=20e9, bw=20e9)
    oop, dt, B, Lp, fmax, orom = _oracle_case(wl, q=20)
    gop = P.Operator.from_workload(wl)
    grom = P.mor_reduce(gop, wl.sources, wl.probes, 20, dt_ref=dt, fmax=fmax, precision="f32",
                        tol=1e-6, defl_tol=defl)
    info = grom.info()
    assert (info["q1"], info["q2"]) == (20, 20)
    g = _as_oracle_rom(grom)
    P_, Q_ = mor.system_pq(oop, dt)
    for z in list(orom.points) + list(np.conj(orom.points[1:])):
        Hf = mor.transfer(P_, Q_, B, Lp, z)
        assert rel_l2(mor.rom_transfer(g, dt, z), Hf) <= 1e-4, z
    V1, V2 = _gpu_basis(gop, oop, grom)
    assert np.allclose(V1.T @ V1, np.eye(V1.shape[1]), atol=1e-12)
    assert np.allclose(V2.T @ V2, np.eye(V2.shape[1]), atol=1e-12)
    ang = max(_max_angle(V1, orom.V1), _max_angle(V2, orom.V2))
    u = W.drive(wl, dt, 600)
    ew = rel_l2(mor.rom_leapfrog(g, dt, u), mor.rom_leapfrog(orom, dt, u))
    log(f"  max angle {ang:.2e} waveform {ew:.2e}")
    # The subspaces themselves are not fixed by solves that stop at a residual
    # of 1e-6: the oracle's own reduction with every exact solve replaced by
    # one with a random residual of that size moves them by angles of
    # 6.3e-3 ... 6.7e-3 and its waveform by 0.8e-4 ... 3.1e-4 (six draws,
    # tests/test_oracle_mor.py::test_inexact_solves_move_the_subspaces_not_the_moments),
    # while the transfer function at the points stays matched.  The bounds
    # are that spread with margin; the transfer check above is the parity pin.
    assert ang <= 1e-2
    assert ew <= 1e-3


@pytest.mark.parametrize("case", ["cavity", "graded"])
def test_mor_reduce_3d_fp64_fused_and_two_sweep_matvecs(case):
    """3-D FP64 reductions through the fused single-sweep Schur kernel and the
    two-sweep kernel pair: both match the full model's transfer function at
    the expansion points and the oracle's waveform, and agree with each other
    to the solve accuracy.  The graded board exercises non-uniform z spacing
    and PEC strips; the cavity has ragged xy tiles."""
    require_gpu()
    import paper_1406_7042_amd as P
    log(f"mor 3d fp64 {case}")
    if case == "cavity":
        wl = W.cavity3d(n=11, ny=10, nz=9, d=1e-3, seed=4, block=3, nports=2, margin=2,
                        f0=20e9, bw=20e9)
    else:
        wl = W.board3d(nx=12, ny=10, nz_fine=2, nz_coarse=5, d=1e-3, dz_fine=0.3e-3,
                       strip=(2, 10, 4, 6))
    oop, dt, B, Lp, fmax, orom = _oracle_case(wl, q=20)
    gop = P.Operator.from_workload(wl)
    P_, Q_ = mor.system_pq(oop, dt)
    u = W.drive(wl, dt, 600)
    yo = mor.rom_leapfrog(orom, dt, u)
    ys = []
    for mv in ("auto", "two_sweep"):
        grom = P.mor_reduce(gop, wl.sources, wl.probes, 20, dt_ref=dt, fmax=fmax,
                            precision="f64", tol=1e-12, matvec=mv)
        info = grom.info()
        assert (info["q1"], info["q2"]) == (20, 20) and info["relres_max"] <= 1e-12
        g = _as_oracle_rom(grom)
        for z in orom.points:
            assert rel_l2(mor.rom_transfer(g, dt, z), mor.transfer(P_, Q_, B, Lp, z)) <= 1e-10
        ys.append(mor.rom_leapfrog(g, dt, u))
        ew = rel_l2(ys[-1], yo)
        log(f"  {mv}: iters {info['solve_iters']} waveform vs oracle {ew:.2e}")
        assert ew <= 1e-8
    assert rel_l2(ys[0], ys[1]) <= 1e-8


@pytest.mark.parametrize("case,precision", [("cavity", "f64"), ("absorber", "f64"),
                                            ("cavity", "f32")])
def test_mor_reduce_2d_one_pass_and_two_sweep_matvecs(case, precision):
    """2-D reductions through the one-pass iteration (matvec="one_pass":
    k_cocg_fused2, also the automatic choice in 2-D; several
    64 x 8 tiles with ragged edges; the guide has graded sigma_e, sigma_m, so
    per-sample magnetic coefficients, and PEC walls) and through the two-sweep
    matvec: both reach the full model's transfer function at the expansion
    points (FP64: 1e-10 of its largest value over the points; at the cavity's
    third point it is 1e-6 of that, where the oracle's own reduced model is
    1.8e-8 off in relative terms) and give the same waveform; the one-pass
    iterates are the two-sweep ones up to rounding, so the iteration counts
    agree.  (FP32 solves on the guide at q = 20 leave both paths ~0.65 from
    the oracle's model, as FP32 solves do on the iris guide at M = 1.1: no
    comparison is made there.)"""
    require_gpu()
    import paper_1406_7042_amd as P
    log(f"mor 2d one-pass vs two sweeps: {case} {precision}")
    if case == "cavity":
        wl = W.cavity2d(nx=70, ny=45, d=1e-3, seed=3, eps_block=5, eps_range=(1.0, 4.0),
                        sigma_range=(0.0, 0.01))
    else:
        wl = W.waveguide2d()
    q = 20
    oop, dt, B, Lp, fmax, orom = _oracle_case(wl, q=q)
    gop = P.Operator.from_workload(wl)
    P_, Q_ = mor.system_pq(oop, dt)
    u = W.drive(wl, dt, 800)
    yo = mor.rom_leapfrog(orom, dt, u)
    tol = 1e-12 if precision == "f64" else 1e-4
    ys, its = [], []
    for mv in ("one_pass", "two_sweep"):
        grom = P.mor_reduce(gop, wl.sources, wl.probes, q, dt_ref=dt, fmax=fmax,
                            precision=precision, tol=tol, max_iter=20000, matvec=mv)
        info = grom.info()
        assert info["relres_max"] <= tol
        g = _as_oracle_rom(grom)
        if precision == "f64":
            assert (info["q1"], info["q2"]) == (q, q)
            full = [mor.transfer(P_, Q_, B, Lp, z) for z in orom.points]
            scale = max(np.linalg.norm(f) for f in full)
            for z, f in zip(orom.points, full):
                assert np.linalg.norm(mor.rom_transfer(g, dt, z) - f) <= 1e-10 * scale
        ys.append(mor.rom_leapfrog(g, dt, u))
        its.append(info["solve_iters"])
        log(f"  {mv}: iters {info['solve_iters']} q1 {info['q1']} waveform vs oracle "
            f"{rel_l2(ys[-1], yo):.2e}")
    assert abs(its[0] - its[1]) <= max(2, (0.02 if precision == "f64" else 0.05) * its[1])
    cross = rel_l2(ys[0], ys[1])
    e_one, e_two = rel_l2(ys[0], yo), rel_l2(ys[1], yo)
    log(f"  one-pass vs two sweeps: waveform {cross:.2e}")
    if precision == "f64":  # the guide's two paths are both 3e-8 from the oracle's model
        assert e_one <= 1e-7 and cross <= 1e-7
    else:
        # FP32 solves to 1e-4: the later blocks carry the solve error, the
        # same way for either path (both ~5e-2 from the oracle's exact-solve
        # model on the cavity at q = 20); the one-pass path is no worse and
        # the two differ by a fraction of that
        assert e_one <= 1.25 * e_two + 1e-4
        assert cross <= 0.2 * max(e_one, e_two) + 1e-4
    gop.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_mor_reduce_3d_fused_kernel_multi_tile(precision):
    """On a 40 x 36 x 33 cavity (several xy tiles with ragged edges, several z
    chunks per tile) the one-pass COCG iteration and the two-sweep matvec give
    the same reduced model: the iterates are the same up to rounding, so in
    FP64 the reduced matrices agree to 1e-9 and in FP32 (solves to 1e-6) to
    1e-3.  Point 0 is a real shift (real-arithmetic kernel), the others are
    complex."""
    require_gpu()
    import paper_1406_7042_amd as P
    log(f"mor 3d fused kernel multi-tile {precision}")
    wl = W.cavity3d(n=40, ny=36, nz=33, d=1e-3, seed=6, block=5, nports=2, margin=3,
                    f0=10e9, bw=10e9)
    gop = P.Operator.from_workload(wl)
    dt = 0.99 * gop.dt_max
    tol, bound = (1e-12, 1e-9) if precision == "f64" else (1e-6, 1e-3)
    mats = {}
    for mv in ("auto", "two_sweep"):
        grom = P.mor_reduce(gop, wl.sources, wl.probes, 20, dt_ref=dt, fmax=2e10,
                            precision=precision, tol=tol, max_iter=20000, matvec=mv)
        info = grom.info()
        log(f"  {mv}: iters {info['solve_iters']} relres {info['relres_max']:.2e}")
        assert (info["q1"], info["q2"]) == (20, 20) and info["relres_max"] <= tol
        mats[mv] = grom.matrices()
    for k, a in mats["auto"].items():
        b = mats["two_sweep"][k]
        d = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        assert d <= bound, (k, d)


@pytest.mark.parametrize("nports", [1, 3])
def test_mor_reduce_3d_fused_single_and_padded_batches(nports):
    """One right-hand side per solve (1 port) and a batch padded to the kernel's
    column count (3 ports solved as 4 columns, one of them empty): the one-pass
    COCG (grid planned over the columns still iterating, x updated on every
    other pass with a final fix-up) and the two-sweep matvec give the same
    reduced model in FP64 (solves to 1e-12), and both match the full model's
    transfer function at the expansion points."""
    require_gpu()
    import paper_1406_7042_amd as P
    log(f"mor 3d fused {nports} port(s)")
    wl = W.cavity3d(n=14, ny=12, nz=11, d=1e-3, seed=11, block=4, nports=nports, margin=2,
                    f0=15e9, bw=15e9)
    oop, dt, B, Lp, fmax, orom = _oracle_case(wl, q=5 * nports)
    gop = P.Operator.from_workload(wl)
    P_, Q_ = mor.system_pq(oop, dt)
    mats = {}
    for mv in ("auto", "two_sweep"):
        grom = P.mor_reduce(gop, wl.sources, wl.probes, 5 * nports, dt_ref=dt, fmax=fmax,
                            precision="f64", tol=1e-12, max_iter=20000, matvec=mv)
        info = grom.info()
        log(f"  {mv}: iters {info['solve_iters']} matvecs {info['matvecs']}")
        assert (info["q1"], info["q2"]) == (5 * nports, 5 * nports)
        assert info["relres_max"] <= 1e-12
        g = _as_oracle_rom(grom)
        for z in orom.points:
            assert rel_l2(mor.rom_transfer(g, dt, z), mor.transfer(P_, Q_, B, Lp, z)) <= 1e-9
        mats[mv] = grom.matrices()
    for k, a in mats["auto"].items():
        b = mats["two_sweep"][k]
        d = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        assert d <= 1e-8, (k, d)


@pytest.mark.parametrize("q,precision", [(30, "f64"), (60, "f64"), (120, "f64"), (200, "f64"),
                                         (30, "f32"), (90, "f32"), (200, "f32")])
def test_mor_reduce_projections_equal_explicit_products(q, precision):
    """The projections of eq. (R_and_Freduced), V1^T De V1, V1^T Dse V1,
    V2^T Dm V2 and V1^T (K V2), formed on the matrix cores over the full grid,
    equal the same products taken in FP64 from the returned basis; the orders
    span every row-chunk size of the Gram and two-operand kernels (up to 32,
    64, 128 and 256 columns).  With FP32 solves the basis is orthonormalised
    by the deflating CholQR2 whose V R^-1 runs in place on the matrix cores
    (every chunk size: up to 64, 128 and 256 columns): V1 and V2 come out
    orthonormal to 1e-10."""
    require_gpu()
    import paper_1406_7042_amd as P
    log(f"mor projections q={q} {precision}")
    wl = W.cavity3d(n=20, ny=16, nz=14, d=1e-3, seed=5, block=4, nports=2, margin=2,
                    f0=15e9, bw=15e9)
    oop = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(oop.grid)
    gop = P.Operator.from_workload(wl)
    tol = 1e-10 if precision == "f64" else 1e-4
    grom = P.mor_reduce(gop, wl.sources, wl.probes, q, dt_ref=dt, fmax=wl.f0 + wl.bw,
                        precision=precision, tol=tol, max_iter=20000)
    info = grom.info()
    log(f"  q1 {info['q1']} q2 {info['q2']} relres {info['relres_max']:.2e}")
    assert info["relres_max"] <= tol
    V1, V2 = _gpu_basis(gop, oop, grom)
    assert V1.shape[1] == info["q1"] and V2.shape[1] == info["q2"]
    assert info["q1"] > 0.75 * q and info["q2"] > 0.75 * q
    assert np.abs(V1.T @ V1 - np.eye(V1.shape[1])).max() <= 1e-10
    assert np.abs(V2.T @ V2 - np.eye(V2.shape[1])).max() <= 1e-10
    m = grom.matrices()
    want = {"De": V1.T @ (oop.De[:, None] * V1), "Dse": V1.T @ (oop.Dse[:, None] * V1),
            "Dm": V2.T @ (oop.Dm[:, None] * V2), "K": V1.T @ (oop.K @ V2)}
    for k, b in want.items():
        a = m[k]
        assert a.shape == b.shape and (k == "K" or np.array_equal(a, a.T)), k
        d = np.linalg.norm(a - b) / np.linalg.norm(b)
        log(f"  {k}: {d:.2e}")
        assert d <= 1e-12, (k, d)
    gop.close()


def test_mor_reduce_waveguide_matched_absorber():
    """The matched-absorber guide (graded sigma_e and sigma_m, non-uniform
    magnetic materials: two-sweep Schur matvec) with a line source and two
    line probes: the reduced model matches the full model's transfer function
    at the expansion points (Sec. II-C), as the oracle's does, and carries the
    projected magnetic losses Dsm~."""
    require_gpu()
    import paper_1406_7042_amd as P
    log("mor waveguide matched absorber")
    wl = W.waveguide2d()
    q = 20
    oop, dt, B, Lp, fmax, orom = _oracle_case(wl, q=q)
    gop = P.Operator.from_workload(wl)
    grom = P.mor_reduce(gop, wl.sources, wl.probes, q, dt_ref=dt, fmax=fmax, precision="f64",
                        tol=1e-12, max_iter=20000)
    info = grom.info()
    assert (info["q1"], info["q2"]) == (orom.q1, orom.q2) == (q, q)
    assert info["relres_max"] <= 1e-12
    V1, V2 = _gpu_basis(gop, oop, grom)
    assert np.allclose(V1.T @ V1, np.eye(q), atol=1e-12)
    m = grom.matrices()
    want = V2.T @ (oop.Dsm[:, None] * V2)
    assert np.linalg.norm(m["Dsm"]) > 0
    assert np.linalg.norm(m["Dsm"] - want) <= 1e-12 * np.linalg.norm(want)
    P_, Q_ = mor.system_pq(oop, dt)
    g = _as_oracle_rom(grom)
    for z in orom.points:
        full = mor.transfer(P_, Q_, B, Lp, z)
        dg, do = rel_l2(mor.rom_transfer(g, dt, z), full), rel_l2(mor.rom_transfer(orom, dt, z), full)
        log(f"  H(z = {z:.4f}): gpu {dg:.2e} oracle {do:.2e}")
        assert dg <= 1e-8 and do <= 1e-8
    gop.close()


def test_mor_reduce_3d_matched_absorber_walls():
    """3-D lossy cavity whose two x walls carry 3-cell 4th-order matched
    absorbers (graded sigma_e and sigma_m = sigma_e mu / eps): the magnetic
    losses make the magnetic materials non-uniform, so the reduction runs the
    two-sweep Schur matvec in 3-D; the reduced model matches the full model's
    transfer function at the expansion points and projects D_sigma_m exactly."""
    require_gpu()
    import paper_1406_7042_amd as P
    log("mor 3d matched absorber walls")
    wl = W.cavity3d(n=14, ny=12, nz=11, d=1e-3, seed=11, block=4, nports=2, margin=2,
                    f0=15e9, bw=15e9)
    prof = W.graded_absorber(3, 4, W.absorber_sigma_max(3, 4, 1e-3, 1.0, np.exp(-8.0)))
    eps0 = 1.0 / (W.MU0_WL * W.C0 ** 2)
    sig_m = np.zeros_like(wl.eps_r)
    for a, sv in enumerate(prof):
        for i in (a, wl.nx - 1 - a):
            wl.sigma_e[:, :, i] += sv
            sig_m[:, :, i] = wl.sigma_e[:, :, i] * W.MU0_WL / (eps0 * wl.eps_r[:, :, i])
    wl.sigma_m = sig_m
    q = 10
    oop, dt, B, Lp, fmax, orom = _oracle_case(wl, q=q)
    gop = P.Operator.from_workload(wl)
    grom = P.mor_reduce(gop, wl.sources, wl.probes, q, dt_ref=dt, fmax=fmax, precision="f64",
                        tol=1e-12, max_iter=20000)
    info = grom.info()
    assert (info["q1"], info["q2"]) == (orom.q1, orom.q2) == (q, q)
    V1, V2 = _gpu_basis(gop, oop, grom)
    want = V2.T @ (oop.Dsm[:, None] * V2)
    got = grom.matrices()["Dsm"]
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    P_, Q_ = mor.system_pq(oop, dt)
    g = _as_oracle_rom(grom)
    for z in orom.points:
        d = rel_l2(mor.rom_transfer(g, dt, z), mor.transfer(P_, Q_, B, Lp, z))
        log(f"  H(z = {z:.4f}): {d:.2e}")
        assert d <= 1e-9
    gop.close()


def test_mor_reduce_full_size_fused_vs_two_sweep():
    """The 128^3 lossy cavity with 4 ports, the launch configuration the
    benchmark times (128 x 8 FP32 tiles whose last x tile borders the padding
    column i = nx, 4 right-hand sides per pass, the grid re-planned as columns
    converge): the one-pass COCG iteration and the two-sweep matvec (separate
    kernels, no tiling) build the same reduced model up to the FP32 solve
    accuracy; both bases come out orthonormal and zero at padding positions.
    The reduced matrices depend on the basis, which the block Krylov
    recurrence fixes only to the solve error amplified over the blocks (K moves
    by a few 1e-3 here), so the comparison is on what the basis does not
    change: the reduced transfer function (Sec. II-C) at and between the
    expansion points, and the reduced waveform."""
    require_gpu()
    import torch

    import paper_1406_7042_amd as P
    log("mor 128^3 fused vs two-sweep")
    wl = W.cavity3d(n=128, d=1e-3, seed=1, block=8, nports=4, f0=1.5e9, bw=1.5e9)
    gop = P.Operator.from_workload(wl)
    dt = 0.99 * gop.dt_max
    fmax, M, L = 3e9, 1.1, 2
    roms = {}
    for mv in ("auto", "two_sweep"):
        grom = P.mor_reduce(gop, wl.sources, wl.probes, 20, dt_ref=dt, fmax=fmax, M=M, L=L,
                            precision="f32", tol=1e-6, max_iter=20000, matvec=mv)
        info = grom.info()
        log(f"  {mv}: iters {info['solve_iters']} matvecs {info['matvecs']} "
            f"relres {info['relres_max']:.2e}")
        assert (info["q1"], info["q2"]) == (20, 20) and info["relres_max"] <= 1e-6
        V1, V2 = grom.basis(gop)  # q x (padded slots)
        for V in (V1, V2):
            G = (V @ V.T).double().cpu().numpy()
            assert np.abs(G - np.eye(20)).max() <= 1e-10
        # the padding column i = nx and row j = ny are never unknowns: zero
        pad = [gop.slot(c, 128, j, k) for c in range(3) for j in (0, 5, 64, 127)
               for k in (1, 77)] + [gop.slot(c, i, 128, 9) for c in range(3) for i in (0, 64)]
        assert torch.count_nonzero(V1[:, pad]).item() == 0
        roms[mv] = _as_oracle_rom(grom)
    pts = mor.expansion_points(M, L, fmax, dt)
    zs = list(pts) + list(np.conj(pts[1:])) + [M * np.exp(0.5j * (np.angle(pts[1]) + np.angle(pts[2])))]
    for z in zs:
        a, b = (mor.rom_transfer(roms[mv], dt, z) for mv in ("auto", "two_sweep"))
        d = rel_l2(a, b)
        log(f"  H(z = {z:.4f}): {d:.2e}")
        assert d <= 1e-8, (z, d)
    u = W.drive(wl, dt, 2000)
    ya, yb = (mor.rom_leapfrog(roms[mv], dt, u) for mv in ("auto", "two_sweep"))
    d = rel_l2(ya, yb)
    log(f"  waveform: {d:.2e}")
    assert d <= 1e-4
    gop.close()


def test_mor_reduce_rejects_bad_order():
    require_gpu()
    import paper_1406_7042_amd as P
    wl = W.cavity2d()
    gop = P.Operator.from_workload(wl)
    with pytest.raises(P.YeeromError):
        P.mor_reduce(gop, wl.sources, wl.probes, 41, dt_ref=0.99 * gop.dt_max, fmax=1e11)


# --------------------------------------------------------------------------- perturbation


@pytest.fixture(scope="module")
def small_rom():
    # drive band (5-15 GHz, f_max 20 GHz) well below the Nyquist frequency of
    # the largest reduced time step used here (s = 4.95: 43 GHz)
    wl = W.cavity2d(nx=14, ny=12, seed=5, eps_block=3, eps_range=(1, 4), sigma_range=(0, 2.0),
                    f0=10e9, bw=10e9)
    oop, dt, B, Lp, fmax, orom = _oracle_case(wl, q=30)
    return wl, oop, dt, orom


def _gpu_rom_from(orom):
    import paper_1406_7042_amd as P
    return P.Rom.from_matrices(orom.De, orom.Dm, orom.K, orom.B1, orom.L1, Dse=orom.Dse,
                               Dsm=orom.Dsm, B2=orom.B2, L2=orom.L2)


@pytest.mark.parametrize("s", [0.99, 4.95])
def test_rom_perturb_matches_oracle(small_rom, s):
    """Sec. III-A on identical inputs: K~' and the singular values agree with
    the oracle (symmetric square roots) to 1e-10; nothing is clamped below CFL."""
    require_gpu()
    import paper_1406_7042_amd as P
    log(f"perturb s={s}")
    wl, oop, dt0, orom = small_rom
    dt = dt0 / 0.99 * s
    Kp, n, sig, _ = perturb.perturb(orom.De, orom.Dm, orom.K, dt, 0.9999)
    grom = _gpu_rom_from(orom)
    ng = P.rom_perturb(grom, dt, 0.9999, dtype="f64")
    assert ng == n
    if s < 1:
        assert n == 0
    else:
        assert n > 0
    ek = rel_l2(grom.get(P.yeerom.ROM_KP), Kp)
    log(f"  K' rel err {ek:.2e} clamped {n}")
    assert ek <= 1e-10
    assert rel_l2(grom.get(P.yeerom.ROM_SIGMA), np.sort(sig)[::-1]) <= 1e-12
    assert grom.info()["guard_margin"] > 0


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_rom_step_matches_oracle_beyond_cfl(small_rom, prec, tol):
    """Reduced leapfrog at s = 4.95 after the clamp, lossy model: output
    waveform equals the oracle's eq. (reducedMNAform) with K~ -> K~'."""
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    log(f"rom_step {prec}")
    wl, oop, dt0, orom = small_rom
    dt = dt0 / 0.99 * 4.95
    Kp, _, _, _ = perturb.perturb(orom.De, orom.Dm, orom.K, dt, 0.9999)
    nsteps = 3000
    u = W.drive(wl, dt, nsteps)
    y_ref = mor.rom_leapfrog(orom, dt, u, K=Kp)
    grom = _gpu_rom_from(orom)
    P.rom_perturb(grom, dt, 0.9999, dtype=prec)
    tdt = torch.float64 if prec == "f64" else torch.float32
    y = P.rom_step([grom], dt, nsteps, [torch.tensor(u, dtype=tdt, device="cuda")],
                   dtype=prec)[0]
    torch.cuda.synchronize()
    err = rel_l2(y.cpu().numpy(), y_ref)
    log(f"  rom_step {prec} rel err {err:.2e}")
    assert err <= tol


def test_rom_lift_reconstructs_the_oracle_full_state():
    """Full-field reconstruction x ~ V x~ (eq. (V)) of the reduced state left by
    rom_step equals the oracle's V x~ (basis-invariant), its probe gather is
    rom_step's last output (L~ = V^T L), states lift linearly in batches, and
    FP32 states lift to the FP64 field at FP32 accuracy."""
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    log("rom_lift")
    wl = W.cavity2d()
    q = 20
    oop, dt, B, Lp, fmax, orom = _oracle_case(wl, q=q)
    c = _collected_condition(oop, dt, B, fmax, q)
    gop = P.Operator.from_workload(wl)
    grom = P.mor_reduce(gop, wl.sources, wl.probes, q, dt_ref=dt, fmax=fmax, precision="f64",
                        tol=1e-13)
    P.rom_perturb(grom, dt, 0.9999, dtype="f64")
    info = grom.info()
    nsteps = 400
    u = W.drive(wl, dt, nsteps)
    st = torch.zeros(info["q1"] + info["q2"], dtype=torch.float64, device="cuda")
    y = P.rom_step([grom], dt, nsteps, [torch.tensor(u, dtype=torch.float64, device="cuda")],
                   dtype="f64", states=[st])[0]
    x = P.rom_lift(gop, grom, st)
    torch.cuda.synchronize()
    xo = state_to_oracle(gop, oop, x)
    _, Xo = mor.rom_leapfrog(orom, dt, u, return_states=True)
    xt = Xo[-1]
    ref = np.concatenate([orom.V1 @ xt[:orom.q1], orom.V2 @ xt[orom.q1:]])
    err = rel_l2(xo, ref)
    eprobe = rel_l2(Lp.T @ xo, y[-1].cpu().numpy())
    log(f"  lift vs oracle V x~ {err:.2e}, probe identity {eprobe:.2e}")
    assert err <= max(1e-9, 1e-13 / c)
    assert eprobe <= 1e-12
    # off the unknowns the lifted buffer is exactly zero
    mask = np.ones(gop.field_len, bool)
    mask[slots_of(gop, oop.ne.keys)] = False
    mask[slots_of(gop, oop.nh.keys)] = False
    assert np.all(x.cpu().numpy()[mask] == 0)
    # batches (5 states: one full pass of 4 and a ragged one) lift linearly
    fac = [1.0, 2.0, 0.0, -0.5, 1.0]
    X5 = P.rom_lift(gop, grom, torch.stack([f * st for f in fac]))
    for i, f in enumerate(fac):
        assert torch.equal(X5[i], f * x)
    x32 = P.rom_lift(gop, grom, st.float())
    assert rel_l2(x32.double().cpu().numpy(), x.cpu().numpy()) <= 1e-6


def test_rom_step_batch_of_uneven_orders_equals_single_runs():
    """Many reduced models of different orders stepped in one launch give the
    same outputs as each model alone (and as the oracle)."""
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    log("rom_step batch")
    roms, orcs, us = [], [], []
    for i, (n, q) in enumerate([(10, 15), (13, 25), (9, 10), (12, 30)]):
        wl = W.cavity2d(nx=n, ny=n, seed=10 + i, eps_block=3, eps_range=(1, 6), f0=10e9, bw=10e9)
        oop, dt0, B, Lp, fmax, orom = _oracle_case(wl, q=q)
        orcs.append((orom, wl, dt0))
    dt = max(o[2] for o in orcs) / 0.99 * 4.95
    nsteps = 1500
    for orom, wl, _ in orcs:
        r = _gpu_rom_from(orom)
        roms.append(r)
        us.append(torch.tensor(W.drive(wl, dt, nsteps), dtype=torch.float64, device="cuda"))
    P.rom_perturb(roms, dt, 0.9999, dtype="f64")
    ys = P.rom_step(roms, dt, nsteps, us, dtype="f64")
    for r, u, y, (orom, wl, _) in zip(roms, us, ys, orcs):
        y1 = P.rom_step([r], dt, nsteps, [u], dtype="f64")[0]
        assert torch.equal(y, y1)
        Kp, _, _, _ = perturb.perturb(orom.De, orom.Dm, orom.K, dt, 0.9999)
        y_ref = mor.rom_leapfrog(orom, dt, u.cpu().numpy(), K=Kp)
        err = rel_l2(y.cpu().numpy(), y_ref)
        log(f"  batch model rel err {err:.2e}")
        assert err <= 1e-10


def test_rom_step_state_roundtrip_and_errors(small_rom):
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    wl, oop, dt0, orom = small_rom
    grom = _gpu_rom_from(orom)
    u = torch.tensor(W.drive(wl, dt0, 200), dtype=torch.float64, device="cuda")
    with pytest.raises(P.YeeromError) as e:  # not prepared
        P.rom_step([grom], dt0, 200, [u], dtype="f64")
    assert e.value.status == P.yeerom.YR_ESTATE
    P.rom_perturb(grom, dt0, 0.9999, dtype="f64")
    q = grom.info()["q1"] + grom.info()["q2"]
    st = torch.zeros(q, dtype=torch.float64, device="cuda")
    ya = P.rom_step([grom], dt0, 100, [u[:100].contiguous()], dtype="f64", states=[st])[0]
    yb = P.rom_step([grom], dt0, 100, [u[100:].contiguous()], dtype="f64", states=[st])[0]
    yall = P.rom_step([grom], dt0, 200, [u], dtype="f64")[0]
    assert torch.allclose(torch.cat([ya, yb]), yall, rtol=1e-12, atol=1e-300)


def test_rom_perturb_certificate_rejects_unstable_stepping(small_rom):
    """gamma > 1 keeps singular values beyond 2/dt: the FP64 certificate of
    condition (Dstability2) fails and the model is not prepared."""
    require_gpu()
    import paper_1406_7042_amd as P
    wl, oop, dt0, orom = small_rom
    dt = dt0 / 0.99 * 4.95
    grom = _gpu_rom_from(orom)
    with pytest.raises(P.YeeromError) as e:
        P.rom_perturb(grom, dt, 1.5, dtype="f64")
    assert e.value.status == P.yeerom.YR_EUNSTABLE
    assert grom.info()["step_dt"] < 0


# --------------------------------------------------------------------------- reduced adjoint


def test_rom_adjoint_matches_oracle(small_rom):
    """Reduced adjoint at s = 4.95 on identical inputs: J, dJ/dDe~, dJ/dK~' and
    the parameter derivative (clamp frozen, and through the clamp) agree with
    the oracle (symmetric square roots) to 1e-9."""
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    from oracle import adjoint as oadj
    log("rom adjoint")
    wl = W.cavity2d(nx=14, ny=12, seed=5, eps_block=3, eps_range=(1, 4), sigma_range=(0, 2.0),
                    f0=10e9, bw=10e9)
    oop, dt0, B, Lp, fmax, orom = _oracle_case(wl, q=20)
    assert orom.q1 == orom.q2 == 20
    dt = dt0 / 0.99 * 4.95
    nsteps = 400
    u = W.drive(wl, dt, nsteps)
    V = W.random_vectors(21, (orom.q1, orom.q1))
    dDe = 0.5 * (V + V.T) * np.abs(orom.De).max() * 1e-2
    J, dJ, gDe, gDse, gK = oadj.reduced_theta_gradient(orom, dt, u, dDe)
    _, dJf, *_ = oadj.reduced_theta_gradient(orom, dt, u, dDe, through_clamp=False)
    grom = _gpu_rom_from(orom)
    # dJ/dy = 2 dt y for the probe energy: y from the FP64 oracle run
    Kp, _, _, _ = perturb.perturb(orom.De, orom.Dm, orom.K, dt, 0.9999)
    y = mor.rom_leapfrog(orom, dt, u, K=Kp)
    ud = torch.tensor(u, dtype=torch.float64, device="cuda")
    gy = torch.tensor(2 * dt * y, dtype=torch.float64, device="cuda")
    r = P.yeerom.rom_adjoint(grom, dt, nsteps, ud, gy, dDe=dDe)
    log(f"  J {r['J']:.6e} vs {J:.6e}; dJ {r['dJ']:.6e} vs {dJ:.6e}; frozen {r['dJ_frozen']:.6e} vs {dJf:.6e}")
    assert r["J"] == pytest.approx(J, rel=1e-10)
    assert rel_l2(r["gDe"], gDe) <= 1e-9
    assert rel_l2(r["gDse"], gDse) <= 1e-9
    assert rel_l2(r["gK"], gK) <= 1e-9
    assert r["dJ_frozen"] == pytest.approx(dJf, rel=1e-9)
    assert r["dJ"] == pytest.approx(dJ, rel=1e-8)


def test_rom_function_gradients_match_oracle():
    """ROMFunction (autograd over the clamp + reduced leapfrog, backward
    through the reduced adjoint): for J = dt sum y^2 and two parameters that
    move De~ along seeded symmetric directions, theta.grad equals the oracle's
    reduced_theta_gradient through the clamp (s = 4.95) to 1e-8, and the
    forward waveform equals the oracle's clamped reduced leapfrog to 1e-10."""
    require_gpu()
    import torch
    from oracle import adjoint as oadj
    from paper_1406_7042_amd.autograd import ROMFunction
    log("ROMFunction")
    wl = W.cavity2d(nx=14, ny=12, seed=5, eps_block=3, eps_range=(1, 4), sigma_range=(0, 2.0),
                    f0=10e9, bw=10e9)
    oop, dt0, B, Lp, fmax, orom = _oracle_case(wl, q=20)
    dt = dt0 / 0.99 * 4.95
    nsteps = 400
    u = W.drive(wl, dt, nsteps)
    dirs = []
    for seed in (31, 32):
        V = W.random_vectors(seed, (orom.q1, orom.q1))
        dirs.append(0.5 * (V + V.T) * np.abs(orom.De).max() * 1e-2)
    ref = [oadj.reduced_theta_gradient(orom, dt, u, d)[1] for d in dirs]
    Kp, _, _, _ = perturb.perturb(orom.De, orom.Dm, orom.K, dt, 0.9999)
    y_ref = mor.rom_leapfrog(orom, dt, u, K=Kp)
    grom = _gpu_rom_from(orom)
    theta = torch.zeros(2, dtype=torch.float64, requires_grad=True)
    ud = torch.tensor(u, dtype=torch.float64, device="cuda")
    y = ROMFunction.apply(theta, grom, orom.De, dirs, dt, nsteps, ud)
    assert rel_l2(y.detach().cpu().numpy(), y_ref) <= 1e-10
    J = dt * (y ** 2).sum()
    J.backward()
    g = theta.grad.numpy()
    log(f"  dJ/dtheta {g} vs oracle {ref}")
    for a, b in zip(g, ref):
        assert a == pytest.approx(b, rel=1e-8)


def test_rom_adjoint_slab_eps_graded_board_vs_finite_differences():
    """Graded-mesh board (fine substrate under coarse air, PEC strip, 2 line
    ports): reduce, then d/d(slab eps_r) of the reduced probe energy at 9.9x
    the fine-cell CFL step, through the clamp, with the basis frozen, equals
    FP64 central differences of clamp + reduced leapfrog (GPU, FP64)."""
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    log("rom adjoint board")
    wl = W.board3d(nx=20, ny=12, nz_fine=3, nz_coarse=5, d=1e-3, dz_fine=0.2e-3,
                   strip=(4, 16, 5, 7), f0=10e9, bw=10e9)
    oop = yee.assemble(wl)
    dt_fine = 0.99 * yee.cfl_dt_max(oop.grid)
    gop = P.Operator.from_workload(wl)
    rom = P.mor_reduce(gop, wl.sources, wl.probes, 20, dt_ref=dt_fine, fmax=20e9, precision="f64",
                       tol=1e-12)
    # projecting the structure's own eps_r reproduces De~
    De = rom.get(P.yeerom.ROM_DE)
    assert rel_l2(P.yeerom.rom_project_cells(gop, rom, wl.eps_r, "eps"), De) <= 1e-12
    slab = np.zeros_like(wl.eps_r)
    slab[:3] = 1.0
    dDe = P.yeerom.rom_project_cells(gop, rom, slab, "eps")
    dt = 10 * dt_fine  # s = 9.9
    nsteps = 600
    u = torch.tensor(W.drive(wl, dt, nsteps), dtype=torch.float64, device="cuda")
    m = rom.matrices()

    def J_of(theta):
        r = P.Rom.from_matrices(m["De"] + theta * dDe, m["Dm"], m["K"], m["B1"], m["L1"],
                                Dse=m["Dse"], Dsm=m["Dsm"], B2=m["B2"], L2=m["L2"])
        n = P.rom_perturb(r, dt, 0.9999, dtype="f64")
        y = P.rom_step([r], dt, nsteps, [u], dtype="f64")[0]
        return float(dt * (y ** 2).sum()), n, y

    J0, n0, y0 = J_of(0.0)
    assert n0 > 0
    res = P.yeerom.rom_adjoint(rom, dt, nsteps, u, (2 * dt * y0).contiguous(), dDe=dDe)
    assert res["J"] == pytest.approx(J0, rel=1e-9)
    h = 1e-5
    (jp, n1, _), (jm, n2, _) = J_of(h), J_of(-h)
    assert n1 == n2 == n0
    fd = (jp - jm) / (2 * h)
    log(f"  clamped {n0}: adjoint {res['dJ']:.8e} FD {fd:.8e} frozen {res['dJ_frozen']:.8e}")
    assert res["dJ"] == pytest.approx(fd, rel=1e-5)
