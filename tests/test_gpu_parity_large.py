"""Parity on the launch paths the benchmark workloads take, against the FP64
oracle.

* rom_perturb (Sec. III-A) and rom_step (eq. (reducedMNAform)) on reduced
  models of the orders the benchmarks use: oracle reductions of lossy 2-D
  96 x 96 cavities at q = 100, 200, 400 and 600 (min(q1, q2) = 79 ... 338,
  which selects every block size of the block-Jacobi SVD), stepped 2048
  times at s = 4.95 (the length from which the stepper's workgroup size is
  autotuned), alone and inside one launch of 64 models of uneven order.
  Inputs are identical on both sides (the oracle's reduced matrices).
* The one-pass FP32 COCG kernel on a box wider than one 128-cell x tile,
  against the full model's transfer function (Sec. II-C moment matching).
* The 20 x 20 cavity at its own order q = 40, through quantities the data
  determine well: the reduced transfer function and its derivative at each
  expansion point against the full model.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mor, perturb, yee
from tests.gpuutil import log, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

ORDERS = (100, 200, 400, 600)


def _cavity96(seed):
    # lossy blocks (sigma_e up to 0.5 S/m) so that the loss eigenvectors of the
    # clamp are exercised too; drive band 5-15 GHz, f_max 20 GHz, far below the
    # Nyquist frequency of s = 4.95 (43 GHz)
    return W.cavity2d(nx=96, ny=96, d=1e-3, seed=seed, eps_block=8, eps_range=(1, 6),
                      sigma_range=(0.0, 0.5), f0=10e9, bw=10e9)


@pytest.fixture(scope="module")
def roms96():
    require_gpu()
    out = {}
    for i, q in enumerate(ORDERS):
        wl = _cavity96(2000 + i)
        oop = yee.assemble(wl)
        dt0 = 0.99 * yee.cfl_dt_max(oop.grid)
        B = yee.port_matrix(oop, wl.sources, True)
        Lp = yee.port_matrix(oop, wl.probes, False)
        log(f"oracle reduction 96x96 q={q}")
        out[q] = (wl, dt0, mor.mor_reduce(oop, B, Lp, q=q, dt_ref=dt0, fmax=20e9, M=1.1,
                                           npts_half=2))
    return out


def _gpu_rom(orom):
    import paper_1406_7042_amd as P
    return P.Rom.from_matrices(orom.De, orom.Dm, orom.K, orom.B1, orom.L1, Dse=orom.Dse,
                               Dsm=orom.Dsm, B2=orom.B2, L2=orom.L2)


def _truncate(orom, a, b):
    """The model projected on the first a columns of V1 and b of V2: itself a
    reduced model of eq. (R_and_Freduced) (a congruence of the full one)."""
    return mor.Reduced(V1=orom.V1[:, :a], V2=orom.V2[:, :b], De=orom.De[:a, :a],
                       Dse=orom.Dse[:a, :a], Dm=orom.Dm[:b, :b], Dsm=orom.Dsm[:b, :b],
                       K=orom.K[:a, :b], B1=orom.B1[:a], B2=orom.B2[:b], L1=orom.L1[:a],
                       L2=orom.L2[:b])


@pytest.mark.parametrize("q", ORDERS)
def test_rom_perturb_large_orders_match_oracle(roms96, q):
    """K~' and the singular values of De~^-1/2 K~ Dm~^-1/2 at s = 4.95 agree
    with the oracle's symmetric-root route to 1e-10 (the singular values to
    1e-12), the clamp count is the same and the FP64 certificate holds."""
    require_gpu()
    import paper_1406_7042_amd as P
    wl, dt0, orom = roms96[q]
    dt = dt0 / 0.99 * 4.95
    log(f"perturb q={q} (q1 {orom.q1}, q2 {orom.q2})")
    Kp, n, sig, _ = perturb.perturb(orom.De, orom.Dm, orom.K, dt, 0.9999)
    g = _gpu_rom(orom)
    ng = P.rom_perturb(g, dt, 0.9999, dtype="f64")
    ek = rel_l2(g.get(P.yeerom.ROM_KP), Kp)
    es = rel_l2(g.get(P.yeerom.ROM_SIGMA), np.sort(sig)[::-1])
    log(f"  clamped {ng}/{n}  K' {ek:.2e}  sigma {es:.2e}")
    assert ng == n > 0
    assert ek <= 1e-10
    assert es <= 1e-12
    assert g.info()["guard_margin"] > 0


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
@pytest.mark.parametrize("q", ORDERS)
def test_rom_step_large_orders_match_oracle(roms96, q, prec, tol):
    """2048 reduced steps at s = 4.95 after the clamp (autotuned workgroup
    size): output waveform against the oracle's eq. (reducedMNAform) with
    K~ -> K~'."""
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    wl, dt0, orom = roms96[q]
    dt = dt0 / 0.99 * 4.95
    nsteps = 2048
    log(f"rom_step q={q} {prec}")
    Kp, _, _, _ = perturb.perturb(orom.De, orom.Dm, orom.K, dt, 0.9999)
    u = W.drive(wl, dt, nsteps)
    y_ref = mor.rom_leapfrog(orom, dt, u, K=Kp)
    g = _gpu_rom(orom)
    P.rom_perturb(g, dt, 0.9999, dtype=prec)
    tdt = torch.float64 if prec == "f64" else torch.float32
    y = P.rom_step([g], dt, nsteps, [torch.tensor(u, dtype=tdt, device="cuda")], dtype=prec)[0]
    torch.cuda.synchronize()
    err = rel_l2(y.cpu().numpy(), y_ref)
    log(f"  rel err {err:.2e}")
    assert err <= tol


@pytest.fixture(scope="module")
def batch64(roms96):
    """64 models: the four full models and 60 truncations to ~U[50, q1] leading
    columns, one dt (every grid is 96 x 96 at 1 mm), with the oracle's
    clamped waveforms over 2048 steps at s = 4.95."""
    require_gpu()
    rng = np.random.default_rng(64)
    models = [roms96[q] for q in ORDERS]
    while len(models) < 64:
        wl, dt0, orom = roms96[ORDERS[int(rng.integers(0, len(ORDERS)))]]
        a = int(rng.integers(50, orom.q1 + 1))
        b = min(orom.q2, a + int(rng.integers(0, 3)))
        models.append((wl, dt0, _truncate(orom, a, b)))
    dt = roms96[ORDERS[0]][1] / 0.99 * 4.95
    nsteps = 2048
    log("oracle references of the 64-model batch")
    refs = []
    for wl, _, o in models:
        Kp, _, _, _ = perturb.perturb(o.De, o.Dm, o.K, dt, 0.9999)
        u = W.drive(wl, dt, nsteps)
        refs.append((u, mor.rom_leapfrog(o, dt, u, K=Kp)))
    return models, dt, nsteps, refs


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_rom_step_batch_of_64_uneven_large_orders_matches_oracle(batch64, prec, tol):
    """One rom_step launch over 64 models of uneven order, clamped together by
    rom_perturb_batch, 2048 steps at s = 4.95: every model's waveform against
    the oracle."""
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    models, dt, nsteps, refs = batch64
    tdt = torch.float64 if prec == "f64" else torch.float32
    log(f"rom_step batch of {len(models)} ({prec})")
    grs = [_gpu_rom(o) for _, _, o in models]
    P.rom_perturb(grs, dt, 0.9999, dtype=prec)
    us = [torch.tensor(u, dtype=tdt, device="cuda") for u, _ in refs]
    ys = P.rom_step(grs, dt, nsteps, us, dtype=prec)
    torch.cuda.synchronize()
    errs = [rel_l2(y.cpu().numpy(), y_ref) for y, (_, y_ref) in zip(ys, refs)]
    log(f"  worst rel err {max(errs):.2e}")
    for (_, _, o), e in zip(models, errs):
        assert e <= tol, (o.q1, o.q2, e)


# ------------------------------------------------------------- one-pass COCG, 2 x tiles


@pytest.fixture(scope="module")
def wide_box():
    require_gpu()
    wl = W.cavity3d(n=140, ny=10, nz=8, d=1e-3, seed=7, block=5, nports=2, margin=2,
                    f0=15e9, bw=15e9)
    oop = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(oop.grid)
    B = yee.port_matrix(oop, wl.sources, True)
    Lp = yee.port_matrix(oop, wl.probes, False)
    pts = mor.expansion_points(1.1, 2, wl.f0 + wl.bw, dt)
    zs = list(pts) + list(np.conj(pts[1:]))
    log("oracle transfer functions 140x10x8")
    H = [Lp.T @ mor.schur_solve(oop, dt, z, B.astype(complex)) for z in zs]
    return wl, oop, dt, B, Lp, zs, H


@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_fused_fp32_cocg_two_x_tiles_matches_full_transfer(wide_box, tol):
    """140 x 10 x 8 cavity (two 128-cell x tiles, two y tiles, both ragged),
    FP32 one-pass COCG at the benchmark's tolerance 1e-4 and at 1e-6: the
    reduced model matches the full transfer function at every expansion point
    and its conjugate to 1e-4 (the projection error is quadratic in the solve
    error)."""
    require_gpu()
    import paper_1406_7042_amd as P
    wl, oop, dt, B, Lp, zs, H = wide_box
    gop = P.Operator.from_workload(wl)
    log(f"fused fp32 2 x tiles tol={tol}")
    g = P.mor_reduce(gop, wl.sources, wl.probes, 20, dt_ref=dt, fmax=wl.f0 + wl.bw,
                     precision="f32", tol=tol, defl_tol=1e-6, max_iter=20000)
    info = g.info()
    assert info["relres_max"] <= tol
    m = g.matrices()
    orom = mor.Reduced(V1=np.zeros((1, info["q1"])), V2=np.zeros((1, info["q2"])), **m)
    errs = [rel_l2(mor.rom_transfer(orom, dt, z), h) for z, h in zip(zs, H)]
    log(f"  q1 {info['q1']} q2 {info['q2']} iters {info['solve_iters']}  "
        f"transfer errors {' '.join(f'{e:.1e}' for e in errs)}")
    assert max(errs) <= 1e-4
    gop.close()


# ------------------------------------------------------ 20 x 20 cavity at q = 40


def test_config0_q40_moments_match_full_model_fp64():
    """The 2-D 20 x 20 cavity at its order q = 40 (FP64 COCG to 1e-13): the
    reduced transfer function and its first derivative equal the full
    model's at every expansion point and conjugate to 1e-10 (moment matching,
    Sec. II-C), though the basis itself is determined only to ~1e-5 there."""
    require_gpu()
    import scipy.sparse.linalg as spla
    import paper_1406_7042_amd as P
    wl = W.cavity2d()
    oop = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(oop.grid)
    B = yee.port_matrix(oop, wl.sources, True)
    Lp = yee.port_matrix(oop, wl.probes, False)
    fmax = wl.f0 + wl.bw
    gop = P.Operator.from_workload(wl)
    log("config0 q=40 moments")
    g = P.mor_reduce(gop, wl.sources, wl.probes, 40, dt_ref=dt, fmax=fmax, precision="f64",
                     tol=1e-13)
    m = g.matrices()
    orom = mor.Reduced(V1=np.zeros((1, 40)), V2=np.zeros((1, 40)), **m)
    Pf, Qf = mor.system_pq(oop, dt)
    Rr, Fr = mor.reduced_R_F(orom, dt)
    Pr, Qr = Rr + Fr, Rr - Fr
    Br = np.vstack([orom.B1, orom.B2]).astype(complex)
    Lr = np.vstack([orom.L1, orom.L2])
    pts = mor.expansion_points(1.1, 2, fmax, dt)
    worst = [0.0, 0.0]
    for z in list(pts) + list(np.conj(pts[1:])):
        lu = spla.splu((z * Pf - Qf).tocsc().astype(complex))
        X = lu.solve(B.astype(complex))
        Hf, dHf = Lp.T @ X, -(Lp.T @ lu.solve(Pf @ X))
        Ar = z * Pr - Qr
        Xr = np.linalg.solve(Ar, Br)
        Hr, dHr = Lr.T @ Xr, -(Lr.T @ np.linalg.solve(Ar, Pr @ Xr))
        e0, e1 = rel_l2(Hr, Hf), rel_l2(dHr, dHf)
        worst = [max(worst[0], e0), max(worst[1], e1)]
        assert e0 <= 1e-10 and e1 <= 1e-10, (z, e0, e1)
    log(f"  H {worst[0]:.2e}  dH/dz {worst[1]:.2e}")
