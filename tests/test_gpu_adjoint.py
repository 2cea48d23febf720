"""fdtd_adjoint (HIP reverse-time adjoint) against the oracle's discrete
adjoint and against central finite differences of the GPU FP64 forward run.

Objective J = dt * sum_n sum_p y_p^n^2 (probe energy), dJ/dy = 2 dt y.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import yee
from tests.gpuutil import log, rel_l2, require_gpu

pytestmark = pytest.mark.gpu


def _gpu_grads(wl, dt, nsteps, dtype, ckpt, signs=None):
    import torch
    import paper_1406_7042_amd as P
    gop = P.Operator.from_workload(wl)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u = torch.tensor(W.drive(wl, dt, nsteps, signs), dtype=tdt, device="cuda")
    f = gop.new_fields(tdt)
    y = torch.zeros((nsteps, len(wl.probes)), dtype=tdt, device="cuda")
    P.fdtd_step(gop, dt, nsteps, f, wl.sources, u, wl.probes, y)
    dJdy = (2.0 * dt * y).contiguous()
    ge, gs = P.yeerom.fdtd_adjoint(gop, dt, nsteps, wl.sources, u, wl.probes, dJdy, ckpt)
    torch.cuda.synchronize()
    J = float(dt * (y.double() ** 2).sum())
    return J, ge.cpu().numpy(), gs.cpu().numpy()


def _oracle_grads(wl, dt, nsteps, signs=None):
    op = yee.assemble(wl)
    B = yee.port_matrix(op, wl.sources, True)
    L = yee.port_matrix(op, wl.probes, False)
    u = W.drive(wl, dt, nsteps, signs)
    J, gDe, gDse = oadj.full_adjoint(op, dt, B, u, L)
    ge, gs = oadj.cell_gradients(op, wl, gDe, gDse)
    return J, ge, gs


@pytest.mark.parametrize("case", ["2d", "3d", "graded"])
def test_adjoint_matches_oracle_fp64(case):
    require_gpu()
    log(f"adjoint {case}")
    if case == "2d":
        wl = W.cavity2d(nx=19, ny=15, seed=3, eps_block=3, eps_range=(1, 4), sigma_range=(0, 3.0),
                        nsrc=1, nprobe=2)
        wl.pec = [(2, 9, j, 0) for j in range(2, 6)]
    elif case == "3d":
        wl = W.cavity3d(n=9, ny=8, nz=7, d=1e-3, seed=2, block=3, nports=2, margin=2,
                        sigma_range=(0, 2.0))
    else:
        wl = W.board3d(nx=10, ny=8, nz_fine=2, nz_coarse=3, d=1e-3, dz_fine=0.3e-3,
                       strip=(2, 8, 3, 5))
        wl.sigma_e = np.random.default_rng(4).uniform(0, 1.0, size=wl.eps_r.shape)
    oop = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(oop.grid)
    nsteps = 150
    Jo, geo, gso = _oracle_grads(wl, dt, nsteps)
    Jg, ge, gs = _gpu_grads(wl, dt, nsteps, "f64", ckpt=16)
    assert Jg == pytest.approx(Jo, rel=1e-10)
    assert rel_l2(ge, geo) <= 1e-10
    assert rel_l2(gs, gso) <= 1e-10
    # checkpoint interval does not change the result
    _, ge2, gs2 = _gpu_grads(wl, dt, nsteps, "f64", ckpt=nsteps)
    assert rel_l2(ge2, ge) <= 1e-13 and rel_l2(gs2, gs) <= 1e-13


def test_autograd_function_backward():
    require_gpu()
    import torch
    from paper_1406_7042_amd.autograd import FDTDFunction, geometry_of
    wl = W.cavity2d(nx=16, ny=14, seed=6, eps_block=2, eps_range=(1, 4), sigma_range=(0, 2.0))
    oop = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(oop.grid)
    nsteps = 120
    eps = torch.tensor(wl.eps_r, dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(wl.sigma_e, dtype=torch.float64, requires_grad=True)
    u = torch.tensor(W.drive(wl, dt, nsteps), dtype=torch.float64, device="cuda")
    y = FDTDFunction.apply(eps, sig, geometry_of(wl), dt, nsteps, u, 32)
    J = dt * (y ** 2).sum()
    J.backward()
    Jo, geo, gso = _oracle_grads(wl, dt, nsteps)
    assert float(J.detach()) == pytest.approx(Jo, rel=1e-10)
    assert rel_l2(eps.grad.numpy(), geo) <= 1e-10
    assert rel_l2(sig.grad.numpy(), gso) <= 1e-10


def test_config3_design_region_gradients_vs_central_differences():
    """2-D 512x512 PEC box, 128x128 design region (per-cell eps_r ~ U[1,4],
    sigma_e ~ U[0,0.01] S/m), PEC strips 2 cells wide every 16; 3000 FP32
    steps, checkpoint every 64.  The FP64 adjoint matches FP64 central
    differences (h = 1e-4) on 16 seeded cells per parameter; the FP32
    adjoint matches the FP64 adjoint over the whole design region."""
    require_gpu()
    import copy
    import torch
    import paper_1406_7042_amd as P
    log("adjoint config3")
    wl = W.design2d()
    n = wl.nx
    dt = 0.99 * 0.5e-3 / (yee.C0 * np.sqrt(2.0))
    nsteps = 3000
    J64, ge64, gs64 = _gpu_grads(wl, dt, nsteps, "f64", ckpt=64)
    J32, ge32, gs32 = _gpu_grads(wl, dt, nsteps, "f32", ckpt=64)
    c0 = (n - 128) // 2
    reg = (slice(c0, c0 + 128), slice(c0, c0 + 128))
    e32 = rel_l2(ge32[reg], ge64[reg])
    s32 = rel_l2(gs32[reg], gs64[reg])
    log(f"  J64 {J64:.6e} J32 rel {abs(J32 - J64) / J64:.2e}  fp32 grad rel err eps {e32:.2e} sig {s32:.2e}")
    assert e32 <= 2e-3 and s32 <= 2e-3

    def J_of(eps=None, sig=None):
        w2 = copy.copy(wl)
        if eps is not None:
            w2.eps_r = eps
        if sig is not None:
            w2.sigma_e = sig
        gop = P.Operator.from_workload(w2)
        u = torch.tensor(W.drive(w2, dt, nsteps), dtype=torch.float64, device="cuda")
        f = gop.new_fields(torch.float64)
        y = torch.zeros((nsteps, 1), dtype=torch.float64, device="cuda")
        P.fdtd_step(gop, dt, nsteps, f, w2.sources, u, w2.probes, y)
        return float(dt * (y ** 2).sum())

    rng = np.random.default_rng(33)
    cells = [(c0 + int(rng.integers(0, 128)), c0 + int(rng.integers(0, 128))) for _ in range(16)]
    h = 1e-4
    worst = 0.0
    for (j, i) in cells:
        for which, g in (("eps", ge64), ("sig", gs64)):
            if which == "sig" and wl.sigma_e[j, i] < h:
                continue  # keep the conductivity non-negative
            a = (wl.eps_r if which == "eps" else wl.sigma_e).copy()
            b = a.copy()
            a[j, i] += h
            b[j, i] -= h
            fd = ((J_of(eps=a) - J_of(eps=b)) if which == "eps" else
                  (J_of(sig=a) - J_of(sig=b))) / (2 * h)
            scale = np.abs(g[reg]).max()
            err = abs(g[j, i] - fd) / scale
            worst = max(worst, err)
            assert err <= 1e-6, (which, j, i, g[j, i], fd)
    log(f"  worst FD mismatch / max|grad| {worst:.2e}")
