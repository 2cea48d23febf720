"""fdtd_step (HIP) against the FP64 oracle's leapfrog, eq. (MNAform).

Tolerances: FP64 fields and probes 1e-10 relative L2; FP32 probes 1e-4
relative L2 (the precision targets of the hot path).
"""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import yee
from tests.gpuutil import log, oracle_to_state, rel_l2, require_gpu, state_to_oracle

pytestmark = pytest.mark.gpu


def _run_pair(wl, nsteps, s=0.99, dtype="f64", x0_seed=None, signs=None, leapfrog="auto"):
    import torch
    import paper_1406_7042_amd as P
    oop = yee.assemble(wl)
    dt = s * yee.cfl_dt_max(oop.grid)
    B = yee.port_matrix(oop, wl.sources, True)
    L = yee.port_matrix(oop, wl.probes, False)
    u = W.drive(wl, dt, nsteps, signs)
    x0 = None if x0_seed is None else W.random_vectors(x0_seed, oop.N)
    y_ref, x_ref = yee.leapfrog(oop, dt, B, u, L, x0=x0)
    gop = P.Operator.from_workload(wl)
    gop.set_leapfrog(leapfrog)
    assert (gop.n_e, gop.n_h) == (oop.Ne, oop.Nh)
    assert gop.dt_max == pytest.approx(yee.cfl_dt_max(oop.grid), rel=1e-14)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    f = (gop.new_fields(tdt) if x0 is None else oracle_to_state(gop, oop, x0, tdt))
    ud = torch.tensor(u, dtype=tdt, device="cuda")
    yd = torch.zeros((nsteps, len(wl.probes)), dtype=tdt, device="cuda")
    P.fdtd_step(gop, dt, nsteps, f, wl.sources, ud, wl.probes, yd)
    torch.cuda.synchronize()
    return y_ref, x_ref, yd.cpu().numpy(), state_to_oracle(gop, oop, f), f, gop, oop


def test_config0_cavity2d_fp64():
    """2-D Ez-pol PEC cavity 20x20, 1 mm, vacuum, 2000 steps at 0.99 CFL."""
    require_gpu()
    log("fdtd config0 fp64")
    wl = W.cavity2d()
    y_ref, x_ref, y, x, *_ = _run_pair(wl, 2000)
    assert rel_l2(y, y_ref) <= 1e-10
    assert rel_l2(x, x_ref) <= 1e-10


def test_config0_cavity2d_fp32():
    require_gpu()
    log("fdtd config0 fp32")
    wl = W.cavity2d()
    y_ref, _, y, *_ = _run_pair(wl, 2000, dtype="f32")
    assert rel_l2(y, y_ref) <= 1e-4


def test_2d_lossy_materials_pec_ragged():
    """Several 256-thread tiles and a ragged tail, lossy blocks, PEC strip."""
    require_gpu()
    log("fdtd 2d lossy pec")
    wl = W.cavity2d(nx=37, ny=29, d=1e-3, seed=5, eps_block=4, eps_range=(1, 4),
                    sigma_range=(0, 5.0), nsrc=2, nprobe=3)
    wl.pec = [(2, 30, j, 0) for j in range(5, 20)]
    wl.sources = [s for s in wl.sources]
    y_ref, x_ref, y, x, *_ = _run_pair(wl, 300, x0_seed=7)
    assert rel_l2(y, y_ref) <= 1e-10
    assert rel_l2(x, x_ref) <= 1e-10


def test_3d_lossy_blocks_fp64_and_fp32():
    require_gpu()
    log("fdtd 3d lossy")
    wl = W.cavity3d(n=13, ny=11, nz=9, d=1e-3, seed=1, block=4, nports=3, margin=2)
    y_ref, x_ref, y, x, *_ = _run_pair(wl, 200, x0_seed=3, signs=W.port_signs(1, 3))
    assert rel_l2(y, y_ref) <= 1e-10
    assert rel_l2(x, x_ref) <= 1e-10
    y_ref, x_ref, y, x, *_ = _run_pair(wl, 200, dtype="f32", signs=W.port_signs(1, 3))
    assert rel_l2(y, y_ref) <= 1e-4


@pytest.mark.parametrize("nsteps,mu", [(61, False), (60, True)])
def test_3d_larger_box_many_ports(nsteps, mu):
    """A 70 x 40 x 40 cavity (many launch blocks, none aligned with the box),
    six ports spread over it, random initial fields: every field value and
    probe sample matches the oracle to 1e-10 (FP64), with uniform or per-cell
    magnetic materials; positions that are not unknowns stay zero."""
    require_gpu()
    import torch
    log(f"fdtd 3d larger box nsteps={nsteps} mu={mu}")
    wl = W.cavity3d(n=70, ny=40, nz=40, d=1e-3, seed=7, block=5, nports=6, margin=3)
    if mu:
        rng = np.random.default_rng(8)
        wl.mu_r = rng.uniform(1, 2, size=wl.eps_r.shape)
        wl.sigma_m = rng.uniform(0, 20.0, size=wl.eps_r.shape)
    y_ref, x_ref, y, x, f, gop, oop = _run_pair(wl, nsteps, x0_seed=5, signs=W.port_signs(2, 6))
    assert rel_l2(y, y_ref) <= 1e-10
    assert rel_l2(x, x_ref) <= 1e-10
    pattern = oracle_to_state(gop, oop, np.ones(oop.N), torch.float64)
    assert torch.count_nonzero(f[pattern == 0]).item() == 0
    y_ref, x_ref, y, x, *_ = _run_pair(wl, nsteps, dtype="f32", signs=W.port_signs(2, 6))
    assert rel_l2(y, y_ref) <= 1e-4


def test_3d_graded_mesh_pec_strip_line_ports():
    """Graded z spacing (fine substrate under coarse air), PEC strip, line ports."""
    require_gpu()
    log("fdtd 3d graded")
    wl = W.board3d(nx=14, ny=10, nz_fine=3, nz_coarse=4, d=1e-3, dz_fine=0.25e-3,
                   strip=(3, 11, 4, 6))
    rng = np.random.default_rng(0)
    wl.sigma_e = rng.uniform(0, 0.5, size=wl.eps_r.shape)
    y_ref, x_ref, y, x, *_ = _run_pair(wl, 150, s=0.99, x0_seed=2)
    assert rel_l2(y, y_ref) <= 1e-10
    assert rel_l2(x, x_ref) <= 1e-10


def test_3d_nonuniform_mu_sigma_m():
    """Magnetic losses and mu_r != 1 (the D_mu, D_sigma_m path of eq. (matrix))."""
    require_gpu()
    wl = W.cavity3d(n=8, ny=7, nz=6, d=1e-3, seed=2, block=3, nports=1, margin=2)
    rng = np.random.default_rng(3)
    wl.mu_r = rng.uniform(1, 2, size=wl.eps_r.shape)
    wl.sigma_m = rng.uniform(0, 50.0, size=wl.eps_r.shape)
    y_ref, x_ref, y, x, *_ = _run_pair(wl, 80, x0_seed=4)
    assert rel_l2(y, y_ref) <= 1e-10
    assert rel_l2(x, x_ref) <= 1e-10


@pytest.mark.parametrize("n,leapfrog", [(128, "split"), (128, "fused"), (256, "fused")])
def test_full_size_config1_light_cone_sample(n, leapfrog):
    """Full 128^3 lossy cavity (the benchmark launch configuration, FP32 and
    FP64, both leapfrog paths) and a 256^3 one (one-pass path): within the light cone of a source the
    leapfrog only sees the cells it has reached, so the oracle on a 36^3
    sub-box with the same materials reproduces the full-size run exactly for
    12 steps."""
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    log(f"fdtd {n}^3 light cone {leapfrog}")
    full = W.cavity3d(n=n, d=1e-3, seed=1, block=8, nports=4)
    src = [[(2, 64, 61, 67, 1.0)]]
    prb = [[(2, 64, 61, 67, 1.0)], [(2, 66, 63, 65, 1.0)], [(0, 60, 62, 70, 1.0)]]
    lo = np.array([46, 43, 49])  # sub-box origin (cells)
    n = 36
    sub = copy.deepcopy(full)
    sub.nx = sub.ny = sub.nz = n
    sub.dx, sub.dy, sub.dz = full.dx[:n], full.dy[:n], full.dz[:n]
    sub.eps_r = full.eps_r[lo[2]:lo[2] + n, lo[1]:lo[1] + n, lo[0]:lo[0] + n].copy()
    sub.sigma_e = full.sigma_e[lo[2]:lo[2] + n, lo[1]:lo[1] + n, lo[0]:lo[0] + n].copy()
    shift = lambda port: [(c, i - lo[0], j - lo[1], k - lo[2], w) for (c, i, j, k, w) in port]
    sub.sources = [shift(p) for p in src]
    sub.probes = [shift(p) for p in prb]
    full.sources, full.probes = src, prb
    nsteps = 12
    oop = yee.assemble(sub)
    dt = 0.99 * yee.cfl_dt_max(oop.grid)
    u = W.drive(full, dt, nsteps) * 0 + 1.0  # constant drive: strongest light-cone test
    B = yee.port_matrix(oop, sub.sources, True)
    L = yee.port_matrix(oop, sub.probes, False)
    y_ref, _ = yee.leapfrog(oop, dt, B, u, L)
    gop = P.Operator.from_workload(full)
    gop.set_leapfrog(leapfrog)
    for tdt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        f = gop.new_fields(tdt)
        ud = torch.tensor(u, dtype=tdt, device="cuda")
        yd = torch.zeros((nsteps, 3), dtype=tdt, device="cuda")
        P.fdtd_step(gop, dt, nsteps, f, full.sources, ud, full.probes, yd)
        torch.cuda.synchronize()
        assert rel_l2(yd.cpu().numpy(), y_ref) <= tol, tdt


def test_error_paths():
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    wl = W.cavity2d(nx=10, ny=10)
    gop = P.Operator.from_workload(wl)
    f = gop.new_fields(torch.float64)
    with pytest.raises(P.YeeromError) as e:
        P.fdtd_step(gop, 1.01 * gop.dt_max, 5, f)
    assert e.value.status == P.yeerom.YR_EUNSTABLE
    with pytest.raises(P.YeeromError) as e:  # tangential on the wall: not an unknown
        P.fdtd_step(gop, 0.5 * gop.dt_max, 1, f, [[(2, 0, 3, 0, 1.0)]],
                    torch.zeros((1, 1), dtype=torch.float64, device="cuda"))
    assert e.value.status == P.yeerom.YR_EINVAL
    P.fdtd_step(gop, 0.5 * gop.dt_max, 0, f)  # empty run is fine
    assert float(f.abs().sum()) == 0.0


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_waveguide_matched_absorber_line_ports(dtype, tol):
    """2-D guide (160 x 16 cells, eps_r 2.5) ended on 5-cell 4th-order matched
    absorbers (graded sigma_e and sigma_m), driven by a mode-shaped line source
    (15 weighted Ez entries) and read by two line probes: the D_sigma_m path
    and multi-entry ports against the oracle, 2000 steps at 0.99 CFL."""
    require_gpu()
    log(f"fdtd waveguide matched absorber {dtype}")
    wl = W.waveguide2d()
    y_ref, x_ref, y, x, *_ = _run_pair(wl, 2000, dtype=dtype)
    assert rel_l2(y, y_ref) <= tol
    if dtype == "f64":
        assert rel_l2(x, x_ref) <= tol


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-4)])
@pytest.mark.parametrize("leapfrog", ["split", "fused"])
def test_plane_source_and_plane_probe(dtype, tol, leapfrog):
    """Sec. V-C drives with a plane of uniform sources and reads probes on the
    far side of a screen: a 40 x 40 plane of Ez sources (1600 entries, one
    port) plus a point port, probed by a 40 x 40 plane (one port of 1600
    entries) and a line of point probes along the axis, in a lossy 3-D box;
    600 steps against the oracle."""
    require_gpu()
    import dataclasses
    log(f"fdtd plane source / plane probe {dtype}")
    wl = W.cavity3d(n=48, ny=46, nz=30, d=1e-3, seed=21, block=6, eps_range=(1, 3),
                    sigma_range=(0, 0.02), nports=1, margin=4, f0=30e9, bw=30e9)
    plane_src = [(2, i, j, 8, 1.0) for j in range(3, 43) for i in range(4, 44)]
    plane_prb = [(2, i, j, 20, 1.0 / 1600) for j in range(3, 43) for i in range(4, 44)]
    axis = [[(2, 24, 23, k, 1.0)] for k in range(12, 26, 2)]
    wl = dataclasses.replace(wl, sources=[plane_src, [(0, 30, 9, 14, 1.0)]],
                             probes=[plane_prb] + axis)
    y_ref, x_ref, y, x, *_ = _run_pair(wl, 600, dtype=dtype, signs=np.array([1.0, -1.0]),
                                       leapfrog=leapfrog)
    log(f"  probes rel err {rel_l2(y, y_ref):.2e}")
    assert rel_l2(y, y_ref) <= tol
    if dtype == "f64":
        assert rel_l2(x, x_ref) <= tol


def _one_pass_cases():
    rng = np.random.default_rng(8)
    lossy = W.cavity3d(n=13, ny=11, nz=9, d=1e-3, seed=1, block=4, nports=3, margin=2)
    big = W.cavity3d(n=70, ny=40, nz=40, d=1e-3, seed=7, block=5, nports=6, margin=3)
    mu = copy.deepcopy(big)
    mu.mu_r = rng.uniform(1, 2, size=mu.eps_r.shape)
    mu.sigma_m = rng.uniform(0, 20.0, size=mu.eps_r.shape)
    board = W.board3d(nx=70, ny=36, nz_fine=3, nz_coarse=12, d=1e-3, dz_fine=0.25e-3,
                      strip=(5, 60, 15, 19))
    board.sigma_e = rng.uniform(0, 0.5, size=board.eps_r.shape)
    return {"lossy": (lossy, 3), "big": (big, 6), "mu": (mu, 6), "board": (board, 2)}


@pytest.mark.parametrize("case", ["lossy", "big", "mu", "board"])
@pytest.mark.parametrize("nsteps", [41, 60])
def test_3d_one_pass_leapfrog_matches_oracle(case, nsteps):
    """The one-pass leapfrog (E and H of a step in one sweep, fields
    alternating between two buffers) on boxes of several tiles in x and y
    (FP32: 128 x 8 at nx = 70, 64 x 16 at nx = 13; FP64: 64 x 8) and several
    z chunks, with uniform and per-cell magnetic materials,
    a graded mesh with a PEC strip and line ports, random initial fields, an
    odd and an even step count (the final fields land in either buffer):
    FP64 1e-10 (fields and probes), FP32 1e-4 (probes); positions that are not
    unknowns stay zero."""
    require_gpu()
    import torch
    log(f"fdtd one-pass {case} nsteps={nsteps}")
    wl, nports = _one_pass_cases()[case]
    signs = W.port_signs(2, nports)
    y_ref, x_ref, y, x, f, gop, oop = _run_pair(wl, nsteps, x0_seed=5, signs=signs,
                                                leapfrog="fused")
    assert rel_l2(y, y_ref) <= 1e-10
    assert rel_l2(x, x_ref) <= 1e-10
    pattern = oracle_to_state(gop, oop, np.ones(oop.N), torch.float64)
    assert torch.count_nonzero(f[pattern == 0]).item() == 0
    y_ref, _, y, *_ = _run_pair(wl, nsteps, dtype="f32", signs=signs, leapfrog="fused")
    assert rel_l2(y, y_ref) <= 1e-4


@pytest.mark.parametrize("leapfrog", ["split", "fused"])
@pytest.mark.parametrize("shape", [(48, 46, 30), (120, 30, 20)])
def test_3d_per_cell_materials_32bit_material_numbers(leapfrog, shape):
    """Per-cell random eps_r and sigma_e on a 48 x 46 x 30 and a 120 x 30 x
    20 box: the electric samples take ~2e5 distinct (D_eps, D_sigma_e) pairs,
    past the 16-bit material numbers, so the leapfrog reads 32-bit numbers and
    the (ca, cb) table; FP64 1e-10 (fields and probes), FP32 1e-4, both paths
    (the one-pass FP32 step on 64 x 16 tiles for the first box, 128 x 8 for
    the second)."""
    require_gpu()
    log(f"fdtd per-cell materials {leapfrog} {shape}")
    nx, ny, nz = shape
    wl = W.cavity3d(n=nx, ny=ny, nz=nz, d=1e-3, seed=23, block=6, nports=3, margin=4)
    rng = np.random.default_rng(24)
    wl.eps_r = rng.uniform(1, 4, size=wl.eps_r.shape)
    wl.sigma_e = rng.uniform(0, 0.05, size=wl.eps_r.shape)
    signs = W.port_signs(3, 3)
    y_ref, x_ref, y, x, *_ = _run_pair(wl, 120, x0_seed=9, signs=signs, leapfrog=leapfrog)
    assert rel_l2(y, y_ref) <= 1e-10
    assert rel_l2(x, x_ref) <= 1e-10
    y_ref, _, y, *_ = _run_pair(wl, 120, dtype="f32", signs=signs, leapfrog=leapfrog)
    assert rel_l2(y, y_ref) <= 1e-4
