"""rom_step_noalloc (the entry point for callers that cannot allocate device
memory) against rom_step on the same prepared models: both launch the same
kernel with the same workgroup size, so the outputs and final states must be
identical.  Two calls in a row, the second with fewer models, fewer steps and
given initial states (the shared descriptor table keeps the first call's
contents)."""
import numpy as np
import pytest

import workloads as W
from tests.gpuutil import log, require_gpu

pytestmark = pytest.mark.gpu


def _models(P, dt, dtype):
    """Reduced models of three 2-D cavities (1 mm cells, so one dt fits all),
    reduced on the GPU and prepared for dt beyond the CFL limit."""
    out = []
    for k, (n, q) in enumerate(((20, 20), (24, 30), (30, 40))):
        wl = W.cavity2d(nx=n, ny=n, seed=50 + k, eps_block=4, eps_range=(1, 3),
                        sigma_range=(0.0, 0.2))
        gop = P.Operator.from_workload(wl)
        rom = P.mor_reduce(gop, wl.sources, wl.probes, q, dt_ref=dt / 5.0,
                           fmax=wl.f0 + wl.bw, precision="f64", tol=1e-12)
        P.rom_perturb(rom, dt, dtype=dtype)
        out.append((wl, rom))
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rom_step_noalloc_equals_rom_step(dtype):
    require_gpu()
    import torch
    import paper_1406_7042_amd as P
    from oracle import yee
    wl0 = W.cavity2d()
    dt = 4.95 * yee.cfl_dt_max(yee.assemble(wl0).grid)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    models = _models(P, dt, dtype)
    roms = [r for _, r in models]

    def inputs(ms, nsteps):
        return [torch.tensor(W.drive(wl, dt, nsteps), dtype=tdt, device="cuda") for wl, _ in ms]

    # call 1: all models, 2048 steps (rom_step picks its workgroup size by
    # timing first; the allocation-free call reuses that choice)
    n1 = 2048
    us = inputs(models, n1)
    log(f"rom_step vs rom_step_noalloc {dtype}: 3 models, {n1} steps")
    y_ref = P.rom_step(roms, dt, n1, us, dtype=dtype)
    ys = [torch.full((n1, 1), float("nan"), dtype=tdt, device="cuda") for _ in roms]
    P.rom_step_noalloc(roms, dt, n1, us, ys, dtype=dtype)
    torch.cuda.synchronize()
    for a, b in zip(ys, y_ref):
        assert torch.equal(a, b)
        assert float(b.abs().max()) > 0

    # call 2: two models, 700 steps, from given states; states come back
    n2 = 700
    sub = models[1:]
    us2 = inputs(sub, n2)
    st0 = [torch.tensor(np.random.default_rng(7 + m).standard_normal(r.info()["q1"] + r.info()["q2"]),
                        dtype=tdt, device="cuda") * 1e-3 for m, (_, r) in enumerate(sub)]
    st_ref = [s.clone() for s in st0]
    st_new = [s.clone() for s in st0]
    log(f"second call: 2 models, {n2} steps, initial states")
    y2_ref = P.rom_step([r for _, r in sub], dt, n2, us2, dtype=dtype, states=st_ref)
    y2 = [torch.full((n2, 1), float("nan"), dtype=tdt, device="cuda") for _ in sub]
    P.rom_step_noalloc([r for _, r in sub], dt, n2, us2, y2, dtype=dtype, states=st_new)
    torch.cuda.synchronize()
    for a, b in zip(y2, y2_ref):
        assert torch.equal(a, b)
    for a, b, s in zip(st_new, st_ref, st0):
        assert torch.equal(a, b)
        assert not torch.equal(a, s)


def test_rom_step_noalloc_rejects_too_many_models():
    require_gpu()
    import paper_1406_7042_amd as P
    import ctypes as C
    n = 4097
    arr = (C.c_void_p * n)()
    st = P.lib().rom_step_noalloc(arr, n, 1e-12, 10, P.YR_F32, None, None, None, None)
    assert st == -1
    assert b"4096" in P.lib().yr_last_error()
