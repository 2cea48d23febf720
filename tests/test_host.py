"""Host-side logic: seeded input generators and argument marshalling."""
import numpy as np
import pytest

import workloads as W


def test_pulse_is_odd_about_t0_and_has_no_dc():
    f0, bw = 10e9, 10e9
    tau = 2 / (np.pi * bw)
    t0 = 4 * tau
    m = 300
    dt = t0 / m  # t0 on the sample grid: samples (n+1/2) dt mirror onto each other
    u = W.pulse(f0, bw, dt, 2 * m)
    # odd symmetry about t0: u[n] = -u[2m-1-n]
    a = u
    assert np.allclose(a[:m], -a[::-1][:m], atol=1e-12)
    assert abs(u.sum()) < 1e-6 * np.abs(u).sum()


def test_cavity3d_blocks_and_ports():
    wl = W.cavity3d(n=32, block=8, nports=4, seed=1)
    assert wl.eps_r.shape == (32, 32, 32)
    blk = wl.eps_r[:8, :8, :8]
    assert np.all(blk == blk[0, 0, 0])
    assert 1 <= wl.eps_r.min() and wl.eps_r.max() <= 4
    assert 0 <= wl.sigma_e.min() and wl.sigma_e.max() <= 0.01
    locs = [p[0][1:4] for p in wl.sources]
    assert len(set(locs)) == 4
    for (i, j, k) in locs:
        assert 8 <= i <= 24 and 8 <= j <= 24 and 8 <= k < 24
    # same seed, same structure
    wl2 = W.cavity3d(n=32, block=8, nports=4, seed=1)
    assert np.array_equal(wl.eps_r, wl2.eps_r) and wl.sources == wl2.sources


def test_design2d_region_and_strips():
    wl = W.design2d(n=64, region=32, strip_period=16)
    c0 = 16
    assert np.all(wl.eps_r[:c0] == 1) and np.all(wl.sigma_e[:, :c0] == 0)
    cols = sorted(set(p[1] for p in wl.pec))
    assert cols == [16, 17, 32, 33]


def test_board3d_graded_spacing_and_line_ports():
    wl = W.board3d(nx=20, ny=12, nz_fine=3, nz_coarse=5, dz_fine=0.2e-3, strip=(4, 16, 5, 7))
    assert np.allclose(wl.dz[:3], 0.2e-3) and np.allclose(wl.dz[3:], 1e-3)
    assert np.all(wl.eps_r[:3] == 3.38) and np.all(wl.eps_r[3:] == 1)
    for port in wl.sources:
        assert [e[3] for e in port] == [0, 1, 2]
        assert all(e[4] == pytest.approx(0.2e-3) for e in port)


def test_rom_batch_orders():
    q = W.rom_batch_orders(7, 256)
    assert q.min() >= 50 and q.max() <= 400 and np.all(q % 5 == 0)


def test_ports_csr_packing():
    from paper_1406_7042_amd.yeerom import Ports
    p = Ports([[(2, 1, 2, 3, 0.5)], [(0, 4, 5, 6, 1.0), (1, 7, 8, 9, 2.0)]])
    assert p.n == 2
    assert list(p._off) == [0, 1, 3]
    assert list(p._smp) == [2, 1, 2, 3, 0, 4, 5, 6, 1, 7, 8, 9]
    assert list(p._w) == [0.5, 1.0, 2.0]
