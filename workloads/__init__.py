"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module only *generates inputs*: Yee grids (cell spacings), per-cell
material tables, PEC object masks, port/probe locations and source
waveforms.  It holds none of the method's arithmetic (no curl operators, no
time stepping, no reduction), so that the CPU oracle and the HIP library stay
independent of each other and meet only here.

Conventions shared by both sides
--------------------------------
* A grid has ``nx x ny (x nz)`` cells; node indices run ``0..n`` per axis.
* Field components are coded ``0,1,2 = Ex,Ey,Ez`` and ``3,4,5 = Hx,Hy,Hz``.
  A component sample ``(c, i, j, k)`` sits at the Yee position
  Ex (i+1/2, j, k), Ey (i, j+1/2, k), Ez (i, j, k+1/2),
  Hx (i, j+1/2, k+1/2), Hy (i+1/2, j, k+1/2), Hz (i+1/2, j+1/2, k).
  In 2-D (Ez-polarisation: Ez, Hx, Hy only) ``k`` is always 0 and Ez sits at
  node (i, j), Hx at (i, j+1/2), Hy at (i+1/2, j).
* Per-cell arrays are indexed ``[k, j, i]`` (2-D: ``[j, i]``).
* A port (source or probe) is a list of ``(c, i, j, k, weight)`` entries on
  electric-field samples.
* The source waveform array ``u[n, p]`` holds the value that drives the
  update producing ``E^{n+1}``; it is the pulse sampled at ``(n + 1/2) dt``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

C0 = 299_792_458.0  # m/s, exact (SI)

Port = List[Tuple[int, int, int, int, float]]


@dataclass
class Workload:
    """One synthetic structure: grid, materials, PEC objects, ports, probes."""

    name: str
    dim: int
    nx: int
    ny: int
    nz: int
    dx: np.ndarray  # (nx,) cell spacings [m]
    dy: np.ndarray  # (ny,)
    dz: np.ndarray  # (nz,) ; 2-D: a single 1.0 (per unit length)
    eps_r: np.ndarray  # per cell, [k, j, i] (2-D: [j, i])
    sigma_e: np.ndarray  # per cell [S/m]
    mu_r: Optional[np.ndarray] = None  # None -> 1 everywhere
    sigma_m: Optional[np.ndarray] = None  # None -> 0 everywhere
    pec: List[Tuple[int, int, int, int]] = field(default_factory=list)  # E samples forced to 0
    sources: List[Port] = field(default_factory=list)
    probes: List[Port] = field(default_factory=list)
    f0: float = 0.0  # pulse centre frequency [Hz]
    bw: float = 0.0  # pulse bandwidth [Hz]

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * (self.nz if self.dim == 3 else 1)


# ----------------------------------------------------------------------------
# waveforms


def pulse(f0: float, bw: float, dt: float, nsteps: int) -> np.ndarray:
    """Sine-modulated Gaussian ``exp(-((t-t0)/tau)^2) sin(2 pi f0 (t-t0))``.

    ``tau = 2/(pi bw)`` (spectrum down by e at f0 +- bw/2), ``t0 = 4 tau``.
    Sampled at ``t = (n + 1/2) dt`` for n = 0..nsteps-1 (the electric source
    sits at half steps in the Yee scheme).  Odd about t0, so it carries no DC.
    """
    tau = 2.0 / (math.pi * bw)
    t0 = 4.0 * tau
    t = (np.arange(nsteps, dtype=np.float64) + 0.5) * dt - t0
    return np.exp(-((t / tau) ** 2)) * np.sin(2.0 * math.pi * f0 * t)


def drive(wl: Workload, dt: float, nsteps: int, signs: Optional[np.ndarray] = None) -> np.ndarray:
    """u[n, p] for every source port of ``wl`` (same pulse, optional signs)."""
    base = pulse(wl.f0, wl.bw, dt, nsteps)
    npt = len(wl.sources)
    s = np.ones(npt) if signs is None else np.asarray(signs, dtype=np.float64)
    return np.ascontiguousarray(base[:, None] * s[None, :])


# ----------------------------------------------------------------------------
# structures


def _interior_nodes(rng, lo, hi, count, dim):
    """Distinct random interior nodes (i, j[, k]) with lo <= idx <= hi."""
    if (hi - lo + 1) ** dim < count:
        raise ValueError("grid too small for the requested number of distinct nodes")
    seen = set()
    out = []
    while len(out) < count:
        p = tuple(int(v) for v in rng.integers(lo, hi + 1, size=dim))
        if p not in seen:
            seen.add(p)
            out.append(p)
    return out


def cavity2d(nx=20, ny=20, d=1e-3, seed=0, f0=75e9, bw=50e9, nsrc=1, nprobe=1,
             eps_block=None, eps_range=(1.0, 1.0), sigma_range=(0.0, 0.0),
             name="cavity2d") -> Workload:
    """2-D Ez-polarised PEC rectangular cavity with seeded point source/probe.

    Source and probe nodes are drawn uniformly (distinct) from interior nodes
    2..n-2.  With ``eps_block`` set, eps_r and sigma_e are constant on
    ``eps_block x eps_block`` cell blocks, drawn uniformly from the ranges.
    """
    rng = np.random.default_rng(seed)
    eps = np.ones((ny, nx))
    sig = np.zeros((ny, nx))
    if eps_block:
        by, bx = -(-ny // eps_block), -(-nx // eps_block)
        te = rng.uniform(*eps_range, size=(by, bx))
        ts = rng.uniform(*sigma_range, size=(by, bx))
        jj, ii = np.meshgrid(np.arange(ny) // eps_block, np.arange(nx) // eps_block, indexing="ij")
        eps = te[jj, ii]
        sig = ts[jj, ii]
    lo = 2 if min(nx, ny) >= 6 else 1
    nodes = _interior_nodes(rng, lo, min(nx, ny) - lo, nsrc + nprobe, 2)
    src = [[(2, i, j, 0, 1.0)] for (i, j) in nodes[:nsrc]]
    prb = [[(2, i, j, 0, 1.0)] for (i, j) in nodes[nsrc:]]
    return Workload(name=name, dim=2, nx=nx, ny=ny, nz=1,
                    dx=np.full(nx, d), dy=np.full(ny, d), dz=np.ones(1),
                    eps_r=eps, sigma_e=sig, sources=src, probes=prb, f0=f0, bw=bw)


def cavity3d(n=128, d=1e-3, seed=1, block=8, eps_range=(1.0, 4.0), sigma_range=(0.0, 0.01),
             nports=4, f0=1.5e9, bw=1.5e9, margin=8, ny=None, nz=None, name="cavity3d") -> Workload:
    """3-D lossy PEC cavity, eps_r and sigma_e piecewise constant on block^3 cells.

    ``nports`` z-directed point ports at seeded interior Ez edges at least
    ``margin`` cells from every wall; each port is also a probe.
    """
    nx = n
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    rng = np.random.default_rng(seed)
    bz, by, bx = -(-nz // block), -(-ny // block), -(-nx // block)
    te = rng.uniform(*eps_range, size=(bz, by, bx))
    ts = rng.uniform(*sigma_range, size=(bz, by, bx))
    kk = (np.arange(nz) // block)[:, None, None]
    jj = (np.arange(ny) // block)[None, :, None]
    ii = (np.arange(nx) // block)[None, None, :]
    eps = np.broadcast_to(te[kk, jj, ii], (nz, ny, nx)).copy()
    sig = np.broadcast_to(ts[kk, jj, ii], (nz, ny, nx)).copy()
    m = min(margin, (min(nx, ny, nz) - 2) // 2)
    seen = set()
    ports = []
    while len(ports) < nports:
        i = int(rng.integers(m, nx - m + 1))
        j = int(rng.integers(m, ny - m + 1))
        k = int(rng.integers(m, nz - m))
        if (i, j, k) in seen or not (1 <= i <= nx - 1 and 1 <= j <= ny - 1):
            continue
        seen.add((i, j, k))
        ports.append([(2, i, j, k, 1.0)])
    return Workload(name=name, dim=3, nx=nx, ny=ny, nz=nz,
                    dx=np.full(nx, d), dy=np.full(ny, d), dz=np.full(nz, d),
                    eps_r=eps, sigma_e=sig, sources=ports, probes=[list(p) for p in ports],
                    f0=f0, bw=bw)


MU0_WL = 1.25663706212e-6  # H/m (CODATA 2018), for absorber profiles only


def graded_absorber(ncell: int, order: int, sigma_max: float) -> np.ndarray:
    """Conductivity of the ``ncell`` absorber cells, outermost first:
    sigma_max * (depth / ncell)^order at each cell centre (depth measured
    from the inner face of the absorber)."""
    depth = (np.arange(ncell, 0, -1) - 0.5) / ncell
    return sigma_max * depth ** order


def absorber_sigma_max(ncell: int, order: int, d: float, eps_r: float, refl: float) -> float:
    """Peak conductivity for which a matched layer of ``ncell`` cells of size
    ``d`` backed by PEC reflects ``refl`` at normal incidence in the
    continuum: the attenuation in a matched medium is sigma_e * eta, so the
    round trip gives refl = exp(-2 eta sigma_max ncell d / (order + 1))."""
    eta = MU0_WL * C0 / math.sqrt(eps_r)
    return -(order + 1) * math.log(refl) / (2.0 * eta * ncell * d)


def waveguide2d(nx=160, ny=16, d=1e-3, eps_r=2.5, absorber=5, order=4, refl=math.exp(-8.0),
                matched=True, src_x=40, probe_x=(60, 120), f0=12e9, bw=8e9,
                name="waveguide2d") -> Workload:
    """2-D Ez-polarised parallel-plate guide along x (PEC plates at j = 0 and
    j = ny), filled with eps_r, both ends terminated on ``absorber`` cells of
    graded loss (order ``order``) in front of the PEC end walls: the 5-cell
    4th-order matched termination of the open structures of Sec. V-B to V-D
    (the peak loss is not given there; ``refl`` sets it by the continuum rule).

    Matched absorber: sigma_m / mu = sigma_e / eps in every absorber cell, so
    the layer's wave impedance equals the guide's.  ``matched=False`` keeps
    sigma_e and sets sigma_m = 0 (an electric-only layer, for comparison);
    ``absorber=0`` leaves plain PEC ends.  The source is a line of Ez nodes
    across the guide at i = src_x with the fundamental mode's weights
    sin(pi j / ny); each probe is the same line at one of ``probe_x``.
    """
    eps = np.full((ny, nx), float(eps_r))
    sig_e = np.zeros((ny, nx))
    sig_m = np.zeros((ny, nx))
    if absorber:
        smax = absorber_sigma_max(absorber, order, d, eps_r, refl)
        prof = graded_absorber(absorber, order, smax)
        sig_e[:, :absorber] = prof[None, :]
        sig_e[:, nx - absorber:] = prof[::-1][None, :]
        if matched:
            eps0 = 1.0 / (MU0_WL * C0 * C0)
            sig_m = sig_e * MU0_WL / (eps0 * eps)
    w = np.sin(np.pi * np.arange(1, ny) / ny)

    def line(i):
        return [(2, i, j, 0, float(w[j - 1])) for j in range(1, ny)]

    return Workload(name=name, dim=2, nx=nx, ny=ny, nz=1,
                    dx=np.full(nx, d), dy=np.full(ny, d), dz=np.ones(1),
                    eps_r=eps, sigma_e=sig_e, sigma_m=sig_m, sources=[line(src_x)],
                    probes=[line(i) for i in probe_x], f0=f0, bw=bw)


def iris_guide2d(nx=401, ny=41, d=1.25e-3, eps_r=2.5, absorber=5, order=4,
                 refl=math.exp(-8.0), n_iris=5, iris_len=10, iris_depth=8, spacing=40,
                 src_x=10, probe_x=390, f0=1.5e9, bw=3e9, name="iris_guide2d") -> Workload:
    """The 2-D waveguide filter of Sec. V-B: a parallel-plate guide of
    ny x nx cells (41 x 401 of 1.25 mm: 5 cm x 50 cm) along x, filled with
    eps_r = 2.5, PEC plates at j = 0 and j = ny, ends on 5-cell 4th-order
    matched absorbers (as ``waveguide2d``).  ``n_iris`` irises evenly placed
    ``spacing`` cells apart (5 cm) about the middle of the guide, each a pair
    of PEC blocks ``iris_len`` cells along the guide (1.25 cm) reaching
    ``iris_depth`` cells (1 cm) in from each plate, which leaves an opening of
    ny - 2 iris_depth cells (3 cm).  A mode-shaped line source at i = src_x
    (one end), a line probe at i = probe_x (the other end).  Pulse: f0 =
    1.5 GHz, bandwidth 3 GHz (the band below 3 GHz).  The layout figure is
    not available: the text gives the iris length, "aperture size" and
    separation; an opening of only 1 cm would be cut off for the TM mode over
    the whole band (five such irises pass ~1e-9 of the field), so the 1 cm is
    read as the depth of each block."""
    wl = waveguide2d(nx=nx, ny=ny, d=d, eps_r=eps_r, absorber=absorber, order=order, refl=refl,
                     src_x=src_x, probe_x=(probe_x,), f0=f0, bw=bw, name=name)
    mid = nx // 2
    pec = []
    for m in range(n_iris):
        c = mid + (m - (n_iris - 1) // 2) * spacing
        i0 = c - iris_len // 2
        for i in range(i0, i0 + iris_len + 1):
            for j in range(1, ny):
                if j <= iris_depth or j >= ny - iris_depth:
                    pec.append((2, i, j, 0))
    wl.pec = pec
    return wl


def port_signs(seed: int, nports: int) -> np.ndarray:
    """Seeded +-1 drive signs for driving several ports together."""
    rng = np.random.default_rng(seed + 7919)
    return rng.choice([-1.0, 1.0], size=nports)


def design2d(n=512, d=0.5e-3, seed=3, region=128, strip_period=16, strip_width=2,
             f0=15e9, bw=10e9, name="design2d") -> Workload:
    """2-D Ez-pol PEC box with a central design region of per-cell eps_r, sigma_e.

    Region cells ``[c0, c0+region)`` in x and y with ``c0 = (n-region)//2``;
    eps_r ~ U[1,4], sigma_e ~ U[0, 0.01] S/m there, vacuum elsewhere.  PEC
    strips: node columns ``x = c0 + p*strip_period + s`` (s < strip_width)
    across the full height of the region.  Source node (n/8, n/2), probe
    node (7n/8, n/2).
    """
    rng = np.random.default_rng(seed)
    c0 = (n - region) // 2
    eps = np.ones((n, n))
    sig = np.zeros((n, n))
    eps[c0:c0 + region, c0:c0 + region] = rng.uniform(1.0, 4.0, size=(region, region))
    sig[c0:c0 + region, c0:c0 + region] = rng.uniform(0.0, 0.01, size=(region, region))
    pec = []
    for p in range(0, region, strip_period):
        for s in range(strip_width):
            i = c0 + p + s
            if not (1 <= i <= n - 1):
                continue
            for j in range(max(c0, 1), min(c0 + region, n - 1) + 1):
                pec.append((2, i, j, 0))
    src = [[(2, n // 8, n // 2, 0, 1.0)]]
    prb = [[(2, (7 * n) // 8, n // 2, 0, 1.0)]]
    return Workload(name=name, dim=2, nx=n, ny=n, nz=1, dx=np.full(n, d), dy=np.full(n, d),
                    dz=np.ones(1), eps_r=eps, sigma_e=sig, pec=pec, sources=src, probes=prb,
                    f0=f0, bw=bw)


def board3d(nx=256, ny=128, nz_fine=8, nz_coarse=56, d=1e-3, dz_fine=0.1e-3, eps_sub=3.38,
            strip=(16, 240, 62, 66), nport_edges=None, f0=10e9, bw=10e9, name="board3d") -> Workload:
    """3-D graded-mesh board: substrate slab on fine dz under coarse dz, PEC strip.

    z spacing: ``nz_fine`` cells of ``dz_fine`` (substrate, eps_r = eps_sub),
    then ``nz_coarse`` cells of ``d``.  The ground plane is the z = 0 wall.
    The PEC strip lies on node plane k = nz_fine over x in [x0, x1), y in
    [y0, y1) (Ex and Ey samples on that plane are forced to zero).  Two line
    ports: the column of Ez edges k = 0..nz_fine-1 under each strip end
    (weights = dz, i.e. the port voltage); each port is also a probe.
    """
    x0, x1, y0, y1 = strip
    nz = nz_fine + nz_coarse
    dz = np.concatenate([np.full(nz_fine, dz_fine), np.full(nz_coarse, d)])
    eps = np.ones((nz, ny, nx))
    eps[:nz_fine] = eps_sub
    sig = np.zeros((nz, ny, nx))
    kk = nz_fine
    pec = []
    for j in range(y0, y1 + 1):
        for i in range(x0, x1):
            if 1 <= j <= ny - 1:
                pec.append((0, i, j, kk))  # Ex on the strip plane
    for j in range(y0, y1):
        for i in range(x0, x1 + 1):
            if 1 <= i <= nx - 1:
                pec.append((1, i, j, kk))  # Ey on the strip plane
    jm = (y0 + y1) // 2
    ports = []
    for ie in (x0 + 1, x1 - 1):
        ports.append([(2, ie, jm, k, float(dz[k])) for k in range(nz_fine)])
    return Workload(name=name, dim=3, nx=nx, ny=ny, nz=nz, dx=np.full(nx, d), dy=np.full(ny, d),
                    dz=dz, eps_r=eps, sigma_e=sig, pec=pec, sources=[list(p) for p in ports],
                    probes=[list(p) for p in ports], f0=f0, bw=bw)


def rom_batch_orders(seed: int, count: int, lo=50, hi=400, step=5) -> np.ndarray:
    """Orders q_i = step * round(U[lo, hi] / step) for a batch of reduced models."""
    rng = np.random.default_rng(seed)
    return (step * np.round(rng.uniform(lo, hi, size=count) / step)).astype(np.int64)


def random_vectors(seed: int, shape, dtype=np.float64) -> np.ndarray:
    """Standard-normal test vectors (used by operator/adjoint consistency tests)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape).astype(dtype)
