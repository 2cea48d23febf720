"""Yee-grid matrices and full-order leapfrog (Sec. II-A, eqs. (CFL), (matrix),
(MNAform), (R_and_F), (x)).  FP64, SciPy sparse.  Test infrastructure only.

Discretisation (the paper states the matrices, not the index bookkeeping):
* Unknowns are the Yee samples strictly inside a PEC box: electric samples
  tangential to a wall and magnetic samples normal to a wall are identically
  zero and are not unknowns.  2-D is Ez-polarisation (Ez, Hx, Hy).
* K is defined from Ampere's law only: ``-K H`` is the dual-grid curl of H
  at each electric sample (weighted, see below).  The magnetic rows use
  ``K^T`` exactly as eq. (matrix) does; Faraday's law is then a consequence
  that the tests check independently.
* Non-uniform grids (the paper asserts eq. (matrix) holds, Sec. II-A, without
  formulas): finite-integration weights.  Electric row e is multiplied by
  ``W_e = dual_area_e * primal_length_e / V_ref`` and magnetic row f by
  ``W_f = primal_area_f * dual_length_f / V_ref`` with ``V_ref`` the volume of
  cell (0,0,0).  On a uniform grid every weight is 1 and the matrices are the
  paper's: D_eps = eps per sample, K with entries +-1/Delta.
* Per-cell materials are averaged onto samples with dual-area (electric) or
  dual-length (magnetic) weights; on uniform grids this is the plain mean of
  the 4 (electric) or 2 (magnetic) cells touching the sample.
* The CFL limit eq. (CFL) uses the vacuum speed and the smallest spacings.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

C0 = 299_792_458.0
MU0 = 1.25663706212e-6  # H/m (CODATA 2018)
EPS0 = 1.0 / (MU0 * C0 * C0)  # F/m
ETA0 = math.sqrt(MU0 / EPS0)


@dataclass
class Grid:
    dim: int
    nx: int
    ny: int
    nz: int
    dx: np.ndarray
    dy: np.ndarray
    dz: np.ndarray

    @staticmethod
    def of(wl) -> "Grid":
        return Grid(wl.dim, wl.nx, wl.ny, wl.nz if wl.dim == 3 else 1,
                    np.asarray(wl.dx, float), np.asarray(wl.dy, float),
                    np.asarray(wl.dz if wl.dim == 3 else np.ones(1), float))

    def dual(self, a: np.ndarray) -> np.ndarray:
        """Dual spacing at nodes 0..n (mean of the adjacent cell spacings)."""
        n = len(a)
        out = np.zeros(n + 1)
        out[1:n] = 0.5 * (a[:-1] + a[1:])
        out[0] = 0.5 * a[0]
        out[n] = 0.5 * a[-1]
        return out


def cfl_dt_max(g: Grid) -> float:
    """eq. (CFL): dt <= 1 / (c sqrt(1/dx^2 + 1/dy^2 [+ 1/dz^2])), smallest cells."""
    s = 1.0 / g.dx.min() ** 2 + 1.0 / g.dy.min() ** 2
    if g.dim == 3:
        s += 1.0 / g.dz.min() ** 2
    return 1.0 / (C0 * math.sqrt(s))


# component codes: 0,1,2 = Ex,Ey,Ez ; 3,4,5 = Hx,Hy,Hz


def component_ranges(g: Grid, c: int) -> Tuple[range, range, range]:
    """Index ranges (i, j, k) of the unknown samples of component c."""
    nx, ny, nz = g.nx, g.ny, g.nz
    if g.dim == 2:
        table = {2: (range(1, nx), range(1, ny), range(0, 1)),
                 3: (range(1, nx), range(0, ny), range(0, 1)),
                 4: (range(0, nx), range(1, ny), range(0, 1))}
        return table[c]
    table = {0: (range(0, nx), range(1, ny), range(1, nz)),
             1: (range(1, nx), range(0, ny), range(1, nz)),
             2: (range(1, nx), range(1, ny), range(0, nz)),
             3: (range(1, nx), range(0, ny), range(0, nz)),
             4: (range(0, nx), range(1, ny), range(0, nz)),
             5: (range(0, nx), range(0, ny), range(1, nz))}
    return table[c]


def e_components(g: Grid) -> Sequence[int]:
    return (2,) if g.dim == 2 else (0, 1, 2)


def h_components(g: Grid) -> Sequence[int]:
    return (3, 4) if g.dim == 2 else (3, 4, 5)


class Numbering:
    """Oracle's own ordering of unknowns: component, then k, j, i (i fastest)."""

    def __init__(self, g: Grid, comps: Sequence[int], removed=()):
        self.g = g
        removed = set((int(c), int(i), int(j), int(k)) for (c, i, j, k) in removed)
        self.index: Dict[Tuple[int, int, int, int], int] = {}
        self.keys: List[Tuple[int, int, int, int]] = []
        for c in comps:
            ri, rj, rk = component_ranges(g, c)
            for k in rk:
                for j in rj:
                    for i in ri:
                        key = (c, i, j, k)
                        if key in removed:
                            continue
                        self.index[key] = len(self.keys)
                        self.keys.append(key)

    def __len__(self):
        return len(self.keys)

    def get(self, c, i, j, k):
        return self.index.get((c, i, j, k))


def count_unknowns_2d(nx: int, ny: int) -> int:
    """Ez-pol interior unknowns: (nx-1)(ny-1) + (nx-1)ny + nx(ny-1)."""
    return (nx - 1) * (ny - 1) + (nx - 1) * ny + nx * (ny - 1)


@dataclass
class Operator:
    """The diagonal matrices and K of eq. (matrix) for one structure."""

    grid: Grid
    ne: Numbering
    nh: Numbering
    De: np.ndarray  # D_eps  (N_e,)
    Dse: np.ndarray  # D_sigma_e (N_e,)
    Dm: np.ndarray  # D_mu (N_h,)
    Dsm: np.ndarray  # D_sigma_m (N_h,)
    K: sp.csr_matrix  # N_e x N_h
    We: np.ndarray  # row weights of the electric rows (1 on uniform grids)
    Wh: np.ndarray

    @property
    def Ne(self):
        return len(self.ne)

    @property
    def Nh(self):
        return len(self.nh)

    @property
    def N(self):
        return self.Ne + self.Nh


def _cell(a: np.ndarray, g: Grid, i: int, j: int, k: int) -> float:
    if g.dim == 2:
        return float(a[j, i])
    return float(a[k, j, i])


def _lengths(g: Grid):
    return (g.dx, g.dy, g.dz, g.dual(g.dx), g.dual(g.dy), g.dual(g.dz))


def _edge_cells(g: Grid, c: int, i: int, j: int, k: int):
    """Cells touching electric sample (c,i,j,k) with their dual-area weights."""
    dx, dy, dz = g.dx, g.dy, g.dz
    out = []
    if g.dim == 2:  # Ez at node (i, j): cells (i-1..i, j-1..j)
        for a in (i - 1, i):
            for b in (j - 1, j):
                out.append(((a, b, 0), 0.25 * dx[a] * dy[b]))
        return out
    if c == 0:  # Ex(i+1/2, j, k): cells (i, j-1..j, k-1..k)
        for b in (j - 1, j):
            for cc in (k - 1, k):
                out.append(((i, b, cc), 0.25 * dy[b] * dz[cc]))
    elif c == 1:
        for a in (i - 1, i):
            for cc in (k - 1, k):
                out.append(((a, j, cc), 0.25 * dx[a] * dz[cc]))
    else:
        for a in (i - 1, i):
            for b in (j - 1, j):
                out.append(((a, b, k), 0.25 * dx[a] * dy[b]))
    return out


def _face_cells(g: Grid, c: int, i: int, j: int, k: int):
    """Cells touching magnetic sample (c,i,j,k) with their dual-length weights."""
    dx, dy, dz = g.dx, g.dy, g.dz
    if g.dim == 2:
        if c == 3:  # Hx(i, j+1/2): cells (i-1, j), (i, j)
            return [((i - 1, j, 0), 0.5 * dx[i - 1]), ((i, j, 0), 0.5 * dx[i])]
        return [((i, j - 1, 0), 0.5 * dy[j - 1]), ((i, j, 0), 0.5 * dy[j])]
    if c == 3:
        return [((i - 1, j, k), 0.5 * dx[i - 1]), ((i, j, k), 0.5 * dx[i])]
    if c == 4:
        return [((i, j - 1, k), 0.5 * dy[j - 1]), ((i, j, k), 0.5 * dy[j])]
    return [((i, j, k - 1), 0.5 * dz[k - 1]), ((i, j, k), 0.5 * dz[k])]


def edge_average_weights(g: Grid, c, i, j, k):
    cells = _edge_cells(g, c, i, j, k)
    tot = sum(w for _, w in cells)
    return [(cell, w / tot) for cell, w in cells]


def face_average_weights(g: Grid, c, i, j, k):
    cells = _face_cells(g, c, i, j, k)
    tot = sum(w for _, w in cells)
    return [(cell, w / tot) for cell, w in cells]


def row_weight_e(g: Grid, c, i, j, k) -> float:
    """dual area x primal length / V_ref for electric sample (c,i,j,k)."""
    dx, dy, dz, dxd, dyd, dzd = _lengths(g)
    vref = dx[0] * dy[0] * (dz[0] if g.dim == 3 else 1.0)
    if g.dim == 2:
        return dxd[i] * dyd[j] * 1.0 / vref
    if c == 0:
        return dyd[j] * dzd[k] * dx[i] / vref
    if c == 1:
        return dxd[i] * dzd[k] * dy[j] / vref
    return dxd[i] * dyd[j] * dz[k] / vref


def row_weight_h(g: Grid, c, i, j, k) -> float:
    """primal area x dual length / V_ref for magnetic sample (c,i,j,k)."""
    dx, dy, dz, dxd, dyd, dzd = _lengths(g)
    vref = dx[0] * dy[0] * (dz[0] if g.dim == 3 else 1.0)
    if g.dim == 2:
        if c == 3:
            return dy[j] * 1.0 * dxd[i] / vref
        return dx[i] * 1.0 * dyd[j] / vref
    if c == 3:
        return dy[j] * dz[k] * dxd[i] / vref
    if c == 4:
        return dx[i] * dz[k] * dyd[j] / vref
    return dx[i] * dy[j] * dzd[k] / vref


def _dual_curl_terms(g: Grid, c, i, j, k):
    """Ampere: (curl H) at electric sample (c,i,j,k) as [(h_key, coeff)].

    Central differences of the neighbouring magnetic samples over the dual
    spacing, e.g. Ex: dHz/dy - dHy/dz.
    """
    dx, dy, dz, dxd, dyd, dzd = _lengths(g)
    if g.dim == 2:  # eps dEz/dt = dHy/dx - dHx/dy
        return [((4, i, j, 0), 1 / dxd[i]), ((4, i - 1, j, 0), -1 / dxd[i]),
                ((3, i, j, 0), -1 / dyd[j]), ((3, i, j - 1, 0), 1 / dyd[j])]
    if c == 0:  # dHz/dy - dHy/dz
        return [((5, i, j, k), 1 / dyd[j]), ((5, i, j - 1, k), -1 / dyd[j]),
                ((4, i, j, k), -1 / dzd[k]), ((4, i, j, k - 1), 1 / dzd[k])]
    if c == 1:  # dHx/dz - dHz/dx
        return [((3, i, j, k), 1 / dzd[k]), ((3, i, j, k - 1), -1 / dzd[k]),
                ((5, i, j, k), -1 / dxd[i]), ((5, i - 1, j, k), 1 / dxd[i])]
    # dHy/dx - dHx/dy
    return [((4, i, j, k), 1 / dxd[i]), ((4, i - 1, j, k), -1 / dxd[i]),
            ((3, i, j, k), -1 / dyd[j]), ((3, i, j - 1, k), 1 / dyd[j])]


def assemble(wl, eps0=EPS0, mu0=MU0) -> Operator:
    """Build D_eps, D_sigma_e, D_mu, D_sigma_m and K of eq. (matrix)."""
    g = Grid.of(wl)
    ne = Numbering(g, e_components(g), removed=wl.pec)
    nh = Numbering(g, h_components(g))
    mu_r = wl.mu_r if wl.mu_r is not None else np.ones_like(wl.eps_r)
    sig_m = wl.sigma_m if wl.sigma_m is not None else np.zeros_like(wl.eps_r)
    De = np.zeros(len(ne))
    Dse = np.zeros(len(ne))
    We = np.zeros(len(ne))
    for r, (c, i, j, k) in enumerate(ne.keys):
        w = row_weight_e(g, c, i, j, k)
        avg = edge_average_weights(g, c, i, j, k)
        er = sum(a * _cell(wl.eps_r, g, *cell) for cell, a in avg)
        se = sum(a * _cell(wl.sigma_e, g, *cell) for cell, a in avg)
        We[r] = w
        De[r] = eps0 * er * w
        Dse[r] = se * w
    Dm = np.zeros(len(nh))
    Dsm = np.zeros(len(nh))
    Wh = np.zeros(len(nh))
    for r, (c, i, j, k) in enumerate(nh.keys):
        w = row_weight_h(g, c, i, j, k)
        avg = face_average_weights(g, c, i, j, k)
        mr = sum(a * _cell(mu_r, g, *cell) for cell, a in avg)
        sm = sum(a * _cell(sig_m, g, *cell) for cell, a in avg)
        Wh[r] = w
        Dm[r] = mu0 * mr * w
        Dsm[r] = sm * w
    rows, cols, vals = [], [], []
    for r, (c, i, j, k) in enumerate(ne.keys):
        w = We[r]
        for hkey, coef in _dual_curl_terms(g, c, i, j, k):
            col = nh.index.get(hkey)
            if col is None:  # magnetic sample normal to a PEC wall: zero
                continue
            rows.append(r)
            cols.append(col)
            vals.append(-w * coef)  # -K H = W_e curl H
    K = sp.csr_matrix((vals, (rows, cols)), shape=(len(ne), len(nh)))
    return Operator(g, ne, nh, De, Dse, Dm, Dsm, K, We, Wh)


def R_F(op: Operator, dt: float):
    """eq. (R_and_F): R = [[De/dt, -K/2], [-K^T/2, Dm/dt]], F = [[Dse/2, K/2], [-K^T/2, Dsm/2]]."""
    K = op.K
    R = sp.bmat([[sp.diags(op.De / dt), -0.5 * K], [-0.5 * K.T, sp.diags(op.Dm / dt)]], format="csr")
    F = sp.bmat([[sp.diags(op.Dse / 2), 0.5 * K], [-0.5 * K.T, sp.diags(op.Dsm / 2)]], format="csr")
    return R, F


def port_matrix(op: Operator, ports, scale_rows: bool) -> np.ndarray:
    """Columns for a list of ports on electric samples.

    Sources (B, eq. (matrix)): entry weight * W_e, i.e. 1 at a point source
    on a uniform grid.  Probes (L): plain weights on the field samples.
    Returns an N x nports dense array (magnetic rows zero).
    """
    M = np.zeros((op.N, len(ports)))
    for p, port in enumerate(ports):
        for (c, i, j, k, w) in port:
            r = op.ne.get(c, i, j, k)
            if r is None:
                raise ValueError(f"port entry {(c, i, j, k)} is not an electric unknown")
            M[r, p] += w * (op.We[r] if scale_rows else 1.0)
    return M


def leapfrog(op: Operator, dt: float, B: np.ndarray, u: np.ndarray, L: np.ndarray,
             x0=None, return_states=False):
    """eq. (MNAform): (R+F) x^{n+1} = (R-F) x^n + B u^{n+1}.

    (R+F) is block lower triangular with diagonal diagonal blocks, so each
    step is the block forward substitution: first the electric rows,
        (De/dt + Dse/2) E^{n+1} = (De/dt - Dse/2) E^n - K H^{n+1/2} + B_e u^{n+1},
    then the magnetic rows,
        (Dm/dt + Dsm/2) H^{n+3/2} = (Dm/dt - Dsm/2) H^{n+1/2} + K^T E^{n+1} + B_h u^{n+1}.
    ``u[n]`` drives the step producing x^{n+1}.  Returns y[n] = L^T x^{n+1}.
    """
    ne = op.Ne
    x = np.zeros(op.N) if x0 is None else np.array(x0, dtype=float)
    E, H = x[:ne].copy(), x[ne:].copy()
    pe, me = op.De / dt + op.Dse / 2, op.De / dt - op.Dse / 2
    pm, mm = op.Dm / dt + op.Dsm / 2, op.Dm / dt - op.Dsm / 2
    Be, Bh = B[:ne], B[ne:]
    KT = op.K.T.tocsr()
    nsteps = u.shape[0]
    y = np.zeros((nsteps, L.shape[1]))
    states = []
    for n in range(nsteps):
        E = (me * E - op.K @ H + Be @ u[n]) / pe
        H = (mm * H + KT @ E + Bh @ u[n]) / pm
        xn = np.concatenate([E, H])
        y[n] = L.T @ xn
        if return_states:
            states.append(xn)
    if return_states:
        return y, np.array(states)
    return y, np.concatenate([E, H])


def energy(R, x: np.ndarray) -> float:
    """W = x^T R x, the quadratic form of condition (Dstability2)."""
    return float(x @ (R @ x))


def fields_from_x(op: Operator, x: np.ndarray) -> Dict[Tuple[int, int, int, int], float]:
    """Map a state vector back to {(c,i,j,k): value}."""
    out = {}
    for r, key in enumerate(op.ne.keys):
        out[key] = x[r]
    for r, key in enumerate(op.nh.keys):
        out[key] = x[op.Ne + r]
    return out
