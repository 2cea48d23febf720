"""Structure-preserving reduction (Sec. II-C, IV-A, IV-B).  FP64, exact sparse
LU solves.  Test infrastructure only.

Steps, in the paper's order:
1. expansion points z_l = M exp(j 2 pi (l/L) f_max dt), eq. (distrib);
   l = 0..L (the conjugate points l < 0 are covered by the real split, 4.);
2. per point, a block Krylov (Arnoldi) basis of A_l = (z_l P - Q)^{-1} P
   started from (z_l P - Q)^{-1} B, with P = R + F, Q = R - F.  Reading of
   eq. (linear_system_solution): the shifted matrix is z (R+F) - (R-F), the
   resolvent of eq. (MNAform), which equals 2F at z = 1 (static conditions,
   as Sec. IV-A states);
3. inner products in the energy-balanced scaling diag(I, eta0 I) (E and H
   rows differ by the wave impedance; the Krylov subspace itself does not
   depend on the inner product), modified Gram-Schmidt twice, a column is
   deflated when its norm drops below ``defl_tol`` times its norm before
   orthogonalisation;
4. real basis: the real vectors of z_0 and Re/Im of the complex vectors of
   z_1..z_L;
5. SPRIM split, eq. (V): V1 = orth(electric rows), V2 = orth(magnetic rows),
   by SVD keeping singular values above ``rank_tol`` times the largest;
6. projection, eq. (R_and_Freduced), D-blocks symmetrised;
7. reduced leapfrog, eq. (reducedMNAform) with input u^{n+1} (reading: the
   printed u^n and the time index of eq. (projection) are typos against
   eq. (MNAform)).

Moments per point (the paper gives only the total order): with q real
columns, 2L+1 points and b ports, every point gets k = q/(2L+1) real
columns: z_0 contributes k/b real block moments; each z_l, l >= 1, k/b
complex block moments whose Re/Im parts give 2k columns covering the pair
(z_l, conj z_l); in total k + 2Lk = q.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import yee


def expansion_points(M: float, L: int, fmax: float, dt: float) -> np.ndarray:
    """eq. (distrib) for l = 0..L."""
    return np.array([M * np.exp(2j * math.pi * (l / L) * fmax * dt) if L > 0 else M
                     for l in range(L + 1)])


def system_pq(op: yee.Operator, dt: float):
    """P = R + F, Q = R - F of eq. (MNAform)."""
    R, F = yee.R_F(op, dt)
    return (R + F).tocsc(), (R - F).tocsc()


def shifted_matrix(op: yee.Operator, dt: float, z: complex):
    """z (R + F) - (R - F)  (reading of eq. (linear_system_solution))."""
    P, Q = system_pq(op, dt)
    return (z * P - Q).tocsc()


def schur_complement(op: yee.Operator, dt: float, z: complex):
    """S = A11 - A12 A22^{-1} A21 of the shifted matrix (eq. (reduced_linear_system_solution1)),
    with A11 = (z-1) De/dt + (z+1) Dse/2, A12 = K, A21 = -z K^T,
    A22 = (z-1) Dm/dt + (z+1) Dsm/2 (the diagonal blocks of z (R+F) - (R-F))."""
    a11 = (z - 1) * op.De / dt + (z + 1) * op.Dse / 2
    a22 = (z - 1) * op.Dm / dt + (z + 1) * op.Dsm / 2
    A12 = op.K.astype(complex)
    A21 = (-z) * op.K.T.astype(complex)
    return (sp.diags(a11) - A12 @ sp.diags(1.0 / a22) @ A21).tocsc()


def schur_solve(op: yee.Operator, dt: float, z: complex, b: np.ndarray) -> np.ndarray:
    """Solve the shifted system through its 2x2 block Schur complement.

    eqs. (reduced_linear_system_solution1/2): with A11, A22 diagonal,
    (A11 - A12 A22^{-1} A21) x1 = b1 - A12 A22^{-1} b2,
    x2 = A22^{-1} (b2 - A21 x1).  Here A11 = (z-1) De/dt + (z+1) Dse/2,
    A12 = K, A21 = -z K^T, A22 = (z-1) Dm/dt + (z+1) Dsm/2.
    """
    ne = op.Ne
    a22 = (z - 1) * op.Dm / dt + (z + 1) * op.Dsm / 2
    A12 = op.K.astype(complex)
    A21 = (-z) * op.K.T.astype(complex)
    b1, b2 = b[:ne], b[ne:]
    S = schur_complement(op, dt, z)
    x1 = spla.splu(S).solve(np.asarray(b1 - A12 @ (b2 / a22 if b2.ndim == 1 else b2 / a22[:, None]),
                                       dtype=complex))
    rhs2 = b2 - A21 @ x1
    x2 = rhs2 / (a22 if rhs2.ndim == 1 else a22[:, None])
    return np.concatenate([x1, x2])


@dataclass
class Reduced:
    """Reduced model of eq. (reducedMNAform) plus its projection basis."""

    V1: np.ndarray
    V2: np.ndarray
    De: np.ndarray
    Dse: np.ndarray
    Dm: np.ndarray
    Dsm: np.ndarray
    K: np.ndarray
    B1: np.ndarray
    B2: np.ndarray
    L1: np.ndarray
    L2: np.ndarray
    points: np.ndarray = field(default_factory=lambda: np.zeros(0))
    deflated: int = 0

    @property
    def q1(self):
        return self.V1.shape[1]

    @property
    def q2(self):
        return self.V2.shape[1]


def _balance(op: yee.Operator) -> np.ndarray:
    """diag(I, eta0 I): energy-balanced row scaling for inner products."""
    return np.concatenate([np.ones(op.Ne), np.full(op.Nh, yee.ETA0)])


def arnoldi_point(lu, P, B: np.ndarray, nblocks: int, scale: np.ndarray,
                  defl_tol: float) -> List[np.ndarray]:
    """Block Arnoldi at one expansion point (Sec. II-C, Sec. IV-A).

    ``lu`` factors (z P - Q).  Returns the orthonormal (in the scaled inner
    product) basis columns, unscaled, as a list of vectors.
    """
    basis_s: List[np.ndarray] = []  # scaled, orthonormal
    X = lu.solve(np.asarray(B, dtype=lu_dtype(lu)))
    for m in range(nblocks):
        if m > 0:
            X = lu.solve(np.asarray(P @ prev, dtype=lu_dtype(lu)))
        kept = []
        for col in (X.T if X.ndim == 2 else [X]):
            y = scale * col
            n0 = np.linalg.norm(y)
            if n0 == 0:
                continue
            for _ in range(2):  # modified Gram-Schmidt, twice
                for v in basis_s:
                    y = y - v * np.vdot(v, y)
            n1 = np.linalg.norm(y)
            if n1 < defl_tol * n0:
                continue  # deflation
            y = y / n1
            basis_s.append(y)
            kept.append(y / scale)
        if not kept:
            break
        prev = np.array(kept).T
    return [v / scale for v in basis_s]


def lu_dtype(lu):
    return lu.U.dtype


def orth_svd(A: np.ndarray, rank_tol: float) -> np.ndarray:
    """Orthonormal basis of range(A) from its SVD, singular values > rank_tol*s1."""
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    if s.size == 0 or s[0] == 0:
        return U[:, :0]
    r = int(np.sum(s > rank_tol * s[0]))
    return U[:, :r]


def project(op: yee.Operator, V1: np.ndarray, V2: np.ndarray, B: np.ndarray, L: np.ndarray) -> dict:
    """eq. (R_and_Freduced): De~ = V1^T De V1, ..., K~ = V1^T K V2, B~ = V^T B."""
    ne = op.Ne
    sym = lambda A: 0.5 * (A + A.T)
    return dict(
        De=sym(V1.T @ (op.De[:, None] * V1)),
        Dse=sym(V1.T @ (op.Dse[:, None] * V1)),
        Dm=sym(V2.T @ (op.Dm[:, None] * V2)),
        Dsm=sym(V2.T @ (op.Dsm[:, None] * V2)),
        K=V1.T @ (op.K @ V2),
        B1=V1.T @ B[:ne], B2=V2.T @ B[ne:],
        L1=V1.T @ L[:ne], L2=V2.T @ L[ne:],
    )


def mor_reduce(op: yee.Operator, B: np.ndarray, L: np.ndarray, q: int, dt_ref: float,
               fmax: float, M: float = 1.1, npts_half: int = 2, defl_tol: float = 1e-10,
               rank_tol: float = 1e-12, pair_only: bool = False) -> Reduced:
    """Sec. II-C + IV-A: SPRIM reduction with complex frequency hopping.

    pair_only: the single conjugate pair z = M exp(+-j 2 pi f_max dt_ref) of
    Sec. V-C (single-frequency drive) instead of eq. (distrib): all q columns
    come from the complex block moments at z, whose real and imaginary parts
    cover z and its conjugate (q/2 complex vectors)."""
    b = B.shape[1]
    Lh = npts_half
    if pair_only:
        if q % 2:
            raise ValueError("q must be even for a conjugate pair")
        k = q // 2
        pts = np.array([M * np.exp(2j * math.pi * fmax * dt_ref)])
    else:
        if q % (2 * Lh + 1):
            raise ValueError("q must be a multiple of the number of expansion points 2L+1")
        k = q // (2 * Lh + 1)
        pts = expansion_points(M, Lh, fmax, dt_ref)
    if k % b:
        raise ValueError("columns per point must be a multiple of the port count")
    P, Q = system_pq(op, dt_ref)
    scale = _balance(op)
    cols = []
    for l, z in enumerate(pts):
        nblk = k // b
        if l == 0 and not pair_only:
            lu = spla.splu((z.real * P - Q).tocsc())
            vecs = arnoldi_point(lu, P, B, nblk, scale, defl_tol)
            cols += [v.real for v in vecs]
        else:
            lu = spla.splu((z * P - Q).tocsc())
            vecs = arnoldi_point(lu, P, B.astype(complex), nblk, scale, defl_tol)
            for v in vecs:
                cols += [v.real, v.imag]
    Vhat = np.array(cols).T
    ne = op.Ne
    V1 = orth_svd(Vhat[:ne], rank_tol)
    V2 = orth_svd(Vhat[ne:], rank_tol)
    pr = project(op, V1, V2, B, L)
    return Reduced(V1=V1, V2=V2, points=pts, deflated=q - Vhat.shape[1], **pr)


def reduced_R_F(rom: Reduced, dt: float, K: Optional[np.ndarray] = None):
    """eq. (R_and_Freduced) as dense matrices."""
    K = rom.K if K is None else K
    R = np.block([[rom.De / dt, -0.5 * K], [-0.5 * K.T, rom.Dm / dt]])
    F = np.block([[rom.Dse / 2, 0.5 * K], [-0.5 * K.T, rom.Dsm / 2]])
    return R, F


def rom_leapfrog(rom: Reduced, dt: float, u: np.ndarray, K: Optional[np.ndarray] = None,
                 return_states=False):
    """eq. (reducedMNAform), solved in leapfrog order (Sec. II-C, last remark):
    (De~/dt + Dse~/2) e^{n+1} = (De~/dt - Dse~/2) e^n - K~ h + B1~ u^{n+1},
    (Dm~/dt + Dsm~/2) h^{n+1} = (Dm~/dt - Dsm~/2) h + K~^T e^{n+1} + B2~ u^{n+1}.
    Output y^{n+1} = L1~^T e^{n+1} + L2~^T h^{n+1}.
    """
    K = rom.K if K is None else K
    ce = sla.cho_factor(rom.De / dt + rom.Dse / 2)
    cm = sla.cho_factor(rom.Dm / dt + rom.Dsm / 2)
    Me = rom.De / dt - rom.Dse / 2
    Mm = rom.Dm / dt - rom.Dsm / 2
    e = np.zeros(rom.q1)
    h = np.zeros(rom.q2)
    y = np.zeros((u.shape[0], rom.L1.shape[1]))
    states = []
    for n in range(u.shape[0]):
        e = sla.cho_solve(ce, Me @ e - K @ h + rom.B1 @ u[n])
        h = sla.cho_solve(cm, Mm @ h + K.T @ e + rom.B2 @ u[n])
        y[n] = rom.L1.T @ e + rom.L2.T @ h
        if return_states:
            states.append(np.concatenate([e, h]))
    if return_states:
        return y, np.array(states)
    return y


def transfer(P, Q, B: np.ndarray, L: np.ndarray, z: complex) -> np.ndarray:
    """H(z) = L^T (z P - Q)^{-1} B of the discrete system eq. (MNAform)."""
    if sp.issparse(P):
        X = spla.splu((z * P - Q).tocsc().astype(complex)).solve(B.astype(complex))
    else:
        X = np.linalg.solve(z * P - Q, B.astype(complex))
    return L.T @ X


def rom_transfer(rom: Reduced, dt: float, z: complex, K=None) -> np.ndarray:
    R, F = reduced_R_F(rom, dt, K)
    B = np.vstack([rom.B1, rom.B2])
    L = np.vstack([rom.L1, rom.L2])
    return transfer(R + F, R - F, B, L, z)
