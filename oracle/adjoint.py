"""Discrete adjoint of the leapfrog eq. (MNAform) and of the reduced leapfrog
eq. (reducedMNAform) for the probe-energy objective.  Not in the paper: it
is derived here from the same equations.  FP64.  Test infrastructure only.

Objective  J = sum_{n=1..N} dt * sum_p (L_p^T x^n)^2.

Lagrangian stationarity gives, with lambda^{N+1} = 0 and n = N..1,
    P^T lambda^n = Q^T lambda^{n+1} + dJ/dx^n,
where P = R + F (block lower triangular) so P^T is block upper triangular:
the magnetic rows are solved first, then the electric rows,
    (Dm/dt + Dsm/2) lh^n = (Dm/dt - Dsm/2) lh^{n+1} - K^T le^{n+1} + dJ/dh^n
    (De/dt + Dse/2) le^n = (De/dt - Dse/2) le^{n+1} + K lh^n + dJ/de^n.
Gradients with respect to the diagonal entries (per electric unknown):
    dJ/dDe_e  = -sum_n le_e^{n+1} (E_e^{n+1} - E_e^n) / dt
    dJ/dDse_e = -sum_n le_e^{n+1} (E_e^{n+1} + E_e^n) / 2
and per cell through the averaging of materials onto samples.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import yee
from .mor import Reduced


def objective(y: np.ndarray, dt: float) -> float:
    return float(dt * np.sum(y ** 2))


def full_adjoint(op: yee.Operator, dt: float, B: np.ndarray, u: np.ndarray, L: np.ndarray):
    """Gradient of J w.r.t. the diagonals De, Dse (per electric unknown)."""
    y, X = yee.leapfrog(op, dt, B, u, L, return_states=True)
    ne = op.Ne
    nsteps = u.shape[0]
    Xall = np.vstack([np.zeros(op.N), X])  # x^0 .. x^N
    pe, me = op.De / dt + op.Dse / 2, op.De / dt - op.Dse / 2
    pm, mm = op.Dm / dt + op.Dsm / 2, op.Dm / dt - op.Dsm / 2
    KT = op.K.T.tocsr()
    le = np.zeros(ne)
    lh = np.zeros(op.Nh)
    gDe = np.zeros(ne)
    gDse = np.zeros(ne)
    for n in range(nsteps, 0, -1):  # lambda^{n}, uses lambda^{n+1} = (le, lh)
        g = 2.0 * dt * (L @ (L.T @ Xall[n]))
        lh_new = (mm * lh - KT @ le + g[ne:]) / pm
        le_new = (me * le + op.K @ lh_new + g[:ne]) / pe
        le, lh = le_new, lh_new
        # this lambda^n multiplies the step producing x^n from x^{n-1}
        En, Ep = Xall[n][:ne], Xall[n - 1][:ne]
        gDe += -le * (En - Ep) / dt
        gDse += -le * (En + Ep) / 2
    return objective(y, dt), gDe, gDse


def cell_gradients(op: yee.Operator, wl, gDe: np.ndarray, gDse: np.ndarray):
    """Chain dJ/dDe_e, dJ/dDse_e to per-cell eps_r and sigma_e."""
    g = op.grid
    ge = np.zeros_like(wl.eps_r, dtype=float)
    gs = np.zeros_like(wl.sigma_e, dtype=float)
    for r, (c, i, j, k) in enumerate(op.ne.keys):
        for cell, a in yee.edge_average_weights(g, c, i, j, k):
            idx = (cell[1], cell[0]) if g.dim == 2 else (cell[2], cell[1], cell[0])
            ge[idx] += gDe[r] * yee.EPS0 * op.We[r] * a
            gs[idx] += gDse[r] * op.We[r] * a
    return ge, gs


def reduced_adjoint(rom: Reduced, dt: float, u: np.ndarray, K=None):
    """Adjoint of eq. (reducedMNAform) for J = dt sum (L~^T x~^n)^2.

    Returns J and dJ/dDe~, dJ/dDse~ (q1 x q1 matrices; the chain to a
    parameter theta is trace(dJ/dDe~^T dDe~/dtheta)) and dJ/dK~.
    """
    from .mor import rom_leapfrog
    K = rom.K if K is None else K
    y, X = rom_leapfrog(rom, dt, u, K=K, return_states=True)
    q1 = rom.q1
    nsteps = u.shape[0]
    Xall = np.vstack([np.zeros(X.shape[1]), X])
    Pe = rom.De / dt + rom.Dse / 2
    Me = rom.De / dt - rom.Dse / 2
    Pm = rom.Dm / dt + rom.Dsm / 2
    Mm = rom.Dm / dt - rom.Dsm / 2
    L = np.vstack([rom.L1, rom.L2])
    le = np.zeros(q1)
    lh = np.zeros(rom.q2)
    gDe = np.zeros((q1, q1))
    gDse = np.zeros((q1, q1))
    gK = np.zeros_like(K)
    for n in range(nsteps, 0, -1):
        g = 2.0 * dt * (L @ (L.T @ Xall[n]))
        lh_new = sla.solve(Pm.T, Mm.T @ lh - K.T @ le + g[q1:])
        le_new = sla.solve(Pe.T, Me.T @ le + K @ lh_new + g[:q1])
        le, lh = le_new, lh_new
        En, Ep = Xall[n][:q1], Xall[n - 1][:q1]
        Hn, Hp = Xall[n][q1:], Xall[n - 1][q1:]
        # P x^n - Q x^{n-1}: electric rows (De/dt+Dse/2)En - (De/dt-Dse/2)Ep + K Hp
        gDe += -np.outer(le, (En - Ep) / dt)
        gDse += -np.outer(le, (En + Ep) / 2)
        # K enters the electric rows (+K Hp) and the magnetic rows (-K^T En)
        gK += -np.outer(le, Hp) + np.outer(En, lh)
    return objective(y, dt), gDe, gDse, gK


def clamp_derivative(A: np.ndarray, dA: np.ndarray, smax: float) -> np.ndarray:
    """Directional derivative of A -> U min(S, smax) W^T (the clamp of Sec. III-A).

    Divided differences of the singular-value function f(s) = min(s, smax)
    (square A, distinct singular values): with dX = U^T dA W,
    [U^T df W]_ij = sym(dX)_ij (f_i - f_j)/(s_i - s_j) + skew(dX)_ij (f_i + f_j)/(s_i + s_j),
    [U^T df W]_ii = f'(s_i) dX_ii.
    """
    U, s, Wt = np.linalg.svd(A)
    W = Wt.T
    f = np.minimum(s, smax)
    dX = U.T @ dA @ W
    Ps = 0.5 * (dX + dX.T)
    Sk = 0.5 * (dX - dX.T)
    q = len(s)
    G = np.zeros_like(dX)
    for i in range(q):
        for j in range(q):
            if i == j:
                G[i, i] = (1.0 if s[i] < smax else 0.0) * dX[i, i]
            else:
                G[i, j] = (Ps[i, j] * (f[i] - f[j]) / (s[i] - s[j])
                           + Sk[i, j] * (f[i] + f[j]) / (s[i] + s[j]))
    return U @ G @ Wt


def sqrt_derivative(D: np.ndarray, dD: np.ndarray):
    """(S, dS) with S = D^{1/2} (principal root) and S dS + dS S = dD."""
    w, Q = np.linalg.eigh(0.5 * (D + D.T))
    r = np.sqrt(w)
    S = (Q * r) @ Q.T
    dS = Q @ ((Q.T @ dD @ Q) / (r[:, None] + r[None, :])) @ Q.T
    return S, dS


def perturbed_K_derivative(De: np.ndarray, Dm: np.ndarray, K: np.ndarray, dt: float,
                           gamma: float, dDe: np.ndarray) -> np.ndarray:
    """d K~' for a change dDe of De~ (Dm~, K~ fixed), symmetric-square-root form of
    K~' = De~^{1/2} f(De~^{-1/2} K~ Dm~^{-1/2}) Dm~^{1/2}, f the singular-value clamp."""
    from .perturb import sym_sqrt
    Se, dSe = sqrt_derivative(De, dDe)
    Sei = np.linalg.inv(Se)
    Sm = sym_sqrt(Dm)
    Smi = np.linalg.inv(Sm)
    A = Sei @ K @ Smi
    dA = -(Sei @ dSe @ Sei) @ K @ Smi
    smax = gamma * 2.0 / dt
    U, s, Wt = np.linalg.svd(A)
    fA = (U * np.minimum(s, smax)) @ Wt
    return dSe @ fA @ Sm + Se @ clamp_derivative(A, dA, smax) @ Sm


def reduced_theta_gradient(rom: Reduced, dt: float, u: np.ndarray, dDe: np.ndarray,
                           gamma: float = 0.9999, through_clamp: bool = True):
    """dJ/dtheta for the reduced leapfrog at dt after the clamp, for a parameter
    theta that moves De~ by dDe (V frozen: dDe = V1^T (dDe/dtheta) V1).

    J = dt sum (L~^T x~^n)^2.  Reverse mode through the time stepping gives
    dJ/dDe~ and dJ/dK~'; forward mode through the clamp gives dK~'/dtheta.
    With through_clamp = False the clamped K~' is held fixed.
    """
    from .perturb import perturb
    Kp, _, _, _ = perturb(rom.De, rom.Dm, rom.K, dt, gamma)
    J, gDe, gDse, gK = reduced_adjoint(rom, dt, u, K=Kp)
    dJ = float(np.sum(gDe * dDe))
    if through_clamp:
        dKp = perturbed_K_derivative(rom.De, rom.Dm, rom.K, dt, gamma, dDe)
        dJ += float(np.sum(gK * dKp))
    return J, dJ, gDe, gDse, gK
