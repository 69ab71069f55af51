"""Two-grid cycle with PML-aware coarsening (oracle), Sec. 4 and App. A.

* Coarse mesh (Sec. 4, "Using PML layers in the two-grid method"): per axis
  the w_pml outer-PML cells on each side are not coarsened, the N - 2 w_pml
  interior cells are coarsened 2:1.
* Prolongation by tent functions: (P u)_{i_FP(i)} = u_i and
  (P u)_{i_FP(i)+1} = (u_i + u_{i+1})/2 when coarse cell i+1/2 is refined;
  restriction R = P^T.
* Coarse coefficients (App. A, coarse level optimized finite elements):
  cell k^2 by tensor products of 1-D averages of the fine node values with
  weights (1/2, 1/2) on unrefined cells and (1/4, 1/2, 1/4) on refined
  cells; alpha evaluated at the coarse cell midpoints.
* Cycle: nu omega-Jacobi pre-smoothing steps from x = 0, residual,
  restriction, an (inexact) coarse solve, prolongation and correction, nu
  post-smoothing steps (V-cycle with omega-Jacobi, Sec. 4).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .discretization import Axis


def coarsen_axis(fine, w_pml):
    """Coarse axis and its maps.  Returns (coarse Axis, i_FP, refined) where
    i_FP[i] is the fine node of coarse node i and refined[p] tells whether
    coarse cell p (between coarse nodes p, p+1) is a refined (2-cell) cell."""
    N = fine.n_cells
    n_int = N - 2 * w_pml
    if n_int % 2:
        raise ValueError("interior cell count must be even for 2:1 coarsening")
    ifp = list(range(0, w_pml + 1))
    ifp += [w_pml + 2 * m for m in range(1, n_int // 2 + 1)]
    ifp += [N - w_pml + q for q in range(1, w_pml + 1)]
    ifp = np.array(ifp)
    refined = np.diff(ifp) == 2
    coarse = Axis(fine.x[ifp], fine.sigma, 2.0 * fine.h_nom)
    return coarse, ifp, refined


def prolongation_1d(ifp, refined, n_fine_cells):
    """Tent prolongation on one axis restricted to the unknowns:
    shape (N_f - 1, N_c - 1).  Coarse Dirichlet nodes 0, N_c are zero."""
    Nc = len(ifp) - 1
    rows, cols, vals = [], [], []
    for i in range(1, Nc):
        rows.append(ifp[i] - 1); cols.append(i - 1); vals.append(1.0)
    for p in range(Nc):
        if refined[p]:
            r = ifp[p] + 1          # fine node between coarse nodes p, p+1
            for i in (p, p + 1):
                if 1 <= i <= Nc - 1:
                    rows.append(r - 1); cols.append(i - 1); vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_fine_cells - 1, Nc - 1))


def cell_average_1d(ifp, refined, n_fine_cells):
    """(N_c, N_f + 1) weights taking fine node values to coarse cell values:
    (1/2, 1/2) on an unrefined cell, (1/4, 1/2, 1/4) on a refined cell."""
    Nc = len(ifp) - 1
    W = np.zeros((Nc, n_fine_cells + 1))
    for p in range(Nc):
        i0 = ifp[p]
        if refined[p]:
            W[p, i0:i0 + 3] = (0.25, 0.5, 0.25)
        else:
            W[p, i0:i0 + 2] = (0.5, 0.5)
    return W


class TwoGrid:
    """Two-grid preconditioner x = TG(r) with a pluggable coarse solver."""

    def __init__(self, A_fine, P, A_coarse, coarse_solve, nu, omega_jac):
        self.A = A_fine.tocsr()
        self.P = P.tocsr()
        self.R = self.P.T.tocsr()
        self.Ac = A_coarse
        self.coarse_solve = coarse_solve
        self.nu = nu
        self.wj = omega_jac
        self.dinv = 1.0 / self.A.diagonal()

    def smooth(self, x, r, steps):
        """omega-Jacobi: x <- x + omega D^{-1} (r - A x), ``steps`` times."""
        for _ in range(steps):
            x = x + self.wj * self.dinv * (r - self.A @ x)
        return x

    def apply(self, r):
        r = np.asarray(r, dtype=complex).ravel()
        x = self.smooth(np.zeros_like(r), r, self.nu)
        rc = self.R @ (r - self.A @ x)
        ec = self.coarse_solve(rc)
        x = x + self.P @ np.asarray(ec).ravel()
        x = self.smooth(x, r, self.nu)
        return x
