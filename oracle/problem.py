"""Setup / apply / solve driver of the oracle, mirroring the GPU library.

Problem (Sec. 1, Sec. 2.1): -Laplace u - k^2 u = f, k = omega / c, on a
rectangle with PML layers and homogeneous Dirichlet values outside.  The
mesh has N = n + 1 + 2 w cells per axis (n interior nodes, w outer-PML cells
per side), spacing h, unknown nodes 1..N-1.  ``c`` is given at all unknown
nodes (PML nodes included), shape (N1-1, N2-1).

Preconditioners:
* one-level: the X (or UD) sweep on the fine operator itself;
* two-grid (TGSP, Sec. 4): omega-Jacobi on the fine operator, coarse level
  = optimized finite elements on the PML-aware coarse mesh (App. A), coarse
  solve = one X (or UD) sweep application, or an exact solve.

Fine operator: the 5-point PML FD of eq. define_pml_fd (``fine='fd5'``) or
the finite-element 9-point form with Table (a) coefficients at the fine
1/G (``fine='fe9'``).  Both are FE scaled (multiplied by h^2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import discretization as D
from . import dd as DD
from . import twogrid as TG
from .krylov import fgmres


class Level2D:
    """One discretization level: axes, coefficients, operator kind."""

    def __init__(self, ax, ay, omega, kind, k2_nodes=None, k2_cells=None, k2_coef_cells=None):
        self.ax, self.ay, self.omega, self.kind = ax, ay, omega, kind
        self.k2_nodes = k2_nodes
        self.k2_cells = k2_cells
        # real cell k^2 the Table (a) coefficients are taken at (the k^2 of
        # the operator itself is complex inside sponge layers)
        self.k2_coef_cells = k2_coef_cells
        self.n1, self.n2 = ax.n_unknowns, ay.n_unknowns

    def coefs(self, k2_cells=None):
        if k2_cells is None:
            k2_cells = self.k2_cells if self.k2_coef_cells is None else self.k2_coef_cells
        return D.cell_coefs_2d(k2_cells, self.ax.h_nom, "opt")

    def matrix(self):
        if self.kind == "fd5":
            return D.fd5_matrix(self.ax, self.ay, self.k2_nodes, self.omega)
        return D.fe9_matrix(self.ax, self.ay, self.k2_cells, self.coefs(), self.omega)

    def slab_level(self, beta, j, w, strength, c_pml):
        """Level of subdomain j (Sec. 2.1, subdomains): layers x0..x1, DD-PML
        of thickness w h_nom beyond b_j = x_{beta_j + 1/2} and before
        b~_{j-1} = x_{beta_{j-1} - 1/2}, k continued as a constant (per row)
        from the core boundary into the added layers."""
        J = len(beta) - 1
        x0, x1 = DD.slab_extent(beta, j, w)
        gx = self.ax.x
        loc_x = gx[x0 - 1:x1 + 2]
        d = w * self.ax.h_nom
        C = strength * c_pml / d ** 3
        bl = 0.5 * (gx[beta[j - 1] - 1] + gx[beta[j - 1]]) if j > 1 else None
        br = 0.5 * (gx[beta[j]] + gx[beta[j] + 1]) if j < J else None
        gsig = self.ax.sigma

        def sig(x):
            x = np.asarray(x, dtype=float)
            s = gsig(x)
            if bl is not None:
                s = np.where(x < bl, C * (bl - x) ** 2, s)
            if br is not None:
                s = np.where(x > br, C * (x - br) ** 2, s)
            return s

        sax = D.Axis(loc_x, sig, self.ax.h_nom)
        if self.kind == "fd5":
            lo = beta[j - 1] if j > 1 else 1
            hi = beta[j] if j < J else self.n1
            src = np.clip(np.arange(x0, x1 + 1), lo, hi)
            return Level2D(sax, self.ay, self.omega, "fd5", k2_nodes=self.k2_nodes[src - 1])
        lo = beta[j - 1] - 1 if j > 1 else 0
        hi = beta[j] if j < J else self.ax.n_cells - 1
        src = np.clip(np.arange(x0 - 1, x1 + 1), lo, hi)
        kc = None if self.k2_coef_cells is None else self.k2_coef_cells[src]
        return Level2D(sax, self.ay, self.omega, "fe9", k2_cells=self.k2_cells[src], k2_coef_cells=kc)


def make_sweep(level, J, w, strength, c_pml, w_outer):
    beta = DD.partition(level.n1, w_outer, J)
    ext = [DD.slab_extent(beta, j, w) for j in range(1, J + 1)]
    for j in range(1, J + 1):
        if beta[j] - beta[j - 1] < 3:
            raise ValueError("core thinner than 3 layers")
    if J > 1 and (ext[1][0] < 1 or ext[-2][1] > level.n1):
        raise ValueError("DD-PML layers leave the domain")

    def slab_matrix(j):
        return level.slab_level(beta, j, w, strength, c_pml).matrix()

    return DD.SweepDD(level.matrix(), level.n1, level.n2, beta, ext, slab_matrix)


class Problem2D:
    def __init__(self, c, omega, h, w_outer, S_outer=None, c_pml=None, J=4, w_dd=4,
                 S_dd=None, fine="fd5", two_grid=False, nu=3, omega_jac=0.8,
                 sweep="x", coarse="sweep", ncell=2, boundary="pml"):
        """``boundary``: 'pml' (outer PML layers of w_outer cells) or 'sponge'
        (sponge layers of w_outer cells, Sec. 2.1: k -> k (1 + i beta), no
        PML; S_outer then gives beta at the outer edge, None selects
        sponge_beta_default).  With sponge layers the two-grid method uses
        the standard coarsening of every cell (Sec. 4, the two-grid method in
        absence of PML layers: full weighting R = P^T, linear P) and the
        partition spreads the cores over all layers."""
        c = np.asarray(c, dtype=float)
        wx, wy = (w_outer, w_outer) if np.isscalar(w_outer) else tuple(w_outer)
        N1, N2 = c.shape[0] + 1, c.shape[1] + 1
        self.omega, self.h = omega, h
        self.c_pml = float(c.mean()) if c_pml is None or c_pml <= 0 else float(c_pml)
        S_dd = 5.0 * w_dd if S_dd is None or S_dd <= 0 else S_dd
        k2u = omega ** 2 / c ** 2
        sponge = boundary == "sponge"
        if sponge:
            ax = D.uniform_axis(N1, h, 0, 0.0, self.c_pml)
            ay = D.uniform_axis(N2, h, 0, 0.0, self.c_pml)
            bmax = [S_outer if S_outer is not None and S_outer > 0 else
                    (D.sponge_beta_default(omega, self.c_pml, wa, h) if wa > 0 else 0.0) for wa in (wx, wy)]
            bx = D.sponge_profile(N1, h, wx, bmax[0])[1:-1]
            by = D.sponge_profile(N2, h, wy, bmax[1])[1:-1]
            k2n = k2u * (1.0 + 1j * (bx[:, None] + by[None, :])) ** 2
            dd_outer = 0
        elif boundary == "pml":
            S_o = 5.0 * max(wx, wy) if S_outer is None else S_outer
            ax = D.uniform_axis(N1, h, wx, S_o, self.c_pml)
            ay = D.uniform_axis(N2, h, wy, S_o, self.c_pml)
            k2n = k2u
            dd_outer = wx
        else:
            raise ValueError(f"unknown boundary {boundary}")
        if fine == "fd5":
            self.fine = Level2D(ax, ay, omega, "fd5", k2_nodes=k2n)
        else:
            k2c = D.node_to_cell_average_2d(D.pad_nodes_edge(k2n))
            k2cu = D.node_to_cell_average_2d(D.pad_nodes_edge(k2u)) if sponge else None
            self.fine = Level2D(ax, ay, omega, "fe9", k2_cells=k2c, k2_coef_cells=k2cu)
        self.A = self.fine.matrix().tocsr()
        self.rhs_scale = D.fd5_rhs_scale(ax, ay, omega)
        self.shape = c.shape
        self.sweep_kind = sweep
        if two_grid:
            cwx, cwy = (0, 0) if sponge else (wx, wy)  # cells that are not coarsened
            cax, ifx, rfx = TG.coarsen_axis(ax, cwx)
            cay, ify, rfy = TG.coarsen_axis(ay, cwy)
            W1 = TG.cell_average_1d(ifx, rfx, N1)
            W2 = TG.cell_average_1d(ify, rfy, N2)
            k2c = W1 @ D.pad_nodes_edge(k2n) @ W2.T
            k2cu = W1 @ D.pad_nodes_edge(k2u) @ W2.T if sponge else None
            self.coarse = Level2D(cax, cay, omega, "fe9", k2_cells=k2c, k2_coef_cells=k2cu)
            P = sp.kron(TG.prolongation_1d(ifx, rfx, N1), TG.prolongation_1d(ify, rfy, N2))
            Ac = self.coarse.matrix().tocsc()
            if coarse == "exact":
                lu = spla.splu(Ac)
                csolve = lu.solve
                self.dd = None
            else:
                self.dd = make_sweep(self.coarse, J, w_dd, S_dd, self.c_pml, dd_outer)
                csolve = self._sweep_map(sweep, ncell)
            self.tg = TG.TwoGrid(self.A, P, Ac, lambda r: csolve(r).ravel(), nu, omega_jac)
            self.precond = self.tg.apply
        else:
            self.coarse = None
            self.dd = make_sweep(self.fine, J, w_dd, S_dd, self.c_pml, dd_outer)
            ap = self._sweep_map(sweep, ncell)
            self.precond = lambda r: ap(r).ravel()

    def _sweep_map(self, sweep, ncell):
        """The sweep of Table 3: 'x' (SweepingPrecX), 'ud' (SweepingPrecUD)
        or 'nx' (SweepingPrecNX over ncell groups)."""
        if sweep == "x":
            return self.dd.apply_x
        if sweep == "ud":
            return self.dd.apply_ud
        if sweep == "nx":
            self.dd.nx_cells(ncell)  # validates the groups
            return lambda f: self.dd.apply_nx(f, ncell)
        raise ValueError(f"unknown sweep {sweep}")

    def rhs(self, f):
        return (self.rhs_scale * np.asarray(f).reshape(self.shape)).ravel()

    def matvec(self, x):
        return self.A @ x

    def solve(self, f, tol=1e-6, maxit=200, restart=None, callback=None):
        b = self.rhs(f)
        return fgmres(self.matvec, self.precond, b, tol=tol, maxit=maxit,
                      restart=restart, callback=callback)

    def direct(self, f):
        return spla.splu(self.A.tocsc()).solve(self.rhs(f))
