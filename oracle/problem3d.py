"""Setup / apply / solve driver of the oracle in three dimensions.

Same method as ``problem`` (Sec. 2-4), on a box: -Laplace u - k^2 u = f with
PML layers on every face and homogeneous Dirichlet values outside.  The mesh
has N_a = n_a + 1 + 2 w_a cells per axis, spacing h, unknown nodes
1..N_a - 1; ``c`` is given at all unknown nodes, shape (N1-1, N2-1, N3-1), x
(the sweep axis) slowest and z fastest.

Operators (FE scaled, i.e. multiplied by h^3):
* fine level: the standard 7-point PML finite differences (``fine='fd7'``,
  the 3-D form of eq. define_pml_fd, the paper's fine level) or the 27-point
  finite-element form with Table (b) coefficients at the fine 1/G
  (``fine='fe27'``);
* coarse level (two-grid, Sec. 4): the 27-point finite-element operator of
  eq. define_H_FE with eq. def_IJ_opt and Table (b) at the coarse 1/G, on the
  mesh that is not coarsened inside the PML layers;
* domain decomposition (Sec. 2.2): slabs of x layers, each layer an
  (n2 x n3) plane; the sweeps of Tables 2 and 3 are the same code as in 2-D
  with a layer of n2 n3 unknowns.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import discretization as D
from . import dd as DD
from . import twogrid as TG
from .krylov import fgmres


def pad_nodes_edge_3d(v):
    """Unknown-node values (N1-1, N2-1, N3-1) extended to all nodes by
    copying the nearest unknown node (medium only)."""
    return np.pad(v, 1, mode="edge")


def node_to_cell_average_3d(k2_full):
    """Cell values as the mean of the 8 corner nodes of each cell."""
    a = k2_full
    return 0.125 * (a[:-1, :-1, :-1] + a[1:, :-1, :-1] + a[:-1, 1:, :-1] + a[1:, 1:, :-1]
                    + a[:-1, :-1, 1:] + a[1:, :-1, 1:] + a[:-1, 1:, 1:] + a[1:, 1:, 1:])


class Level3D:
    """One discretization level: three axes, the operator kind and its medium."""

    def __init__(self, ax, ay, az, omega, kind, k2_nodes=None, k2_cells=None):
        self.ax, self.ay, self.az, self.omega, self.kind = ax, ay, az, omega, kind
        self.k2_nodes = k2_nodes
        self.k2_cells = k2_cells
        self.n1, self.n2, self.n3 = ax.n_unknowns, ay.n_unknowns, az.n_unknowns

    def coefs(self):
        return D.cell_coefs_3d(self.k2_cells, self.ax.h_nom, "opt")

    def matrix(self):
        if self.kind == "fd7":
            return D.fd7_matrix(self.ax, self.ay, self.az, self.k2_nodes, self.omega)
        return D.fe27_matrix(self.ax, self.ay, self.az, self.k2_cells, self.coefs(), self.omega)

    def slab_level(self, beta, j, w, strength, c_pml):
        """Level of subdomain j (Sec. 2.1): x layers x0..x1, DD-PML of
        thickness w h_nom beyond b_j = x_{beta_j + 1/2} and before
        b~_{j-1} = x_{beta_{j-1} - 1/2}, k continued from the core boundary
        into the added layers (copied along x, per (y, z) line)."""
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
        if self.kind == "fd7":
            lo = beta[j - 1] if j > 1 else 1
            hi = beta[j] if j < J else self.n1
            src = np.clip(np.arange(x0, x1 + 1), lo, hi)
            return Level3D(sax, self.ay, self.az, self.omega, "fd7", k2_nodes=self.k2_nodes[src - 1])
        lo = beta[j - 1] - 1 if j > 1 else 0
        hi = beta[j] if j < J else self.ax.n_cells - 1
        src = np.clip(np.arange(x0 - 1, x1 + 1), lo, hi)
        return Level3D(sax, self.ay, self.az, self.omega, "fe27", k2_cells=self.k2_cells[src])


def make_sweep3d(level, J, w, strength, c_pml, w_outer):
    beta = DD.partition(level.n1, w_outer, J)
    ext = [DD.slab_extent(beta, j, w) for j in range(1, J + 1)]
    for j in range(1, J + 1):
        if beta[j] - beta[j - 1] < 3:
            raise ValueError("core thinner than 3 layers")
    if J > 1 and (ext[1][0] < 1 or ext[-2][1] > level.n1):
        raise ValueError("DD-PML layers leave the domain")

    def slab_matrix(j):
        return level.slab_level(beta, j, w, strength, c_pml).matrix()

    return DD.SweepDD(level.matrix(), level.n1, level.n2 * level.n3, beta, ext, slab_matrix)


def cell_average_3d(W1, W2, W3, v_full):
    """Tensor product of the 1-D averages (App. A, coarse level): cell value
    (a, b, c) = sum W1[a, i] W2[b, j] W3[c, k] v[i, j, k]."""
    t = np.tensordot(W1, v_full, axes=(1, 0))            # (Nc1, N2+1, N3+1)
    t = np.tensordot(W2, t, axes=(1, 1))                 # (Nc2, Nc1, N3+1)
    t = np.tensordot(W3, t, axes=(1, 2))                 # (Nc3, Nc2, Nc1)
    return np.transpose(t, (2, 1, 0))


class Problem3D:
    def __init__(self, c, omega, h, w_outer, S_outer=None, c_pml=None, J=4, w_dd=3,
                 S_dd=None, fine="fd7", two_grid=False, nu=3, omega_jac=0.6,
                 sweep="x", coarse="sweep", ncell=2):
        c = np.asarray(c, dtype=float)
        ws = (w_outer,) * 3 if np.isscalar(w_outer) else tuple(w_outer)
        Ns = [s + 1 for s in c.shape]
        self.omega, self.h = omega, h
        self.c_pml = float(c.mean()) if c_pml is None or c_pml <= 0 else float(c_pml)
        S_o = 5.0 * max(ws) if S_outer is None else S_outer
        S_dd = 5.0 * w_dd if S_dd is None or S_dd <= 0 else S_dd
        axes = [D.uniform_axis(N, h, w, S_o, self.c_pml) for N, w in zip(Ns, ws)]
        k2n = omega ** 2 / c ** 2
        if fine == "fd7":
            self.fine = Level3D(*axes, omega, "fd7", k2_nodes=k2n)
        else:
            k2c = node_to_cell_average_3d(pad_nodes_edge_3d(k2n))
            self.fine = Level3D(*axes, omega, "fe27", k2_cells=k2c)
        self.A = self.fine.matrix().tocsr()
        self.rhs_scale = D.fd7_rhs_scale(*axes, omega)
        self.shape = c.shape
        if two_grid:
            cax, Ws, Ps = [], [], []
            for a, w, N in zip(axes, ws, Ns):
                ca, ifp, ref = TG.coarsen_axis(a, w)
                cax.append(ca)
                Ws.append(TG.cell_average_1d(ifp, ref, N))
                Ps.append(TG.prolongation_1d(ifp, ref, N))
            k2c = cell_average_3d(*Ws, pad_nodes_edge_3d(k2n))
            self.coarse = Level3D(*cax, omega, "fe27", k2_cells=k2c)
            P = sp.kron(Ps[0], sp.kron(Ps[1], Ps[2]))
            Ac = self.coarse.matrix().tocsc()
            if coarse == "exact":
                csolve = spla.splu(Ac).solve
                self.dd = None
            else:
                self.dd = make_sweep3d(self.coarse, J, w_dd, S_dd, self.c_pml, ws[0])
                csolve = self._sweep_map(sweep, ncell)
            self.tg = TG.TwoGrid(self.A, P, Ac, lambda r: csolve(r).ravel(), nu, omega_jac)
            self.P = P
            self.precond = self.tg.apply
        else:
            self.coarse = None
            self.dd = make_sweep3d(self.fine, J, w_dd, S_dd, self.c_pml, ws[0])
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
