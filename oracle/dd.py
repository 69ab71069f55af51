"""Double-sweep domain decomposition with PML transmission (oracle).

Follows Sec. 2.2 (discrete formulation) and the procedures of Tables 2 and 3
(SubdomSolve, ForwardSweep, BackwardSweep, MidSolveIn, MidSolveOut,
SweepingPrecUD, SweepingPrecX).

Layers are the unknown node planes x = const, numbered 1..n1 (global).  A
vector is an (n1, n2) array, layer i = row i-1.  The subdomain boundaries
b_j, b~_j sit at half nodes beta_j + 1/2 and beta~_j + 1/2 with
beta~_j = beta_j - 1 for 0 < j < J (Sec. 2.2).  Subdomain j spans layers
x0_j..x1_j: its core beta_{j-1}..beta_j plus w DD-PML layers on each side
that has a neighbour.  Missing transmission data (a buffer never written)
is zero, and T^(1) = T~^(J) = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def partition(n1, w_outer, J):
    """Subdomain boundaries beta_0..beta_J on the n1 unknown layers.

    The outer-PML layers join the first and last cores and the
    n1 - 2 w_outer interior layers are split as evenly as integer division
    allows: beta_j = w_outer + floor((j n_int + floor(J/2)) / J)."""
    n_int = n1 - 2 * w_outer
    beta = [0]
    for j in range(1, J):
        beta.append(w_outer + (j * n_int + J // 2) // J)
    beta.append(n1)
    return beta


def beta_tilde(beta):
    """beta~_0 = beta_0, beta~_J = beta_J, beta~_j = beta_j - 1 otherwise."""
    J = len(beta) - 1
    return [beta[0]] + [beta[j] - 1 for j in range(1, J)] + [beta[J]]


def slab_extent(beta, j, w):
    """First and last global layer of subdomain j (1-based j)."""
    J = len(beta) - 1
    x0 = 1 if j == 1 else beta[j - 1] - w
    x1 = beta[J] if j == J else beta[j] + w
    return x0, x1


class SweepDD:
    """Discrete sweeping preconditioner on one level.

    ``A``            global sparse matrix (n1*n2 square), layer-major.
    ``n1, n2``       number of layers and unknowns per layer.
    ``beta``         partition beta_0..beta_J.
    ``extents``      list of (x0, x1) per subdomain.
    ``slab_matrix``  callable j -> sparse matrix of A^(j) on layers x0..x1.
    """

    def __init__(self, A, n1, n2, beta, extents, slab_matrix):
        self.A = A.tocsr()
        self.n1, self.n2 = n1, n2
        self.beta = list(beta)
        self.bt = beta_tilde(beta)
        self.J = len(beta) - 1
        self.extents = list(extents)
        self.lu = []
        for j in range(1, self.J + 1):
            Aj = slab_matrix(j).tocsc()
            self.lu.append(spla.splu(Aj))

    # ---- index helpers ---------------------------------------------------
    def block(self, p, q):
        """n2 x n2 block A_{p,q} of the global matrix between layers p, q."""
        n2 = self.n2
        return self.A[(p - 1) * n2:p * n2, (q - 1) * n2:q * n2]

    # ---- SubdomSolve (Table 2) -------------------------------------------
    def subdom_solve(self, u, f, j, a, b, at, bt, t1, B1, t2, t3, B3, t4):
        """One subdomain solve and update.  Returns (B2, B4): the outgoing
        forward transmission layers (beta_j, beta_j+1) if t2 and the
        outgoing backward layers (beta~_{j-1}, beta~_{j-1}+1) if t4."""
        x0, x1 = self.extents[j - 1]
        nl = x1 - x0 + 1
        fd = np.zeros((nl, self.n2), dtype=complex)
        # f_d = J(j,a,b) f : layers a+1..b
        for g in range(a + 1, b + 1):
            fd[g - x0] += f[g - 1]
        # f_d += (J_in)^t T^(j) B1 : layers beta_{j-1}, beta_{j-1}+1
        if t1 and B1 is not None:
            be = self.beta[j - 1]
            fd[be - x0] += self.block(be, be + 1) @ B1[1]
            fd[be + 1 - x0] -= self.block(be + 1, be) @ B1[0]
        # f_d += (J~_in)^t T~^(j) B3 : layers beta~_j, beta~_j+1
        if t3 and B3 is not None:
            bb = self.bt[j]
            fd[bb - x0] -= self.block(bb, bb + 1) @ B3[1]
            fd[bb + 1 - x0] += self.block(bb + 1, bb) @ B3[0]
        ud = self.lu[j - 1].solve(fd.ravel()).reshape(nl, self.n2)
        # u += J(j, a~, b~)^T u_d : layers a~+1..b~
        for g in range(at + 1, bt + 1):
            u[g - 1] += ud[g - x0]
        B2 = B4 = None
        if t2:
            be = self.beta[j]
            B2 = np.array([ud[be - x0], ud[be + 1 - x0]])
        if t4:
            bb = self.bt[j - 1]
            B4 = np.array([ud[bb - x0], ud[bb + 1 - x0]])
        return B2, B4

    # ---- helper procedures (Table 2) -----------------------------------
    def forward_sweep(self, u, f, j0, j1, B):
        J, be = self.J, self.beta
        for j in range(j0, j1 + 1):
            B2, _ = self.subdom_solve(u, f, j, be[j - 1], be[j], be[j - 1], be[j],
                                      j > 1, B, j < J, False, None, False)
            if j < J:
                B = B2
        return B

    def backward_sweep(self, u, f, j0, j1, B):
        J, bt = self.J, self.bt
        for j in range(j0, j1 - 1, -1):
            _, B4 = self.subdom_solve(u, f, j, bt[j - 1], bt[j], bt[j - 1], bt[j],
                                      False, None, False, j < J, B, j > 1)
            if j > 1:
                B = B4
        return B

    def mid_solve_in(self, u, f, j, B1, B2):
        be, bt = self.beta, self.bt
        self.subdom_solve(u, f, j, be[j - 1], bt[j], be[j - 1], bt[j],
                          j > 1, B1, False, j < self.J, B2, False)

    def mid_solve_out(self, u, f, j):
        """Returns (forward-out buffer, backward-out buffer).  An outgoing
        buffer toward a missing neighbour (j = 1 or j = J) is not formed."""
        be, bt = self.beta, self.bt
        return self.subdom_solve(u, f, j, bt[j - 1], be[j], bt[j - 1], be[j],
                                 False, None, j < self.J, False, None, j > 1)

    # ---- the preconditioners (Table 3) ----------------------------------
    def residual(self, f, u):
        return f - (self.A @ u.ravel()).reshape(u.shape)

    def apply_ud(self, f):
        """SweepingPrecUD: forward sweep, residual, backward sweep."""
        f = f.reshape(self.n1, self.n2)
        u = np.zeros_like(f, dtype=complex)
        self.forward_sweep(u, f, 1, self.J, None)
        g = self.residual(f, u)
        self.backward_sweep(u, g, self.J, 1, None)
        return u

    def j_mid(self):
        """Intersection subdomain; J/2 + 1 for even J (Sec. 2.1), floor(J/2)+1
        in general."""
        return self.J // 2 + 1

    def apply_x(self, f):
        """SweepingPrecX: simultaneous sweeps meeting at j_mid."""
        f = f.reshape(self.n1, self.n2)
        u = np.zeros_like(f, dtype=complex)
        J, jm = self.J, self.j_mid()
        B1 = self.forward_sweep(u, f, 1, jm - 1, None)
        B2 = self.backward_sweep(u, f, J, jm + 1, None)
        self.mid_solve_in(u, f, jm, B1, B2)
        g = self.residual(f, u)
        # MidSolveOut(u, g, j_mid, B2, B1): its forward output feeds the
        # forward sweep to the right, its backward output the backward sweep
        # to the left.
        Bf, Bb = self.mid_solve_out(u, g, jm)
        self.backward_sweep(u, g, jm - 1, 1, Bb)
        self.forward_sweep(u, g, jm + 1, J, Bf)
        return u

    def nx_cells(self, ncell):
        """Groups of the partial sweeps (Sec. 2.2, SweepingPrecNX): boundary
        subdomains j_cell,m = round(m (J + 1) / N_cell) for 0 < m < N_cell,
        with j_cell,0 = 0 and j_cell,N_cell = J + 1 (the paper writes -1 for
        j_cell,0, which would start the first sweep at subdomain 0; read as
        0), and the centre j_mid,m = floor((j_cell,m-1 + j_cell,m + 1) / 2)
        of the subdomains strictly between two boundaries.  N_cell = 1 gives
        the X-sweep's j_mid.  Every group needs at least one subdomain."""
        J, N = self.J, ncell
        if N < 1 or 2 * N - 1 > J:
            raise ValueError("NX-sweep needs 1 <= N_cell and 2 N_cell - 1 <= J")
        jc = [0] + [(m * (J + 1) + N // 2) // N for m in range(1, N)] + [J + 1]
        if any(jc[m] - jc[m - 1] < 2 for m in range(1, N + 1)):
            raise ValueError("a group of the NX-sweep has no subdomain")
        jm = [None] + [(jc[m - 1] + jc[m] + 1) // 2 for m in range(1, N + 1)]
        return jc, jm

    def apply_nx(self, f, ncell):
        """SweepingPrecNX: X-sweeps over N_cell groups of subdomains, coupled
        through the boundary subdomains between the groups.  The groups are
        independent within each half (the partial sweeps are meant to run in
        parallel), so the order taken is: the boundary subdomains'
        MidSolveOut, the sweeps of every group and its MidSolveIn; the
        residual; every group's MidSolveOut and outward sweeps; then the
        boundary subdomains' MidSolveIn, which needs the sweeps of both
        neighbouring groups.  Buffer B_{2m-1} carries the forward data of
        group m, B_{2m} its backward data."""
        f = f.reshape(self.n1, self.n2)
        u = np.zeros_like(f, dtype=complex)
        jc, jm = self.nx_cells(ncell)
        N = ncell
        fwd_in = [None] * (N + 2)   # B_{2m-1} entering group m from the left
        bwd_in = [None] * (N + 2)   # B_{2m} entering group m from the right
        for m in range(1, N):       # boundary subdomains, first half
            fo, bo = self.mid_solve_out(u, f, jc[m])
            fwd_in[m + 1] = fo
            bwd_in[m] = bo
        for m in range(1, N + 1):
            B1 = self.forward_sweep(u, f, jc[m - 1] + 1, jm[m] - 1, fwd_in[m])
            B2 = self.backward_sweep(u, f, jc[m] - 1, jm[m] + 1, bwd_in[m])
            self.mid_solve_in(u, f, jm[m], B1, B2)
        g = self.residual(f, u)
        left_of = [None] * (N + 2)  # forward data arriving at boundary j_cell,m
        right_of = [None] * (N + 2)  # backward data arriving at boundary j_cell,m
        for m in range(1, N + 1):
            fo, bo = self.mid_solve_out(u, g, jm[m])
            right_of[m - 1] = self.backward_sweep(u, g, jm[m] - 1, jc[m - 1] + 1, bo)
            left_of[m] = self.forward_sweep(u, g, jm[m] + 1, jc[m] - 1, fo)
        for m in range(1, N):       # boundary subdomains, second half
            self.mid_solve_in(u, g, jc[m], left_of[m], right_of[m])
        return u

    # ---- written layer ranges (for the partition check) -------------------
    def written_ranges(self, kind):
        """Layer ranges (a~+1..b~) written by each solve of one preconditioner
        application, split into the two halves around g = f - A u."""
        J, be, bt, jm = self.J, self.beta, self.bt, self.j_mid()
        if kind == "ud":
            first = [(be[j - 1] + 1, be[j]) for j in range(1, J + 1)]
            second = [(bt[j - 1] + 1, bt[j]) for j in range(J, 0, -1)]
        else:
            first = ([(be[j - 1] + 1, be[j]) for j in range(1, jm)]
                     + [(bt[j - 1] + 1, bt[j]) for j in range(J, jm, -1)]
                     + [(be[jm - 1] + 1, bt[jm])])
            second = ([(bt[jm - 1] + 1, be[jm])]
                      + [(bt[j - 1] + 1, bt[j]) for j in range(jm - 1, 0, -1)]
                      + [(be[j - 1] + 1, be[j]) for j in range(jm + 1, J + 1)])
        return first, second
