"""Discrete Helmholtz operators with PML (oracle, complex128).

Conventions
-----------
* Time factor exp(-i omega t); outgoing waves behave like exp(+i k r).
* An axis with N cells has nodes 0..N; nodes 0 and N carry homogeneous
  Dirichlet values, the unknowns are nodes 1..N-1 (Sec. 2.2, discrete
  formulation).  Cell p lies between nodes p and p+1.
* 2-D unknown (i, k) (x index i, y index k, both 1-based) has flat index
  (i-1)*(N2-1) + (k-1): x is the slowest axis, the sweep axis.
* "FE scaling": every operator here is the FD operator multiplied by h^dim,
  as the paper does for the fine level of its two-grid method (App. A,
  coarse level optimized finite elements).  The right-hand side is scaled
  the same way.

PML (Sec. 2.1): d/dx -> alpha d/dx with alpha = 1/(1 + i sigma/omega) and
sigma = C * dist^2 inside a layer, C = S_pml * c_pml / d_pml^3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# --------------------------------------------------------------------------
# Optimized finite-difference coefficients, App. A, Table "optFD_coeff".
# Columns: 1/G_k, then c_1..c_3 (2-D, table (a)) or c_1..c_5 (3-D, table (b)).
# --------------------------------------------------------------------------
OPT_TABLE_2D = np.array([
    [0.00, 0.61953, 0.45295, 0.77363],
    [0.04, 0.63691, 0.47535, 0.87242],
    [0.08, 0.62988, 0.48633, 0.86400],
    [0.12, 0.62610, 0.48880, 0.84984],
    [0.16, 0.62289, 0.48759, 0.83017],
    [0.20, 0.62596, 0.47106, 0.80852],
    [0.24, 0.62213, 0.46478, 0.78215],
    [0.28, 0.61036, 0.47016, 0.74857],
    [0.32, 0.59107, 0.48468, 0.70553],
    [0.36, 0.56369, 0.50746, 0.65062],
    [0.40, 0.52412, 0.54163, 0.57676],
])

OPT_TABLE_3D = np.array([
    [0.00, 0.56428, 0.35970, 0.20490, 0.77998, 0.17505],
    [0.04, 0.56571, 0.36071, 0.20541, 0.78635, 0.17442],
    [0.08, 0.56298, 0.36150, 0.20719, 0.78273, 0.16881],
    [0.12, 0.56540, 0.35620, 0.20287, 0.76438, 0.18678],
    [0.16, 0.56370, 0.35299, 0.20299, 0.74684, 0.19603],
    [0.20, 0.55813, 0.35277, 0.20452, 0.72755, 0.20131],
    [0.24, 0.54673, 0.35830, 0.20693, 0.70298, 0.20847],
    [0.28, 0.52423, 0.38368, 0.19633, 0.66863, 0.22424],
    [0.32, 0.49946, 0.39740, 0.20725, 0.62734, 0.23845],
    [0.36, 0.47567, 0.40216, 0.22132, 0.58198, 0.25329],
    [0.40, 0.45011, 0.36784, 0.29962, 0.53417, 0.23589],
])

# The 5-point (2-D) scheme written in the same family: all mass on the
# centre node (c1 = 1, c2 = 0) and no cross stiffness (c3 = 1).
FIVE_POINT_COEFS_2D = (1.0, 0.0, 1.0)


def opt_coefs_2d(inv_g):
    """c_1, c_2, c_3 at 1/G by linear interpolation in Table (a) (App. A,
    optimized finite differences).  1/G is clamped to the table range
    [0, 0.40].  Returns three arrays shaped like ``inv_g``."""
    x = np.clip(np.asarray(inv_g, dtype=float), OPT_TABLE_2D[0, 0], OPT_TABLE_2D[-1, 0])
    return tuple(np.interp(x, OPT_TABLE_2D[:, 0], OPT_TABLE_2D[:, j]) for j in (1, 2, 3))


def opt_coefs_3d(inv_g):
    """c_1..c_5 at 1/G by linear interpolation in Table (b), clamped."""
    x = np.clip(np.asarray(inv_g, dtype=float), OPT_TABLE_3D[0, 0], OPT_TABLE_3D[-1, 0])
    return tuple(np.interp(x, OPT_TABLE_3D[:, 0], OPT_TABLE_3D[:, j]) for j in range(1, 6))


def fe_constants_2d(c1, c2, c3):
    """2-D analogue of eq. def_IJ_opt: integrals I_0..I_2, J_0..J_1 that make
    the finite-element rows equal h^2 times the optimized FD rows.

    Mass:  I_0 = c1/4, I_1 = c2/8, I_2 = (1 - c1 - c2)/4  (4, 2, 1 cells)
    Stiff: J_0 = c3/2, J_1 = (1 - c3)/2                   (2, 1 cells)
    """
    return (c1 / 4.0, c2 / 8.0, (1.0 - c1 - c2) / 4.0), (c3 / 2.0, (1.0 - c3) / 2.0)


# --------------------------------------------------------------------------
# PML profiles (Sec. 2.1)
# --------------------------------------------------------------------------
def alpha_of_sigma(sigma, omega):
    """alpha = 1 / (1 + i sigma / omega)."""
    return 1.0 / (1.0 + 1j * np.asarray(sigma, dtype=float) / omega)


class Axis:
    """One axis of a rectilinear mesh.

    ``x``      node coordinates, length N+1 (nodes 0..N).
    ``sigma``  vectorised callable: PML damping sigma(x) (0 outside layers).
    ``h_nom``  nominal spacing of the level (used for 1/G of the optimized
               coefficients and for the DD-PML thickness).
    """

    def __init__(self, x, sigma, h_nom):
        self.x = np.asarray(x, dtype=float)
        self.sigma = sigma
        self.h_nom = float(h_nom)

    @property
    def n_cells(self):
        return len(self.x) - 1

    @property
    def n_unknowns(self):
        return len(self.x) - 2

    def widths(self):
        return np.diff(self.x)

    def mid(self):
        return 0.5 * (self.x[:-1] + self.x[1:])

    def alpha_nodes(self, omega):
        return alpha_of_sigma(self.sigma(self.x), omega)

    def alpha_cells(self, omega):
        """alpha at cell midpoints = at half nodes i+1/2."""
        return alpha_of_sigma(self.sigma(self.mid()), omega)


def outer_pml_sigma(x_lo, x_hi, width, strength, c_pml):
    """sigma(x) for PML layers of thickness ``width`` outside [x_lo, x_hi]:
    C (x_lo - x)^2 left of x_lo, C (x - x_hi)^2 right of x_hi, 0 between, with
    C = S c_pml / d^3 (Sec. 2.1).  ``width`` <= 0 gives no PML."""
    if width <= 0:
        return lambda x: np.zeros_like(np.asarray(x, dtype=float))
    C = strength * c_pml / width ** 3

    def sig(x):
        x = np.asarray(x, dtype=float)
        return C * (np.maximum(x_lo - x, 0.0) ** 2 + np.maximum(x - x_hi, 0.0) ** 2)

    return sig


def sponge_profile(n_cells, h, width, beta_max):
    """Sponge layers (Sec. 2.1): k is replaced by k (1 + i beta) with beta
    continuous and quadratically increasing over ``width`` cells from each
    end, beta = beta_max (dist / d)^2, d = width h.  Returns beta at the nodes
    0..N of the axis (0 in the interior)."""
    x = h * np.arange(n_cells + 1)
    if width <= 0:
        return np.zeros_like(x)
    d = width * h
    dist = np.maximum(np.maximum(d - x, x - (n_cells - width) * h), 0.0)
    return beta_max * (dist / d) ** 2


def sponge_beta_default(omega, c_ref, width, h):
    """beta_max for which a wave crossing the layer once is damped by about
    1e-2 (round trip 1e-4, the middle of the paper's 1e-2..1e-4): with
    beta = beta_max (s/d)^2 the damping is exp(-k beta_max d / 3)."""
    k = omega / c_ref
    return 3.0 * np.log(100.0) / (k * width * h)


def uniform_axis(n_cells, h, pml_cells, strength, c_pml):
    """Uniform axis with ``pml_cells`` outer PML cells on each side.  The PML
    onset is node ``pml_cells`` (and node N - pml_cells); d_pml = pml_cells*h."""
    x = h * np.arange(n_cells + 1)
    d = pml_cells * h
    sig = outer_pml_sigma(d, (n_cells - pml_cells) * h, d, strength, c_pml)
    return Axis(x, sig, h)


# --------------------------------------------------------------------------
# 5-point PML finite differences, eq. define_pml_fd (Sec. 4), FE scaling
# --------------------------------------------------------------------------
def fd5_matrix(ax, ay, k2_nodes, omega):
    """Assemble h^2 * (5-point operator of eq. define_pml_fd) as CSR.

    Row (i,k):  [ -a1(i-1/2) u(i-1,k) + (a1(i-1/2)+a1(i+1/2)) u(i,k)
                  - a1(i+1/2) u(i+1,k) ] / a2(k)
              + [ -a2(k-1/2) u(i,k-1) + (a2(k-1/2)+a2(k+1/2)) u(i,k)
                  - a2(k+1/2) u(i,k+1) ] / a1(i)
              - h^2 k^2(i,k) u(i,k) / (a1(i) a2(k))
    ``k2_nodes`` has shape (N1-1, N2-1).  Requires a uniform spacing h.
    """
    hx = ax.widths()
    hy = ay.widths()
    h = hx[0]
    assert np.allclose(hx, h) and np.allclose(hy, h), "5-point FD needs a uniform mesh"
    a1n = ax.alpha_nodes(omega)
    a1h = ax.alpha_cells(omega)       # a1h[i] = alpha at i+1/2
    a2n = ay.alpha_nodes(omega)
    a2h = ay.alpha_cells(omega)
    n1, n2 = ax.n_unknowns, ay.n_unknowns
    I, K = np.meshgrid(np.arange(1, n1 + 1), np.arange(1, n2 + 1), indexing="ij")
    idx = (I - 1) * n2 + (K - 1)
    w = -a1h[I - 1] / a2n[K]
    e = -a1h[I] / a2n[K]
    s = -a2h[K - 1] / a1n[I]
    nn = -a2h[K] / a1n[I]
    c = -(w + e + s + nn) - h * h * k2_nodes / (a1n[I] * a2n[K])
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [c.ravel()]
    for di, dk, v in ((-1, 0, w), (1, 0, e), (0, -1, s), (0, 1, nn)):
        m = (I + di >= 1) & (I + di <= n1) & (K + dk >= 1) & (K + dk <= n2)
        rows.append(idx[m])
        cols.append(((I + di - 1) * n2 + (K + dk - 1))[m])
        vals.append(v[m])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n1 * n2, n1 * n2))
    return A


def fd5_rhs_scale(ax, ay, omega):
    """Factor h^2 / (a1(i) a2(k)) that turns the physical source f into the
    right-hand side of the FE-scaled system (right side of eq. define_pml_fd)."""
    h = ax.widths()[0]
    a1n = ax.alpha_nodes(omega)[1:-1]
    a2n = ay.alpha_nodes(omega)[1:-1]
    return h * h / (a1n[:, None] * a2n[None, :])


# --------------------------------------------------------------------------
# Finite-element form of the compact 9-point operator (App. A), 2-D
# --------------------------------------------------------------------------
def fe9_element_values(hx, hy, a1, a2, k2, c1, c2, c3):
    """Per-cell element-matrix values of H_FE = -M_FE - sum D (x) N.

    For a cell with widths hx, hy, PML factors a1, a2 (at its midpoint),
    squared wavenumber k2 and coefficients c1..c3, the contribution to
    H[node a, node b] for two corners a, b of the cell depends only on
    (dx, dy) = (|a_x - b_x|, |a_y - b_y|):

      e(dx,dy) = sx * sgn(dx) * J_dy + sy * sgn(dy) * J_dx - m * I_{dx+dy}

    with sx = (a1/hx)(hy/a2), sy = (a2/hy)(hx/a1), m = hx hy k2/(a1 a2),
    sgn(0) = +1, sgn(1) = -1 (the 1-D stiffness of one cell is
    (a/h) [[1,-1],[-1,1]], i.e. minus D_2,FE), and the I, J constants of
    fe_constants_2d.  Returns (e00, e10, e01, e11).
    """
    (I0, I1, I2), (J0, J1) = fe_constants_2d(c1, c2, c3)
    sx = (a1 / hx) * (hy / a2)
    sy = (a2 / hy) * (hx / a1)
    m = hx * hy * k2 / (a1 * a2)
    e00 = sx * J0 + sy * J0 - m * I0
    e10 = -sx * J0 + sy * J1 - m * I1
    e01 = sx * J1 - sy * J0 - m * I1
    e11 = -sx * J1 - sy * J1 - m * I2
    return e00, e10, e01, e11


def fe9_matrix(ax, ay, k2_cells, coefs, omega):
    """Assemble the 2-D finite-element operator H_FE (eq. define_H_FE, 2-D
    analogue) on the rectilinear mesh ax x ay as a sum of cell element
    matrices.  ``k2_cells`` (N1, N2) and ``coefs`` = (c1, c2, c3), each an
    (N1, N2) array, are cellwise constant as App. A assumes."""
    hx = ax.widths()
    hy = ay.widths()
    a1 = ax.alpha_cells(omega)
    a2 = ay.alpha_cells(omega)
    N1, N2 = ax.n_cells, ay.n_cells
    n1, n2 = N1 - 1, N2 - 1
    P, Q = np.meshgrid(np.arange(N1), np.arange(N2), indexing="ij")
    e = fe9_element_values(hx[P], hy[Q], a1[P], a2[Q], k2_cells, *coefs)
    eval_ = {(0, 0): e[0], (1, 0): e[1], (0, 1): e[2], (1, 1): e[3]}
    rows, cols, vals = [], [], []
    corners = [(0, 0), (1, 0), (0, 1), (1, 1)]
    for ca in corners:
        for cb in corners:
            ia, ka = P + ca[0], Q + ca[1]
            ib, kb = P + cb[0], Q + cb[1]
            m = ((ia >= 1) & (ia <= n1) & (ka >= 1) & (ka <= n2)
                 & (ib >= 1) & (ib <= n1) & (kb >= 1) & (kb <= n2))
            v = eval_[(abs(ca[0] - cb[0]), abs(ca[1] - cb[1]))]
            rows.append(((ia - 1) * n2 + (ka - 1))[m])
            cols.append(((ib - 1) * n2 + (kb - 1))[m])
            vals.append(v[m])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n1 * n2, n1 * n2))
    A.sum_duplicates()
    return A


def cell_coefs_2d(k2_cells, h_nom, mode="opt"):
    """Cellwise (c1, c2, c3): Table (a) at 1/G = h_nom k / (2 pi) per cell
    (``mode='opt'``), or the 5-point set (``mode='fd5'``)."""
    if mode == "fd5":
        one = np.ones_like(k2_cells)
        return (FIVE_POINT_COEFS_2D[0] * one, FIVE_POINT_COEFS_2D[1] * one,
                FIVE_POINT_COEFS_2D[2] * one)
    inv_g = h_nom * np.sqrt(k2_cells) / (2.0 * np.pi)
    return opt_coefs_2d(inv_g)


def node_to_cell_average_2d(k2_nodes_full):
    """Cell values as the mean of the 4 corner nodes; ``k2_nodes_full`` has
    shape (N1+1, N2+1) (boundary nodes included)."""
    a = k2_nodes_full
    return 0.25 * (a[:-1, :-1] + a[1:, :-1] + a[:-1, 1:] + a[1:, 1:])


def pad_nodes_edge(v_unknowns):
    """Extend unknown-node values (N1-1, N2-1) to all nodes (N1+1, N2+1) by
    copying the nearest unknown node (used for the medium only)."""
    return np.pad(v_unknowns, 1, mode="edge")


# --------------------------------------------------------------------------
# Three dimensions
# --------------------------------------------------------------------------
# Flat index of unknown (i, j, k) (x, y, z, 1-based): ((i-1) n2 + (j-1)) n3 + (k-1).
# x is the sweep axis (slowest), z the fastest.

# The 7-point scheme written in the 3-D family of App. A: all mass on the
# centre (c1 = 1, c2 = c3 = 0) and no transverse mass spreading in the
# stiffness (c4 = 1, c5 = 0).
SEVEN_POINT_COEFS_3D = (1.0, 0.0, 0.0, 1.0, 0.0)


def fd7_matrix(ax, ay, az, k2_nodes, omega):
    """h^3 times the 3-D analogue of eq. define_pml_fd (standard second order
    finite differences with PML, the paper's fine level in 3-D, Sec. 4):

      sum over axes l of  (1/h^2) [-a_l(i-1/2) u(i-1) + (a_l(i-1/2) + a_l(i+1/2)) u(i)
                                    - a_l(i+1/2) u(i+1)] / (product of the other two a at the node)
      - k^2 u / (a_1 a_2 a_3)

    with the 1-D second-order operator of Sec. 4 along each axis.
    ``k2_nodes`` has shape (N1-1, N2-1, N3-1).  Requires a uniform spacing h."""
    h = ax.widths()[0]
    for a in (ax, ay, az):
        assert np.allclose(a.widths(), h), "7-point FD needs a uniform mesh"
    an = [a.alpha_nodes(omega) for a in (ax, ay, az)]
    ah = [a.alpha_cells(omega) for a in (ax, ay, az)]
    n = [ax.n_unknowns, ay.n_unknowns, az.n_unknowns]
    I, Jg, K = np.meshgrid(*[np.arange(1, m + 1) for m in n], indexing="ij")
    idx = ((I - 1) * n[1] + (Jg - 1)) * n[2] + (K - 1)
    pos = (I, Jg, K)
    # transverse node factors: 1 / (product of the alphas of the other axes)
    tr = [1.0 / (an[1][Jg] * an[2][K]), 1.0 / (an[0][I] * an[2][K]), 1.0 / (an[0][I] * an[1][Jg])]
    diag = -h * h * h * k2_nodes / (an[0][I] * an[1][Jg] * an[2][K])
    rows, cols, vals = [], [], []
    for l in range(3):
        p = pos[l]
        lo = -h * ah[l][p - 1] * tr[l]      # coefficient of u(p-1) (h^3 / h^2 = h)
        hi = -h * ah[l][p] * tr[l]          # coefficient of u(p+1)
        diag = diag - lo - hi
        for d, v in ((-1, lo), (1, hi)):
            q = [I, Jg, K]
            q[l] = q[l] + d
            m = (q[l] >= 1) & (q[l] <= n[l])
            rows.append(idx[m])
            cols.append((((q[0] - 1) * n[1] + (q[1] - 1)) * n[2] + (q[2] - 1))[m])
            vals.append(v[m])
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    N = n[0] * n[1] * n[2]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def fd7_rhs_scale(ax, ay, az, omega):
    """h^3 / (a1 a2 a3) at the unknown nodes: turns the physical source into
    the right-hand side of the FE-scaled 3-D system."""
    h = ax.widths()[0]
    a = [v.alpha_nodes(omega)[1:-1] for v in (ax, ay, az)]
    return h ** 3 / (a[0][:, None, None] * a[1][None, :, None] * a[2][None, None, :])


def fe_constants_3d(c1, c2, c3, c4, c5):
    """eq. def_IJ_opt: I_0 = c1/8, I_1 = c2/24, I_2 = c3/24,
    I_3 = (1 - c1 - c2 - c3)/8; J_0 = c4/4, J_1 = c5/8, J_2 = (1 - c4 - c5)/4."""
    return ((c1 / 8.0, c2 / 24.0, c3 / 24.0, (1.0 - c1 - c2 - c3) / 8.0),
            (c4 / 4.0, c5 / 8.0, (1.0 - c4 - c5) / 4.0))


def fe27_element_values(h1, h2, h3, a1, a2, a3, k2, c1, c2, c3, c4, c5):
    """Cell contributions of eq. define_H_FE (H = -M_FE - sum_l D^(l) (x) N).

    For two corners a, b of one cell with |a - b| = (d1, d2, d3), d in {0,1}:
      e = s1 sgn(d1) J_{d2+d3} + s2 sgn(d2) J_{d1+d3} + s3 sgn(d3) J_{d1+d2} - m I_{d1+d2+d3}
    with s1 = (a1/h1)(h2 h3/(a2 a3)) (the cell's share of D^(1) times its
    share of N^(2,3)), s2, s3 alike, m = h1 h2 h3 k^2 / (a1 a2 a3) (the cell's
    share of M_FE), sgn(0) = +1, sgn(1) = -1.  Returns a dict keyed by
    (d1, d2, d3)."""
    (I0, I1, I2, I3), (J0, J1, J2) = fe_constants_3d(c1, c2, c3, c4, c5)
    Iv = (I0, I1, I2, I3)
    Jv = (J0, J1, J2)
    s = ((a1 / h1) * (h2 * h3 / (a2 * a3)),
         (a2 / h2) * (h1 * h3 / (a1 * a3)),
         (a3 / h3) * (h1 * h2 / (a1 * a2)))
    m = h1 * h2 * h3 * k2 / (a1 * a2 * a3)
    out = {}
    for d1 in (0, 1):
        for d2 in (0, 1):
            for d3 in (0, 1):
                d = (d1, d2, d3)
                e = -m * Iv[d1 + d2 + d3]
                for l in range(3):
                    sg = -1.0 if d[l] else 1.0
                    e = e + s[l] * sg * Jv[sum(d) - d[l]]
                out[d] = e
    return out


def fe27_matrix(ax, ay, az, k2_cells, coefs, omega):
    """Assemble the 3-D finite-element operator H_FE of eq. define_H_FE on the
    rectilinear mesh ax x ay x az as a sum of cell element matrices.
    ``k2_cells`` (N1, N2, N3) and ``coefs`` = (c1, ..., c5), each (N1, N2, N3),
    are cellwise constant, and the alphas are taken at cell midpoints
    (App. A, coarse level)."""
    h = [a.widths() for a in (ax, ay, az)]
    al = [a.alpha_cells(omega) for a in (ax, ay, az)]
    Nc = [ax.n_cells, ay.n_cells, az.n_cells]
    n = [m - 1 for m in Nc]
    P, Q, R = np.meshgrid(*[np.arange(m) for m in Nc], indexing="ij")
    e = fe27_element_values(h[0][P], h[1][Q], h[2][R], al[0][P], al[1][Q], al[2][R], k2_cells, *coefs)
    corners = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    rows, cols, vals = [], [], []

    def flat(i, j, k):
        return ((i - 1) * n[1] + (j - 1)) * n[2] + (k - 1)

    def inside(i, j, k):
        return (i >= 1) & (i <= n[0]) & (j >= 1) & (j <= n[1]) & (k >= 1) & (k <= n[2])

    for ca in corners:
        ia, ja, ka = P + ca[0], Q + ca[1], R + ca[2]
        ma = inside(ia, ja, ka)
        for cb in corners:
            ib, jb, kb = P + cb[0], Q + cb[1], R + cb[2]
            m = ma & inside(ib, jb, kb)
            v = e[(abs(ca[0] - cb[0]), abs(ca[1] - cb[1]), abs(ca[2] - cb[2]))]
            rows.append(flat(ia, ja, ka)[m])
            cols.append(flat(ib, jb, kb)[m])
            vals.append(np.broadcast_to(v, m.shape)[m])
    N = n[0] * n[1] * n[2]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    A.sum_duplicates()
    return A


def cell_coefs_3d(k2_cells, h_nom, mode="opt"):
    """Cellwise (c1, ..., c5): Table (b) at 1/G = h_nom k / (2 pi) per cell, or
    the 7-point set (``mode='fd7'``)."""
    if mode == "fd7":
        one = np.ones_like(k2_cells)
        return tuple(v * one for v in SEVEN_POINT_COEFS_3D)
    inv_g = h_nom * np.sqrt(k2_cells) / (2.0 * np.pi)
    return opt_coefs_3d(inv_g)
