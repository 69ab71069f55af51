"""Pins of the oracle's finite-element operators, two-grid cycle and 3-D
discretization against what the paper and the mathematics fix.

* Galerkin special case: with the constants of the standard bilinear
  (trilinear) test functions, the finite-element form of eq. define_H_FE is
  the plain Galerkin discretization of the PML weak form (eq. weak_form)
  with alpha and k^2 constant per cell and alpha taken at cell midpoints
  (App. A).  The reference matrices below are built by Gauss quadrature of
  that weak form, cell by cell, with their own shape functions and their own
  PML profile; they share nothing with the oracle's assembly.
* Green's function: the FE form with PML converges at second order to
  (i/4) H0(k r).
* Two-grid: the error propagator of the cycle of Sec. 4 with an exact coarse
  solve is S^nu (I - P Ac^-1 P^T A) S^nu, S = I - omega D^-1 A.
* 3-D: rows of the 27-point form equal h^3 H_FDOpt (eq. define_H_FDOPT) built
  from the paper's M_j / N_j definitions; plane waves solving the symbols are
  null vectors; Table (b) matches the 7-point phase speed at h = H/2; the
  7-point operator on a sine mode in z is the (pinned) 5-point operator with
  a shifted k^2.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.optimize import brentq
from scipy.special import hankel1

from oracle import discretization as D
from oracle import dd as DD
from oracle import twogrid as TG
from oracle.problem import Problem2D
from oracle.problem3d import Problem3D, Level3D, make_sweep3d, cell_average_3d
from synth.media import layered_medium_2d, extend_into_pml, point_source, random_rhs, resample_nodes

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Standard bilinear / trilinear Galerkin constants expressed as Table
# coefficients: 2-D I = (1/9, 1/18, 1/36), J = (1/3, 1/6); 3-D
# I = (1/27, 1/54, 1/108, 1/216), J = (1/9, 1/18, 1/36).
Q1_COEFS_2D = (4.0 / 9.0, 4.0 / 9.0, 2.0 / 3.0)
Q1_COEFS_3D = (8.0 / 27.0, 4.0 / 9.0, 2.0 / 9.0, 4.0 / 9.0, 4.0 / 9.0)

GAUSS2 = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))


def _pml_alpha(x, L, d, S, c_pml, omega):
    """alpha = 1/(1 + i sigma/omega), sigma = C dist^2 within d of either end
    of [0, L], C = S c_pml / d^3 (Sec. 2.1), written out independently."""
    if d <= 0:
        return np.ones_like(x, dtype=complex)
    C = S * c_pml / d ** 3
    sig = C * (np.maximum(d - x, 0.0) ** 2 + np.maximum(x - (L - d), 0.0) ** 2)
    return 1.0 / (1.0 + 1j * sig / omega)


def _galerkin(xs, alphas, k2_cells):
    """Galerkin matrix of the weak form: sum over cells of
    int [ sum_l alpha_l^2/(prod alpha) d_l phi_a d_l phi_b - k^2/(prod alpha) phi_a phi_b ]
    with tensor-product linear shape functions, 2-point Gauss per axis
    (exact here), alpha and k^2 constant per cell.  ``xs``: node coordinates
    per axis; ``alphas``: alpha per cell per axis.  Unknowns: interior nodes,
    x slowest."""
    dim = len(xs)
    Nc = [len(x) - 1 for x in xs]
    n = [m - 1 for m in Nc]
    N = int(np.prod(n))
    rows, cols, vals = [], [], []
    corners = [tuple((c >> (dim - 1 - a)) & 1 for a in range(dim)) for c in range(2 ** dim)]
    qpts = [tuple((q >> (dim - 1 - a)) & 1 for a in range(dim)) for q in range(2 ** dim)]

    def phi(c, t):
        return t if c else 1.0 - t

    def dphi(c):
        return 1.0 if c else -1.0

    for cell in np.ndindex(*Nc):
        hs = [xs[a][cell[a] + 1] - xs[a][cell[a]] for a in range(dim)]
        al = [alphas[a][cell[a]] for a in range(dim)]
        pa = np.prod(al)
        vol = np.prod(hs)
        Ke = np.zeros((2 ** dim, 2 ** dim), complex)
        for q in qpts:
            t = [GAUSS2[q[a]] for a in range(dim)]
            wq = 0.5 ** dim
            for ia, ca in enumerate(corners):
                for ib, cb in enumerate(corners):
                    val = 0.0
                    for l in range(dim):
                        g = dphi(ca[l]) * dphi(cb[l]) / hs[l] ** 2
                        for m in range(dim):
                            if m != l:
                                g *= phi(ca[m], t[m]) * phi(cb[m], t[m])
                        val += al[l] ** 2 / pa * g
                    mass = 1.0
                    for m in range(dim):
                        mass *= phi(ca[m], t[m]) * phi(cb[m], t[m])
                    val -= k2_cells[cell] / pa * mass
                    Ke[ia, ib] += wq * vol * val
        for ia, ca in enumerate(corners):
            na = [cell[a] + ca[a] for a in range(dim)]
            if any(v < 1 or v > n[a] for a, v in enumerate(na)):
                continue
            ra = np.ravel_multi_index([v - 1 for v in na], n)
            for ib, cb in enumerate(corners):
                nb = [cell[a] + cb[a] for a in range(dim)]
                if any(v < 1 or v > n[a] for a, v in enumerate(nb)):
                    continue
                rows.append(ra)
                cols.append(np.ravel_multi_index([v - 1 for v in nb], n))
                vals.append(Ke[ia, ib])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def _coarse_like_axis(n_int_cells, w, h, S, c_pml):
    """A PML-aware coarse axis (PML cells of width h, interior cells of 2h)."""
    fine = D.uniform_axis(n_int_cells + 2 * w, h, w, S, c_pml)
    ca, _, _ = TG.coarsen_axis(fine, w)
    return fine, ca


# ---------------------------------------------------------------------------
# 2-D finite-element form: Galerkin special case with PML
# ---------------------------------------------------------------------------
def test_fe9_equals_bilinear_galerkin_with_pml():
    """With the bilinear constants (c1, c2, c3) = (4/9, 4/9, 2/3) the
    FE-form matrix equals the Galerkin matrix of the PML weak form, on a
    non-uniform (PML-aware coarse) mesh with PML on both axes and a random
    cellwise k^2.  A swapped alpha_1 / alpha_2, alpha at nodes instead of
    cell midpoints, or a transposed element value fails this."""
    h, S, c_pml, om = 0.1, 12.0, 1.3, 7.0
    fx, ax = _coarse_like_axis(12, 3, h, S, c_pml)
    fy, ay = _coarse_like_axis(10, 4, h, S, c_pml)
    rng = np.random.default_rng(5)
    k2 = rng.uniform(10.0, 60.0, size=(ax.n_cells, ay.n_cells))
    coefs = tuple(np.full(k2.shape, v) for v in Q1_COEFS_2D)
    A = D.fe9_matrix(ax, ay, k2, coefs, om).toarray()
    Lx, Ly = fx.x[-1], fy.x[-1]
    alx = _pml_alpha(0.5 * (ax.x[:-1] + ax.x[1:]), Lx, 3 * h, S, c_pml, om)
    aly = _pml_alpha(0.5 * (ay.x[:-1] + ay.x[1:]), Ly, 4 * h, S, c_pml, om)
    G = _galerkin([ax.x, ay.x], [alx, aly], k2).toarray()
    assert np.max(np.abs(A - G)) < 1e-12 * np.max(np.abs(G))
    # the PML is active on both axes in this mesh
    assert np.min(np.abs(alx - 1)) == 0 and np.max(np.abs(alx - 1)) > 0.1
    assert np.max(np.abs(aly - 1)) > 0.1


@pytest.mark.slow
def test_fe9_greens_function_second_order_with_pml():
    """The 9-point FE form with Table (a) at the fine 1/G and outer PML
    converges at second order to (i/4) H0(k r) (P04 for the FE form): the
    error in a ring inside the PML frame drops by about 4 per halving of h
    at fixed k."""
    k = 2 * np.pi * 4.0
    errs = []
    for n_half in (48, 96, 192):
        n = 2 * n_half - 1
        h = 1.0 / (n + 1)
        w = n_half // 4
        N = n + 1 + 2 * w
        ax = D.uniform_axis(N, h, w, 30.0, 1.0)
        k2c = np.full((N, N), k * k)
        A = D.fe9_matrix(ax, ax, k2c, D.cell_coefs_2d(k2c, h, "opt"), k)
        b = (D.fd5_rhs_scale(ax, ax, k) * point_source((N - 1, N - 1), (N // 2 - 1, N // 2 - 1), h)).ravel()
        u = spla.splu(A.tocsc()).solve(b).reshape(N - 1, N - 1)
        xs = h * np.arange(1, N)
        X, Y = np.meshgrid(xs, xs, indexing="ij")
        r = np.hypot(X - xs[N // 2 - 1], Y - xs[N // 2 - 1])
        ring = (r > 0.15) & (r < 0.35)
        g = 0.25j * hankel1(0, k * r[ring])
        errs.append(np.max(np.abs(u[ring] - g)) / np.max(np.abs(g)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert errs[2] < 0.02, errs
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, errs


def test_coarse_level_coefficients_follow_table_a_at_coarse_inv_g():
    """App. A (coarse level): the coarse operator takes Table (a) at the
    coarse 1/G = H k / (2 pi).  At 10 points per wavelength on the fine mesh
    the coarse mesh has 5, i.e. 1/G = 0.20: every coarse cell must carry the
    0.20 row of the table typed from the paper, and the fine-level 9-point
    form the 0.10 interpolant."""
    tab = np.loadtxt(os.path.join(GOLDEN, "optfd_table_a.txt"), comments="#")
    n, w = 39, 4
    h = 1.0 / (n + 1)
    om = 2 * np.pi / (10 * h)                 # c = 1: k h = 2 pi / 10
    c = np.ones((n + 2 * w, n + 2 * w))
    P = Problem2D(c, om, h, w, J=2, two_grid=True)
    row = tab[np.isclose(tab[:, 0], 0.20)][0, 1:]
    cc = P.coarse.coefs()
    for v, t in zip(cc, row):
        assert np.allclose(v, t, rtol=0, atol=1e-12)
    Pf = Problem2D(c, om, h, w, J=2, fine="fe9")
    cf = Pf.fine.coefs()
    mid = 0.5 * (tab[np.isclose(tab[:, 0], 0.08)][0, 1:] + tab[np.isclose(tab[:, 0], 0.12)][0, 1:])
    for v, t in zip(cf, mid):
        assert np.allclose(v, t, rtol=0, atol=1e-12)


def _small_layered(n=31, w=4, ppw=8.0, seed=1412046):
    h = 10.24 / (n + 1)
    c = extend_into_pml(resample_nodes(layered_medium_2d(255, 255, seed), n), w)
    return c, h, 2 * np.pi * 1.5 / (ppw * h), w


def test_two_grid_error_propagator_identity():
    """Sec. 4 cycle with an exact coarse solve: for any r,
    A^-1 r - TG(r) = S^nu (I - P Ac^-1 P^T A) S^nu A^-1 r with the omega-Jacobi
    iteration matrix S = I - omega_J D^-1 A, D = diag(A).  A dropped or extra
    smoothing step, a mis-scaled restriction or a wrong correction sign fails."""
    c, h, om, w = _small_layered(n=19, w=3)
    for nu, wj in ((3, 0.8), (2, 0.6)):
        Pb = Problem2D(c, om, h, w, two_grid=True, coarse="exact", nu=nu, omega_jac=wj)
        A = Pb.A.toarray()
        Pm = Pb.tg.P.toarray()
        Ac = Pb.tg.Ac.toarray()
        n = A.shape[0]
        S = np.eye(n) - wj * (A / np.diag(A)[:, None])
        Snu = np.linalg.matrix_power(S, nu)
        E = Snu @ (np.eye(n) - Pm @ np.linalg.solve(Ac, Pm.T @ A)) @ Snu
        r = random_rhs((n,), 17)
        x = np.linalg.solve(A, r)
        lhs = x - Pb.tg.apply(r)
        rhs = E @ x
        assert np.linalg.norm(lhs - rhs) < 1e-11 * np.linalg.norm(x)


def test_two_grid_stagnates_at_6ppw_with_exact_coarse_solve():
    """The reason configuration 3 stops at 8 points per wavelength: on the
    layered medium the two-grid method with an EXACT coarse solve (so no
    sweep is involved) does not reach 1e-6 at 6 points per wavelength (the
    coarse mesh then has 3), while it converges in under 25 iterations at 8.
    The paper's experiments all use at least 10 points per wavelength."""
    c, h, om6, w = _small_layered(n=127, w=16, ppw=6.0)
    om8 = om6 * 6.0 / 8.0
    f = point_source(c.shape, (c.shape[0] // 2, c.shape[1] // 8), h)
    P6 = Problem2D(c, om6, h, w, J=4, two_grid=True, coarse="exact")
    _, it6, _, rr6 = P6.solve(f, tol=1e-6, maxit=100)
    P8 = Problem2D(c, om8, h, w, J=4, two_grid=True, coarse="exact")
    _, it8, _, rr8 = P8.solve(f, tol=1e-6, maxit=100)
    assert rr8 < 1e-6 and it8 < 25
    assert it6 == 100 and rr6 > 1e-4


# ---------------------------------------------------------------------------
# 3-D finite-element form (eq. define_H_FE, eq. def_IJ_opt, Table (b))
# ---------------------------------------------------------------------------
def test_fe27_equals_trilinear_galerkin_with_pml():
    """With the trilinear constants the 27-point FE form equals the Galerkin
    matrix of the 3-D PML weak form on a non-uniform mesh with PML on all
    three axes and random cellwise k^2."""
    h, S, c_pml, om = 0.1, 12.0, 1.1, 6.0
    fx, ax = _coarse_like_axis(4, 2, h, S, c_pml)
    fy, ay = _coarse_like_axis(4, 2, h, S, c_pml)
    fz, az = _coarse_like_axis(2, 3, h, S, c_pml)
    rng = np.random.default_rng(11)
    k2 = rng.uniform(10.0, 60.0, size=(ax.n_cells, ay.n_cells, az.n_cells))
    coefs = tuple(np.full(k2.shape, v) for v in Q1_COEFS_3D)
    A = D.fe27_matrix(ax, ay, az, k2, coefs, om).toarray()
    al = [_pml_alpha(0.5 * (a.x[:-1] + a.x[1:]), f.x[-1], wv * h, S, c_pml, om)
          for a, f, wv in ((ax, fx, 2), (ay, fy, 2), (az, fz, 3))]
    G = _galerkin([ax.x, ay.x, az.x], al, k2).toarray()
    assert np.max(np.abs(A - G)) < 1e-12 * np.max(np.abs(G))


def _no_pml_axis(n_cells, h):
    return D.Axis(h * np.arange(n_cells + 1), lambda x: np.zeros_like(np.asarray(x, float)), h)


def test_fe27_with_7pt_coefficients_equals_fd7_without_pml():
    """(c1..c5) = (1, 0, 0, 1, 0) puts all mass on the centre and no
    transverse mass in the stiffness: the 27-point form is then the 7-point
    operator (constant k, no PML)."""
    h, N = 0.1, 7
    ax = _no_pml_axis(N, h)
    k = 3.0
    k2c = np.full((N, N, N), k * k)
    coefs = tuple(np.full(k2c.shape, v) for v in D.SEVEN_POINT_COEFS_3D)
    A = D.fe27_matrix(ax, ax, ax, k2c, coefs, 1.0).toarray()
    B = D.fd7_matrix(ax, ax, ax, np.full((N - 1,) * 3, k * k), 1.0).toarray()
    assert np.max(np.abs(A - B)) < 1e-13 * np.max(np.abs(B))


def _kappa_7pt(kh, d):
    f = lambda q: sum(2 - 2 * np.cos(q * di) for di in d) - kh ** 2
    return brentq(f, 1e-12, np.pi * 0.999)


def _symbol_opt3(A, B, C, kH, c):
    c1, c2, c3, c4, c5 = c
    ca, cb, cc = np.cos(A), np.cos(B), np.cos(C)
    M1 = (ca + cb + cc) / 3
    M2 = (ca * cb + ca * cc + cb * cc) / 3
    M3 = ca * cb * cc
    Ntil = lambda p, q: c4 + c5 * (p + q) / 2 + (1 - c4 - c5) * p * q
    return ((2 - 2 * ca) * Ntil(cb, cc) + (2 - 2 * cb) * Ntil(ca, cc) + (2 - 2 * cc) * Ntil(ca, cb)
            - kH ** 2 * (c1 + c2 * M1 + c3 * M2 + (1 - c1 - c2 - c3) * M3))


def _kappa_opt3(kH, d, c):
    return brentq(lambda q: _symbol_opt3(q * d[0], q * d[1], q * d[2], kH, c), 1e-12, np.pi * 0.999)


def test_fe27_rows_equal_h3_fdopt_and_plane_wave_null_vector():
    """P02/P01 in 3-D: interior rows of the FE form with eq. def_IJ_opt equal
    h^3 H_FDOpt (eq. define_H_FDOPT built here from M0..M3, N0..N2 and D2),
    and a plane wave whose wavenumber solves the 27-point symbol is a null
    vector of the interior rows."""
    h, N = 1.0 / 9, 9
    ax = _no_pml_axis(N, h)
    k = 2 * np.pi / (6 * h)
    c = D.opt_coefs_3d(h * k / (2 * np.pi))
    k2c = np.full((N, N, N), k * k)
    A = D.fe27_matrix(ax, ax, ax, k2c, tuple(np.full(k2c.shape, v) for v in c), 1.0)
    n = N - 1
    rng = np.random.default_rng(4)
    U = np.zeros((n + 2,) * 3, complex)
    U[1:-1, 1:-1, 1:-1] = rng.standard_normal((n,) * 3) + 1j * rng.standard_normal((n,) * 3)
    sh = lambda a, b, cc: U[1 + a:n + 1 + a, 1 + b:n + 1 + b, 1 + cc:n + 1 + cc]
    offs = [(a, b, cc) for a in (-1, 0, 1) for b in (-1, 0, 1) for cc in (-1, 0, 1)]
    Mj = [sum(sh(*o) for o in offs if sum(map(abs, o)) == m) for m in range(4)]
    Mj = [Mj[0], Mj[1] / 6, Mj[2] / 12, Mj[3] / 8]
    c1, c2, c3, c4, c5 = c
    mass = c1 * Mj[0] + c2 * Mj[1] + c3 * Mj[2] + (1 - c1 - c2 - c3) * Mj[3]
    out = -k * k * mass
    for l in range(3):
        others = [m for m in range(3) if m != l]

        def Nt(dl):
            def at(a, b):
                o = [0, 0, 0]
                o[l] = dl
                o[others[0]] = a
                o[others[1]] = b
                return sh(*o)
            N0 = at(0, 0)
            N1 = 0.25 * (at(-1, 0) + at(1, 0) + at(0, -1) + at(0, 1))
            N2 = 0.25 * (at(-1, -1) + at(1, -1) + at(-1, 1) + at(1, 1))
            return c4 * N0 + c5 * N1 + (1 - c4 - c5) * N2

        out = out - (Nt(-1) - 2 * Nt(0) + Nt(1)) / h ** 2
    got = (A @ U[1:-1, 1:-1, 1:-1].ravel()).reshape((n,) * 3)
    inner = (slice(1, -1),) * 3
    assert np.max(np.abs(got[inner] - h ** 3 * out[inner])) < 1e-12 * np.max(np.abs(got))
    d = np.array([0.3, 0.5, 0.81])
    d /= np.linalg.norm(d)
    kap = _kappa_opt3(k * h, d, c) / h
    I = np.arange(1, n + 1)
    X, Y, Z = np.meshgrid(I, I, I, indexing="ij")
    u = np.exp(1j * kap * h * (d[0] * X + d[1] * Y + d[2] * Z)).ravel()
    r = (A @ u).reshape((n,) * 3)
    assert np.max(np.abs(r[inner])) < 1e-11 * abs(A).max()


def _max_phase_err_3d(inv_gs, roles):
    worst = 0.0
    dirs = []
    for th in np.linspace(0.0, np.pi / 4, 6):
        for ph in np.linspace(0.0, np.arccos(1 / np.sqrt(3)), 6):
            dirs.append(np.array([np.cos(th) * np.sin(ph), np.sin(th) * np.sin(ph), np.cos(ph)]))
    for ig in inv_gs:
        kH = 2 * np.pi * ig
        c = D.opt_coefs_3d(ig)
        c = tuple(c[i] for i in roles)
        for d in dirs:
            try:
                kc = _kappa_opt3(kH, d, c)
            except ValueError:
                return np.inf
            kf = _kappa_7pt(kH / 2, d)
            worst = max(worst, abs((kH / kc) / ((kH / 2) / kf) - 1))
    return worst


def test_p12_3d_phase_speed_matches_fine_7pt():
    """App. A, Table (b): the 27-point scheme at H with the coefficients at the
    coarse 1/G matches the phase speed of the standard 7-point scheme at
    h = H/2 to a few 1e-4 over all directions (the paper: about 2e-4); with
    the mass and stiffness coefficient roles exchanged it does not."""
    inv_gs = np.linspace(0.02, 0.30, 8)
    assert _max_phase_err_3d(inv_gs, (0, 1, 2, 3, 4)) <= 4e-4
    assert _max_phase_err_3d(inv_gs, (3, 4, 2, 0, 1)) > 4e-3


def test_fd7_plane_wave_null_vector():
    """P01: exp(i kappa d.x) with 2-2cos terms summing to k^2 h^2 is a null
    vector of the interior rows of the 7-point operator."""
    h, N = 0.1, 10
    ax = _no_pml_axis(N, h)
    k = 2 * np.pi / (7 * h)
    A = D.fd7_matrix(ax, ax, ax, np.full((N - 1,) * 3, k * k), 1.0)
    d = np.array([0.2, 0.7, 0.4])
    d /= np.linalg.norm(d)
    kap = _kappa_7pt(k * h, d) / h
    I = np.arange(1, N)
    X, Y, Z = np.meshgrid(I, I, I, indexing="ij")
    u = np.exp(1j * kap * h * (d[0] * X + d[1] * Y + d[2] * Z)).ravel()
    r = (A @ u).reshape((N - 1,) * 3)
    assert np.max(np.abs(r[1:-1, 1:-1, 1:-1])) < 1e-12 * abs(A).max()


def test_fd7_sine_mode_reduces_to_pinned_fd5():
    """With PML on x and y only, u = v(x, y) sin(pi m z_k / L_z) is mapped by
    the 7-point operator to h (A5(k^2 - lambda_m) v) sin(...), A5 the pinned
    5-point PML operator (Green's function, reciprocity) and
    lambda_m = (2 - 2 cos(pi m / N3)) / h^2: this ties the 3-D PML terms to
    the 2-D ones."""
    h, om = 0.05, 20.0
    N1, N2, N3 = 16, 13, 9
    ax = D.uniform_axis(N1, h, 3, 15.0, 1.0)
    ay = D.uniform_axis(N2, h, 4, 15.0, 1.0)
    az = _no_pml_axis(N3, h)
    rng = np.random.default_rng(8)
    k2 = rng.uniform(200.0, 400.0, size=(N1 - 1, N2 - 1))
    A7 = D.fd7_matrix(ax, ay, az, np.repeat(k2[:, :, None], N3 - 1, axis=2), om)
    v = rng.standard_normal((N1 - 1, N2 - 1)) + 1j * rng.standard_normal((N1 - 1, N2 - 1))
    for m in (1, 3):
        s = np.sin(np.pi * m * np.arange(1, N3) / N3)
        lam = (2 - 2 * np.cos(np.pi * m / N3)) / h ** 2
        A5 = D.fd5_matrix(ax, ay, k2 - lam, om)
        lhs = (A7 @ (v[:, :, None] * s[None, None, :]).ravel()).reshape(N1 - 1, N2 - 1, N3 - 1)
        rhs = h * (A5 @ v.ravel()).reshape(N1 - 1, N2 - 1)[:, :, None] * s[None, None, :]
        assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


def _small_3d(n=(13, 9, 11), w=3, ppw=6.0, seed=3):
    from synth.media import smooth_medium_3d
    h = 0.1
    c = np.pad(smooth_medium_3d(*n, seed, corr_len=3.0), w, mode="edge")
    return c, h, 2 * np.pi * 1.5 / (ppw * h), w


@pytest.mark.parametrize("fine", ["fd7", "fe27"])
def test_3d_symmetry_and_reciprocity(fine):
    """P03 in 3-D: A = A^T with PML and variable k; u_a(x_b) = u_b(x_a)."""
    c, h, om, w = _small_3d()
    P = Problem3D(c, om, h, w, J=2, fine=fine)
    A = P.A
    assert abs(A - A.T).max() < 1e-13 * abs(A).max()
    lu = spla.splu(A.tocsc())
    n = A.shape[0]
    a, b = 37, n - 101
    ea = np.zeros(n, complex)
    eb = np.zeros(n, complex)
    ea[a] = eb[b] = 1.0
    assert abs(lu.solve(ea)[b] - lu.solve(eb)[a]) < 1e-12 * abs(lu.solve(ea)[b])


def test_3d_coarse_operator_symmetric_and_coefficients():
    """The 3-D coarse operator is symmetric; at 10 points per wavelength on the
    fine mesh every coarse cell takes the 0.20 row of Table (b)."""
    tab = np.loadtxt(os.path.join(GOLDEN, "optfd_table_b.txt"), comments="#")
    n, w, h = 11, 2, 0.1
    om = 2 * np.pi / (10 * h)
    P = Problem3D(np.ones((n + 2 * w,) * 3), om, h, w, J=2, two_grid=True, coarse="exact")
    Ac = P.tg.Ac
    assert abs(Ac - Ac.T).max() < 1e-13 * abs(Ac).max()
    row = tab[np.isclose(tab[:, 0], 0.20)][0, 1:]
    for v, t in zip(P.coarse.coefs(), row):
        assert np.allclose(v, t, rtol=0, atol=1e-12)


def test_3d_prolongation_reproduces_trilinear_functions():
    """The tensor tent prolongation maps a coarse trilinear function to the
    same function on the fine nodes (away from the Dirichlet faces), and the
    3-D cell averages reproduce a trilinear function at cell midpoints."""
    n, w, h = 9, 2, 0.1
    P = Problem3D(np.ones((n + 2 * w,) * 3), 2.0, h, w, J=2, two_grid=True, coarse="exact")
    ca = [P.coarse.ax, P.coarse.ay, P.coarse.az]
    fa = [P.fine.ax, P.fine.ay, P.fine.az]
    f = lambda x, y, z: 1 + 2 * x - y + 0.5 * z + x * y * z
    Xc = np.meshgrid(*[a.x[1:-1] for a in ca], indexing="ij")
    Xf = np.meshgrid(*[a.x[1:-1] for a in fa], indexing="ij")
    uf = (P.P @ f(*Xc).ravel()).reshape(Xf[0].shape)
    ex = f(*Xf)
    # fine nodes whose coarse cell has no Dirichlet corner
    m = np.ones(ex.shape, bool)
    for a, (c_ax, f_ax) in enumerate(zip(ca, fa)):
        lo, hi = c_ax.x[1], c_ax.x[-2]
        sl = (f_ax.x[1:-1] >= lo) & (f_ax.x[1:-1] <= hi)
        shp = [1, 1, 1]
        shp[a] = -1
        m &= sl.reshape(shp)
    assert np.allclose(uf[m], ex[m])
    Ws = []
    for f_ax, wv in zip(fa, (w, w, w)):
        _, ifp, ref = TG.coarsen_axis(f_ax, wv)
        Ws.append(TG.cell_average_1d(ifp, ref, f_ax.n_cells))
    Xn = np.meshgrid(*[a.x for a in fa], indexing="ij")
    avg = cell_average_3d(*Ws, f(*Xn))
    mids = np.meshgrid(*[0.5 * (a.x[:-1] + a.x[1:]) for a in ca], indexing="ij")
    # x y z is not reproduced exactly by the (1/4,1/2,1/4) weights: test the linear part
    g = lambda x, y, z: 1 + 2 * x - y + 0.5 * z
    assert np.allclose(cell_average_3d(*Ws, g(*Xn)), g(*mids))


def test_3d_two_grid_error_propagator_identity():
    """The two-grid identity of Sec. 4 in 3-D (27-point coarse level)."""
    c, h, om, w = _small_3d(n=(7, 5, 5), w=2, ppw=8.0)
    Pb = Problem3D(c, om, h, w, two_grid=True, coarse="exact", nu=3, omega_jac=0.6)
    A = Pb.A.toarray()
    Pm = Pb.tg.P.toarray()
    Ac = Pb.tg.Ac.toarray()
    n = A.shape[0]
    S = np.eye(n) - 0.6 * (A / np.diag(A)[:, None])
    S3 = np.linalg.matrix_power(S, 3)
    E = S3 @ (np.eye(n) - Pm @ np.linalg.solve(Ac, Pm.T @ A)) @ S3
    r = random_rhs((n,), 23)
    x = np.linalg.solve(A, r)
    assert np.linalg.norm(x - Pb.tg.apply(r) - E @ x) < 1e-11 * np.linalg.norm(x)


@pytest.mark.parametrize("kind", ["fd7", "fe27"])
def test_3d_slab_core_rows_equal_global_rows(kind):
    """A^(j) restricted to its core rows equals the global operator's rows
    (the DD-PML starts at the half node beyond the core, Sec. 2.2), so the
    transmission blocks taken from A are those of the subdomain operators."""
    c, h, om, w = _small_3d(n=(15, 7, 6), w=2)
    P = Problem3D(c, om, h, w, J=3, fine=kind, w_dd=2)
    lev = P.fine
    beta = DD.partition(lev.n1, w, 3)
    A = P.A.tocsr()
    L = lev.n2 * lev.n3
    for j in (1, 2, 3):
        x0, x1 = DD.slab_extent(beta, j, 2)
        Aj = lev.slab_level(beta, j, 2, 10.0, P.c_pml).matrix().tocsr()
        lo = beta[j - 1] + 1 if j > 1 else 1
        hi = beta[j] if j < 3 else lev.n1
        for layer in range(lo, hi + 1):
            rl = slice((layer - x0) * L, (layer - x0 + 1) * L)
            rg = slice((layer - 1) * L, layer * L)
            lc0 = max(layer - 1, x0)
            lc1 = min(layer + 1, x1)
            a = Aj[rl][:, (lc0 - x0) * L:(lc1 - x0 + 1) * L].toarray()
            g = A[rg][:, (lc0 - 1) * L:lc1 * L].toarray()
            assert np.allclose(a, g, rtol=0, atol=1e-13 * abs(A).max())


def test_3d_single_slab_exact_and_two_slabs_x_equals_ud():
    """P07 / P08 in 3-D: J = 1 gives A^-1; J = 2 gives P_X = P_UD."""
    c, h, om, w = _small_3d(n=(9, 6, 5), w=2)
    P1 = Problem3D(c, om, h, w, J=1)
    r = random_rhs((P1.A.shape[0],), 5)
    x = spla.splu(P1.A.tocsc()).solve(r)
    assert np.linalg.norm(P1.dd.apply_x(r).ravel() - x) < 1e-11 * np.linalg.norm(x)
    P2 = Problem3D(c, om, h, w, J=2, w_dd=2)
    assert np.linalg.norm(P2.dd.apply_x(r).ravel() - P2.dd.apply_ud(r).ravel()) < 1e-12 * np.linalg.norm(x)


def test_3d_two_grid_sweep_converges():
    """Context (iteration counts are unpinned): the 3-D two-grid sweep with
    J = 3 converges to 1e-6 in a few tens of iterations on a small random
    medium, and its solution matches the direct solve."""
    c, h, om, w = _small_3d(n=(21, 9, 9), w=3, ppw=10.0)
    P = Problem3D(c, om, h, w, J=3, w_dd=2, two_grid=True)
    f = point_source(c.shape, tuple(s // 2 for s in c.shape), h)
    u, it, _, rr = P.solve(f, tol=1e-8, maxit=80)
    ud = P.direct(f)
    assert rr < 1e-8 and it < 40
    assert np.linalg.norm(u - ud) < 1e-6 * np.linalg.norm(ud)
