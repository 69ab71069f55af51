"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these tests uses the GPU library.  Each one is chosen so that a
plausible mistake in the oracle (a dropped term, a wrong sign or index, a
transposed operand) fails it.
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
from oracle.krylov import fgmres
from oracle.problem import Problem2D, Level2D
from synth.media import layered_medium_2d, extend_into_pml, point_source, random_rhs

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_table(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def _no_pml_axis(n_cells, h):
    return D.Axis(h * np.arange(n_cells + 1), lambda x: np.zeros_like(np.asarray(x, float)), h)


# ---------------------------------------------------------------------------
# Tables (App. A) and the coefficient roles (P12)
# ---------------------------------------------------------------------------
def test_coefficient_tables_match_paper():
    assert np.array_equal(_load_table("optfd_table_a.txt"), D.OPT_TABLE_2D)
    assert np.array_equal(_load_table("optfd_table_b.txt"), D.OPT_TABLE_3D)
    # linear interpolation between support points
    c = D.opt_coefs_2d(0.10)
    assert np.allclose(c, 0.5 * (D.OPT_TABLE_2D[2, 1:] + D.OPT_TABLE_2D[3, 1:]))


def _kappa_5pt(kh, th):
    f = lambda q: (2 - 2 * np.cos(q * np.cos(th))) + (2 - 2 * np.cos(q * np.sin(th))) - kh ** 2
    return brentq(f, 1e-12, np.pi * 0.999)


def _kappa_opt(kH, th, m1, m2, s):
    def f(q):
        A, B = q * np.cos(th), q * np.sin(th)
        return ((2 - 2 * np.cos(A)) * (s + (1 - s) * np.cos(B))
                + (2 - 2 * np.cos(B)) * (s + (1 - s) * np.cos(A))
                - kH ** 2 * (m1 + m2 * (np.cos(A) + np.cos(B)) / 2 + (1 - m1 - m2) * np.cos(A) * np.cos(B)))
    return brentq(f, 1e-12, np.pi * 0.999)


def _max_phase_err(roles, inv_gs):
    worst = 0.0
    for ig in inv_gs:
        kH = 2 * np.pi * ig
        kh = kH / 2
        c = D.opt_coefs_2d(ig)
        m1, m2, s = (c[0], c[1], c[2]) if roles == "mass,mass,stiff" else (c[1], c[2], c[0])
        for th in np.linspace(0, np.pi / 4, 16):
            try:
                kc = _kappa_opt(kH, th, m1, m2, s)
            except ValueError:
                return np.inf
            kf = _kappa_5pt(kh, th)
            worst = max(worst, abs((kH / kc) / (kh / kf) - 1))
    return worst


def test_p12_phase_speed_matches_fine_5pt():
    """P12 (App. A): coarse optimized scheme at H with Table (a) at the coarse
    1/G matches the standard 5-point scheme at h = H/2 to about 2e-4."""
    claim = dict(l.split() for l in open(os.path.join(GOLDEN, "phase_speed_claim.txt"))
                 if l.strip() and not l.startswith("#"))
    tol, igmax = float(claim["max_rel_phase_speed_diff"]), float(claim["inv_g_coarse_max"])
    inv_gs = np.linspace(0.01, igmax, 13)
    assert _max_phase_err("mass,mass,stiff", inv_gs) <= tol
    # the other role assignment is far off: the mapping is pinned
    assert _max_phase_err("stiff,mass,mass", inv_gs) > 10 * tol


def test_plane_wave_symbol_fe9_and_fdopt():
    """P01/P02: a discrete plane wave solving the optimized symbol is a null
    vector of the interior rows of the FE-form operator (no PML, constant k),
    and those rows equal h^2 times H_FDOpt built from the paper's N0, N1, N2
    and D2 (x) N-tilde definitions."""
    h = 1.0 / 24
    N = 24
    ax = ay = _no_pml_axis(N, h)
    k = 2 * np.pi / (6 * h)
    k2c = np.full((N, N), k * k)
    c1, c2, c3 = D.opt_coefs_2d(h * k / (2 * np.pi))
    coefs = (np.full((N, N), c1), np.full((N, N), c2), np.full((N, N), c3))
    A = D.fe9_matrix(ax, ay, k2c, coefs, omega=1.0).toarray()
    n = N - 1
    th = 0.37
    kap = _kappa_opt(k * h, th, c1, c2, c3) / h
    I, K = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1), indexing="ij")
    u = np.exp(1j * kap * h * (np.cos(th) * I + np.sin(th) * K)).ravel()
    inner = ((I > 1) & (I < n) & (K > 1) & (K < n)).ravel()
    r = A @ u
    assert np.max(np.abs(r[inner])) < 1e-11 * np.max(np.abs(A))
    # H_FDOpt (2-D): -k^2 (c1 N0 + c2 N1 + (1-c1-c2) N2) - D2x (x) (c3 + (1-c3) avg_y)
    #                 - D2y (x) (c3 + (1-c3) avg_x), times h^2
    U = np.zeros((n + 2, n + 2), complex)
    rng = np.random.default_rng(3)
    U[1:-1, 1:-1] = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    C = U[1:-1, 1:-1]
    Ux = lambda di, dk: U[1 + di:n + 1 + di, 1 + dk:n + 1 + dk]
    N1 = 0.25 * (Ux(-1, 0) + Ux(1, 0) + Ux(0, -1) + Ux(0, 1))
    N2 = 0.25 * (Ux(-1, -1) + Ux(1, -1) + Ux(-1, 1) + Ux(1, 1))
    mass = c1 * C + c2 * N1 + (1 - c1 - c2) * N2
    d2x = lambda dk: Ux(-1, dk) - 2 * Ux(0, dk) + Ux(1, dk)
    d2y = lambda di: Ux(di, -1) - 2 * Ux(di, 0) + Ux(di, 1)
    sx = c3 * d2x(0) + (1 - c3) * 0.5 * (d2x(-1) + d2x(1))
    sy = c3 * d2y(0) + (1 - c3) * 0.5 * (d2y(-1) + d2y(1))
    hfd = -(k * h) ** 2 * mass - sx - sy
    assert np.allclose((A @ C.ravel()).reshape(n, n), hfd, rtol=0, atol=1e-12 * np.abs(hfd).max())


def test_fe9_with_5pt_coefficients_equals_fd5_interior():
    """The FE form with (c1, c2, c3) = (1, 0, 1) is the 5-point scheme: with no
    PML and constant k its matrix equals the FD operator of eq. define_pml_fd."""
    N, h = 20, 0.05
    ax = ay = _no_pml_axis(N, h)
    k2 = 30.0
    one = np.ones((N, N))
    A9 = D.fe9_matrix(ax, ay, k2 * one, (one, 0 * one, one), omega=1.0)
    A5 = D.fd5_matrix(ax, ay, np.full((N - 1, N - 1), k2), omega=1.0)
    assert abs(A9 - A5).max() < 1e-13


def test_p01_fd5_plane_wave_null_vector():
    N, h = 30, 1.0 / 30
    ax = ay = _no_pml_axis(N, h)
    k = 2 * np.pi / (10 * h)
    A = D.fd5_matrix(ax, ay, np.full((N - 1, N - 1), k * k), omega=1.0)
    th = 0.61
    kap = _kappa_5pt(k * h, th) / h
    n = N - 1
    I, K = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1), indexing="ij")
    u = np.exp(1j * kap * h * (np.cos(th) * I + np.sin(th) * K)).ravel()
    inner = ((I > 1) & (I < n) & (K > 1) & (K < n)).ravel()
    assert np.abs((A @ u)[inner]).max() < 1e-12
    # a wrong wavenumber is not a null vector
    u2 = np.exp(1j * 1.01 * kap * h * (np.cos(th) * I + np.sin(th) * K)).ravel()
    assert np.abs((A @ u2)[inner]).max() > 1e-4


# ---------------------------------------------------------------------------
# Symmetry, reciprocity, direct solves (P03, P05)
# ---------------------------------------------------------------------------
def _small_layered(n=31, w=6):
    c = extend_into_pml(layered_medium_2d(n, n, 11, n_layers=5, corr_len=4.0), w)
    h = 0.05
    om = 2 * np.pi * 1.5 / (8 * h)
    return c, h, om, w


@pytest.mark.parametrize("fine", ["fd5", "fe9"])
def test_p03_symmetry_and_reciprocity(fine):
    c, h, om, w = _small_layered()
    P = Problem2D(c, om, h, w, J=2, fine=fine)
    A = P.A
    assert abs(A - A.T).max() < 1e-13 * abs(A).max()
    assert abs(A - A.conj().T).max() > 1e-3   # complex symmetric, not Hermitian
    lu = spla.splu(A.tocsc())
    n = A.shape[0]
    a, b = 100, n - 130
    ea = np.zeros(n, complex); ea[a] = 1
    eb = np.zeros(n, complex); eb[b] = 1
    ua, ub = lu.solve(ea), lu.solve(eb)
    assert abs(ua[b] - ub[a]) < 1e-11 * abs(ua[b])


def test_p03_coarse_fe_operator_symmetric():
    c, h, om, w = _small_layered(n=39, w=6)
    P = Problem2D(c, om, h, w, J=2, two_grid=True)
    Ac = P.coarse.matrix()
    assert abs(Ac - Ac.T).max() < 1e-13 * abs(Ac).max()


def test_p05_dense_equals_sparse_direct():
    c, h, om, w = _small_layered(n=15, w=4)
    P = Problem2D(c, om, h, w, J=1)
    f = random_rhs(c.shape, 5)
    b = P.rhs(f)
    ud = np.linalg.solve(P.A.toarray(), b)
    us = spla.splu(P.A.tocsc()).solve(b)
    assert np.linalg.norm(ud - us) < 1e-12 * np.linalg.norm(ud)


# ---------------------------------------------------------------------------
# Green's function: O(h^2) convergence to (i/4) H0^(1)(k r) (P04)
# ---------------------------------------------------------------------------
@pytest.mark.slow
def test_p04_greens_function_second_order():
    k = 2 * np.pi * 4.0
    errs = []
    for n_half in (48, 96, 192):
        n = 2 * n_half - 1                  # interior nodes; centre node exists
        h = 1.0 / (n + 1)
        w = n_half // 4                     # PML thickness 1/8 for every h
        N = n + 1 + 2 * w
        ax = D.uniform_axis(N, h, w, 30.0, 1.0)
        A = D.fd5_matrix(ax, ax, np.full((N - 1, N - 1), k * k), omega=k)
        b = (D.fd5_rhs_scale(ax, ax, k) * point_source((N - 1, N - 1), (N // 2 - 1, N // 2 - 1), h)).ravel()
        u = spla.splu(A.tocsc()).solve(b).reshape(N - 1, N - 1)
        xs = h * np.arange(1, N)
        X, Y = np.meshgrid(xs, xs, indexing="ij")
        r = np.hypot(X - xs[N // 2 - 1], Y - xs[N // 2 - 1])
        ring = (r > 0.15) & (r < 0.35)
        g = 0.25j * hankel1(0, k * r[ring])
        errs.append(np.max(np.abs(u[ring] - g)) / np.max(np.abs(g)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert errs[2] < 0.02
    assert 3.2 < r1 < 4.8 and 3.2 < r2 < 4.8, errs


def test_greens_function_outgoing_sign():
    """A wrong sign of the PML (or of the time convention) turns the
    solution into the incoming wave; the phase must advance like +k r."""
    k = 2 * np.pi * 4.0
    n = 127
    h = 1.0 / (n + 1)
    w = 16
    N = n + 1 + 2 * w
    ax = D.uniform_axis(N, h, w, 30.0, 1.0)
    A = D.fd5_matrix(ax, ax, np.full((N - 1, N - 1), k * k), omega=k)
    b = (D.fd5_rhs_scale(ax, ax, k) * point_source((N - 1, N - 1), (N // 2 - 1, N // 2 - 1), h)).ravel()
    u = spla.splu(A.tocsc()).solve(b).reshape(N - 1, N - 1)
    ic = N // 2 - 1
    pts = [ic + m for m in (20, 30, 40)]
    g = 0.25j * hankel1(0, k * h * (np.array(pts) - ic))
    assert np.max(np.abs(u[pts, ic] - g)) < 0.1 * np.max(np.abs(g))


# ---------------------------------------------------------------------------
# Sweeps: degenerate cases, partition, exactness (P07-P11)
# ---------------------------------------------------------------------------
def test_p09_written_ranges_partition():
    for n1, J in ((60, 4), (61, 5), (100, 7), (40, 2), (30, 1)):
        beta = DD.partition(n1, 4, J)
        sw = DD.SweepDD.__new__(DD.SweepDD)
        sw.J, sw.beta, sw.bt = J, beta, DD.beta_tilde(beta)
        for kind in ("ud", "x"):
            for half in sw.written_ranges(kind):
                cover = np.zeros(n1 + 2, int)
                for lo, hi in half:
                    cover[lo:hi + 1] += 1
                assert np.all(cover[1:n1 + 1] == 1) and cover[0] == 0 and cover[n1 + 1] == 0


def test_p07_single_subdomain_is_exact():
    c, h, om, w = _small_layered(n=31, w=6)
    P = Problem2D(c, om, h, w, J=1)
    f = random_rhs(c.shape, 9)
    u, it, hist, rr = P.solve(f, tol=1e-10)
    assert it == 1 and rr < 1e-11
    z = P.precond(P.rhs(f))
    assert np.linalg.norm(z - P.direct(f)) < 1e-11 * np.linalg.norm(z)


def test_p08_two_subdomains_x_equals_ud():
    c, h, om, w = _small_layered(n=31, w=6)
    Px = Problem2D(c, om, h, w, J=2, sweep="x")
    Pu = Problem2D(c, om, h, w, J=2, sweep="ud")
    r = random_rhs((Px.A.shape[0],), 4)
    zx, zu = Px.precond(r), Pu.precond(r)
    assert np.linalg.norm(zx - zu) < 1e-12 * np.linalg.norm(zu)
    # for J > 2 they differ
    Px3 = Problem2D(c, om, h, w, J=3, sweep="x")
    Pu3 = Problem2D(c, om, h, w, J=3, sweep="ud")
    assert np.linalg.norm(Px3.precond(r) - Pu3.precond(r)) > 1e-6 * np.linalg.norm(zu)


def _exact_closure_1d(n1, kh):
    """1-D -u'' - k^2 u with the exact discrete radiation condition
    u_{n+1} = e^{i theta} u_n, 2 - 2 cos(theta) = (kh)^2, at both ends."""
    eith = np.exp(1j * np.arccos(1 - kh * kh / 2))
    main = np.full(n1, 2 - kh * kh, complex)
    main[0] -= eith
    main[-1] -= eith
    A = sp.diags([np.full(n1 - 1, -1.0), main, np.full(n1 - 1, -1.0)], [-1, 0, 1], format="csr")
    return A, eith


@pytest.mark.parametrize("J,w", [(4, 1), (5, 2), (6, 3), (3, 1)])
def test_p10_one_dimensional_sweeps_are_exact(J, w):
    """P10 (Sec. 3.1): in 1-D with constant k and exact absorbing ends on every
    subdomain, both the UD and the X sweep reproduce A^{-1} exactly.  This
    pins the transmission layers, the signs of T and T~ and the schedules."""
    n1, kh = 90, 0.6
    A, eith = _exact_closure_1d(n1, kh)
    beta = DD.partition(n1, 0, J)
    ext = [DD.slab_extent(beta, j, w) for j in range(1, J + 1)]

    def slab(j):
        x0, x1 = ext[j - 1]
        return _exact_closure_1d(x1 - x0 + 1, kh)[0]

    sw = DD.SweepDD(A, n1, 1, beta, ext, slab)
    f = random_rhs((n1,), 17)
    u_ex = spla.spsolve(A.tocsc(), f)
    for ap in (sw.apply_ud, sw.apply_x):
        u = ap(f).ravel()
        assert np.linalg.norm(u - u_ex) < 1e-11 * np.linalg.norm(u_ex)
    # a sign error in the transmission breaks exactness
    sw3 = DD.SweepDD(A, n1, 1, beta, ext, slab)
    sw3.A = sw3.A.copy(); sw3.A.data = sw3.A.data.copy()
    blk_bad = sw3.block

    def flipped(p, q):
        return -blk_bad(p, q)

    sw3.block = flipped
    assert np.linalg.norm(sw3.apply_x(f).ravel() - u_ex) > 1e-3 * np.linalg.norm(u_ex)


def test_p11_strip_theorem_few_iterations():
    """Theorem 1 (Sec. 3.2): constant k on a strip with absorbing layers only
    at x = 0, L gives A P_X f ~ f; with real PMLs a handful of iterations."""
    n1, n2, w = 127, 47, 10
    h = 1.0 / 128
    c = np.ones((n1 + 2 * w, n2))
    om = 2 * np.pi / (10 * h)
    P = Problem2D(c, om, h, (w, 0), S_outer=50, J=6, w_dd=4)
    f = random_rhs(c.shape, 2)
    u, it, hist, rr = P.solve(f, tol=1e-6)
    assert it <= 4 and rr < 1e-6


# ---------------------------------------------------------------------------
# Slab operators (Sec. 2.1 subdomains, discrete transmission)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["fd5", "fe9"])
def test_slab_core_rows_equal_global_rows(kind):
    """Rows of A^(j) in the core (layers beta_{j-1}..beta_j) equal the global
    rows: the DD-PML and the k continuation start strictly beyond b_j and
    before b~_{j-1}, so the transmission blocks taken from A agree with
    those of A^(j-1)."""
    c, h, om, w = _small_layered(n=41, w=6)
    fine = Problem2D(c, om, h, w, J=4, fine=kind).fine
    A = fine.matrix().tocsr()
    n2 = fine.n2
    beta = DD.partition(fine.n1, w, 4)
    for j in (1, 2, 3, 4):
        x0, x1 = DD.slab_extent(beta, j, 3)
        Aj = fine.slab_level(beta, j, 3, 15.0, 2.0).matrix().tocsr()
        lo = beta[j - 1] if j > 1 else 1
        for g in range(lo, beta[j] + 1):
            rg = A[(g - 1) * n2:g * n2, (x0 - 1) * n2:x1 * n2].toarray()
            rj = Aj[(g - x0) * n2:(g - x0 + 1) * n2, :].toarray()
            assert np.allclose(rg, rj, rtol=0, atol=1e-13 * abs(A).max())
        # the added layers differ (they carry the DD-PML)
        if j < 4:
            g = beta[j] + 2
            rg = A[(g - 1) * n2:g * n2, (g - 1) * n2:g * n2].toarray()
            rj = Aj[(g - x0) * n2:(g - x0 + 1) * n2, (g - x0) * n2:(g - x0 + 1) * n2].toarray()
            assert not np.allclose(rg, rj)


# ---------------------------------------------------------------------------
# Two-grid pieces (Sec. 4, App. A)
# ---------------------------------------------------------------------------
def test_coarsening_and_prolongation():
    w = 5
    ax = D.uniform_axis(10 + 2 * w, 0.1, w, 20.0, 1.0)
    cax, ifp, ref = TG.coarsen_axis(ax, w)
    assert cax.n_cells == 5 + 2 * w and ifp[0] == 0 and ifp[-1] == 20
    assert not ref[:w].any() and not ref[-w:].any() and ref[w:-w].all()
    assert np.allclose(np.diff(cax.x)[w:-w], 0.2) and np.allclose(np.diff(cax.x)[:w], 0.1)
    P1 = TG.prolongation_1d(ifp, ref, ax.n_cells).toarray()
    # tent prolongation reproduces any function that is linear on every coarse
    # cell, and vanishes at the Dirichlet ends
    xc = cax.x[1:-1]
    vc = np.sin(3 * xc) + xc
    vf = P1 @ vc
    for p in range(cax.n_cells):
        i0 = ifp[p]
        if ref[p]:
            left = vc[p - 1] if p >= 1 else 0.0
            right = vc[p] if p < cax.n_cells - 1 else 0.0
            assert np.isclose(vf[i0], 0.5 * (left + right))
    W = TG.cell_average_1d(ifp, ref, ax.n_cells)
    assert np.allclose(W.sum(1), 1.0)
    xm = 0.5 * (cax.x[:-1] + cax.x[1:])
    assert np.allclose(W @ ax.x, xm)      # averages reproduce linear functions at midpoints


def test_two_grid_exact_coarse_iterations_context():
    """Table 3 context (unpinned): constant medium, 10 ppw, two-grid with an
    exact coarse solve needs about 10 iterations; the sweep as coarse solver
    costs about the same."""
    n, w = 255, 8
    h = 1.0 / (n + 1)
    c = np.ones((n + 2 * w, n + 2 * w))
    om = 2 * np.pi / (10 * h)
    f = point_source(c.shape, (c.shape[0] // 2, c.shape[1] // 2), h)
    its = {}
    for coarse in ("exact", "sweep"):
        P = Problem2D(c, om, h, w, J=8, w_dd=4, two_grid=True, coarse=coarse)
        u, it, hist, rr = P.solve(f, tol=1e-6)
        assert rr < 1e-6
        its[coarse] = it
    assert its["exact"] <= 14 and abs(its["sweep"] - its["exact"]) <= 3


# ---------------------------------------------------------------------------
# FGMRES (P13)
# ---------------------------------------------------------------------------
def test_p13_fgmres_iterates_minimise_residual():
    """The k-th FGMRES iterate with a fixed linear preconditioner M minimises
    ||b - A x|| over x in M K_k(A M, b); checked against an explicit
    Krylov basis and a least-squares solve, and against GMRES."""
    c, h, om, w = _small_layered(n=23, w=4)
    P = Problem2D(c, om, h, w, J=3)
    b = P.rhs(random_rhs(c.shape, 21))
    A, M = P.A, P.precond
    iters = {}
    fgmres(P.matvec, M, b, tol=1e-14, maxit=5, callback=lambda k, x: iters.__setitem__(k, x))
    giters = {}
    fgmres(P.matvec, M, b, tol=1e-14, maxit=5, flexible=False,
           callback=lambda k, x: giters.__setitem__(k, x))
    K = [b / np.linalg.norm(b)]
    for k in range(1, 6):
        Q, _ = np.linalg.qr(np.array(K).T)
        Y = np.array([M(q) for q in Q.T]).T
        cc, *_ = np.linalg.lstsq(A @ Y, b, rcond=None)
        x = Y @ cc
        assert np.linalg.norm(iters[k] - x) < 1e-8 * np.linalg.norm(x)
        assert np.linalg.norm(giters[k] - x) < 1e-8 * np.linalg.norm(x)
        K.append(A @ M(Q[:, -1]))
