"""Pins of the oracle's sponge-layer boundary (Sec. 2.1: k -> k (1 + i beta)
with beta continuous and quadratic in the layer, no PML) and of the
two-grid method used without PML layers (Sec. 4: standard coarsening of
every cell, full weighting R = P^T, linear prolongation).

* With alpha = 1 the FE-scaled operator is the textbook 5-point Laplacian
  (Kronecker sum of 1-D second differences) minus h^2 k^2 (1 + i beta)^2 on
  the diagonal.
* A wave entering the layer decays like exp(-int k beta dx) (the paper's
  1-D estimate), checked at a quarter, half and three quarters of the layer.
* The point-source solution converges at second order to (i/4) H0(k r) at
  fixed k (the sponge's reflection is small enough not to stop it).
* The coarse mesh coarsens every cell, the restriction is the transpose of
  linear interpolation (full weighting up to the FE scaling), and the
  two-grid sweep preconditioner converges.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.special import hankel1

from oracle import discretization as D
from oracle.problem import Problem2D
from synth.media import point_source, random_rhs

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def test_sponge_operator_is_laplacian_minus_damped_k2():
    n1, n2, w, h = 30, 22, 6, 0.05
    c = 1.0 + 0.3 * np.random.default_rng(3).random((n1 + 2 * w, n2 + 2 * w))
    om = 9.0
    P = Problem2D(c, om, h, w, J=2, boundary="sponge")
    m1, m2 = c.shape
    T1 = sp.diags([-1.0, 2.0, -1.0], [-1, 0, 1], shape=(m1, m1))
    T2 = sp.diags([-1.0, 2.0, -1.0], [-1, 0, 1], shape=(m2, m2))
    lap = sp.kron(T1, sp.eye(m2)) + sp.kron(sp.eye(m1), T2)
    N1, N2 = m1 + 1, m2 + 1
    bmax = D.sponge_beta_default(om, float(c.mean()), w, h)
    xs, ys = h * np.arange(1, N1), h * np.arange(1, N2)
    dx = np.maximum(np.maximum(w * h - xs, xs - (N1 - w) * h), 0) / (w * h)
    dy = np.maximum(np.maximum(w * h - ys, ys - (N2 - w) * h), 0) / (w * h)
    beta = bmax * (dx[:, None] ** 2 + dy[None, :] ** 2)
    mass = (h * h * om ** 2 / c ** 2 * (1 + 1j * beta) ** 2).ravel()
    ref = lap - sp.diags(mass)
    assert abs(P.A - ref).max() < 1e-12 * abs(ref).max()
    assert np.allclose(P.rhs(np.ones(c.shape)), h * h)


def test_sponge_decay_follows_exp_minus_integral_k_beta():
    n1, n2, w = 255, 31, 40
    h = 1.0 / 256
    N1, N2 = n1 + 1 + 2 * w, n2 + 1
    om = 2 * np.pi / (10 * h)
    c = np.ones((N1 - 1, N2 - 1))
    P = Problem2D(c, om, h, (w, 0), J=4, boundary="sponge")
    ky = np.pi / (N2 * h)
    f = np.zeros(c.shape)
    f[N1 // 2 - 1, :] = np.sin(ky * h * np.arange(1, N2)) / h
    amp = np.abs(P.direct(f).reshape(c.shape)[:, (N2 - 1) // 2])
    bmax = D.sponge_beta_default(om, 1.0, w, h)
    d, onset = w * h, N1 - w
    for frac, tol in ((0.25, 0.1), (0.5, 0.1), (0.75, 0.2)):
        node = int(round(onset + frac * w))
        pred = np.exp(-om * bmax * (frac * d) ** 3 / (3 * d * d))
        assert abs(amp[node - 1] / amp[onset - 1] / pred - 1) < tol, (frac, amp[node - 1] / amp[onset - 1], pred)


def test_sponge_greens_function_second_order():
    k = 2 * np.pi * 4.0
    errs = []
    for n_half in (48, 96):
        n = 2 * n_half - 1
        h = 1.0 / (n + 1)
        w = int(round(0.75 / h))  # three wavelengths
        N = n + 1 + 2 * w
        c = np.ones((N - 1, N - 1))
        P = Problem2D(c, k, h, w, J=2, boundary="sponge")
        u = P.direct(point_source(c.shape, (N // 2 - 1, N // 2 - 1), h)).reshape(c.shape)
        xs = h * np.arange(1, N)
        X, Y = np.meshgrid(xs, xs, indexing="ij")
        r = np.hypot(X - xs[N // 2 - 1], Y - xs[N // 2 - 1])
        ring = (r > 0.15) & (r < 0.35)
        g = 0.25j * hankel1(0, k * r[ring])
        errs.append(np.max(np.abs(u[ring] - g)) / np.max(np.abs(g)))
    assert errs[1] < 0.006 and errs[0] / errs[1] > 3.0, errs


def test_two_grid_without_pml_coarsens_every_cell():
    n, w = 63, 20
    h = 1.0 / (n + 1)
    c = np.ones((n + 2 * w, n + 2 * w))
    om = 2 * np.pi / (10 * h)
    P = Problem2D(c, om, h, w, J=4, w_dd=4, two_grid=True, boundary="sponge")
    N = n + 1 + 2 * w
    assert P.coarse.n1 == N // 2 - 1
    # linear interpolation of a coarse linear function (Dirichlet-free part)
    xc = P.coarse.ax.x[1:-1]
    Pm = P.tg.P.toarray()
    lin = np.add.outer(xc, 0.5 * P.coarse.ay.x[1:-1]).ravel()
    fine = Pm @ lin
    xf = P.fine.ax.x[1:-1]
    ref = np.add.outer(xf, 0.5 * P.fine.ay.x[1:-1]).ravel()
    inner = np.add.outer((xf > 2 * h) & (xf < xf[-1] - h), (xf > 2 * h) & (xf < xf[-1] - h)).ravel() == 2
    assert np.allclose(fine[inner], ref[inner], atol=1e-12)
    # full weighting: interior rows of R = P^T are (1/2, 1, 1/2) per axis
    R1 = P.tg.P.T.tocsr()
    row = R1[(n // 2) * P.coarse.n2 + P.coarse.n2 // 2].toarray().ravel()
    vals = np.sort(row[row != 0])
    assert np.allclose(vals, np.sort([0.25] * 4 + [0.5] * 4 + [1.0]))
    f = random_rhs(c.shape, 4)
    _, it, _, rr = P.solve(f, tol=1e-6, maxit=100)
    assert rr < 1e-6 and it < 40
