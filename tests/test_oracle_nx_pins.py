"""Pins of the oracle's partial-sweep preconditioner SweepingPrecNX (Sec. 2.2,
main-algorithm table): groups of subdomains swept simultaneously from both
ends, coupled through the boundary subdomains between the groups.

* With one group it is the X-sweep.
* In 1-D with constant k and exact absorbing ends on every subdomain the
  sweeps inside one group are an X-sweep of that group, which is exact
  there (Sec. 3.1): a source inside a group is reproduced exactly on the
  group's layers and on the boundary subdomain to its left (completed by
  the group's outward half-sweep), and a source inside a boundary subdomain
  exactly on both neighbouring groups.  A sign error in the transmission
  or swapped group buffers break this.
* Each half of the preconditioner writes every layer exactly once.
* Iteration counts exceed the X-sweep's (Table 4: partial sweeps need more
  iterations); context only.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import dd as DD
from oracle.problem import Problem2D
from synth.media import layered_medium_2d, extend_into_pml, random_rhs

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def _exact_closure_1d(n1, kh):
    eith = np.exp(1j * np.arccos(1 - kh * kh / 2))
    main = np.full(n1, 2 - kh * kh, complex)
    main[0] -= eith
    main[-1] -= eith
    return sp.diags([np.full(n1 - 1, -1.0), main, np.full(n1 - 1, -1.0)], [-1, 0, 1], format="csr")


def _sweep_1d(n1, J, w, kh=0.6):
    A = _exact_closure_1d(n1, kh)
    beta = DD.partition(n1, 0, J)
    ext = [DD.slab_extent(beta, j, w) for j in range(1, J + 1)]
    return A, beta, DD.SweepDD(A, n1, 1, beta, ext, lambda j: _exact_closure_1d(ext[j - 1][1] - ext[j - 1][0] + 1, kh))


def test_nx_cells_and_one_group_is_x():
    n1, n2, w = 61, 45, 6
    c = extend_into_pml(layered_medium_2d(n1, n2, 1412046, n_layers=7, corr_len=6.0), w)
    h = 0.02
    om = 2 * np.pi * 1.5 / (8.0 * h)
    P = Problem2D(c, om, h, w, J=5, w_dd=4)
    assert P.dd.nx_cells(1) == ([0, 6], [None, 3])
    assert P.dd.nx_cells(2) == ([0, 3, 6], [None, 2, 5])
    with pytest.raises(ValueError):
        P.dd.nx_cells(4)
    r = random_rhs(c.shape, 3).ravel()
    zx = P.dd.apply_x(r)
    assert np.linalg.norm(P.dd.apply_nx(r, 1) - zx) < 1e-14 * np.linalg.norm(zx)
    assert np.linalg.norm(P.dd.apply_nx(r, 2) - zx) > 1e-3 * np.linalg.norm(zx)


@pytest.mark.parametrize("n1,J,w,N", [(90, 9, 3, 2), (120, 12, 2, 3), (84, 7, 1, 2)])
def test_nx_1d_exact_on_the_source_group(n1, J, w, N):
    A, beta, sw = _sweep_1d(n1, J, w)
    jc, jm = sw.nx_cells(N)
    lu = spla.splu(A.tocsc())
    for j in range(1, J + 1):
        f = np.zeros(n1, complex)
        a, b = beta[j - 1] + 1, beta[j]
        f[a - 1:b] = random_rhs((b - a + 1,), 3 + j)
        ue = lu.solve(f)
        u = sw.apply_nx(f, N).ravel()
        if j in jc:
            m = jc.index(j)
            lo, hi = max(jc[m - 1], 1), jc[m + 1] - 1
        else:
            m = next(q for q in range(1, N + 1) if jc[q - 1] < j < jc[q])
            lo, hi = max(jc[m - 1], 1), jc[m] - 1
        rows = slice(beta[lo - 1], beta[hi])
        err = np.linalg.norm(u[rows] - ue[rows]) / np.linalg.norm(ue)
        assert err < 1e-11, (j, lo, hi, err)
    # a flipped transmission sign breaks it
    blk = sw.block
    sw.block = lambda p, q: -blk(p, q)
    f = np.zeros(n1, complex)
    a, b = beta[jc[1] - 1] + 1, beta[jc[1]]
    f[a - 1:b] = 1.0
    assert np.linalg.norm(sw.apply_nx(f, N).ravel() - lu.solve(f)) > 1e-3 * np.linalg.norm(lu.solve(f))


def test_nx_halves_write_every_layer_once():
    n1, J, w, N = 120, 12, 2, 3
    A, beta, sw = _sweep_1d(n1, J, w)
    calls, half = [], [0]
    orig_solve, orig_res = sw.subdom_solve, sw.residual

    def solve(u, f, j, a, b, at, bt, *rest):
        calls.append((half[0], at, bt))
        return orig_solve(u, f, j, a, b, at, bt, *rest)

    def residual(f, u):
        half[0] = 1
        return orig_res(f, u)

    sw.subdom_solve, sw.residual = solve, residual
    sw.apply_nx(random_rhs((n1,), 5), N)
    for h in (0, 1):
        cover = np.zeros(n1, int)
        for hh, at, bt in calls:
            if hh == h:
                cover[at:bt] += 1  # layers at+1..bt (1-based)
        assert (cover == 1).all(), (h, cover)
    assert len(calls) == 2 * J


def test_nx_two_groups_needs_more_iterations_than_x():
    n1, n2, w = 95, 63, 8
    c = extend_into_pml(layered_medium_2d(n1, n2, 1412046, n_layers=7, corr_len=6.0), w)
    h = 0.02
    om = 2 * np.pi * 1.5 / (8.0 * h)
    f = random_rhs(c.shape, 9)
    its = {}
    for sweep, ncell in (("x", 1), ("nx", 2)):
        P = Problem2D(c, om, h, w, J=6, w_dd=4, two_grid=True, sweep=sweep, ncell=ncell)
        _, it, _, rr = P.solve(f, tol=1e-6, maxit=200)
        assert rr < 1e-6
        its[sweep] = it
    assert its["nx"] > its["x"]
