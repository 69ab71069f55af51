"""GPU parity of the three-dimensional path against the CPU oracle.

Operators, transfers, smoothing, slab solves, sweeps, the two-grid
preconditioner and FGMRES on seeded smooth random 3-D media (the depth-trend
medium of the 3-D experiments, Sec. 6.2, at small sizes).  The slab planes
have 60-1240 unknowns, so the dense-block factorization runs several panels
of 32 columns, several 64 x 64 update tiles with ragged edges, and (one case)
more than 1024 rows per panel.  Tolerances: FP64 kernels 1e-12 relative;
complex64 maps (slab factors from the FP32 matrix cores, sweeps, two-grid)
2e-4 relative; solves to 1e-6 with iteration counts within +-1 of the
oracle's FGMRES.  Both slab factorizations are covered: block tridiagonal
along y with dense blocks, and the nested dissection of the slab planes
(multifrontal fronts of up to a few hundred unknowns, children's Schur
complements assembled into their parents).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

from oracle.problem3d import Problem3D  # noqa: E402
from synth.media import smooth_medium_3d, point_source, random_rhs  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")]

TOL32 = 2e-4


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


# (name, interior nodes, pml, J, fine, two_grid, sweep, ppw)
CASES = {
    "fd7_1lvl_x": ((17, 8, 9), 3, 3, "fd7", False, "x", 8.0),
    "fd7_1lvl_ud": ((15, 7, 8), 3, 2, "fd7", False, "ud", 8.0),
    "fe27_1lvl_x": ((16, 7, 9), 3, 3, "fe27", False, "x", 10.0),
    "tg_x": ((25, 9, 11), 4, 3, "fd7", True, "x", 10.0),
    "tg_ud": ((21, 7, 9), 4, 2, "fd7", True, "ud", 10.0),
}


def _medium(n, w, seed=1412047):
    c = smooth_medium_3d(*n, seed, corr_len=3.0)
    return np.pad(c, w, mode="edge")


SF = ["block", "nd"]


def _build(name, J=None, w_dd=2, slab_factor="nd"):
    n, w, J0, fine, tg, sweep, ppw = CASES[name]
    J = J0 if J is None else J
    c = _medium(n, w)
    h = 0.05
    om = 2 * np.pi * 1.5 / (ppw * h)
    print(f"[3d case {name} J={J} shape={c.shape} slab_factor={slab_factor}]", flush=True)
    ref = Problem3D(c, om, h, w, J=J, w_dd=w_dd, fine=fine, two_grid=tg, sweep=sweep, omega_jac=0.6)
    from paper_1412_0464_amd import Helmholtz
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, J, fine_stencil=7 if fine == "fd7" else 27,
                   two_grid=tg, sweep=sweep, w_dd=w_dd, omega_jac=0.6, slab_factor=slab_factor)
    assert hs.slab_factor == slab_factor
    return c, ref, hs


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device=_dev())


def _relerr(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name", list(CASES))
def test_partition_matches(name):
    c, ref, hs = _build(name)
    dd = ref.dd
    assert hs.beta == list(dd.beta)
    assert [(a, b) for a, b in zip(hs.x0, hs.x1)] == [tuple(e) for e in dd.extents]
    hs.close()


@pytest.mark.parametrize("name", ["fd7_1lvl_x", "fe27_1lvl_x", "tg_x"])
def test_fine_operator_and_rhs(name):
    c, ref, hs = _build(name)
    try:
        x = random_rhs(c.shape, 11)
        y = hs.apply_operator(_t(x)).cpu().numpy().ravel()
        assert _relerr(y, ref.matvec(x.ravel())) < 1e-12
        f = random_rhs(c.shape, 12)
        assert _relerr(hs.rhs(_t(f)).cpu().numpy(), ref.rhs(f)) < 1e-13
    finally:
        hs.close()


def test_coarse_operator_and_transfers():
    c, ref, hs = _build("tg_x")
    try:
        Ac = ref.tg.Ac
        xc = random_rhs(hs.n_coarse, 13)
        yc = hs.apply_level_operator(1, _t(xc)).cpu().numpy().ravel()
        assert _relerr(yc, Ac @ xc.ravel()) < 2e-6
        rf = random_rhs(c.shape, 14)
        rc = hs.restrict(_t(rf)).cpu().numpy().ravel()
        assert _relerr(rc, ref.P.T @ rf.ravel()) < 1e-13
        ec = random_rhs(hs.n_coarse, 15)
        xf = random_rhs(c.shape, 16)
        out = hs.prolong_add(_t(ec), _t(xf)).cpu().numpy().ravel()
        assert _relerr(out, xf.ravel() + ref.P @ ec.ravel()) < 1e-13
        r = random_rhs(c.shape, 17)
        for steps in (1, 3):
            xs = hs.smooth(_t(r), steps).cpu().numpy().ravel()
            xo = ref.tg.smooth(np.zeros(r.size, complex), r.ravel(), steps)
            assert _relerr(xs, xo) < 1e-12
    finally:
        hs.close()


@pytest.mark.parametrize("sf", SF)
@pytest.mark.parametrize("name", ["fd7_1lvl_x", "fe27_1lvl_x", "tg_x"])
def test_slab_solves(name, sf):
    c, ref, hs = _build(name, slab_factor=sf)
    try:
        for j in range(hs.J):
            nl = hs.x1[j] - hs.x0[j] + 1
            shape = (nl,) + tuple(hs.dd_shape[1:])
            b = random_rhs(shape, 20 + j)
            x = hs.slab_solve(j, _t(b)).cpu().numpy().ravel()
            xo = ref.dd.lu[j].solve(b.ravel())
            err = _relerr(x, xo)
            print(f"[3d slab {j}: {nl} layers, plane {nl * shape[2]} unknowns, rel err {err:.2e}, "
                  f"pivot growth {hs.pivot_growth:.3f}]", flush=True)
            assert err < TOL32, f"slab {j}: {err:.2e}"
    finally:
        hs.close()


@pytest.mark.parametrize("sf", SF)
def test_single_slab_plane_of_more_than_1024_unknowns(sf):
    """J = 1: the sweep is the exact inverse; slab planes of 40 x 31 = 1240
    unknowns (block form: rows beyond 1024 of each panel live in LDS; nested
    dissection: fronts of 40-layer separators)."""
    n, w = (34, 3, 25), 3
    c = _medium(n, w)
    h = 0.05
    om = 2 * np.pi * 1.5 / (8.0 * h)
    print(f"[3d single slab, shape {c.shape}]", flush=True)
    ref = Problem3D(c, om, h, w, J=1, w_dd=2)
    from paper_1412_0464_amd import Helmholtz
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, 1, w_dd=2, slab_factor=sf)
    try:
        assert hs.x1[0] - hs.x0[0] + 1 == 40 and hs.n_fine[2] == 31
        f = random_rhs(c.shape, 30)
        u = hs.sweep(_t(f)).cpu().numpy().ravel()
        uo = spla.splu(ref.A.tocsc()).solve(f.ravel())
        assert _relerr(u, uo) < TOL32
    finally:
        hs.close()


@pytest.mark.parametrize("sf", SF)
@pytest.mark.parametrize("name", list(CASES))
def test_sweep(name, sf):
    c, ref, hs = _build(name, slab_factor=sf)
    try:
        f = random_rhs(hs.dd_shape, 40)
        u = hs.sweep(_t(f)).cpu().numpy().ravel()
        ap = ref.dd.apply_x if CASES[name][5] == "x" else ref.dd.apply_ud
        uo = ap(f.ravel()).ravel()
        assert _relerr(u, uo) < TOL32
    finally:
        hs.close()


@pytest.mark.parametrize("sf", SF)
@pytest.mark.parametrize("name", list(CASES))
def test_precond(name, sf):
    c, ref, hs = _build(name, slab_factor=sf)
    try:
        r = random_rhs(c.shape, 50)
        z = hs.apply_precond(_t(r)).cpu().numpy().ravel()
        assert _relerr(z, ref.precond(r.ravel())) < TOL32
    finally:
        hs.close()


@pytest.mark.parametrize("sf", SF)
@pytest.mark.parametrize("name", ["fd7_1lvl_x", "tg_x", "tg_ud"])
def test_solve(name, sf):
    c, ref, hs = _build(name, slab_factor=sf)
    try:
        f = point_source(c.shape, tuple(s // 2 for s in c.shape), 0.05)
        u, it, rr = hs.solve(hs.rhs(_t(f)), tol=1e-6, maxit=100)
        uo, ito, _, _ = ref.solve(f, tol=1e-6, maxit=100)
        u = u.cpu().numpy().ravel()
        b = ref.rhs(f)
        rr_o = np.linalg.norm(b - ref.matvec(u)) / np.linalg.norm(b)
        print(f"[3d solve {name}: gpu {it} iterations (relres {rr:.2e}, oracle operator {rr_o:.2e}), "
              f"oracle {ito}]", flush=True)
        assert rr <= 1e-6 and rr_o <= 1.001e-6 and abs(it - ito) <= 1
        assert _relerr(u, uo) < 1e-4
    finally:
        hs.close()


def test_fp64_and_bad_stencil_rejected_in_3d():
    from paper_1412_0464_amd import Helmholtz, HspError
    c = _medium((9, 6, 6), 2)
    with pytest.raises(HspError) as e:
        Helmholtz(torch.tensor(c, device=_dev()), 20.0, 0.05, 2, 1, precision="fp64")
    assert e.value.status == -1 and "HSP_MIXED" in str(e.value)
    with pytest.raises(HspError) as e:
        Helmholtz(torch.tensor(c, device=_dev()), 20.0, 0.05, 2, 1, fine_stencil=5)
    assert e.value.status == -1


@pytest.mark.parametrize("sf", SF)
def test_singular_slab_gives_esingular_in_3d(sf):
    """A separator block forced to zero (debug knob) reaches HSP_ESINGULAR
    through the ABI for both factorizations."""
    from paper_1412_0464_amd import Helmholtz, HspError, hsp
    c = _medium((17, 8, 9), 3)
    print(f"[3d failure path: singular block of slab 1, {sf}]", flush=True)
    hsp.debug_set("singular_slab", 1)
    try:
        with pytest.raises(HspError) as e:
            Helmholtz(torch.tensor(c, device=_dev()), 2 * np.pi * 1.5 / (8.0 * 0.05), 0.05, 3, 3, w_dd=2,
                      slab_factor=sf)
        assert e.value.status == hsp.HSP_ESINGULAR
    finally:
        hsp.debug_set("singular_slab", -1)


def test_nested_dissection_fronts_span_levels():
    """The nested dissection of a 9 x 11 plane has several levels, and its
    pivot growth stays moderate on the two-grid case."""
    c, ref, hs = _build("tg_x")
    try:
        assert hs.slab_factor == "nd" and 0 < hs.pivot_growth < 1e3
    finally:
        hs.close()


def test_slab_factor_rejected_in_2d():
    from paper_1412_0464_amd import Helmholtz, HspError
    c = np.ones((20, 20))
    with pytest.raises(HspError) as e:
        Helmholtz(torch.tensor(c, device=_dev()), 20.0, 0.05, 3, 2, slab_factor="nd")
    assert e.value.status == -1


@pytest.mark.parametrize("sf", SF)
@pytest.mark.parametrize("shape,pml", [((17, 8, 1), (3, 3, 0)), ((17, 1, 9), (3, 0, 3))])
def test_degenerate_planes(shape, pml, sf):
    """Slab planes one node thick in z (or y): the dissection of a line of
    nodes (single-node separators) and block-tridiagonal blocks of n_l (or
    a single block), against the oracle's slab solves, sweep and
    preconditioner."""
    c = np.pad(smooth_medium_3d(*shape, 1412047, corr_len=3.0), [(w, w) for w in pml], mode="edge")
    h = 0.05
    om = 2 * np.pi * 1.5 / (8.0 * h)
    print(f"[3d degenerate plane {c.shape} pml {pml} {sf}]", flush=True)
    ref = Problem3D(c, om, h, pml, J=3, w_dd=2)
    from paper_1412_0464_amd import Helmholtz
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, pml, 3, w_dd=2, slab_factor=sf)
    try:
        for j in range(hs.J):
            nl = hs.x1[j] - hs.x0[j] + 1
            b = random_rhs((nl,) + tuple(hs.dd_shape[1:]), 60 + j)
            assert _relerr(hs.slab_solve(j, _t(b)).cpu().numpy().ravel(), ref.dd.lu[j].solve(b.ravel())) < TOL32
        f = random_rhs(hs.dd_shape, 70)
        assert _relerr(hs.sweep(_t(f)).cpu().numpy(), ref.dd.apply_x(f.ravel())) < TOL32
        r = random_rhs(c.shape, 71)
        assert _relerr(hs.apply_precond(_t(r)).cpu().numpy(), ref.precond(r.ravel())) < TOL32
    finally:
        hs.close()
