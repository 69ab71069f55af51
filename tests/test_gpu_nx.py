"""GPU parity of the partial-sweep preconditioner SweepingPrecNX (Sec. 2.2,
main-algorithm table) against the oracle: the sweep alone, one- and
two-level preconditioners, FGMRES, the batched and grouped forms (groups of
slabs sharing every stage launch) and the 3-D path.  Tolerances as for the
X- and UD-sweeps: FP64 maps 1e-10, complex64 maps 2e-5 (2e-4 in 3-D),
iteration counts within +-1."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.problem import Problem2D  # noqa: E402
from oracle.problem3d import Problem3D  # noqa: E402
from synth.media import layered_medium_2d, extend_into_pml, point_source, random_rhs, smooth_medium_3d  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")]

# (name, n1, n2, w, J, two_grid, ncell)
CASES = {
    "nx2_1lvl": (71, 45, 6, 5, False, 2),
    "nx3_1lvl": (97, 39, 6, 7, False, 3),
    "nx2_tg": (111, 63, 8, 5, True, 2),
    "nx3_tg": (159, 47, 8, 7, True, 3),
}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _build(name, precision="fp64"):
    n1, n2, w, J, tg, ncell = CASES[name]
    c = extend_into_pml(layered_medium_2d(n1, n2, 1412046, n_layers=7, corr_len=6.0), w)
    h = 0.02
    om = 2 * np.pi * 1.5 / (8.0 * h)
    print(f"[nx case {name} precision={precision} shape={c.shape}]", flush=True)
    ref = Problem2D(c, om, h, w, S_outer=5.0 * w, J=J, w_dd=4, two_grid=tg, sweep="nx", ncell=ncell)
    from paper_1412_0464_amd import Helmholtz
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, J, S_outer=5.0 * w, two_grid=tg, sweep="nx",
                   ncell=ncell, precision=precision)
    return c, ref, hs


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device=_dev())


def _relerr(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name", list(CASES))
def test_nx_sweep_and_precond_fp64(name):
    c, ref, hs = _build(name)
    try:
        ncell = CASES[name][5]
        f = random_rhs(hs.dd_shape, 60)
        u = hs.sweep(_t(f)).cpu().numpy()
        assert _relerr(u, ref.dd.apply_nx(f, ncell)) < 1e-10
        r = random_rhs(c.shape, 61)
        assert _relerr(hs.apply_precond(_t(r)).cpu().numpy(), ref.precond(r.ravel())) < 1e-10
    finally:
        hs.close()


@pytest.mark.parametrize("name", ["nx2_1lvl", "nx3_tg"])
def test_nx_solve_fp64(name):
    c, ref, hs = _build(name)
    try:
        f = point_source(c.shape, (c.shape[0] // 2, c.shape[1] // 3), 0.02)
        uo, ito, _, _ = ref.solve(f, tol=1e-6, maxit=150)
        u, it, rr = hs.solve(hs.rhs(_t(f)), tol=1e-6, maxit=150)
        print(f"[nx solve {name}: {it} iterations, oracle {ito}]", flush=True)
        assert abs(it - ito) <= 1 and rr <= 1e-6
        assert _relerr(u.cpu().numpy(), uo) < 1e-6
    finally:
        hs.close()


@pytest.mark.parametrize("tile", [1, 4])
def test_nx_batched_and_grouped_mixed(tile):
    """Batched columns of an NX problem, and a group that mixes it with an
    X-sweep problem (different buffer counts and stage widths)."""
    from paper_1412_0464_amd import Group, Helmholtz
    c, ref, hs = _build("nx3_tg", "mixed")
    n1, n2, w = 63, 79, 8
    c2 = extend_into_pml(layered_medium_2d(n1, n2, 1412046, n_layers=7, corr_len=6.0), w)
    h = 0.02
    om = 2 * np.pi * 1.5 / (8.0 * h)
    ref2 = Problem2D(c2, om, h, w, S_outer=5.0 * w, J=3, w_dd=4, two_grid=True)
    hs2 = Helmholtz(torch.tensor(c2, device=_dev()), om, h, w, 3, S_outer=5.0 * w, two_grid=True, precision="mixed")
    try:
        R = np.stack([random_rhs(c.shape, 70 + j) for j in range(5)])
        Z = hs.apply_precond_batch(_t(R), tile=tile).cpu().numpy()
        for j in range(5):
            assert _relerr(Z[j], ref.precond(R[j].ravel())) < 2e-5
        R2 = np.stack([random_rhs(c2.shape, 80 + j) for j in range(3)])
        Zs = Group([hs, hs2]).apply_precond([_t(R[:2]), _t(R2)], tile=tile)
        for j in range(2):
            assert _relerr(Zs[0][j].cpu().numpy(), ref.precond(R[j].ravel())) < 2e-5
        for j in range(3):
            assert _relerr(Zs[1][j].cpu().numpy(), ref2.precond(R2[j].ravel())) < 2e-5
        f = point_source(c.shape, (c.shape[0] // 2, c.shape[1] // 3), 0.02)
        B = torch.stack([hs.rhs(_t(f))] * 2)
        U, its, rrs = hs.solve_batch(B, tol=1e-6, maxit=150, tile=tile)
        _, ito, _, _ = ref.solve(f, tol=1e-6, maxit=150)
        assert all(abs(i - ito) <= 1 for i in its) and max(rrs) <= 1e-6
    finally:
        hs.close()
        hs2.close()


@pytest.mark.parametrize("sf", ["nd", "block"])
def test_nx_3d_sweep_and_precond(sf):
    n, w, J = (33, 9, 11), 4, 5
    c = np.pad(smooth_medium_3d(*n, 1412047, corr_len=3.0), w, mode="edge")
    h = 0.05
    om = 2 * np.pi * 1.5 / (10.0 * h)
    print(f"[nx 3d, shape {c.shape}, slab_factor {sf}]", flush=True)
    ref = Problem3D(c, om, h, w, J=J, w_dd=2, two_grid=True, sweep="nx", ncell=2, omega_jac=0.6)
    from paper_1412_0464_amd import Helmholtz
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, J, two_grid=True, sweep="nx", ncell=2, w_dd=2,
                   omega_jac=0.6, slab_factor=sf)
    try:
        f = random_rhs(hs.dd_shape, 90)
        assert _relerr(hs.sweep(_t(f)).cpu().numpy(), ref.dd.apply_nx(f.ravel(), 2)) < 2e-4
        r = random_rhs(c.shape, 91)
        assert _relerr(hs.apply_precond(_t(r)).cpu().numpy(), ref.precond(r.ravel())) < 2e-4
    finally:
        hs.close()
