"""GPU parity of the batched multi-right-hand-side path against the CPU oracle.

The batched preconditioner is the same linear map as the single one, applied
to every column: each column is compared with the oracle's preconditioner
(FP64 1e-10, complex64 2e-5 relative).  The batched FGMRES runs one Arnoldi
process per right-hand side with its own stopping test, so each column must
reproduce the oracle's FGMRES on that right-hand side: iteration counts
within +-1 and solutions within 1e-6 (FP64) or, after refinement to 1e-10,
within 1e-4 of the direct solution (mixed).  Batches are ragged with respect
to every tile size, mix sources that converge at different iterations, and
include a zero right-hand side (0 iterations, u = 0).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.problem import Problem2D  # noqa: E402
from oracle.krylov import fgmres  # noqa: E402
from synth.media import layered_medium_2d, extend_into_pml, point_source, random_rhs  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")]

# (n1, n2, w, J, fine, two_grid, sweep, ppw)
CASES = {
    "fd5_1lvl_x": (61, 45, 6, 3, "fd5", False, "x", 8.0),
    "fe9_1lvl_x": (47, 53, 5, 4, "fe9", False, "x", 10.0),
    "tg_ud": (79, 63, 8, 2, "fd5", True, "ud", 8.0),
    "tg_x_j5": (127, 95, 8, 5, "fd5", True, "x", 8.0),
    # thicker slabs (38, 53 and 40 layers): the chain layouts on 64 row lanes
    # with 40 and 64 product columns
    "thick38_1lvl_x": (55, 41, 6, 2, "fd5", False, "x", 8.0),
    "thick53_1lvl_x": (85, 41, 6, 2, "fd5", False, "x", 8.0),
    "thick40_tg_x": (111, 47, 8, 2, "fd5", True, "x", 8.0),
}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _build(name, precision="fp64", chunk=0, restart=40, **extra):
    n1, n2, w, J, fine, tg, sweep, ppw = CASES[name]
    c = extend_into_pml(layered_medium_2d(n1, n2, 1412046, n_layers=7, corr_len=6.0), w)
    h = 0.02
    om = 2 * np.pi * 1.5 / (ppw * h)
    print(f"[batch case {name} precision={precision} chunk={chunk} {extra} shape={c.shape}]", flush=True)
    ref = Problem2D(c, om, h, w, S_outer=5.0 * w, J=J, w_dd=4, fine=fine, two_grid=tg, sweep=sweep)
    from paper_1412_0464_amd import Helmholtz
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, J, S_outer=5.0 * w,
                   fine_stencil=5 if fine == "fd5" else 9, two_grid=tg, sweep=sweep, precision=precision,
                   chunk=chunk, restart=restart, **extra)
    return c, ref, hs


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device=_dev())


def _relerr(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _sources(shape, h, nsrc):
    """Point sources spread over the interior (they converge at different
    iterations), plus a zero right-hand side at index 1."""
    rng = np.random.default_rng(1412047)
    fs = []
    for s in range(nsrc):
        if s == 1:
            fs.append(np.zeros(shape, dtype=complex))
            continue
        i = int(rng.integers(shape[0] // 5, 4 * shape[0] // 5))
        k = int(rng.integers(shape[1] // 5, 4 * shape[1] // 5))
        fs.append(point_source(shape, (i, k), h))
    return fs


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,precision,tol", [
    ("fd5_1lvl_x", "fp64", 1e-10), ("fe9_1lvl_x", "fp64", 1e-10), ("tg_ud", "fp64", 1e-10),
    ("tg_x_j5", "fp64", 1e-10), ("tg_x_j5", "mixed", 2e-5), ("fd5_1lvl_x", "mixed", 2e-5),
    ("thick38_1lvl_x", "fp64", 1e-10), ("thick53_1lvl_x", "fp64", 1e-10), ("thick53_1lvl_x", "mixed", 2e-5),
    ("thick40_tg_x", "fp64", 1e-10), ("thick40_tg_x", "mixed", 2e-5)])
@pytest.mark.parametrize("tile", [1, 2, 4, 8])
def test_batch_precond_columns(name, precision, tol, tile):
    c, ref, hs = _build(name, precision)
    nrhs = 5  # ragged for tiles 2, 4 and 8
    R = np.stack([random_rhs(c.shape, 300 + j) for j in range(nrhs)])
    Z = hs.apply_precond_batch(_t(R), tile=tile).cpu().numpy()
    for j in range(nrhs):
        assert _relerr(Z[j], ref.precond(R[j].ravel())) < tol, f"column {j}"


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 2e-5)])
def test_batch_precond_columns_many(precision, tol):
    """18 right-hand sides: the batched stencil launches take the sources in
    groups (a full group and a ragged one), here in the coarse residual of
    every sweep."""
    c, ref, hs = _build("tg_x_j5", precision)
    nrhs = 18
    R = np.stack([random_rhs(c.shape, 340 + j) for j in range(nrhs)])
    Z = hs.apply_precond_batch(_t(R), tile=4).cpu().numpy()
    for j in range(nrhs):
        assert _relerr(Z[j], ref.precond(R[j].ravel())) < tol, f"column {j}"


def test_batch_solve_many_sources():
    """18 sources (one of them zero) through the batched FGMRES: the
    matvec and coarse-residual launches cover two groups of sources until
    enough of them have converged."""
    c, ref, hs = _build("tg_x_j5")
    fs = _sources(c.shape, 0.02, 18)
    B = torch.stack([hs.rhs(_t(f)) for f in fs])
    U, its, rrs = hs.solve_batch(B, tol=1e-6, maxit=100)
    U = U.cpu().numpy()
    for j, f in enumerate(fs):
        if not np.any(f):
            assert its[j] == 0 and rrs[j] == 0 and not np.any(U[j])
            continue
        uo, ito, _, _ = ref.solve(f, tol=1e-6, maxit=100)
        assert abs(its[j] - ito) <= 1 and rrs[j] <= 1e-6, f"column {j}: {its[j]} vs {ito}, {rrs[j]}"
        assert _relerr(U[j], uo) < 1e-6, f"column {j}"


@pytest.mark.parametrize("chunk", [7, 64])
def test_batch_precond_chunk_geometry(chunk):
    c, ref, hs = _build("tg_x_j5", "fp64", chunk=chunk)
    nrhs = 9
    R = np.stack([random_rhs(c.shape, 320 + j) for j in range(nrhs)])
    Z = hs.apply_precond_batch(_t(R), tile=8).cpu().numpy()
    for j in range(nrhs):
        assert _relerr(Z[j], ref.precond(R[j].ravel())) < 1e-10, f"column {j}"


def test_batch_precond_single_column_equals_single_path():
    c, ref, hs = _build("tg_x_j5", "mixed")
    r = random_rhs(c.shape, 330)
    z1 = hs.apply_precond(_t(r)).cpu().numpy()
    zb = hs.apply_precond_batch(_t(r[None])).cpu().numpy()[0]
    # same factors and the same linear map; only the evaluation order differs
    assert _relerr(zb, z1) < 2e-5


@pytest.mark.parametrize("name", ["fd5_1lvl_x", "tg_x_j5", "tg_ud", "thick53_1lvl_x", "thick40_tg_x"])
def test_batch_solve_fp64(name):
    c, ref, hs = _build(name)
    fs = _sources(c.shape, 0.02, 6)
    B = torch.stack([hs.rhs(_t(f)) for f in fs])
    U, its, rrs = hs.solve_batch(B, tol=1e-6, maxit=100)
    U = U.cpu().numpy()
    for j, f in enumerate(fs):
        if not np.any(f):
            assert its[j] == 0 and rrs[j] == 0 and not np.any(U[j])
            continue
        uo, ito, _, _ = ref.solve(f, tol=1e-6, maxit=100)
        assert abs(its[j] - ito) <= 1 and rrs[j] <= 1e-6, f"column {j}: {its[j]} vs {ito}, {rrs[j]}"
        assert _relerr(U[j], uo) < 1e-6, f"column {j}"


@pytest.mark.parametrize("krylov_fp32", [False, True])
def test_batch_solve_mixed_after_refinement(krylov_fp32):
    """Mixed precision, with the Arnoldi basis in complex128 (default) or in
    complex64 (krylov_fp32): refined to 1e-10 it reaches the direct solution;
    at 1e-6 each column takes the oracle's iteration count within +-1."""
    c, ref, hs = _build("tg_x_j5", "mixed", krylov_fp32=krylov_fp32)
    fs = _sources(c.shape, 0.02, 5)
    B = torch.stack([hs.rhs(_t(f)) for f in fs])
    U, its, rrs = hs.solve_batch(B, tol=1e-10, maxit=200)
    U = U.cpu().numpy()
    for j, f in enumerate(fs):
        if not np.any(f):
            continue
        assert rrs[j] <= 1e-10
        assert _relerr(U[j], ref.direct(f)) < 1e-4, f"column {j}"
    _, its6, rrs6 = hs.solve_batch(B, tol=1e-6, maxit=200)
    for j, f in enumerate(fs):
        if not np.any(f):
            continue
        _, ito6, _, _ = ref.solve(f, tol=1e-6, maxit=200)
        assert rrs6[j] <= 1e-6 and abs(its6[j] - ito6) <= 1, f"column {j}: {its6[j]} vs {ito6}"


def test_batch_solve_profile_classes():
    """Event timing of the batched solve: one matvec, one projection pass and
    one update pass per Arnoldi step of the batch, stage and smoothing classes
    non-empty, byte counts positive."""
    c, ref, hs = _build("tg_x_j5", "mixed")
    fs = _sources(c.shape, 0.02, 4)
    B = torch.stack([hs.rhs(_t(f)) for f in fs])
    hs.solve_batch(B, tol=1e-6, maxit=200)  # warm-up
    hs.profile(True)
    try:
        for cls in ("stage", "smooth", "coarse", "transfer", "krylov", "project", "update"):
            hs.profile_read(cls)
        _, its, rrs = hs.solve_batch(B, tol=1e-6, maxit=200)
        got = {cls: hs.profile_read(cls) for cls in ("stage", "smooth", "krylov", "project", "update")}
    finally:
        hs.profile(False)
    steps = max(its)
    assert got["project"][1] == steps and got["update"][1] == steps and got["krylov"][1] == steps, (got, its)
    for cls, (ms, n, by) in got.items():
        assert n > 0 and ms > 0 and by > 0, (cls, ms, n, by)
    assert max(rrs) <= 1e-6


def test_batch_solve_restarted():
    restart = 4
    c, ref, hs = _build("tg_x_j5", "fp64", restart=restart)
    fs = _sources(c.shape, 0.02, 3)
    B = torch.stack([hs.rhs(_t(f)) for f in fs])
    U, its, rrs = hs.solve_batch(B, tol=1e-8, maxit=200, restart=restart)
    U = U.cpu().numpy()
    for j, f in enumerate(fs):
        if not np.any(f):
            continue
        uo, ito, _, _ = fgmres(ref.matvec, ref.precond, ref.rhs(f), tol=1e-8, maxit=200, restart=restart)
        assert abs(its[j] - ito) <= 1 and rrs[j] <= 1e-8, f"column {j}: {its[j]} vs {ito}"
        assert _relerr(U[j], uo) < 1e-6


def test_batch_conjugate_transpose():
    c, ref, hs = _build("tg_ud")
    B = np.stack([random_rhs(c.shape, 340 + j) for j in range(3)])
    U, its, rrs = hs.solve_batch(_t(B), tol=1e-10, maxit=100, conj_transpose=True)
    U = U.cpu().numpy()
    AH = ref.A.conj().T
    for j in range(3):
        res = AH @ U[j].ravel() - B[j].ravel()
        assert np.linalg.norm(res) / np.linalg.norm(B[j]) < 1e-9


def test_batch_empty_and_tune():
    c, ref, hs = _build("fd5_1lvl_x", "mixed")
    B = torch.zeros((0,) + tuple(c.shape), dtype=torch.complex128, device=_dev())
    U, its, rrs = hs.solve_batch(B)
    assert U.shape[0] == 0 and its == [] and rrs == []
    tile, ms = hs.tune_batch(6)
    assert tile in (1, 2, 4, 8) and ms > 0
    R = np.stack([random_rhs(c.shape, 350 + j) for j in range(6)])
    Z = hs.apply_precond_batch(_t(R)).cpu().numpy()
    for j in range(6):
        assert _relerr(Z[j], ref.precond(R[j].ravel())) < 2e-5


def test_batch_invalid_arguments():
    c, ref, hs = _build("fd5_1lvl_x")
    from paper_1412_0464_amd.hsp import HspError
    B = _t(np.stack([random_rhs(c.shape, 360)]))
    with pytest.raises(HspError):
        hs.solve_batch(B, tile=3)
    with pytest.raises(HspError):
        hs.solve_batch(B, tol=0.0)


# ---------------------------------------------------------------------------
# groups: several problems (sizes, slab counts, sweeps, one- and two-level)
# whose sweep stages share launches
# ---------------------------------------------------------------------------
GROUP = [("tg_x_j5", 3), ("tg_ud", 2), ("fd5_1lvl_x", 5), ("fe9_1lvl_x", 0)]


def _group(precision, **extra):
    from paper_1412_0464_amd import Group
    built = [_build(name, precision, **extra) for name, _ in GROUP]
    return built, Group([hs for _, _, hs in built], restart=40)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 2e-5)])
def test_group_precond_columns(precision, tol):
    built, grp = _group(precision)
    Rs = [np.stack([random_rhs(c.shape, 400 + 10 * p + j) for j in range(k)]) if k else
          np.zeros((0,) + c.shape, dtype=complex) for p, ((c, _, _), (_, k)) in enumerate(zip(built, GROUP))]
    Zs = grp.apply_precond([_t(R) for R in Rs], tile=2)
    for p, ((c, ref, _), (name, k)) in enumerate(zip(built, GROUP)):
        Z = Zs[p].cpu().numpy()
        for j in range(k):
            assert _relerr(Z[j], ref.precond(Rs[p][j].ravel())) < tol, f"{name} column {j}"


def test_group_graph_replays_match_eager():
    built, grp = _group("mixed")
    Rs = [_t(np.stack([random_rhs(c.shape, 450 + 10 * p + j) for j in range(max(k, 1))]))
          for p, ((c, _, _), (_, k)) in enumerate(zip(built, GROUP))]
    eager = [z.cpu().numpy() for z in grp.apply_precond(Rs, tile=4)]
    for rep in range(3):
        # eager work and a synchronisation between the replays
        grp.apply_precond(Rs, tile=1)
        torch.cuda.synchronize()
        got = [z.cpu().numpy() for z in grp.apply_precond(Rs, tile=4, graph=True)]
        for p in range(len(Rs)):
            assert np.array_equal(got[p], eager[p]), f"replay {rep} problem {p}"


@pytest.mark.parametrize("precision,graph,krylov_fp32", [("fp64", False, False), ("mixed", True, False),
                                                         ("mixed", False, True)])
def test_group_solve(precision, graph, krylov_fp32):
    built, grp = _group(precision, krylov_fp32=krylov_fp32)
    fss = [_sources(c.shape, 0.02, k) if k else [] for (c, _, _), (_, k) in zip(built, GROUP)]
    Bs = [torch.stack([hs.rhs(_t(f)) for f in fs]) if fs else
          torch.zeros((0,) + tuple(c.shape), dtype=torch.complex128, device=_dev())
          for (c, _, hs), fs in zip(built, fss)]
    tol = 1e-6 if precision == "fp64" else 1e-10
    Us, its, rrs = grp.solve(Bs, tol=tol, maxit=200, graph=graph)
    for p, ((c, ref, hs), fs) in enumerate(zip(built, fss)):
        U = Us[p].cpu().numpy()
        for j, f in enumerate(fs):
            if not np.any(f):
                assert its[p][j] == 0 and not np.any(U[j])
                continue
            assert rrs[p][j] <= tol
            if precision == "fp64":
                uo, ito, _, _ = ref.solve(f, tol=tol, maxit=200)
                assert abs(its[p][j] - ito) <= 1, f"problem {p} column {j}: {its[p][j]} vs {ito}"
                assert _relerr(U[j], uo) < 1e-6
            else:
                assert _relerr(U[j], ref.direct(f)) < 1e-4


def test_group_rejects_mixed_basis_precisions():
    """The members of a group share one Krylov layout: a group of problems
    whose Arnoldi bases are stored in different precisions is refused."""
    from paper_1412_0464_amd import Group
    from paper_1412_0464_amd.hsp import HspError
    _, _, h1 = _build("tg_x_j5", "mixed")
    _, _, h2 = _build("tg_ud", "mixed", krylov_fp32=True)
    with pytest.raises(HspError):
        Group([h1, h2], restart=40).workspace([1, 1])


def test_autotuner_choice_and_its_preconditioner():
    """hsp_autotune on a small two-grid problem: the chosen chunk length is
    one of the candidates (distinct chunk counts), the tile one of 1, 2, 4,
    8, every candidate was timed; the batched preconditioner set up with the
    choice matches the oracle's columns (complex64 tolerance)."""
    from paper_1412_0464_amd import hsp
    n1, n2, w, J, fine, tg, sweep, ppw = CASES["tg_x_j5"]
    c = extend_into_pml(layered_medium_2d(n1, n2, 1412046, n_layers=7, corr_len=6.0), w)
    h = 0.02
    om = 2 * np.pi * 1.5 / (ppw * h)
    print("[autotuner on tg_x_j5, 6 right-hand sides]", flush=True)
    chunk, tile, ms, table = hsp.autotune(torch.tensor(c, device=_dev()), om, h, w, J, 6, S_outer=5.0 * w,
                                          two_grid=True, precision="mixed")
    assert tile in (1, 2, 4, 8) and ms > 0
    assert len(table) >= 2 and (chunk, tile) in [(m, t) for m, t, _ in table]
    c_ref, ref, hs = _build("tg_x_j5", "mixed", chunk=chunk)
    try:
        ncoarse = hs.n_coarse[1]
        assert len({(ncoarse + m - 1) // m for m, _, _ in table}) == len(table)
        R = np.stack([random_rhs(c.shape, 300 + j) for j in range(6)])
        Z = hs.apply_precond_batch(_t(R), tile=tile).cpu().numpy()
        for j in (0, 5):
            assert _relerr(Z[j], ref.precond(R[j].ravel())) < 2e-5
    finally:
        hs.close()
