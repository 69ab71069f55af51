"""GPU parity: every step of the HIP path against the CPU oracle.

Element-wise comparisons on seeded inputs at sizes that span several
threadblocks and ragged tails; full-size configuration-2 checks on sampled
rows and on properties (true residual).  Tolerances: FP64 kernels 1e-12
relative, FP64 composite maps 1e-10, complex64 maps 1e-5 (the acceptance
bar for solves: 1e-6 in FP64, 1e-4 in mixed precision after refinement,
iteration counts within +-1).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

from oracle.problem import Problem2D  # noqa: E402
from oracle import dd as DD  # noqa: E402
from synth.media import layered_medium_2d, extend_into_pml, point_source, random_rhs  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


# (name, n1, n2, w, J, fine, two_grid, sweep, ppw)
CASES = {
    "fd5_1lvl_x": (61, 45, 6, 3, "fd5", False, "x", 8.0),
    "fd5_1lvl_ud": (51, 39, 5, 4, "fd5", False, "ud", 8.0),
    "fe9_1lvl_x": (47, 53, 5, 4, "fe9", False, "x", 10.0),
    "tg_x": (63, 79, 8, 3, "fd5", True, "x", 8.0),
    "tg_ud": (79, 63, 8, 2, "fd5", True, "ud", 8.0),
    "tg_x_j5": (127, 95, 8, 5, "fd5", True, "x", 8.0),
    # thicker slabs (53 and 40 layers): the chain kernels for thick slabs
    "thick53_1lvl_x": (85, 41, 6, 2, "fd5", False, "x", 8.0),
    "thick40_tg_x": (111, 47, 8, 2, "fd5", True, "x", 8.0),
}


def _build(name, precision="fp64", J=None, chunk=0):
    n1, n2, w, J0, fine, tg, sweep, ppw = CASES[name]
    J = J0 if J is None else J
    c = extend_into_pml(layered_medium_2d(n1, n2, 1412046, n_layers=7, corr_len=6.0), w)
    h = 0.02
    om = 2 * np.pi * 1.5 / (ppw * h)
    print(f"[case {name} precision={precision} J={J} chunk={chunk} shape={c.shape}]", flush=True)
    ref = Problem2D(c, om, h, w, S_outer=5.0 * w, J=J, w_dd=4, fine=fine, two_grid=tg, sweep=sweep)
    from paper_1412_0464_amd import Helmholtz
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, J, S_outer=5.0 * w,
                   fine_stencil=5 if fine == "fd5" else 9, two_grid=tg, sweep=sweep, precision=precision,
                   chunk=chunk)
    return c, ref, hs


def _rand(shape, seed):
    return random_rhs(shape, seed)


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device=_dev())


def _relerr(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _maxrel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(CASES))
def test_partition_matches(name):
    c, ref, hs = _build(name)
    assert hs.beta == ref.dd.beta
    assert [(a, b) for a, b in zip(hs.x0, hs.x1)] == ref.dd.extents


@pytest.mark.parametrize("name", ["fd5_1lvl_x", "fe9_1lvl_x", "tg_x"])
def test_fine_operator_and_rhs(name):
    c, ref, hs = _build(name)
    x = _rand(c.shape, 1)
    y = hs.apply_operator(_t(x)).cpu().numpy()
    assert _maxrel(y.ravel(), ref.A @ x.ravel()) < 1e-12
    f = _rand(c.shape, 2)
    b = hs.rhs(_t(f)).cpu().numpy()
    assert _maxrel(b.ravel(), ref.rhs(f)) < 1e-13


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
def test_coarse_operator(precision, tol):
    c, ref, hs = _build("tg_x_j5", precision)
    Ac = ref.coarse.matrix()
    x = _rand(hs.n_coarse, 3)
    y = hs.apply_level_operator(1, _t(x)).cpu().numpy()
    assert _maxrel(y.ravel(), Ac @ x.ravel()) < tol


def test_transfers_and_smoother():
    c, ref, hs = _build("tg_x_j5")
    tg = ref.tg
    r = _rand(c.shape, 4)
    rc = hs.restrict(_t(r)).cpu().numpy()
    assert _maxrel(rc.ravel(), tg.R @ r.ravel()) < 1e-13
    e = _rand(hs.n_coarse, 5)
    x0 = _rand(c.shape, 6)
    xg = hs.prolong_add(_t(e), _t(x0)).cpu().numpy()
    assert _maxrel(xg.ravel(), x0.ravel() + tg.P @ e.ravel()) < 1e-13
    for steps in (1, 3):
        xs = hs.smooth(_t(r), steps).cpu().numpy()
        xo = tg.smooth(np.zeros(r.size, complex), r.ravel(), steps)
        assert _maxrel(xs.ravel(), xo) < 1e-11


@pytest.mark.parametrize("name,precision,tol", [
    ("fd5_1lvl_x", "fp64", 1e-10), ("fe9_1lvl_x", "fp64", 1e-10), ("tg_x_j5", "fp64", 1e-10),
    ("tg_x_j5", "mixed", 2e-5), ("thick53_1lvl_x", "fp64", 1e-10), ("thick53_1lvl_x", "mixed", 2e-5),
    ("thick40_tg_x", "fp64", 1e-10)])
def test_slab_solves(name, precision, tol):
    c, ref, hs = _build(name, precision)
    for j in range(hs.J):
        nl = hs.x1[j] - hs.x0[j] + 1
        b = _rand((nl, hs.dd_shape[1]), 10 + j)
        x = hs.slab_solve(j, _t(b)).cpu().numpy()
        xo = ref.dd.lu[j].solve(b.ravel())
        assert _relerr(x, xo) < tol, (j, _relerr(x, xo))


@pytest.mark.parametrize("name", list(CASES))
def test_sweep_fp64(name):
    c, ref, hs = _build(name)
    f = _rand(hs.dd_shape, 20)
    u = hs.sweep(_t(f)).cpu().numpy()
    uo = (ref.dd.apply_x if CASES[name][6] == "x" else ref.dd.apply_ud)(f)
    assert _relerr(u, uo) < 1e-10


@pytest.mark.parametrize("chunk", [1, 7, 13, 64])
def test_sweep_chunk_geometry(chunk):
    """The parallel substitutions give the same sweep for any chunk length:
    one block per chunk, ragged last chunks, and a single chunk."""
    c, ref, hs = _build("fd5_1lvl_x", chunk=chunk)
    f = _rand(hs.dd_shape, 22)
    u = hs.sweep(_t(f)).cpu().numpy()
    assert _relerr(u, ref.dd.apply_x(f)) < 1e-10
    for j in range(hs.J):
        nl = hs.x1[j] - hs.x0[j] + 1
        b = _rand((nl, hs.dd_shape[1]), 40 + j)
        x = hs.slab_solve(j, _t(b)).cpu().numpy()
        assert _relerr(x, ref.dd.lu[j].solve(b.ravel())) < 1e-10


def test_sweep_mixed():
    c, ref, hs = _build("tg_x_j5", "mixed")
    f = _rand(hs.dd_shape, 21)
    u = hs.sweep(_t(f)).cpu().numpy()
    assert _relerr(u, ref.dd.apply_x(f)) < 2e-5


@pytest.mark.parametrize("name", list(CASES))
def test_precond_fp64(name):
    c, ref, hs = _build(name)
    r = _rand(c.shape, 30)
    z = hs.apply_precond(_t(r)).cpu().numpy()
    assert _relerr(z, ref.precond(r.ravel())) < 1e-10


@pytest.mark.parametrize("name", ["fd5_1lvl_x", "tg_x_j5"])
def test_precond_mixed(name):
    c, ref, hs = _build(name, "mixed")
    r = _rand(c.shape, 31)
    z = hs.apply_precond(_t(r)).cpu().numpy()
    assert _relerr(z, ref.precond(r.ravel())) < 2e-5


@pytest.mark.parametrize("name", list(CASES))
def test_solve_fp64(name):
    c, ref, hs = _build(name)
    f = point_source(c.shape, (c.shape[0] // 2, c.shape[1] // 3), 0.02)
    uo, ito, _, rro = ref.solve(f, tol=1e-6, maxit=100)
    u, it, rr = hs.solve(hs.rhs(_t(f)), tol=1e-6, maxit=100)
    u = u.cpu().numpy()
    assert abs(it - ito) <= 1 and rr <= 1e-6
    assert _relerr(u, uo) < 1e-6


@pytest.mark.parametrize("name", ["fd5_1lvl_x", "tg_x_j5"])
def test_solve_mixed_after_refinement(name):
    c, ref, hs = _build(name, "mixed")
    f = point_source(c.shape, (c.shape[0] // 3, c.shape[1] // 2), 0.02)
    u_direct = ref.direct(f)
    u, it, rr = hs.solve(hs.rhs(_t(f)), tol=1e-10, maxit=200)
    assert rr <= 1e-10
    assert _relerr(u.cpu().numpy(), u_direct) < 1e-4
    _, it6, rr6 = hs.solve(hs.rhs(_t(f)), tol=1e-6, maxit=200)
    _, ito6, _, _ = ref.solve(f, tol=1e-6, maxit=200)
    assert rr6 <= 1e-6 and abs(it6 - ito6) <= 1


def test_conjugate_transpose_solve():
    c, ref, hs = _build("tg_x")
    b = _rand(c.shape, 40)
    u, it, rr = hs.solve(_t(b), tol=1e-10, maxit=100, conj_transpose=True)
    A = ref.A
    res = A.conj().T @ u.cpu().numpy().ravel() - b.ravel()
    assert np.linalg.norm(res) / np.linalg.norm(b) < 1e-9


# ---------------------------------------------------------------------------
# degenerate cases and errors
# ---------------------------------------------------------------------------
def test_single_slab_is_exact():
    n, w = 31, 5
    c = extend_into_pml(layered_medium_2d(n, n, 3, n_layers=4, corr_len=4.0), w)
    h, om = 0.05, 2 * np.pi * 1.5 / (8 * 0.05)
    from paper_1412_0464_amd import Helmholtz
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, 1)
    ref = Problem2D(c, om, h, w, S_outer=5.0 * w, J=1)
    b = _rand(c.shape, 50)
    u, it, rr = hs.solve(_t(b), tol=1e-10, maxit=10)
    assert it == 1 and rr < 1e-10
    z = hs.apply_precond(_t(b)).cpu().numpy()
    assert _relerr(z, spla.spsolve(ref.A.tocsc(), b.ravel())) < 1e-11


def test_two_slabs_x_equals_ud():
    outs = []
    for sweep in ("x", "ud"):
        CASES["_j2"] = (45, 37, 5, 2, "fd5", False, sweep, 8.0)
        c, ref, hs = _build("_j2")
        outs.append(hs.apply_precond(_t(_rand(c.shape, 60))).cpu().numpy())
    del CASES["_j2"]
    assert _relerr(outs[0], outs[1]) < 1e-12


def test_invalid_medium_rejected():
    from paper_1412_0464_amd import Helmholtz, HspError
    c = np.ones((41, 41))
    c[7, 9] = -1.0
    with pytest.raises(HspError) as e:
        Helmholtz(torch.tensor(c, device=_dev()), 10.0, 0.05, 5, 2)
    assert e.value.status == -1
    c[7, 9] = np.nan
    with pytest.raises(HspError):
        Helmholtz(torch.tensor(c, device=_dev()), 10.0, 0.05, 5, 2)


# ---------------------------------------------------------------------------
# configuration 1 end to end
# ---------------------------------------------------------------------------
def test_config1_end_to_end():
    n, w = 127, 10
    N = n + 1 + 2 * w
    h, om = 1.0 / 128, 2 * np.pi * 12.8
    c = np.ones((N - 1, N - 1))
    f = point_source(c.shape, (73, 73), h)
    print("[case config1 127^2 + 10 PML, 5-pt, J=4, X-sweep, complex128]", flush=True)
    ref = Problem2D(c, om, h, w, S_outer=50, c_pml=1.0, J=4, w_dd=4, S_dd=20)
    uo, ito, _, _ = ref.solve(f, tol=1e-6)
    from paper_1412_0464_amd import Helmholtz
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, 4, S_outer=50, c_pml=1.0, S_dd=20)
    u, it, rr = hs.solve(hs.rhs(_t(f)), tol=1e-6)
    assert it == ito and rr <= 1e-6
    assert _relerr(u.cpu().numpy(), uo) < 1e-6


@pytest.mark.parametrize("fine,nu,precision,tol", [
    ("fd5", 1, "fp64", 1e-10), ("fd5", 2, "mixed", 2e-5), ("fd5", 4, "fp64", 1e-10), ("fe9", 3, "mixed", 2e-5)])
def test_precond_smoothing_variants(fine, nu, precision, tol):
    """Two-grid preconditioner with 1, 2 or 4 smoothing steps and with the
    9-point fine operator (fused single-kernel smoothing phases for the
    5-point fine level with nu <= 3, step-by-step kernels otherwise)."""
    n1, n2, w, J = 79, 63, 8, 3
    c = extend_into_pml(layered_medium_2d(n1, n2, 1412046, n_layers=7, corr_len=6.0), w)
    h = 0.02
    om = 2 * np.pi * 1.5 / (8.0 * h)
    print(f"[smoothing variant fine={fine} nu={nu} {precision}]", flush=True)
    ref = Problem2D(c, om, h, w, S_outer=5.0 * w, J=J, w_dd=4, fine=fine, two_grid=True, nu=nu)
    from paper_1412_0464_amd import Helmholtz
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, J, S_outer=5.0 * w,
                   fine_stencil=5 if fine == "fd5" else 9, two_grid=True, nu=nu, precision=precision)
    r = _rand(c.shape, 70 + nu)
    assert _relerr(hs.apply_precond(_t(r)).cpu().numpy(), ref.precond(r.ravel())) < tol
    R = np.stack([_rand(c.shape, 80 + j) for j in range(3)])
    Z = hs.apply_precond_batch(_t(R), tile=2).cpu().numpy()
    for j in range(3):
        assert _relerr(Z[j], ref.precond(R[j].ravel())) < tol


# ---------------------------------------------------------------------------
# failure paths through the C ABI (Sec. 5: block LU with pivoting inside
# each block; FGMRES that stops at maxit)
# ---------------------------------------------------------------------------
def _small_problem():
    n1, n2, w = 47, 39, 5
    c = extend_into_pml(layered_medium_2d(n1, n2, 1412046, n_layers=7, corr_len=6.0), w)
    h = 0.02
    return c, 2 * np.pi * 1.5 / (8.0 * h), h, w


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_singular_slab_block_gives_esingular(precision):
    from paper_1412_0464_amd import Helmholtz, HspError, hsp
    c, om, h, w = _small_problem()
    print(f"[failure path: singular first block of slab 1, {precision}]", flush=True)
    hsp.debug_set("singular_slab", 1)
    try:
        with pytest.raises(HspError) as e:
            Helmholtz(torch.tensor(c, device=_dev()), om, h, w, 3, precision=precision)
        assert e.value.status == hsp.HSP_ESINGULAR
        assert "pivot" in str(e.value)
    finally:
        hsp.debug_set("singular_slab", -1)
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, 3, precision=precision)
    print(f"[pivot growth {hs.pivot_growth:.4f}]", flush=True)
    assert 0.0 < hs.pivot_growth < 1e3
    hs.close()


def test_pivot_growth_guard():
    """The setup refuses factors whose Schur complements grew beyond the
    limit (here set below the growth measured for this medium)."""
    from paper_1412_0464_amd import Helmholtz, HspError, hsp
    c, om, h, w = _small_problem()
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, 3, precision="mixed")
    g = hs.pivot_growth
    hs.close()
    print(f"[failure path: growth limit below the measured growth {g:.3f}]", flush=True)
    hsp.debug_set("growth_limit", 0.5 * g)
    try:
        with pytest.raises(HspError) as e:
            Helmholtz(torch.tensor(c, device=_dev()), om, h, w, 3, precision="mixed")
        assert e.value.status == hsp.HSP_ESINGULAR and "growth" in str(e.value)
    finally:
        hsp.debug_set("growth_limit", 0.0)


def test_maxit_gives_enoconv_with_last_iterate():
    from paper_1412_0464_amd import Helmholtz, HspError, hsp
    c, om, h, w = _small_problem()
    ref = Problem2D(c, om, h, w, S_outer=5.0 * w, J=3, w_dd=4)
    f = point_source(c.shape, (c.shape[0] // 2, c.shape[1] // 2), h)
    print("[failure path: maxit = 1, single and batched]", flush=True)
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, 3, S_outer=5.0 * w)
    try:
        b = hs.rhs(_t(f))
        with pytest.raises(HspError) as e:
            hs.solve(b, tol=1e-10, maxit=1)
        assert e.value.status == hsp.HSP_ENOCONV
        u, it, rr = hs.solve(b, tol=1e-10, maxit=1, raise_on_noconv=False)
        assert it == 1 and rr > 1e-10
        # the returned iterate is the oracle's first FGMRES iterate
        uo, ito, _, _ = ref.solve(f, tol=1e-10, maxit=1)
        assert ito == 1 and _relerr(u.cpu().numpy(), uo) < 1e-10
        B = torch.stack([b, b])
        with pytest.raises(HspError) as e:
            hs.solve_batch(B, tol=1e-10, maxit=1)
        assert e.value.status == hsp.HSP_ENOCONV
        U, its, rrs = hs.solve_batch(B, tol=1e-10, maxit=1, raise_on_noconv=False)
        assert its == [1, 1] and min(rrs) > 1e-10
        assert _relerr(U[1].cpu().numpy(), uo) < 1e-10
    finally:
        hs.close()
