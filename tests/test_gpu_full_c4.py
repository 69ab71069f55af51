"""Full-size checks of the 3-D workload against the oracle.

The smooth random 3-D medium with 127^3 interior nodes and 8 PML cells per
side, 10 points per wavelength, the two-grid sweeping preconditioner with
the 7-point fine level and the 27-point FE coarse level (79^3), J = 16
coarse slabs with w_dd = 3: the configuration bench.py times.  The oracle
cannot run the whole preconditioner at this size in seconds (16 sparse LU
factorizations of 3-D slabs), so the checks use outputs it can compute one
by one and properties that hold at any size:

* the fine operator on a random vector (one sparse product), 1e-12;
* the solve of one middle slab (planes of 11 x 79 = 869 unknowns; 79 dense
  blocks, or the 1023 fronts of the nested dissection, factored on the FP32
  matrix cores) against the oracle's sparse LU of the same slab matrix,
  2e-4;
* the FGMRES solution of a point source: its true residual, recomputed with
  the oracle's operator, meets the tolerance 1e-6.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

import bench  # noqa: E402
from oracle import discretization as D, dd as DD, problem3d as P3, twogrid as TG  # noqa: E402
from synth.media import point_source, random_rhs  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")]


def _relerr(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def oracle4():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = bench.c4_config()
    c = bench.c4_medium(cfg)
    # the oracle's pieces: fine axes and operator, coarse level, partition
    n, w, h, om = cfg["n"], cfg["w"], cfg["h"], cfg["omega"]
    N = n + 1 + 2 * w
    cp = float(c.mean())
    axes = [D.uniform_axis(N, h, w, 5.0 * w, cp) for _ in range(3)]
    k2n = om ** 2 / c ** 2
    A = D.fd7_matrix(*axes, k2n, om).tocsr()
    cax, Ws = [], []
    for a in axes:
        ca, ifp, ref = TG.coarsen_axis(a, w)
        cax.append(ca)
        Ws.append(TG.cell_average_1d(ifp, ref, N))
    lev = P3.Level3D(*cax, om, "fe27", k2_cells=P3.cell_average_3d(*Ws, P3.pad_nodes_edge_3d(k2n)))
    beta = DD.partition(lev.n1, w, cfg["J"])
    return dict(cfg=cfg, c=c, A=A, axes=axes, lev=lev, beta=beta, cp=cp, slab={})


@pytest.fixture(scope="module", params=["nd", "block"])
def c4(request, oracle4):
    from paper_1412_0464_amd import Helmholtz
    cfg, c = oracle4["cfg"], oracle4["c"]
    print(f"[full size c4] {cfg['workload']}, {c.shape}: GPU setup, slab_factor {request.param}", flush=True)
    hs = Helmholtz(torch.tensor(c, device=torch.device("cuda:0")), cfg["omega"], cfg["h"], cfg["w"], cfg["J"],
                   two_grid=True, w_dd=cfg["w_dd"], omega_jac=cfg["omega_jac"], restart=60,
                   slab_factor=request.param)
    yield dict(oracle4, hs=hs)
    hs.close()


def test_c4_fine_operator(c4):
    x = random_rhs(c4["c"].shape, 1412070)
    y = c4["hs"].apply_operator(torch.tensor(x, dtype=torch.complex128, device="cuda:0")).cpu().numpy().ravel()
    assert _relerr(y, c4["A"] @ x.ravel()) < 1e-12


def test_c4_partition_and_middle_slab_solve(c4):
    hs, lev, beta, cfg = c4["hs"], c4["lev"], c4["beta"], c4["cfg"]
    assert hs.beta == list(beta)
    j = 8  # 1-based slab index of the oracle
    x0, x1 = DD.slab_extent(beta, j, cfg["w_dd"])
    assert (hs.x0[j - 1], hs.x1[j - 1]) == (x0, x1)
    b = random_rhs((x1 - x0 + 1, lev.n2, lev.n3), 1412071)
    if j not in c4["slab"]:
        print(f"[full size c4] oracle sparse LU of slab {j} ({x1 - x0 + 1} layers)", flush=True)
        As = lev.slab_level(beta, j, cfg["w_dd"], 5.0 * cfg["w_dd"], c4["cp"]).matrix().tocsc()
        c4["slab"][j] = spla.splu(As).solve(b.ravel())
    xo = c4["slab"][j]
    x = hs.slab_solve(j - 1, torch.tensor(b, dtype=torch.complex128, device="cuda:0")).cpu().numpy().ravel()
    err = _relerr(x, xo)
    print(f"[full size c4] slab {j} ({hs.slab_factor}): rel err {err:.2e}, pivot growth {hs.pivot_growth:.3f}",
          flush=True)
    assert err < 2e-4


def test_c4_solve_true_residual(c4):
    hs, A, c, cfg = c4["hs"], c4["A"], c4["c"], c4["cfg"]
    f = point_source(c.shape, tuple(s // 2 for s in c.shape), cfg["h"])
    ft = torch.tensor(f, dtype=torch.complex128, device="cuda:0")
    b = hs.rhs(ft)
    print("[full size c4] FGMRES to 1e-6", flush=True)
    u, it, rr = hs.solve(b, tol=1e-6, maxit=200)
    bb = b.cpu().numpy().ravel()
    rr_o = np.linalg.norm(bb - A @ u.cpu().numpy().ravel()) / np.linalg.norm(bb)
    print(f"[full size c4] {it} iterations, relres {rr:.3e}, oracle operator {rr_o:.3e}", flush=True)
    assert rr <= 1e-6 and rr_o <= 1.001e-6 and abs(rr - rr_o) < 1e-9
