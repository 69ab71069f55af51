"""The allocation-free batched preconditioner (hsp_apply_precond_batch_noalloc)
against hsp_apply_precond_batch: same kernels and tile, so the columns agree
bitwise; two calls in a row, the second with fewer right-hand sides (the
fixed scratch keeps the first call's contents); a batch larger than the fixed
scratch is refused."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth.media import layered_medium_2d, extend_into_pml, random_rhs  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("precision,tile", [("mixed", 2), ("fp64", 4)])
def test_noalloc_batch_matches_workspace_batch(precision, tile):
    from paper_1412_0464_amd import Helmholtz, hsp
    n1, n2, w, J = 79, 63, 8, 3
    c = extend_into_pml(layered_medium_2d(n1, n2, 1412046, n_layers=7, corr_len=6.0), w)
    h = 0.02
    om = 2 * np.pi * 1.5 / (8.0 * h)
    print(f"[noalloc batch {precision} tile {tile}]", flush=True)
    hs = Helmholtz(torch.tensor(c, device=_dev()), om, h, w, J, two_grid=True, precision=precision)
    lib = hsp.load()
    try:
        for nrhs in (5, 3):
            R = torch.tensor(np.stack([random_rhs(c.shape, 900 + 7 * nrhs + j) for j in range(nrhs)]),
                             dtype=torch.complex128, device=_dev())
            Zw = hs.apply_precond_batch(R, tile=tile)
            Zs = torch.empty_like(R)
            sb = ctypes.c_size_t()
            st = lib.hsp_apply_precond_batch_noalloc(hs.handle, nrhs, ctypes.c_void_p(R.data_ptr()),
                                                     ctypes.c_void_p(Zs.data_ptr()), tile, ctypes.byref(sb),
                                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            assert st == hsp.HSP_OK, lib.hsp_last_error()
            assert sb.value == 256 << 20
            torch.cuda.synchronize()
            assert torch.equal(Zs, Zw), f"nrhs {nrhs}: max diff {(Zs - Zw).abs().max().item():.3e}"
        # a batch that does not fit the fixed scratch is refused
        need = ctypes.c_size_t()
        big = 1
        while True:
            assert lib.hsp_batch_workspace_size(hs.handle, big, 1, ctypes.byref(need)) == 0
            if need.value > (256 << 20):
                break
            big *= 2
        Rb = torch.zeros((big,) + tuple(hs.n_fine), dtype=torch.complex128, device=_dev())
        with pytest.raises(hsp.HspError) as e:
            hs.apply_precond_batch_noalloc(Rb, tile=tile, out=torch.empty_like(Rb))
        assert e.value.status == hsp.HSP_ENOMEM
    finally:
        hs.close()
