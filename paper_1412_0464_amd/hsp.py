"""Thin Python binding of the C ABI in include/hsp.h (argument marshalling only).

Device memory comes from PyTorch: the workspace is a ``torch.uint8`` tensor on
the GPU, vectors are contiguous ``torch.complex128`` tensors of shape
(N1-1, N2-1) (x slowest), and every call is enqueued on the current torch
stream.  All arithmetic runs in the HIP kernels of ``libhsp.so``; there is no
CPU fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libhsp.so")
_lib = None

HSP_OK, HSP_EINVAL, HSP_ENOMEM, HSP_ESINGULAR, HSP_ENOCONV, HSP_EDEVICE = 0, -1, -2, -3, -4, -5
SWEEP = {"x": 0, "ud": 1, "nx": 2}
PRECISION = {"fp64": 0, "mixed": 1}
SLAB_FACTOR = {"auto": 0, "block": 1, "nd": 2}


class HspError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"hsp status {status}: {message}")
        self.status = status


class HspGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("pml", ctypes.c_int * 3), ("S_outer", ctypes.c_double), ("c_pml", ctypes.c_double),
                ("sponge", ctypes.c_int)]


class HspOptions(ctypes.Structure):
    _fields_ = [("fine_stencil", ctypes.c_int), ("two_grid", ctypes.c_int), ("w_dd", ctypes.c_int),
                ("S_dd", ctypes.c_double), ("nu", ctypes.c_int), ("omega_jac", ctypes.c_double),
                ("sweep", ctypes.c_int), ("precision", ctypes.c_int), ("restart", ctypes.c_int),
                ("chunk", ctypes.c_int), ("krylov_fp32", ctypes.c_int), ("ncell", ctypes.c_int),
                ("slab_factor", ctypes.c_int)]


class HspInfo(ctypes.Structure):
    _fields_ = [("n_fine", ctypes.c_int * 2), ("n_coarse", ctypes.c_int * 2), ("J", ctypes.c_int),
                ("max_slab_layers", ctypes.c_int), ("precision", ctypes.c_int), ("two_grid", ctypes.c_int),
                ("pivot_growth", ctypes.c_double), ("dim", ctypes.c_int), ("n_fine_z", ctypes.c_int),
                ("n_coarse_z", ctypes.c_int), ("slab_factor", ctypes.c_int)]


EXPORTS = ["hsp_default_options", "hsp_workspace_size", "hsp_setup", "hsp_rhs", "hsp_apply_operator",
           "hsp_apply_precond", "hsp_solve", "hsp_destroy", "hsp_last_error", "hsp_get_info",
           "hsp_get_partition", "hsp_apply_level_operator", "hsp_restrict", "hsp_prolong_add",
           "hsp_smooth", "hsp_sweep", "hsp_slab_solve", "hsp_profile_enable", "hsp_profile_read",
           "hsp_gradient_accumulate", "hsp_batch_workspace_size", "hsp_apply_precond_batch",
           "hsp_tune_batch", "hsp_solve_batch", "hsp_group_workspace_size", "hsp_apply_precond_group",
           "hsp_solve_group", "hsp_debug_set", "hsp_apply_precond_batch_noalloc", "hsp_autotune_workspace_size",
           "hsp_autotune"]
DEBUG_KNOBS = {"singular_slab": 0, "growth_limit": 1}
GROUP_GRAPH = 1
PROF_CLASSES = {"stage": 0, "smooth": 1, "coarse": 2, "transfer": 3, "krylov": 4, "project": 5, "update": 6}


def library_path():
    return _LIB_PATH


def load():
    """Load libhsp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"HIP library not built: {_LIB_PATH} is missing "
                           "(run `python -c 'import __graft_entry__ as g; g.build()'`)")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        "hsp_default_options": [ctypes.POINTER(HspOptions)],
        "hsp_workspace_size": [ctypes.POINTER(HspGrid), I, ctypes.POINTER(HspOptions), ctypes.POINTER(S)],
        "hsp_setup": [P, D, ctypes.POINTER(HspGrid), I, ctypes.POINTER(HspOptions), P, S, P,
                      ctypes.POINTER(P)],
        "hsp_rhs": [P, P, P, P],
        "hsp_apply_operator": [P, P, P, P],
        "hsp_apply_precond": [P, P, P, P],
        "hsp_solve": [P, P, P, D, I, I, ctypes.POINTER(I), ctypes.POINTER(D), P],
        "hsp_destroy": [P],
        "hsp_get_info": [P, ctypes.POINTER(HspInfo)],
        "hsp_get_partition": [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)],
        "hsp_apply_level_operator": [P, I, P, P, P],
        "hsp_restrict": [P, P, P, P],
        "hsp_prolong_add": [P, P, P, P],
        "hsp_smooth": [P, P, P, I, P],
        "hsp_sweep": [P, P, P, P],
        "hsp_slab_solve": [P, I, P, P, P],
        "hsp_profile_enable": [P, I],
        "hsp_gradient_accumulate": [P, P, P, P, P],
        "hsp_profile_read": [P, I, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(D)],
        "hsp_batch_workspace_size": [P, I, I, ctypes.POINTER(S)],
        "hsp_apply_precond_batch": [P, I, P, P, I, P, S, P],
        "hsp_tune_batch": [P, I, I, P, S, ctypes.POINTER(I), ctypes.POINTER(D), P],
        "hsp_solve_batch": [P, I, P, P, D, I, I, I, I, P, S, ctypes.POINTER(I), ctypes.POINTER(D), P],
        "hsp_group_workspace_size": [I, ctypes.POINTER(P), ctypes.POINTER(I), I, ctypes.POINTER(S)],
        "hsp_apply_precond_group": [I, ctypes.POINTER(P), ctypes.POINTER(I), ctypes.POINTER(P),
                                    ctypes.POINTER(P), I, I, P, S, P],
        "hsp_solve_group": [I, ctypes.POINTER(P), ctypes.POINTER(I), ctypes.POINTER(P), ctypes.POINTER(P), D, I,
                            I, I, I, I, P, S, ctypes.POINTER(I), ctypes.POINTER(D), P],
        "hsp_debug_set": [I, D],
        "hsp_apply_precond_batch_noalloc": [P, I, P, P, I, ctypes.POINTER(S), P],
        "hsp_autotune_workspace_size": [ctypes.POINTER(HspGrid), I, ctypes.POINTER(HspOptions), I, I,
                                        ctypes.POINTER(S), ctypes.POINTER(S)],
        "hsp_autotune": [P, D, ctypes.POINTER(HspGrid), I, ctypes.POINTER(HspOptions), I, I, P, S, P, S,
                         ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(D),
                         ctypes.POINTER(I), P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.hsp_last_error.argtypes = []
    lib.hsp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def autotune(c, omega, h, pml, J, nrhs, restart=40, S_outer=0.0, c_pml=0.0, sponge=False, **opts):
    """Chunk length and right-hand-side tile of the batched solvers for this
    problem and batch size (hsp_autotune).  Returns (chunk, tile, ms per
    batched preconditioner application, [(chunk, tile, ms) per candidate])."""
    lib = load()
    if not (c.is_cuda and c.dtype == torch.float64 and c.is_contiguous() and c.dim() == 2):
        raise ValueError("c must be a contiguous 2-D float64 CUDA tensor")
    pml = (pml,) * 2 if isinstance(pml, int) else tuple(pml)
    n = tuple(c.shape[a] - 2 * pml[a] for a in range(2))
    g = make_grid(n, h, pml, S_outer, c_pml, sponge)
    o = make_options(**opts)
    wsb, bwsb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.hsp_autotune_workspace_size(ctypes.byref(g), int(J), ctypes.byref(o), int(nrhs), int(restart),
                                           ctypes.byref(wsb), ctypes.byref(bwsb)))
    ws = torch.empty(wsb.value, dtype=torch.uint8, device=c.device)
    bws = torch.empty(bwsb.value, dtype=torch.uint8, device=c.device)
    chunk, tile, ntab = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ms = ctypes.c_double()
    tab = (ctypes.c_double * 24)()
    _check(lib.hsp_autotune(_ptr(c), float(omega), ctypes.byref(g), int(J), ctypes.byref(o), int(nrhs), int(restart),
                            _ptr(ws), wsb.value, _ptr(bws), bwsb.value, ctypes.byref(chunk), ctypes.byref(tile),
                            ctypes.byref(ms), tab, ctypes.byref(ntab), _stream()))
    table = [(int(tab[3 * i]), int(tab[3 * i + 1]), tab[3 * i + 2]) for i in range(ntab.value)]
    return chunk.value, tile.value, ms.value, table


def debug_set(knob, value):
    """Set a process-wide debugging knob of the setup (hsp_debug_set):
    ``singular_slab`` (slab index, -1 off) or ``growth_limit`` (> 0, or <= 0
    for the default)."""
    _check(load().hsp_debug_set(DEBUG_KNOBS[knob] if isinstance(knob, str) else int(knob), float(value)))


def _check(st):
    if st != HSP_OK:
        raise HspError(st, load().hsp_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _vec(t, shape, name):
    if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def make_grid(n, h, pml, S_outer=0.0, c_pml=0.0, sponge=False):
    """hsp_grid for 2 (len(n) == 2) or 3 dimensions; sponge=True makes the
    outer layers sponge layers instead of PML."""
    g = HspGrid()
    d = len(n)
    if d not in (2, 3) or len(pml) != d:
        raise ValueError("n and pml must both have 2 or 3 entries")
    g.dim = d
    for a in range(3):
        g.n[a] = int(n[a]) if a < d else 0
        g.pml[a] = int(pml[a]) if a < d else 0
    g.h = float(h)
    g.S_outer = float(S_outer)
    g.c_pml = float(c_pml)
    g.sponge = int(bool(sponge))
    return g


def make_options(**kw):
    o = HspOptions()
    _check(load().hsp_default_options(ctypes.byref(o)))
    for k, v in kw.items():
        if k == "sweep":
            v = SWEEP[v] if isinstance(v, str) else v
        if k == "precision":
            v = PRECISION[v] if isinstance(v, str) else v
        if k == "slab_factor":
            v = SLAB_FACTOR[v] if isinstance(v, str) else v
        if k in ("two_grid", "krylov_fp32"):
            v = int(bool(v))
        if k not in dict(HspOptions._fields_):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def workspace_size(n, h, pml, J, **opts):
    S = ctypes.c_size_t()
    g = make_grid(n, h, pml)
    o = make_options(**opts)
    _check(load().hsp_workspace_size(ctypes.byref(g), int(J), ctypes.byref(o), ctypes.byref(S)))
    return S.value


class Helmholtz:
    """One medium and frequency: hsp_setup on construction, hsp_destroy on close.

    ``c``   contiguous float64 CUDA tensor of wave speeds at all unknown nodes
            (PML nodes included), shape (N1-1, N2-1) in 2-D or
            (N1-1, N2-1, N3-1) in 3-D.
    ``pml`` outer PML cells per side (int, or one per axis); the interior node
            counts follow from c.shape - 2*pml.  ``sponge=True``: these
            cells are sponge layers instead (S_outer = beta at the edge).
    Options follow hsp_options (fine_stencil, two_grid, w_dd, S_dd, nu,
    omega_jac, sweep 'x'/'ud'/'nx', precision 'fp64'/'mixed', restart, chunk,
    krylov_fp32, ncell, slab_factor 'auto'/'block'/'nd').  In 3-D the defaults are those of the paper's 3-D
    experiments (Sec. 6.2): fine_stencil 7, w_dd 3, omega_jac 0.6, and the
    complex64 slab factors of precision 'mixed'.
    """

    def __init__(self, c, omega, h, pml, J, S_outer=0.0, c_pml=0.0, sponge=False, **opts):
        lib = load()
        if not (c.is_cuda and c.dtype == torch.float64 and c.is_contiguous() and c.dim() in (2, 3)):
            raise ValueError("c must be a contiguous 2-D or 3-D float64 CUDA tensor")
        d = c.dim()
        if d == 3:
            opts.setdefault("fine_stencil", 7)
            opts.setdefault("w_dd", 3)
            opts.setdefault("omega_jac", 0.6)
            opts.setdefault("precision", "mixed")
        pml = (pml,) * d if isinstance(pml, int) else tuple(pml)
        n = tuple(c.shape[a] - 2 * pml[a] for a in range(d))
        self.dim = d
        self.shape = tuple(c.shape)
        self.grid = make_grid(n, h, pml, S_outer, c_pml, sponge)
        self.opts = make_options(**opts)
        self.J = int(J)
        S = ctypes.c_size_t()
        _check(lib.hsp_workspace_size(ctypes.byref(self.grid), self.J, ctypes.byref(self.opts), ctypes.byref(S)))
        self.ws = torch.empty(S.value, dtype=torch.uint8, device=c.device)
        hd = ctypes.c_void_p()
        _check(lib.hsp_setup(_ptr(c), float(omega), ctypes.byref(self.grid), self.J, ctypes.byref(self.opts),
                             _ptr(self.ws), S.value, _stream(), ctypes.byref(hd)))
        self.handle = hd
        inf = HspInfo()
        _check(lib.hsp_get_info(self.handle, ctypes.byref(inf)))
        if d == 3:
            self.n_fine = (inf.n_fine[0], inf.n_fine[1], inf.n_fine_z)
            self.n_coarse = (inf.n_coarse[0], inf.n_coarse[1], inf.n_coarse_z)
        else:
            self.n_fine = tuple(inf.n_fine)
            self.n_coarse = tuple(inf.n_coarse)
        self.max_slab_layers = inf.max_slab_layers
        self.two_grid = bool(inf.two_grid)
        self.pivot_growth = inf.pivot_growth
        self.slab_factor = {1: "block", 2: "nd"}.get(inf.slab_factor, "block")
        beta = (ctypes.c_int * (self.J + 1))()
        x0 = (ctypes.c_int * self.J)()
        x1 = (ctypes.c_int * self.J)()
        _check(lib.hsp_get_partition(self.handle, beta, x0, x1))
        self.beta, self.x0, self.x1 = list(beta), list(x0), list(x1)
        self.dd_shape = self.n_coarse if self.two_grid else self.n_fine

    # -- lifecycle ----------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            load().hsp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls ----------------------------------------------------------------
    def _new(self, shape):
        return torch.empty(shape, dtype=torch.complex128, device=self.ws.device)

    def rhs(self, f):
        _vec(f, self.n_fine, "f")
        b = self._new(self.n_fine)
        _check(load().hsp_rhs(self.handle, _ptr(f), _ptr(b), _stream()))
        return b

    def apply_operator(self, x):
        _vec(x, self.n_fine, "x")
        y = self._new(self.n_fine)
        _check(load().hsp_apply_operator(self.handle, _ptr(x), _ptr(y), _stream()))
        return y

    def apply_level_operator(self, level, x):
        shape = self.n_fine if level == 0 else self.n_coarse
        _vec(x, shape, "x")
        y = self._new(shape)
        _check(load().hsp_apply_level_operator(self.handle, int(level), _ptr(x), _ptr(y), _stream()))
        return y

    def apply_precond(self, r, out=None):
        _vec(r, self.n_fine, "r")
        z = self._new(self.n_fine) if out is None else _vec(out, self.n_fine, "out")
        _check(load().hsp_apply_precond(self.handle, _ptr(r), _ptr(z), _stream()))
        return z

    def restrict(self, rf):
        _vec(rf, self.n_fine, "rf")
        rc = self._new(self.n_coarse)
        _check(load().hsp_restrict(self.handle, _ptr(rf), _ptr(rc), _stream()))
        return rc

    def prolong_add(self, ec, xf):
        _vec(ec, self.n_coarse, "ec")
        _vec(xf, self.n_fine, "xf")
        _check(load().hsp_prolong_add(self.handle, _ptr(ec), _ptr(xf), _stream()))
        return xf

    def smooth(self, r, steps):
        _vec(r, self.n_fine, "r")
        x = self._new(self.n_fine)
        _check(load().hsp_smooth(self.handle, _ptr(r), _ptr(x), int(steps), _stream()))
        return x

    def sweep(self, f):
        _vec(f, self.dd_shape, "f")
        u = self._new(self.dd_shape)
        _check(load().hsp_sweep(self.handle, _ptr(f), _ptr(u), _stream()))
        return u

    def slab_solve(self, j, b):
        nl = self.x1[j] - self.x0[j] + 1
        shape = (nl,) + tuple(self.dd_shape[1:])
        _vec(b, shape, "b")
        x = self._new(shape)
        _check(load().hsp_slab_solve(self.handle, int(j), _ptr(b), _ptr(x), _stream()))
        return x

    def gradient_accumulate(self, u, lam, g):
        """g += h^2 omega^2 Re(conj(lam) u / (alpha_1 alpha_2)) (hsp_gradient_accumulate)."""
        _vec(u, self.n_fine, "u")
        _vec(lam, self.n_fine, "lam")
        if not (g.is_cuda and g.dtype == torch.float64 and g.is_contiguous() and tuple(g.shape) == self.n_fine):
            raise ValueError("g must be a contiguous float64 CUDA tensor of the fine shape")
        _check(load().hsp_gradient_accumulate(self.handle, _ptr(u), _ptr(lam), _ptr(g), _stream()))
        return g

    def profile(self, on=True):
        """Enable or disable per-kernel-class event timing (hsp_profile_enable)."""
        _check(load().hsp_profile_enable(self.handle, int(bool(on))))

    def profile_read(self, cls):
        """(total event ms, launches, algorithmic bytes) of a kernel class since
        the last read; resets the class (hsp_profile_read)."""
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        by = ctypes.c_double()
        c = PROF_CLASSES[cls] if isinstance(cls, str) else int(cls)
        _check(load().hsp_profile_read(self.handle, c, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
        return ms.value, n.value, by.value

    def solve(self, b, tol=1e-6, maxit=200, conj_transpose=False, out=None, raise_on_noconv=True):
        """FGMRES on A u = b (b already FE scaled, see rhs).  Returns
        (u, iterations, true relative residual)."""
        _vec(b, self.n_fine, "b")
        u = self._new(self.n_fine) if out is None else _vec(out, self.n_fine, "out")
        it = ctypes.c_int()
        rr = ctypes.c_double()
        st = load().hsp_solve(self.handle, _ptr(b), _ptr(u), float(tol), int(maxit), int(bool(conj_transpose)),
                              ctypes.byref(it), ctypes.byref(rr), _stream())
        if st == HSP_ENOCONV and not raise_on_noconv:
            return u, it.value, rr.value
        _check(st)
        return u, it.value, rr.value

    # -- batched right-hand sides (one medium and frequency, shared factors) --
    def batch_workspace(self, nrhs, restart=None):
        """Device workspace of the batched calls for up to ``nrhs`` right-hand
        sides and FGMRES restart ``restart`` (cached on the object)."""
        restart = int(restart or self.opts.restart)
        key = (int(nrhs), restart)
        if getattr(self, "_bws_key", None) == key:
            return self._bws
        S = ctypes.c_size_t()
        _check(load().hsp_batch_workspace_size(self.handle, int(nrhs), restart, ctypes.byref(S)))
        self._bws = None
        self._bws = torch.empty(S.value, dtype=torch.uint8, device=self.ws.device)
        self._bws_key = key
        return self._bws

    def _batch(self, t, name):
        if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous() and t.dim() == 3
                and tuple(t.shape[1:]) == tuple(self.n_fine)):
            raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape (nrhs, {self.n_fine[0]}, "
                             f"{self.n_fine[1]})")
        return t

    def apply_precond_batch(self, r, tile=0, out=None):
        """z_j = M r_j for every right-hand side j of r (nrhs, n1, n2)
        (hsp_apply_precond_batch)."""
        self._batch(r, "r")
        nrhs = r.shape[0]
        z = torch.empty_like(r) if out is None else self._batch(out, "out")
        if nrhs == 0:
            return z
        key = getattr(self, "_bws_key", None)
        ws = self._bws if key is not None and key[0] == nrhs else self.batch_workspace(nrhs, 1)
        _check(load().hsp_apply_precond_batch(self.handle, int(nrhs), _ptr(r), _ptr(z), int(tile), _ptr(ws),
                                              ws.numel(), _stream()))
        return z

    def apply_precond_batch_noalloc(self, r, tile=1, out=None):
        """As apply_precond_batch, with the library's fixed device scratch
        instead of a workspace (hsp_apply_precond_batch_noalloc).  ``out``
        lets the caller avoid any allocation as well."""
        self._batch(r, "r")
        z = torch.empty_like(r) if out is None else self._batch(out, "out")
        _check(load().hsp_apply_precond_batch_noalloc(self.handle, int(r.shape[0]), _ptr(r), _ptr(z), int(tile), None,
                                                      _stream()))
        return z

    def tune_batch(self, nrhs, restart=None):
        """Time the batched preconditioner for every right-hand-side tile and
        keep the fastest for this batch size (hsp_tune_batch).  Returns
        (tile, ms per application)."""
        restart = int(restart or self.opts.restart)
        ws = self.batch_workspace(nrhs, restart)
        tile = ctypes.c_int()
        ms = ctypes.c_double()
        _check(load().hsp_tune_batch(self.handle, int(nrhs), restart, _ptr(ws), ws.numel(), ctypes.byref(tile),
                                     ctypes.byref(ms), _stream()))
        return tile.value, ms.value

    def solve_batch(self, b, tol=1e-6, maxit=200, restart=None, tile=0, conj_transpose=False, out=None,
                    raise_on_noconv=True):
        """FGMRES on A u_j = b_j for every right-hand side of b (nrhs, n1, n2),
        each stopped at its own tolerance (hsp_solve_batch).  Returns
        (u, iterations per right-hand side, true relative residuals)."""
        self._batch(b, "b")
        nrhs = b.shape[0]
        u = torch.empty_like(b) if out is None else self._batch(out, "out")
        its = (ctypes.c_int * max(nrhs, 1))()
        rr = (ctypes.c_double * max(nrhs, 1))()
        if nrhs == 0:
            return u, [], []
        restart = int(restart or self.opts.restart)
        ws = self.batch_workspace(nrhs, restart)
        st = load().hsp_solve_batch(self.handle, int(nrhs), _ptr(b), _ptr(u), float(tol), int(maxit), restart,
                                    int(bool(conj_transpose)), int(tile), _ptr(ws), ws.numel(), its, rr, _stream())
        if not (st == HSP_ENOCONV and not raise_on_noconv):
            _check(st)
        return u, list(its)[:nrhs], list(rr)[:nrhs]


# -- groups: right-hand sides of several problems solved together ------------
class Group:
    """Several set-up problems (Helmholtz objects of one precision) whose
    right-hand sides are solved together: the sweep stages of all problems
    share launches (hsp_solve_group).  The group workspace is allocated on
    first use for the given right-hand-side counts and restart."""

    def __init__(self, problems, restart=40):
        self.problems = list(problems)
        self.restart = int(restart)
        self._ws = None
        self._key = None

    def _arrays(self, nrhs):
        n = len(self.problems)
        hds = (ctypes.c_void_p * n)(*[p.handle for p in self.problems])
        cnt = (ctypes.c_int * n)(*[int(k) for k in nrhs])
        return n, hds, cnt

    def workspace(self, nrhs, restart=None):
        restart = int(restart or self.restart)
        key = (tuple(int(k) for k in nrhs), restart)
        if key == self._key:
            return self._ws
        n, hds, cnt = self._arrays(nrhs)
        S = ctypes.c_size_t()
        _check(load().hsp_group_workspace_size(n, hds, cnt, restart, ctypes.byref(S)))
        self._ws = None
        self._ws = torch.empty(S.value, dtype=torch.uint8, device=self.problems[0].ws.device)
        self._key = key
        return self._ws

    def _check_vecs(self, vecs, name):
        if len(vecs) != len(self.problems):
            raise ValueError(f"{name}: one tensor per problem expected")
        for p, v in zip(self.problems, vecs):
            p._batch(v, name)

    def apply_precond(self, rs, tile=0, graph=False):
        """z_j = M_p r_j for every right-hand side of every problem p
        (hsp_apply_precond_group); rs[p] has shape (nrhs_p, n1_p, n2_p)."""
        self._check_vecs(rs, "r")
        zs = [torch.empty_like(r) for r in rs]
        nrhs = [r.shape[0] for r in rs]
        ws = self.workspace(nrhs, self.restart)
        n, hds, cnt = self._arrays(nrhs)
        rp = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rs])
        zp = (ctypes.c_void_p * n)(*[z.data_ptr() for z in zs])
        _check(load().hsp_apply_precond_group(n, hds, cnt, rp, zp, int(tile), GROUP_GRAPH if graph else 0, _ptr(ws),
                                              ws.numel(), _stream()))
        return zs

    def solve(self, bs, tol=1e-6, maxit=200, tile=0, graph=False, conj_transpose=False, outs=None,
              raise_on_noconv=True):
        """FGMRES on every right-hand side of every problem (hsp_solve_group).
        Returns (list of solutions, list of iteration lists, list of
        relative-residual lists), problem by problem."""
        self._check_vecs(bs, "b")
        us = [torch.empty_like(b) for b in bs] if outs is None else list(outs)
        nrhs = [b.shape[0] for b in bs]
        tot = max(sum(nrhs), 1)
        ws = self.workspace(nrhs, self.restart)
        n, hds, cnt = self._arrays(nrhs)
        bp = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
        up = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
        its = (ctypes.c_int * tot)()
        rr = (ctypes.c_double * tot)()
        st = load().hsp_solve_group(n, hds, cnt, bp, up, float(tol), int(maxit), self.restart,
                                    int(bool(conj_transpose)), int(tile), GROUP_GRAPH if graph else 0, _ptr(ws),
                                    ws.numel(), its, rr, _stream())
        if not (st == HSP_ENOCONV and not raise_on_noconv):
            _check(st)
        out_it, out_rr, o = [], [], 0
        for k in nrhs:
            out_it.append(list(its)[o:o + k])
            out_rr.append(list(rr)[o:o + k])
            o += k
        return us, out_it, out_rr
