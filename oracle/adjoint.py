"""Adjoint-state misfit gradient (oracle, complex128, direct solves).

Not in the paper; it differentiates the discrete problem of Sec. 4 (eq.
define_pml_fd, FE scaled) with respect to the squared slowness m = 1/c^2 at
the unknown nodes.  With b_s the scaled point sources, A(m) u_s = b_s,
predicted data d_s = R u_s (R picks receiver nodes) and
L = 1/2 sum_s ||R u_s - d_obs_s||^2:

    dL/dm_i = -sum_s Re( conj(lam_s,i) (dA/dm_i u_s)_i ),   A^H lam_s = R^T r_s,

and the only m-dependent entry of row i is the diagonal term
-h^2 omega^2 m_i / (alpha_1 alpha_2)_i, so
    dL/dm_i = h^2 omega^2 sum_s Re( conj(lam_s,i) u_s,i / (alpha_1 alpha_2)_i ).

The PML reference speed c_pml is a fixed number here (were it mean(c), the
PML profile would depend on m as well).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import discretization as D


def operator(m, omega, h, w_outer, S_outer, c_pml):
    """FE-scaled 5-point operator for squared slowness m (unknown nodes incl.
    PML), its right-hand-side scale h^2/(alpha_1 alpha_2) and the diagonal
    factor h^2 omega^2 / (alpha_1 alpha_2) of dA/dm."""
    N1, N2 = m.shape[0] + 1, m.shape[1] + 1
    ax = D.uniform_axis(N1, h, w_outer, S_outer, c_pml)
    ay = D.uniform_axis(N2, h, w_outer, S_outer, c_pml)
    A = D.fd5_matrix(ax, ay, omega ** 2 * m, omega)
    scale = D.fd5_rhs_scale(ax, ay, omega)          # h^2 / (a1 a2)
    return A, scale, omega ** 2 * scale


def misfit_gradient(m, omega, h, w_outer, S_outer, c_pml, sources, receivers, d_obs):
    """L and dL/dm for physical sources ``sources`` (ns, N1-1, N2-1) and
    receiver flat indices ``receivers``; d_obs (ns, nrec)."""
    A, scale, dscale = operator(m, omega, h, w_outer, S_outer, c_pml)
    lu = spla.splu(A.tocsc())
    L = 0.0
    g = np.zeros(m.size)
    us = []
    for s in range(sources.shape[0]):
        u = lu.solve((scale * sources[s]).ravel())
        r = u[receivers] - d_obs[s]
        L += 0.5 * np.vdot(r, r).real
        rt = np.zeros(m.size, dtype=complex)
        rt[receivers] = r
        lam = lu.solve(rt, trans="H")
        g += (np.conj(lam) * u * dscale.ravel()).real
        us.append(u)
    return L, g.reshape(m.shape), np.array(us)


def predicted_data(m, omega, h, w_outer, S_outer, c_pml, sources, receivers):
    A, scale, _ = operator(m, omega, h, w_outer, S_outer, c_pml)
    lu = spla.splu(A.tocsc())
    return np.array([lu.solve((scale * sources[s]).ravel())[receivers] for s in range(sources.shape[0])])
