"""Direct solve of the THIIM fixed point -- TEST INFRASTRUCTURE ONLY.

Setting E^{n+1} = E^n and H^{n+1/2} = H^{n-1/2} in Eq. (3)/(4) (forward
iteration) or Eq. (5) (back iteration, eps' < 0) of arXiv:1510.05218 Sec. I-A
gives, for every split component q of Eq. (6)/(7) and every cell p, one linear
equation.  Multiplied by tau:

  H rows:  (e^{iwt/2} - e^{-iwt/2} + tau sigma*_q) H_q(p)
           - s_q (tau/h) [G(p) - G(p - e_c)]                   = tau S_H(p)
  E rows (eps' > 0):
           (e^{iwt} - 1 + (tau sigma_q / eps') e^{iwt}) E_q(p)
           - s_q (tau / (eps' h)) e^{iwt/2} [G(p + e_c) - G(p)] = tau S_E(p)
  E rows (eps' < 0):
           (e^{iwt} - 1 + tau sigma_q / eps') E_q(p)
           - s_q (tau / (eps' h)) e^{iwt/2} [G(p + e_c) - G(p)] = tau S_E(p)

where G is the sum of the two split parts of the driving component and s_q,
c are the sign and axis of that derivative in the curl of Eq. (1)/(2).  The
system is assembled here directly from (eps, sigma, omega, tau, h) -- not from
the oracle's coefficient arrays -- and the component table is generated from
the curl formula (curl V)_a = d_b V_c - d_c V_b, (a, b, c) cyclic, rather than
copied from the oracle's table.  The solution is the limit of the THIIM
iteration, so it pins the oracle's coefficients, signs, offsets and
boundaries at once (up to the shared readings listed in the oracle header).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

AX = "xyz"


def split_table():
    """Component table from the curl: list of 12 dicts in the API order."""
    table = []
    for field in ("H", "E"):
        for a in range(3):
            others = [b for b in range(3) if b != a]
            for drv in others:
                # (curl V)_a = d_b V_c - d_c V_b  with (a, b, c) cyclic
                b, c = (a + 1) % 3, (a + 2) % 3
                if drv == c:
                    axis, curl_sign = b, +1
                else:  # drv == b
                    axis, curl_sign = c, -1
                sign = -curl_sign if field == "H" else curl_sign
                table.append(dict(field=field, a=a, drv=drv, axis=axis,
                                  sign=sign,
                                  name=f"{field}_{AX[a]}{AX[drv]}"))
    return table


def _index(field, a, drv):
    others = [b for b in range(3) if b != a]
    return (0 if field == "H" else 6) + 2 * a + others.index(drv)


def _shift_matrix(shape, axis, d, periodic_xy):
    """Sparse N x N matrix S with (S g)(p) = g(p + d e_axis), ghost 0."""
    nz, ny, nx = shape
    N = nx * ny * nz
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                          indexing="ij")
    k, j, i = k.ravel(), j.ravel(), i.ravel()
    idx = [i.copy(), j.copy(), k.copy()]
    n_ax = [nx, ny, nz][axis]
    idx[axis] = idx[axis] + d
    valid = (idx[axis] >= 0) & (idx[axis] < n_ax)
    if axis < 2 and periodic_xy[axis]:
        idx[axis] = idx[axis] % n_ax
        valid = np.ones_like(valid)
    rows = np.arange(N)[valid]
    cols = ((idx[2] * ny + idx[1]) * nx + idx[0])[valid]
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(N, N))


def assemble(eps, sig_e, sig_h, sources, omega, tau=0.5, h=1.0,
             bcx=0, bcy=0):
    """Sparse matrix A and right-hand side b with A x = b at the fixed point.

    Unknown ordering: x[q * N + p], q in the API component order."""
    eps = np.asarray(eps, dtype=np.complex128)
    shape = eps.shape
    nz, ny, nx = shape
    N = nx * ny * nz
    ep = eps.real.ravel()
    sig_mat = omega * eps.imag.ravel()
    kz = np.repeat(np.arange(nz), nx * ny)
    sig_e_cell = np.asarray(sig_e, dtype=np.float64)[kz]
    sig_h_cell = np.asarray(sig_h, dtype=np.float64)[kz]
    periodic = (bcx == 0, bcy == 0)
    eye = sp.identity(N, format="csr")
    ph = np.exp(1j * omega * tau)
    ph2 = np.exp(1j * omega * tau / 2)
    blocks = [[None] * 12 for _ in range(12)]
    b = np.zeros(12 * N, dtype=np.complex128)
    sources = sources or {}
    for q, cm in enumerate(split_table()):
        on_z = cm["axis"] == 2
        if cm["field"] == "H":
            sst = sig_h_cell if on_z else np.zeros(N)
            diag = ph2 - np.conj(ph2) + tau * sst
            # backward difference G(p) - G(p - e_c)
            D = eye - _shift_matrix(shape, cm["axis"], -1, periodic)
            scale = -cm["sign"] * (tau / h) * np.ones(N)
            other = "E"
        else:
            sg = sig_mat + (sig_e_cell if on_z else 0.0)
            fwd = ep > 0
            diag = np.where(fwd, ph - 1 + (tau * sg / ep) * ph,
                            ph - 1 + tau * sg / ep)
            D = _shift_matrix(shape, cm["axis"], +1, periodic) - eye
            scale = -cm["sign"] * (tau / (ep * h)) * ph2
            other = "H"
        blocks[q][q] = sp.diags(diag.astype(np.complex128))
        coupling = sp.diags(scale.astype(np.complex128)) @ D
        for part in [p for p in range(3) if p != cm["drv"]]:
            g = _index(other, cm["drv"], part)
            blocks[q][g] = coupling if blocks[q][g] is None else blocks[q][g] + coupling
        if on_z and cm["a"] < 2:
            key = f"{cm['field']}{AX[cm['a']]}"
            s = sources.get(key)
            if s is not None:
                b[q * N:(q + 1) * N] = tau * np.asarray(s, np.complex128).ravel()
    A = sp.bmat(blocks, format="csc")
    return A, b


def fixed_point(eps, sig_e, sig_h, sources, omega, tau=0.5, h=1.0, bcx=0,
                bcy=0):
    """The THIIM fixed point by sparse LU; returns (12, nz, ny, nx)."""
    A, b = assemble(eps, sig_e, sig_h, sources, omega, tau, h, bcx, bcy)
    x = spla.splu(A).solve(b)
    nz, ny, nx = np.asarray(eps).shape
    return x.reshape(12, nz, ny, nx)
