"""Adjoint gradient of the THIIM fixed point -- TEST INFRASTRUCTURE ONLY.

Objective (an absorption functional of the solar-cell application, Sec. I):
    J = sum_p w_p eps''_p |E_p|^2,
|E|^2 summed over the three physical components, each the sum of its two
split parts (Eq. 6/7).

The fixed point x* = M x* + c of one THIIM iteration Phi (Eq. 3-5) depends on
eps through the E coefficients t, c and Src only (mu = 1; the PML profiles are
inputs of their own).  With g = dJ/dx (the holomorphic derivative, so that
dJ = 2 Re g . dx) and lam the solution of (I - M^T) lam = g,
    dJ/dtheta_p = (explicit term) + 2 Re sum_{q in E parts of p}
                  lam_q(p) dPhi_q/dtheta_p (x*),
    dPhi_q/dtheta = (dt_q/dtheta) E_q + (dc_q/dtheta) D_q + dSrc_q/dtheta,
where D_q = s_q (G(p + e) - G(p)) is the curl difference that multiplies c_q
in Eq. (3)/(5), taken from the H half-step of x*.  theta = eps' or eps''
(sigma_mat = w eps'').  The derivatives of t, c, Src follow from their closed
forms (Eq. 3 forward, Eq. 5 back iteration; sigma the total conductivity):
    forward: d = 1 + tau sigma / eps',  t = e^{-iwt}/d,
             c = tau/(eps' h) e^{-iwt/2}/d,  Src = tau e^{-iwt} S/d
    back:    d = 1 - tau sigma / eps',  t = e^{iwt}/d,
             c = -tau/(eps' h) e^{iwt/2}/d,  Src = -tau S/d
so dt = -t dd/d, dSrc = -Src dd/d, dc = -c dd/d (- c/eps' for theta = eps').

The result is reported as a complex array grad = dJ/deps' + 1j dJ/deps''.
"""
from __future__ import annotations

import numpy as np

from . import adjoint_iterate, coeffs, norm, phi, physical, zero_fields
from . import iterate as _iterate
from .dense import split_table

SRC_OF = {0: "Ex", 2: "Ey"}  # E parts (index within E) carrying a source


def objective(eps, x, w) -> float:
    """J = sum w eps'' |E|^2 with E the physical E field of x."""
    E = physical(x)[3:]
    return float(np.sum(np.asarray(w) * np.asarray(eps).imag * np.sum(np.abs(E) ** 2, axis=0)))


def adjoint_source(eps, x, w):
    """g = dJ/dx: w eps'' conj(E_a) on both split parts of E_a, 0 on H."""
    E = physical(x)[3:]
    g = np.zeros_like(np.asarray(x))
    wei = np.asarray(w) * np.asarray(eps).imag
    for a in range(3):
        g[6 + 2 * a] = wei * np.conj(E[a])
        g[6 + 2 * a + 1] = wei * np.conj(E[a])
    return g


def adjoint_residual(coef, lam, g, bcx=0, bcy=0) -> float:
    """||(M^T lam + g - lam)_E|| / ||g||: the E parts only.

    The gradient reads lam on the E parts alone.  Some H parts of lam never
    settle: on PML planes the two parts of an H pair get the same increments
    but only the z-difference part decays, so the other one (multiplied by
    exp(-i w tau) each iteration) keeps a bounded rotating term; that term lies
    in the kernel of the map back to the E parts."""
    nxt = adjoint_iterate(coef, lam.copy(), g, 1, bcx, bcy)
    gn = norm(g)
    return norm(nxt[6:] - lam[6:]) / gn if gn > 0 else 0.0


def adjoint_solve(coef, g, tol, max_it, bcx=0, bcy=0, check_every=50):
    """lam with (I - M^T) lam = g by the transposed iteration from lam = 0,
    until adjoint_residual <= tol or max_it iterations."""
    lam = np.zeros_like(g)
    it, res = 0, 1.0
    while it < max_it:
        step = min(check_every, max_it - it)
        adjoint_iterate(coef, lam, g, step, bcx, bcy)
        it += step
        res = adjoint_residual(coef, lam, g, bcx, bcy)
        if res <= tol:
            break
    return lam, it, res


def forward_solve_e(coef, tol, max_it, bcx=0, bcy=0, check_every=50):
    """THIIM iteration from x0 = 0 until the physical E field is converged:
    ||P(Phi(x) - x)_E|| / ||P Phi(0)_E|| <= tol.  (J and its gradient depend
    on E only; curl-free H modes excited by H sources are invisible to E.)"""
    _, nz, ny, nx = coef.shape
    x = zero_fields((nz, ny, nx))
    r0 = norm(physical(phi(coef, x, bcx, bcy))[3:])
    it, res = 0, 1.0
    while it < max_it:
        step = min(check_every, max_it - it)
        _iterate(coef, x, step, bcx, bcy)
        it += step
        res = norm(physical(phi(coef, x, bcx, bcy) - x)[3:]) / r0
        if res <= tol:
            break
    return x, it, res


def _shift(a, axis, d, periodic_xy):
    """b(p) = a(p + d e_axis) on (nz, ny, nx) arrays, ghost 0 (axis 0 = x)."""
    ax = {0: 2, 1: 1, 2: 0}[axis]
    b = np.roll(a, -d, axis=ax)
    if not (axis < 2 and periodic_xy[axis]):
        idx = [slice(None)] * 3
        idx[ax] = slice(-1, None) if d > 0 else slice(0, 1)
        b[tuple(idx)] = 0
    return b


def _e_coef_derivs(eps, sigma, omega, tau, h, dsig):
    """(d, dd/deps', dd/deps'', c, t) per cell for one E part with total
    conductivity sigma; dsig = dsigma/deps'' (= omega)."""
    ep = eps.real
    fwd = ep > 0
    sgn = np.where(fwd, 1.0, -1.0)
    d = 1.0 + sgn * tau * sigma / ep
    dd_ep = -sgn * tau * sigma / ep ** 2
    dd_epp = sgn * tau * dsig / ep
    ph = np.exp(1j * omega * tau)
    ph2 = np.exp(1j * omega * tau / 2)
    t = np.where(fwd, np.conj(ph), ph) / d
    c = np.where(fwd, tau / (ep * h) * np.conj(ph2), -tau / (ep * h) * ph2) / d
    s = np.where(fwd, tau * np.conj(ph), -tau + 0j) / d
    return d, dd_ep, dd_epp, t, c, s


def gradient(eps, sig_e, sig_h, sources, omega, tau, h, x, lam, w, bcx=0, bcy=0):
    """dJ/deps' + 1j dJ/deps'' per cell at the state x with adjoint lam."""
    eps = np.asarray(eps, dtype=np.complex128)
    coef = coeffs(eps, sig_e, sig_h, sources, omega, tau, h)
    Hn = physical(phi(coef, x, bcx, bcy))[:3]  # H sums after the H half-step
    E = physical(x)[3:]
    periodic = (bcx == 0, bcy == 0)
    nz = eps.shape[0]
    sig_mat = omega * eps.imag
    sig_pml = np.asarray(sig_e, dtype=np.float64)[:, None, None] * np.ones_like(eps.real)
    ge = np.zeros(eps.shape)
    gee = np.array(np.asarray(w) * np.sum(np.abs(E) ** 2, axis=0), dtype=np.float64)
    sources = sources or {}
    for q, cm in enumerate(split_table()[6:]):
        G = Hn[cm["drv"]]
        D = cm["sign"] * (_shift(G, cm["axis"], +1, periodic) - G)
        on_z = cm["axis"] == 2
        sigma = sig_mat + (sig_pml if on_z else 0.0)
        d, dd_ep, dd_epp, t, c, s = _e_coef_derivs(eps, sigma, omega, tau, h, omega)
        S = sources.get(SRC_OF.get(q, ""), None) if on_z else None
        S = np.zeros_like(eps) if S is None else np.asarray(S, np.complex128)
        base = t * x[6 + q] + c * D + s * S  # Phi_q(x): each term scales with 1/d
        l = lam[6 + q]
        ge += 2.0 * np.real(l * (-(dd_ep / d) * base - (c / eps.real) * D))
        gee += 2.0 * np.real(l * (-(dd_epp / d) * base))
    assert nz == eps.shape[0]
    return ge + 1j * gee


def gradient_of(pb, w, tol=1e-13, max_it=200000, check_every=50):
    """Forward solve, adjoint solve and gradient for a Problem; returns
    (J, grad, x, lam, (forward iterations, adjoint iterations))."""
    coef = coeffs(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h)
    x, itf, _ = forward_solve_e(coef, tol, max_it, pb.bcx, pb.bcy, check_every)
    g = adjoint_source(pb.eps, x, w)
    lam, ita, _ = adjoint_solve(coef, g, tol, max_it, pb.bcx, pb.bcy, check_every)
    grad = gradient(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h, x,
                    lam, w, pb.bcx, pb.bcy)
    return objective(pb.eps, x, w), grad, x, lam, (itf, ita)


__all__ = ["objective", "adjoint_source", "adjoint_residual", "adjoint_solve",
           "forward_solve_e", "gradient", "gradient_of"]
