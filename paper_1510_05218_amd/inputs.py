"""Seeded synthetic THIIM problems (material data, PML profiles, sources).

This module only *describes problems*: it draws the permittivity of
solar-cell-shaped layer stacks (Sec. I-A, Fig. 1 of arXiv:1510.05218: layers
with textured interfaces and SiO2-like particles, PML vertically and periodic
horizontally), the graded PML conductivity profiles and the source planes.
It performs none of the method's arithmetic (no coefficients, no updates) and
is used both by the GPU path and by the CPU oracle in the tests.

Conventions
  * grid arrays are [nz][ny][nx] (x fastest), complex128;
  * ``eps`` holds eps' + 1j*eps'' with eps'' >= 0 the loss; in the paper's
    exp(+i w t) convention the relative permittivity is eps' - i eps'';
  * normalised units eps0 = mu0 = c0 = h = 1, so omega = 2 pi h / lambda;
  * ``sig_e[k]`` is the electric PML conductivity at E plane k (position z=k),
    ``sig_h[k]`` the magnetic one at H plane k (position z=k-1/2); matched
    (sigma*/mu = sigma/eps) with eps the adjacent layer's eps'.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CELL_NM = 20.0


def omega_for(wavelength_nm: float, cell_nm: float = CELL_NM) -> float:
    """Angular frequency in units of c0 / h for a vacuum wavelength."""
    return 2.0 * np.pi * cell_nm / wavelength_nm


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def pml_profiles(nz, npml_lo, npml_hi, eps_lo=1.0, eps_hi=1.0, order=3,
                 r0=1e-6, h=1.0):
    """Graded conductivity sigma(d) = sigma_max (d / npml)^order.

    sigma_max = (order + 1) ln(1/r0) sqrt(eps_side) / (2 npml h), the usual
    polynomial grading for a target normal-incidence reflection r0; d is the
    depth of each component's own position into the layer."""
    sig_e = np.zeros(nz)
    sig_h = np.zeros(nz)
    z_e = np.arange(nz, dtype=np.float64)
    z_h = z_e - 0.5
    for npml, eps_side, lo in ((npml_lo, eps_lo, True), (npml_hi, eps_hi, False)):
        if npml <= 0:
            continue
        smax = (order + 1) * np.log(1.0 / r0) * np.sqrt(eps_side) / (2.0 * npml * h)
        if lo:
            d_e = np.clip(npml_lo - z_e, 0.0, None)
            d_h = np.clip(npml_lo - z_h, 0.0, None)
        else:
            top = nz - 1 - npml_hi
            d_e = np.clip(z_e - top, 0.0, None)
            d_h = np.clip(z_h - top, 0.0, None)
        sig_e += smax * (d_e / npml) ** order
        sig_h += smax * (d_h / npml) ** order / eps_side
    return sig_e, sig_h


def heightmap(ny, nx, amplitude, gen, n_modes=8, max_wavenumber=3):
    """Periodic height map: n_modes random Fourier modes with integer
    wave vectors |m|, |n| <= max_wavenumber, scaled to the given peak
    amplitude and rounded to whole cells."""
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    hm = np.zeros((ny, nx))
    for _ in range(n_modes):
        m = int(gen.integers(-max_wavenumber, max_wavenumber + 1))
        n = int(gen.integers(-max_wavenumber, max_wavenumber + 1))
        if m == 0 and n == 0:
            m = 1
        a = gen.normal()
        ph = gen.uniform(0, 2 * np.pi)
        hm += a * np.cos(2 * np.pi * (m * ii / nx + n * jj / ny) + ph)
    peak = np.max(np.abs(hm))
    if peak > 0:
        hm *= amplitude / peak
    return np.rint(hm).astype(np.int64)


@dataclass
class Problem:
    """One synthetic THIIM problem (material data + source), no coefficients."""
    eps: np.ndarray                 # complex128 (nz, ny, nx): eps' + 1j eps''
    sig_e: np.ndarray               # float64 (nz,)
    sig_h: np.ndarray               # float64 (nz,)
    sources: dict                   # 'Hx'|'Hy'|'Ex'|'Ey' -> complex (nz,ny,nx)
    omega: float
    tau: float = 0.5
    h: float = 1.0
    npml: int = 6
    bcx: int = 0                    # 0 periodic, 1 Dirichlet
    bcy: int = 0
    layers: list = field(default_factory=list)   # (k_lo, k_hi, eps) interior
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.eps.shape


def layer_stack(nx, ny, nz, npml=6, n_layers=3, seed=1, texture_amp=4,
                eps_range=(1.0, 16.0), loss_range=(0.0, 0.5), n_spheres=0,
                sphere_radius=(3.0, 10.0), sphere_eps=2.1, flat=False,
                gen=None):
    """Permittivity of a layered, textured stack (solar-cell shaped).

    The nz - 2*npml interior planes are split into n_layers equal layers with
    eps' ~ U(eps_range) and eps'' ~ U(loss_range).  The interface between the
    first and second layer is displaced by a periodic height map of the given
    amplitude (unless flat).  Spheres of eps = sphere_eps (lossless) are
    placed inside the last layer.  The PML planes repeat the adjacent interior
    material.  Returns (eps, layers, gen)."""
    g = gen if gen is not None else rng(seed)
    n_int = nz - 2 * npml
    assert n_int >= n_layers
    bounds = [npml + (n_int * l) // n_layers for l in range(n_layers + 1)]
    vals = [complex(g.uniform(*eps_range), g.uniform(*loss_range))
            for _ in range(n_layers)]
    kk = np.arange(nz)[:, None, None]
    # layer index per cell: count of interior interfaces below (k >= boundary)
    lay = np.zeros((nz, ny, nx), dtype=np.int8)
    hm = np.zeros((ny, nx), dtype=np.int64)
    if not flat and texture_amp > 0 and n_layers >= 2:
        hm = heightmap(ny, nx, texture_amp, g)
    for l in range(1, n_layers):
        b = bounds[l] + (hm if l == 1 else 0)
        b = np.clip(b, npml + 1, nz - npml - 1)
        lay += (kk >= b[None, :, :] if np.ndim(b) else kk >= b).astype(np.int8)
    table = np.array(vals, dtype=np.complex128)
    eps = table[lay]
    layers = [(bounds[l], bounds[l + 1], vals[l]) for l in range(n_layers)]
    if n_spheres > 0:
        k_lo, k_hi = bounds[-2], bounds[-1]
        _place_spheres(eps, g, n_spheres, sphere_radius, sphere_eps, k_lo, k_hi)
    # PML planes: repeat the adjacent interior plane
    eps[:npml] = eps[npml]
    eps[nz - npml:] = eps[nz - npml - 1]
    return eps, layers, g


def _place_spheres(eps, g, n, radius, value, k_lo, k_hi):
    nz, ny, nx = eps.shape
    for _ in range(n):
        r = g.uniform(*radius)
        rc = int(np.ceil(r))
        cz = g.uniform(k_lo + r, max(k_lo + r, k_hi - r))
        cy = g.uniform(0, ny)
        cx = g.uniform(0, nx)
        ks = np.arange(int(np.floor(cz - rc)), int(np.ceil(cz + rc)) + 1)
        ks = ks[(ks >= k_lo) & (ks < k_hi)]
        js = np.arange(int(np.floor(cy - rc)), int(np.ceil(cy + rc)) + 1)
        is_ = np.arange(int(np.floor(cx - rc)), int(np.ceil(cx + rc)) + 1)
        dz = (ks - cz)[:, None, None]
        dy = (js - cy)[None, :, None]
        dx = (is_ - cx)[None, None, :]
        inside = dz * dz + dy * dy + dx * dx <= r * r
        kk, jj, ii = np.nonzero(inside)
        eps[ks[kk], js[jj] % ny, is_[ii] % nx] = value


def plane_source(shape, k_s, pol="x", amplitude=1.0 + 0j, kx=0, ky=0,
                 field_kind="E"):
    """Soft plane-wave source on plane k_s: S = amplitude exp(-i(kx x + ky y))
    with integer periodic wave numbers kx, ky (cycles per domain)."""
    nz, ny, nx = shape
    s = np.zeros(shape, dtype=np.complex128)
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    s[k_s] = amplitude * np.exp(-2j * np.pi * (kx * ii / nx + ky * jj / ny))
    return {f"{field_kind}{pol}": s}


def solar_cell(nx, ny, nz, seed, npml=6, wavelength_nm=600.0, tau=0.5,
               n_spheres=0, texture_amp=4, flat=False, eps_range=(1.0, 16.0),
               loss_range=(0.0, 0.5), k_s=None, pol="x"):
    """A full synthetic problem: layered textured stack, graded PML in z,
    periodic x/y, normally incident x-polarised soft source one plane inside
    the lower PML interface."""
    eps, layers, _ = layer_stack(nx, ny, nz, npml=npml, seed=seed,
                                 texture_amp=texture_amp, n_spheres=n_spheres,
                                 flat=flat, eps_range=eps_range,
                                 loss_range=loss_range)
    sig_e, sig_h = pml_profiles(nz, npml, npml, eps_lo=layers[0][2].real,
                                eps_hi=layers[-1][2].real)
    if k_s is None:
        k_s = npml + 1
    src = plane_source(eps.shape, k_s, pol=pol)
    return Problem(eps=eps, sig_e=sig_e, sig_h=sig_h, sources=src,
                   omega=omega_for(wavelength_nm), tau=tau, npml=npml,
                   layers=layers,
                   meta=dict(seed=seed, wavelength_nm=wavelength_nm, k_s=k_s,
                             n_spheres=n_spheres, flat=flat))


def random_fields(shape, seed, scale=1.0):
    """Random complex field state (12, nz, ny, nx) for parity tests."""
    g = rng(seed)
    nz, ny, nx = shape
    re = g.standard_normal((12, nz, ny, nx))
    im = g.standard_normal((12, nz, ny, nx))
    return scale * (re + 1j * im)


def random_problem(nx, ny, nz, seed, npml=2, omega=0.3, tau=0.5,
                   all_sources=True, eps_range=(1.0, 6.0),
                   loss_range=(0.05, 0.8), bcx=0, bcy=0):
    """Unstructured random material (per-cell eps), random PML profile and
    random sources on all four source arrays -- for parity tests that must
    touch every coefficient array and every component."""
    g = rng(seed)
    eps = (g.uniform(*eps_range, (nz, ny, nx))
           + 1j * g.uniform(*loss_range, (nz, ny, nx)))
    sig_e, sig_h = pml_profiles(nz, npml, npml, eps_lo=eps_range[0],
                                eps_hi=eps_range[0])
    sources = {}
    keys = ("Hx", "Hy", "Ex", "Ey") if all_sources else ("Ex",)
    for key in keys:
        sources[key] = (g.standard_normal((nz, ny, nx))
                        + 1j * g.standard_normal((nz, ny, nx)))
    return Problem(eps=eps, sig_e=sig_e, sig_h=sig_h, sources=sources,
                   omega=omega, tau=tau, npml=npml, bcx=bcx, bcy=bcy,
                   meta=dict(seed=seed))
