"""THIIM reference oracle -- TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation of the THIIM split-field Yee iteration
(arXiv:1510.05218, Sec. I-A Eq. 3-7 and Sec. III Listings 1-2), used to check
the GPU library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the GPU library and its
Python binding never do.  It shares no code with them: the only common module
is the seeded input generator, which holds none of the method's arithmetic.

Contents
  * ``coeffs``    -- the 28 coefficient arrays from the material data
                     (Eq. 3-5 solved for the new value; C, ``thiim_oracle.c``)
  * ``iterate``   -- n THIIM iterations, one loop nest per split component (C)
  * ``iterate_light`` -- the same without coefficient arrays (memory-light
                     mode for full-size grids; bit-identical)
  * ``residual``  -- ||P(Phi(x) - x)||_2 / ||P Phi(0)||_2 in FP64, P the sum
                     of each split pair (the physical field)
  * ``dense``     -- the time-harmonic fixed-point system assembled directly
                     from eps, sigma, omega, tau and solved by sparse LU
  * ``adjoint``   -- the objective J = sum w eps'' |E|^2, the transposed
                     iteration lam <- M^T lam + g (C) and the gradient of J
                     with respect to eps' and eps''

Array conventions (shared with the C-ABI of the GPU library, by definition):
  fields  : complex128 ndarray (12, nz, ny, nx), component order
            H_xy H_xz H_yx H_yz H_zx H_zy E_xy E_xz E_yx E_yz E_zx E_zy
  coef    : complex128 ndarray (28, nz, ny, nx): t_0..t_11, c_0..c_11,
            Src for H_xy, H_yx, E_xy, E_yx
  eps     : complex128 ndarray (nz, ny, nx) holding eps' + 1j*eps''
            (the physical eps_r = eps' - i eps'' in the exp(+i w t) convention)
  sources : dict with optional keys 'Hx', 'Hy', 'Ex', 'Ey' -> complex (nz,ny,nx)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

SRC_KEYS = ("Hx", "Hy", "Ex", "Ey")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no FP contraction)."""
    from .compile import build_oracle

    return build_oracle(force=force)


def _configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_coeffs.argtypes = [ctypes.c_int] * 3 + [
        dp, dp, dp, ctypes.POINTER(dp), ctypes.c_double, ctypes.c_double,
        ctypes.c_double, ctypes.POINTER(dp)]
    lib.oracle_coeffs.restype = ctypes.c_int
    lib.oracle_iterate.argtypes = [ctypes.c_int] * 5 + [
        ctypes.POINTER(dp), ctypes.POINTER(dp), ctypes.c_int]
    lib.oracle_iterate.restype = ctypes.c_int
    lib.oracle_iterate_light.argtypes = [ctypes.c_int] * 5 + [
        dp, dp, dp, ctypes.POINTER(dp), ctypes.c_double, ctypes.c_double, ctypes.c_double,
        ctypes.POINTER(dp), ctypes.c_int]
    lib.oracle_iterate_light.restype = ctypes.c_int
    lib.oracle_adjoint_iterate.argtypes = [ctypes.c_int] * 5 + [
        ctypes.POINTER(dp), ctypes.POINTER(dp), ctypes.POINTER(dp), ctypes.c_int]
    lib.oracle_adjoint_iterate.restype = ctypes.c_int
    lib.oracle_flops_per_update.argtypes = [ctypes.c_int]
    lib.oracle_flops_per_update.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ptr_array(arrs):
    dp = ctypes.POINTER(ctypes.c_double)
    out = (dp * len(arrs))()
    for i, a in enumerate(arrs):
        out[i] = _ptr(a) if a is not None else dp()
    return out


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loop nests (n >= 1)."""
    _load().oracle_set_threads(int(n))


def flops_per_update(has_src: bool) -> int:
    return _load().oracle_flops_per_update(int(bool(has_src)))


def coeffs(eps, sig_e, sig_h, sources, omega, tau=0.5, h=1.0):
    """The 28 coefficient arrays (complex128, (28, nz, ny, nx))."""
    eps = np.ascontiguousarray(eps, dtype=np.complex128)
    nz, ny, nx = eps.shape
    sig_e = np.ascontiguousarray(sig_e, dtype=np.float64)
    sig_h = np.ascontiguousarray(sig_h, dtype=np.float64)
    assert sig_e.shape == (nz,) and sig_h.shape == (nz,)
    src = []
    for key in SRC_KEYS:
        s = (sources or {}).get(key)
        if s is not None:
            s = np.ascontiguousarray(s, dtype=np.complex128)
            assert s.shape == eps.shape
        src.append(s)
    coef = np.zeros((28, nz, ny, nx), dtype=np.complex128)
    rc = _load().oracle_coeffs(nx, ny, nz, _ptr(eps), _ptr(sig_e), _ptr(sig_h),
                               _ptr_array(src), float(omega), float(tau),
                               float(h), _ptr_array([coef[i] for i in range(28)]))
    if rc != 0:
        raise ValueError("oracle_coeffs: invalid material data")
    return coef


def zero_fields(shape):
    nz, ny, nx = shape
    return np.zeros((12, nz, ny, nx), dtype=np.complex128)


def iterate(coef, fields, n, bcx=0, bcy=0):
    """n THIIM iterations in place on ``fields`` (12, nz, ny, nx)."""
    assert coef.dtype == np.complex128 and fields.dtype == np.complex128
    assert coef.flags["C_CONTIGUOUS"] and fields.flags["C_CONTIGUOUS"]
    _, nz, ny, nx = coef.shape
    assert fields.shape == (12, nz, ny, nx)
    _load().oracle_iterate(nx, ny, nz, int(bcx), int(bcy),
                           _ptr_array([coef[i] for i in range(28)]),
                           _ptr_array([fields[i] for i in range(12)]), int(n))
    return fields


def iterate_light(eps, sig_e, sig_h, sources, omega, tau, h, fields, n, bcx=0, bcy=0):
    """n THIIM iterations in place without coefficient arrays (memory-light
    mode: coefficients evaluated per cell from the material data); bit-
    identical to coeffs() + iterate()."""
    eps = np.ascontiguousarray(eps, dtype=np.complex128)
    nz, ny, nx = eps.shape
    assert fields.shape == (12, nz, ny, nx) and fields.flags["C_CONTIGUOUS"]
    sig_e = np.ascontiguousarray(sig_e, dtype=np.float64)
    sig_h = np.ascontiguousarray(sig_h, dtype=np.float64)
    src = []
    for key in SRC_KEYS:
        s = (sources or {}).get(key)
        src.append(None if s is None else np.ascontiguousarray(s, dtype=np.complex128))
    rc = _load().oracle_iterate_light(nx, ny, nz, int(bcx), int(bcy), _ptr(eps), _ptr(sig_e),
                                      _ptr(sig_h), _ptr_array(src), float(omega), float(tau),
                                      float(h), _ptr_array([fields[i] for i in range(12)]),
                                      int(n))
    if rc != 0:
        raise ValueError("oracle_iterate_light: invalid material data")
    return fields


def phi(coef, x, bcx=0, bcy=0):
    """One THIIM iteration applied to a copy of x."""
    y = np.array(x, copy=True)
    return iterate(coef, y, 1, bcx, bcy)


def norm(x) -> float:
    """FP64 2-norm over all components and cells."""
    return float(np.sqrt(np.sum(np.abs(np.asarray(x)) ** 2)))


def physical(x):
    """The six physical components (H_x, H_y, H_z, E_x, E_y, E_z): each the
    sum of its two split parts (Eq. 6/7)."""
    x = np.asarray(x)
    return x[0::2] + x[1::2]


def residual(coef, x, bcx=0, bcy=0, phi0_norm=None) -> float:
    """Relative residual of the physical fields,
    ||P(Phi(x) - x)||_2 / ||P Phi(0)||_2, with P the split-pair sum.

    The split-difference parts of a pair never act on the other field, and
    where both parts have the same coefficients (outside the PML, lossless)
    they rotate by exp(-i w tau) per iteration for ever; the residual is
    therefore taken on the physical fields."""
    if phi0_norm is None:
        phi0_norm = norm(physical(phi(coef, np.zeros_like(x), bcx, bcy)))
    return norm(physical(phi(coef, x, bcx, bcy) - x)) / phi0_norm


def solve(coef, tol, max_it, bcx=0, bcy=0, check_every=50):
    """Iterate from x0 = 0 until the relative residual is <= tol."""
    _, nz, ny, nx = coef.shape
    x = zero_fields((nz, ny, nx))
    r0 = norm(physical(phi(coef, x, bcx, bcy)))
    it = 0
    res = 1.0
    while it < max_it:
        step = min(check_every, max_it - it)
        iterate(coef, x, step, bcx, bcy)
        it += step
        res = residual(coef, x, bcx, bcy, r0)
        if res <= tol:
            break
    return x, it, res


def adjoint_iterate(coef, lam, g, n, bcx=0, bcy=0):
    """n transposed iterations lam <- M^T lam + g in place (lam, g: (12, nz,
    ny, nx); g may be None).  M is the linear part of one THIIM iteration."""
    assert coef.dtype == np.complex128 and lam.dtype == np.complex128
    assert coef.flags["C_CONTIGUOUS"] and lam.flags["C_CONTIGUOUS"]
    _, nz, ny, nx = coef.shape
    assert lam.shape == (12, nz, ny, nx)
    gs = [None] * 12
    if g is not None:
        g = np.ascontiguousarray(g, dtype=np.complex128)
        assert g.shape == lam.shape
        gs = [g[i] for i in range(12)]
    _load().oracle_adjoint_iterate(nx, ny, nz, int(bcx), int(bcy),
                                   _ptr_array([coef[i] for i in range(28)]),
                                   _ptr_array([lam[i] for i in range(12)]),
                                   _ptr_array(gs), int(n))
    return lam
