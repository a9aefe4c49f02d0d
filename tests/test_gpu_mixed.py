"""GPU checks of the mixed-precision solver (complex64 inner sweeps inside
FP64 defect correction) against the plain FP64 GPU solver and the direct
solve of the fixed point.

With x0 = 0 the first correction d = sum_j M^j r, r = Phi(0), is exactly the
plain iterate after the same number of sweeps, so one outer step pins the
complex64 sweep against the FP64 sweep to single-precision rounding.  After
convergence, the FP64 residual (the kernel pinned against the oracle) must be
below the tolerance, and the physical fields must agree with the FP64 solver
and with the sparse-LU fixed point to the accuracy the tolerance implies."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle import dense  # noqa: E402
from paper_1510_05218_amd import inputs  # noqa: E402
from paper_1510_05218_amd import thiim  # noqa: E402


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _phys(x):
    x = x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)
    return x[0::2] + x[1::2]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _window_passes(pb, T):
    """Passes averaged per correction: one rotation period 2 pi / (w tau)."""
    return max(1, math.floor(2 * math.pi / (pb.omega * pb.tau * T) + 0.5))


@pytest.mark.parametrize("t_block,z_chunk", [(2, 0), (3, 0), (2, 5), (3, 7)])
def test_first_correction_equals_plain_iterates(t_block, z_chunk):
    """From x0 = 0 the residual is r = Phi(0) and the inner iterate after j
    passes is d_j = sum_{k <= jT} M^k r, the plain iterate after 1 + jT
    iterations; one correction adds the mean of d_j over the last Kp passes.
    Its physical fields must equal that mean of plain FP64 iterates (the
    residual's split-difference part is dropped where it cannot reach the
    physical fields, so only P x is comparable)."""
    _require_gpu()
    pb = inputs.random_problem(37, 29, 23, seed=41)
    T = t_block
    m = 9
    kp = _window_passes(pb, T)
    passes = max((m - 1 + T - 1) // T, kp)
    s = thiim.Solver(pb, storage="compact", precision="mixed", t_block=T, z_chunk=z_chunk)
    rc, it, r = s.solve(1e-30, 2, m)
    assert rc == thiim.THIIM_ENOTCONV and it == 2 + passes * T
    x_mixed = _phys(s.fields())
    f = thiim.Solver(pb, storage="compact")
    f.iterate(1 + (passes - kp + 1) * T)
    acc = _phys(f.fields()) / kp
    for _ in range(kp - 1):
        f.iterate(T)
        acc = acc + _phys(f.fields()) / kp
    assert _rel(x_mixed, acc) < 2e-6


def test_mixed_matches_fp64_solver():
    _require_gpu()
    pb = inputs.solar_cell(40, 32, 36, seed=5, npml=6, loss_range=(0.2, 0.5),
                           eps_range=(1.0, 4.0), texture_amp=2)
    pb.omega = 0.6
    tol = 1e-9
    f = thiim.Solver(pb, storage="compact")
    rc, it64, r64 = f.solve(tol, 200000, 200)
    assert rc == thiim.THIIM_OK and r64 <= tol
    s = thiim.Solver(pb, storage="compact", precision="mixed")
    rc, itm, rm = s.solve(tol, 200000, 200)
    assert rc == thiim.THIIM_OK and rm <= tol
    # the FP64 residual of the mixed result, recomputed from scratch
    assert s.residual() <= tol
    assert _rel(_phys(s.fields()), _phys(f.fields())) < 1e-6


def test_mixed_reaches_direct_solve_fixed_point():
    _require_gpu()
    pb = inputs.solar_cell(6, 6, 18, seed=1, npml=6, eps_range=(1.0, 2.0),
                           loss_range=(0.2, 0.5), texture_amp=1)
    pb.omega = 1.0
    xs = dense.fixed_point(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau)
    s = thiim.Solver(pb, storage="compact", precision="mixed")
    rc, it, r = s.solve(1e-11, 400000, 0)  # adaptive inner sweeps
    assert rc == thiim.THIIM_OK and r <= 1e-11
    assert _rel(_phys(s.fields()), oracle.physical(xs)) < 1e-7


@pytest.mark.parametrize("bcx,bcy", [(1, 1), (0, 1)])
def test_mixed_dirichlet_back_iteration_reaches_direct_solve(bcx, bcy):
    """The pair-sum form of the complex64 inner sweeps on Dirichlet x/y walls,
    back-iteration cells (Eq. 5) and a graded PML whose planes keep their x
    and y pairs split: the mixed solve reaches the sparse-LU fixed point."""
    _require_gpu()
    # E sources only: a divergent H source would feed curl-free H, which the
    # iteration only rotates (no fixed point is approached there)
    pb = inputs.random_problem(7, 6, 16, seed=23, npml=4, bcx=bcx, bcy=bcy,
                               loss_range=(0.2, 0.6), all_sources=False)
    g = inputs.rng(24)
    mask = g.random(pb.eps.shape) < 0.15
    pb.eps[mask] = -g.uniform(1, 3, mask.sum()) + 1j * g.uniform(0.2, 0.6, mask.sum())
    xs = dense.fixed_point(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau,
                           pb.h, pb.bcx, pb.bcy)
    s = thiim.Solver(pb, storage="compact", precision="mixed")
    rc, it, r = s.solve(1e-11, 400000, 0)
    assert rc == thiim.THIIM_OK and r <= 1e-11
    # slow convergence (the error shrinks by ~0.06% per iteration) magnifies
    # the residual into the error
    assert _rel(_phys(s.fields()), oracle.physical(xs)) < 1e-6


def test_first_correction_full_size_512():
    """The first-correction identity on the 512^3 benchmark workload in the
    configuration the mixed solves use (T = 3, automatic chunks): the
    physical fields of one correction from x0 = 0 equal the window mean of
    plain FP64 iterates.  Tolerance 1e-5: about 60 complex64 sweeps, each
    rounding at 6e-8 relative."""
    _require_gpu()
    if torch.cuda.get_device_properties(0).total_memory < 250e9:
        pytest.skip("needs the 288 GB of an MI355X")
    n, T, m = 512, 3, 9
    pb = inputs.solar_cell(n, n, n, seed=3, npml=6, n_spheres=200)
    kp = _window_passes(pb, T)
    passes = max((m - 1 + T - 1) // T, kp)
    s = thiim.Solver(pb, storage="compact", precision="mixed", t_block=T)
    rc, it, r = s.solve(1e-30, 2, m)
    assert rc == thiim.THIIM_ENOTCONV and it == 2 + passes * T
    x = s.fields()
    x_mixed = x[0::2] + x[1::2]
    del x
    s.close()
    torch.cuda.empty_cache()
    f = thiim.Solver(pb, storage="compact", kernel="blocked")
    f.iterate(1 + (passes - kp + 1) * T)
    x = f.fields()
    acc = (x[0::2] + x[1::2]) / kp
    for _ in range(kp - 1):
        f.iterate(T)
        x = f.fields()
        acc += (x[0::2] + x[1::2]) / kp
    del x
    f.close()
    err = float(torch.linalg.vector_norm(x_mixed - acc) / torch.linalg.vector_norm(acc))
    print(f"[512 first correction] {passes} passes of T = {T}, rel. error {err:.2e}",
          flush=True)
    assert err < 1e-5
