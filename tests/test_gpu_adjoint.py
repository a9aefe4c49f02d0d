"""GPU checks of the adjoint gradient (thiim_adjoint_grad) and its
torch.autograd interface.

  * parity with the oracle at fixed iteration counts: n forward iterations
    from x0 = 0, then m transposed iterations from lam = 0 and the pointwise
    gradient, on both sides, for every fused tile, z chunking and boundary
    combination, on ragged grids with back-iteration cells -- elementwise
    within 1e-10 of the largest gradient entry (both sides round the same
    formulas in different orders);
  * converged gradient against the converged oracle gradient (which is
    pinned against finite differences of the direct solve);
  * central finite differences (h = 1e-6) of J computed by the GPU solver on
    16 cells of the middle layer, every solve run to the same iteration count
    from x0 = 0, within 1e-5 of the largest gradient entry -- on a small grid
    and on the 128 x 128 x 256 gradient configuration itself;
  * one averaged correction of the mixed-precision adjoint (the complex64
    temporally blocked transposed sweep) against the mean of the oracle's
    transposed iterates over the same window, at a complex64 tolerance;
  * torch.autograd.gradcheck of the differentiable absorption functional.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle import adjoint  # noqa: E402
from paper_1510_05218_amd import inputs  # noqa: E402
from paper_1510_05218_amd import thiim  # noqa: E402


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _with_back_cells(pb, seed, frac=0.05):
    g = inputs.rng(seed)
    mask = g.random(pb.eps.shape) < frac
    pb.eps[mask] = -g.uniform(1, 4, mask.sum()) + 1j * g.uniform(0.1, 1, mask.sum())
    return pb


def _oracle_fixed(pb, w, nf, na):
    coef = oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h)
    x = oracle.iterate(coef, oracle.zero_fields(pb.shape), nf, pb.bcx, pb.bcy)
    g = adjoint.adjoint_source(pb.eps, x, w)
    lam = oracle.adjoint_iterate(coef, np.zeros_like(g), g, na, pb.bcx, pb.bcy)
    grad = adjoint.gradient(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h,
                            x, lam, w, pb.bcx, pb.bcy)
    return adjoint.objective(pb.eps, x, w), grad


@pytest.mark.parametrize("tile,z_chunk,bcx,bcy", [
    ((64, 8), 0, 0, 0), ((32, 8), 5, 1, 0), ((64, 4), 3, 0, 1), ((16, 16), 0, 1, 1),
    ((16, 16), 4, 0, 0)])
def test_adjoint_matches_oracle_fixed_counts(tile, z_chunk, bcx, bcy):
    _require_gpu()
    print(f"[adjoint parity] tile={tile} z_chunk={z_chunk} bc=({bcx},{bcy})", flush=True)
    pb = _with_back_cells(inputs.random_problem(37, 19, 14, seed=21, bcx=bcx, bcy=bcy), 22)
    w = inputs.rng(23).uniform(0, 1, pb.shape)
    nf, na = 40, 35
    s = thiim.Solver(pb, kernel="fused", tile=tile, z_chunk=z_chunk, storage="compact",
                     adjoint=True)
    s.iterate(nf)
    rc, J, grad, it, _ = s.adjoint_grad(w, tol=0.0, max_it=na)
    assert rc == thiim.THIIM_OK and it == na
    grad = grad.cpu().numpy()
    s.close()
    Jo, go = _oracle_fixed(pb, w, nf, na)
    assert abs(J - Jo) <= 1e-12 * abs(Jo)
    scale = np.abs(go).max()
    assert np.abs(grad.real - go.real).max() <= 1e-10 * scale
    assert np.abs(grad.imag - go.imag).max() <= 1e-10 * scale


def test_adjoint_blocked_forward_and_zero_iterations():
    """The forward state may come from the blocked sweep; with max_it = 0 the
    gradient is the explicit term w |E|^2 on eps'' alone."""
    _require_gpu()
    pb = inputs.solar_cell(24, 24, 36, seed=1, npml=6)
    w = np.zeros(pb.shape)
    w[14:22] = 1.0
    s = thiim.Solver(pb, storage="compact", adjoint=True)  # blocked forward
    s.iterate(50)
    rc, J, grad, it, _ = s.adjoint_grad(w, tol=0.0, max_it=0)
    assert rc == thiim.THIIM_OK and it == 0
    x = s.fields().cpu().numpy()
    s.close()
    E = x[6::2] + x[7::2]
    e2 = np.sum(np.abs(E) ** 2, axis=0)
    g = grad.cpu().numpy()
    assert np.all(g.real == 0.0)
    np.testing.assert_allclose(g.imag, w * e2, rtol=1e-14, atol=0)
    np.testing.assert_allclose(J, np.sum(w * pb.eps.imag * e2), rtol=1e-12)


def test_adjoint_converged_matches_converged_oracle():
    _require_gpu()
    pb = _with_back_cells(inputs.random_problem(9, 7, 12, seed=31), 32, 0.03)
    w = inputs.rng(33).uniform(0, 1, pb.shape)
    s = thiim.Solver(pb, storage="compact", adjoint=True)
    s.iterate(9000)
    rc, J, grad, it, r = s.adjoint_grad(w, tol=1e-13, max_it=20000, check_every=100)
    assert rc == thiim.THIIM_OK, (it, r)
    s.close()
    Jo, go, _, _, _ = adjoint.gradient_of(pb, w, tol=1e-13)
    assert abs(J - Jo) <= 1e-10 * abs(Jo)
    assert np.abs(grad.cpu().numpy() - go).max() <= 1e-8 * np.abs(go).max()


def test_adjoint_finite_differences_16_cells():
    """J after n iterations from x0 = 0 (n large enough to converge), for
    eps +- 1e-6 at 16 seeded cells of the weighted middle planes, against the
    adjoint gradient at the unperturbed solution (lossy random medium, random
    x-polarised sources, graded PML)."""
    _require_gpu()
    pb = inputs.random_problem(12, 10, 16, seed=20, all_sources=False)
    w = np.zeros(pb.shape)
    w[6:11] = 1.0
    n = 7000

    def solve_J(eps):
        p = inputs.Problem(**{**pb.__dict__, "eps": eps})
        s = thiim.Solver(p, storage="compact", adjoint=True)
        s.iterate(n)
        out = s.adjoint_grad(w, tol=1e-12, max_it=20000, check_every=200)
        s.close()
        return out

    rc, J0, grad, it, r = solve_J(pb.eps)
    assert rc == thiim.THIIM_OK, (it, r)
    grad = grad.cpu().numpy()
    scale = np.abs(grad).max()
    g = inputs.rng(24)
    cells = [(int(g.integers(6, 11)), int(g.integers(0, 10)), int(g.integers(0, 12)))
             for _ in range(16)]
    hfd = 1e-6
    for c in cells:
        for unit, part in ((1.0, "re"), (1j, "im")):
            ep, em = pb.eps.copy(), pb.eps.copy()
            ep[c] += hfd * unit
            em[c] -= hfd * unit
            fd = (solve_J(ep)[1] - solve_J(em)[1]) / (2 * hfd)
            an = grad[c].real if part == "re" else grad[c].imag
            assert abs(fd - an) <= 1e-5 * scale, (c, part, fd, an)


def test_autograd_gradcheck():
    _require_gpu()
    from paper_1510_05218_amd.autograd import absorption

    pb = inputs.random_problem(4, 4, 8, seed=41, npml=2, all_sources=False)
    w = torch.from_numpy(inputs.rng(42).uniform(0, 1, pb.shape)).cuda()
    eps = torch.from_numpy(pb.eps).cuda().requires_grad_(True)

    def f(e):
        return absorption(e, w, pb, iters=8000, adj_tol=1e-12)

    assert torch.autograd.gradcheck(f, (eps,), eps=1e-6, atol=1e-6, rtol=1e-4,
                                    fast_mode=True)
    J = f(eps)
    J.backward()
    assert eps.grad is not None and eps.grad.dtype == torch.complex128


def test_adjoint_requires_adjoint_workspace():
    _require_gpu()
    pb = inputs.random_problem(8, 8, 8, seed=5)
    s = thiim.Solver(pb, storage="compact")
    with pytest.raises(thiim.ThiimError) as e:
        s.adjoint_grad(np.ones(pb.shape), tol=0.0, max_it=1)
    assert e.value.status == thiim.THIIM_EINVAL
    s.close()


def test_adjoint_directional_fd_128x128x256():
    """The gradient configuration at its full size: a 128 x 128 x 256 textured
    stack (eps'' in [0.1, 0.5]), J over the cells of the middle layer, forward
    and adjoint solved to 1e-10 (forward: the mixed-precision solver with a
    fixed inner count; adjoint: averaged defect correction).  Check: the
    central difference (h = 1e-6) of J along a seeded random direction of eps
    over the middle layer -- both perturbed forward solves run the same sweep
    schedule as the unperturbed one, so their truncation errors correlate --
    against the gradient's inner product with it."""
    _require_gpu()
    pb = inputs.solar_cell(128, 128, 256, seed=20, npml=6, loss_range=(0.1, 0.5))
    mid = pb.layers[1][2]
    w = (pb.eps == mid).astype(np.float64)  # the middle layer's cells
    assert w.sum() > 0
    m = 2000
    kw = dict(storage="compact", precision="mixed", adjoint=True)
    s = thiim.Solver(pb, **kw)
    rc, n_sw, r = s.solve(1e-10, 2000000, m)
    assert rc == thiim.THIIM_OK, (n_sw, r)
    print(f"[adjoint 128x128x256] forward {n_sw} sweeps", flush=True)
    rc, J0, grad, ait, ar = s.adjoint_grad(w, tol=1e-10, max_it=2000000, check_every=m)
    assert rc == thiim.THIIM_OK, (ait, ar)
    print(f"[adjoint 128x128x256] adjoint {ait} sweeps", flush=True)
    grad = grad.cpu().numpy()
    s.close()
    g = inputs.rng(25)
    d = (g.standard_normal(pb.shape) + 1j * g.standard_normal(pb.shape)) * w
    hfd = 1e-6

    def J_at(eps):
        p = inputs.Problem(**{**pb.__dict__, "eps": eps})
        sp = thiim.Solver(p, **kw)
        sp.solve(1e-30, n_sw, m)  # the same schedule, stopped at n_sw sweeps
        out = sp.adjoint_grad(w, tol=0.0, max_it=0)[1]
        sp.close()
        return out

    fd = (J_at(pb.eps + hfd * d) - J_at(pb.eps - hfd * d)) / (2 * hfd)
    an = float(np.sum(grad.real * d.real + grad.imag * d.imag))
    print(f"[adjoint 128x128x256] fd {fd:.10e} adjoint {an:.10e}", flush=True)
    assert abs(fd - an) <= 1e-5 * abs(an)


def test_adjoint_on_mixed_context_matches_fp64():
    """On a mixed-precision context the adjoint's inner sweeps run in
    complex64 (defect, lam and norms in FP64): to the same tolerance the
    gradient equals the one from an FP64 context."""
    _require_gpu()
    pb = inputs.random_problem(24, 20, 28, seed=95, all_sources=False)
    w = inputs.rng(96).uniform(0, 1, pb.shape)
    grads = []
    for prec in ("fp64", "mixed"):
        s = thiim.Solver(pb, storage="compact", precision=prec, adjoint=True)
        rc, it, r = s.solve(1e-12, 400000, 300 if prec == "mixed" else 100)
        assert rc == thiim.THIIM_OK, (prec, it, r)
        rc, J, grad, ait, ar = s.adjoint_grad(w, tol=1e-12, max_it=400000, check_every=300)
        assert rc == thiim.THIIM_OK, (prec, ait, ar)
        print(f"[adjoint {prec}] forward {it}, adjoint {ait} sweeps", flush=True)
        grads.append(grad.cpu().numpy())
        s.close()
    scale = np.abs(grads[0]).max()
    assert np.abs(grads[1] - grads[0]).max() <= 1e-8 * scale


@pytest.mark.parametrize("bcx,bcy", [(0, 0), (1, 1)])
def test_adjoint32_blocked_one_correction_matches_oracle(bcx, bcy):
    """On a mixed-precision context, tol > 0 and max_it = 1 + m stop the
    adjoint after exactly one defect correction: one FP64 transposed sweep
    from lam = 0 gives r = g, then P passes of the complex64 blocked
    transposed sweep (two sweeps each) run d <- M^T d + g from d = g, and lam
    is the mean of d after the last Kq passes.  After j sweeps d equals the
    plain transposed iterate lam_{j+1}, so the oracle's lam is the mean of
    lam_{2p+3} over those passes p; both gradients are formed from the same
    forward state.  Complex64 tolerance: 1e-5 of the largest entry."""
    _require_gpu()
    print(f"[adjoint32 blocked] bc=({bcx},{bcy})", flush=True)
    pb = _with_back_cells(inputs.random_problem(37, 19, 14, seed=61, bcx=bcx, bcy=bcy), 62)
    w = inputs.rng(63).uniform(0, 1, pb.shape)
    nf, m = 40, 100
    s = thiim.Solver(pb, storage="compact", precision="mixed", adjoint=True, kernel="fused")
    s.iterate(nf)
    x = s.fields().cpu().numpy()
    rc, J, grad, it, _ = s.adjoint_grad(w, tol=1e-30, max_it=1 + m, check_every=m)
    assert rc == thiim.THIIM_ENOTCONV, rc
    grad = grad.cpu().numpy()
    s.close()
    wt = pb.omega * pb.tau
    Kp = max(1, int(round(2 * np.pi / wt)))
    Kq = max(1, int(round(2 * np.pi / (wt * 2))))
    mm = max(m, 2 * Kp)
    P = max((mm + 1) // 2, Kq)
    coef = oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h)
    xo = oracle.iterate(coef, oracle.zero_fields(pb.shape), nf, bcx, bcy)
    assert np.linalg.norm(x - xo) <= 1e-12 * np.linalg.norm(xo)
    g = adjoint.adjoint_source(pb.eps, xo, w)
    lam = oracle.adjoint_iterate(coef, np.zeros_like(g), g, 2 * (P - Kq) + 3, bcx, bcy)
    acc = lam.copy()
    for _ in range(Kq - 1):
        lam = oracle.adjoint_iterate(coef, lam, g, 2, bcx, bcy)
        acc += lam
    acc /= Kq
    go = adjoint.gradient(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h,
                          xo, acc, w, bcx, bcy)
    scale = np.abs(go).max()
    err = max(np.abs(grad.real - go.real).max(), np.abs(grad.imag - go.imag).max())
    print(f"[adjoint32 blocked] max error {err / scale:.2e} of the largest entry", flush=True)
    assert err <= 1e-5 * scale


def test_adjoint_fd_16_cells_128x128x256():
    """The gradient configuration at its full size (128 x 128 x 256 textured
    stack, J over the middle layer, forward and adjoint to 1e-10), checked
    cell by cell: for 16 seeded middle-layer cells and both eps' and eps'',
    the central difference (h = 1e-6) of J against the adjoint gradient.
    Every perturbed forward solve runs the unperturbed sweep schedule (fixed
    inner count, stopped at the same sweep count), so the truncation errors
    of the two sides correlate.  J(eps + h) - J(eps - h) is formed cell by
    cell from the two physical E fields,
        w eps''_+ Re((E_+ - E_-) conj(E_+ + E_-)) + w (eps''_+ - eps''_-) |E_-|^2,
    rather than as the difference of two sums of 1.3 million terms, whose
    rounding would exceed the single-cell signal."""
    _require_gpu()
    pb = inputs.solar_cell(128, 128, 256, seed=20, npml=6, loss_range=(0.1, 0.5))
    mid = pb.layers[1][2]
    w = (pb.eps == mid).astype(np.float64)
    m = 2000
    kw = dict(storage="compact", precision="mixed", adjoint=True)
    s = thiim.Solver(pb, **kw)
    rc, n_sw, r = s.solve(1e-10, 2000000, m)
    assert rc == thiim.THIIM_OK, (n_sw, r)
    rc, J0, grad, ait, ar = s.adjoint_grad(w, tol=1e-10, max_it=2000000, check_every=m)
    assert rc == thiim.THIIM_OK, (ait, ar)
    print(f"[adjoint fd 128x128x256] forward {n_sw}, adjoint {ait} sweeps", flush=True)
    grad = grad.cpu().numpy()
    s.close()
    scale = np.abs(grad).max()
    wd = torch.from_numpy(w).cuda()
    g = inputs.rng(26)
    ks, js, is_ = np.nonzero(w)
    pick = g.choice(len(ks), size=16, replace=False)
    cells = [(int(ks[i]), int(js[i]), int(is_[i])) for i in pick]
    hfd = 1e-6

    def E_at(eps):
        p = inputs.Problem(**{**pb.__dict__, "eps": eps})
        sp = thiim.Solver(p, **kw)
        sp.solve(1e-30, n_sw, m)  # the unperturbed schedule, stopped at n_sw sweeps
        x = sp.fields()
        sp.close()
        return x[6::2] + x[7::2]

    worst = 0.0
    for n, c in enumerate(cells):
        for unit, part in ((1.0, "re"), (1j, "im")):
            ep, em = pb.eps.copy(), pb.eps.copy()
            ep[c] += hfd * unit
            em[c] -= hfd * unit
            Ep, Em = E_at(ep), E_at(em)
            dE2 = torch.sum(((Ep - Em) * torch.conj(Ep + Em)).real, dim=0)
            e2m = torch.sum((Em * torch.conj(Em)).real, dim=0)
            epp_p = torch.from_numpy(ep.imag.copy()).cuda()
            epp_m = torch.from_numpy(em.imag.copy()).cuda()
            dJ = float(torch.sum(wd * epp_p * dE2) + torch.sum(wd * (epp_p - epp_m) * e2m))
            del Ep, Em, dE2, e2m
            fd = dJ / (2 * hfd)
            an = grad[c].real if part == "re" else grad[c].imag
            worst = max(worst, abs(fd - an) / scale)
            print(f"[adjoint fd 128x128x256] cell {n} {c} d/deps{part}: fd {fd:.9e} "
                  f"adjoint {an:.9e}", flush=True)
            assert abs(fd - an) <= 1e-5 * scale, (c, part, fd, an, scale)
    print(f"[adjoint fd 128x128x256] worst {worst:.2e} of the largest entry", flush=True)
