"""Pins of the CPU oracle against facts other than itself (no GPU needed).

Each test checks the oracle against something it does not contain:
  * the fixed-point system written out independently from Eq. (3)-(5)
    (``oracle.dense``) -- the exact identity Phi(x*) = x*;
  * the textbook Yee numerical dispersion relation (closed form);
  * the printed loop nests of Listings 1 and 2 (operation order, bitwise);
  * structural invariants: linearity in the source, zero source, x/y
    invariance of a flat stack, mirror symmetry x <-> y;
  * closed forms of the coefficients for sigma = 0.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1510_05218_amd import inputs

P = oracle.physical


def _coef(pb):
    return oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


# --------------------------------------------------------------------------
# Fixed point (Sec. I-A, Eq. 3-5 with E^{n+1} = E^n, H^{n+1/2} = H^{n-1/2})
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed,bcx,bcy,back", [(1, 0, 0, False), (2, 1, 0, True),
                                               (3, 0, 1, True), (4, 1, 1, False)])
def test_fixed_point_identity(oracle_lib, seed, bcx, bcy, back):
    """One oracle iteration leaves the directly solved fixed point unchanged,
    for random per-cell materials, random sources on all four source arrays,
    a graded PML and (optionally) back-iteration cells with eps' < 0."""
    pb = inputs.random_problem(5, 4, 9, seed=seed, bcx=bcx, bcy=bcy)
    if back:
        g = inputs.rng(seed + 100)
        mask = g.random(pb.eps.shape) < 0.15
        pb.eps[mask] = -g.uniform(1, 5, mask.sum()) + 1j * g.uniform(0.1, 1, mask.sum())
    coef = _coef(pb)
    xs = dense.fixed_point(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega,
                           pb.tau, pb.h, bcx, bcy)
    y = oracle.phi(coef, xs, bcx, bcy)
    for q in range(12):
        assert _rel(y[q], xs[q]) < 1e-13 or np.linalg.norm(y[q] - xs[q]) < 1e-13 * np.linalg.norm(xs)
    assert _rel(y, xs) < 1e-14


def test_fixed_point_detects_wrong_sign(oracle_lib):
    """The identity is sensitive: a dense system with one curl sign flipped
    is not a fixed point of the oracle."""
    pb = inputs.random_problem(4, 4, 8, seed=7)
    coef = _coef(pb)
    orig = dense.split_table

    def flipped():
        t = orig()
        t[3] = dict(t[3], sign=-t[3]["sign"])
        return t

    dense.split_table = flipped
    try:
        xs = dense.fixed_point(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau)
    finally:
        dense.split_table = orig
    assert _rel(oracle.phi(coef, xs), xs) > 1e-3


def test_iteration_converges_to_fixed_point(oracle_lib):
    """From x0 = 0 the iterates approach the direct solution (physical
    fields) on a lossy textured stack with PML; the residual falls with them."""
    pb = inputs.solar_cell(6, 6, 18, seed=1, npml=6, eps_range=(1.0, 2.0),
                           loss_range=(0.2, 0.5), texture_amp=1)
    pb.omega = 1.0
    coef = _coef(pb)
    xs = dense.fixed_point(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau)
    x = oracle.zero_fields(pb.shape)
    errs, res = [], []
    for _ in range(5):
        oracle.iterate(coef, x, 2000)
        errs.append(_rel(P(x), P(xs)))
        res.append(oracle.residual(coef, x))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert all(b < a for a, b in zip(res, res[1:]))
    assert errs[-1] < 1e-6
    assert oracle.residual(coef, xs) < 1e-13


# --------------------------------------------------------------------------
# Textbook Yee numerical dispersion
# --------------------------------------------------------------------------
def _yee_kz(eps, omega, tau, kt):
    """sin^2(kz h/2) = eps sin^2(w tau/2)/tau^2 - sin^2(kt h/2), h = 1, with the
    branch of a wave travelling (or decaying) towards +z: exp(-i kz z)."""
    s2 = eps * np.sin(omega * tau / 2) ** 2 / tau ** 2 - np.sin(kt / 2) ** 2
    kz = 2 * np.arcsin(np.sqrt(complex(s2)))
    if kz.imag > 0:
        kz = np.conj(kz)
    return kz


@pytest.mark.parametrize("kind,pol,axis", [("E", "y", "x"), ("H", "y", "x"),
                                           ("E", "x", "y"), ("H", "x", "y")])
@pytest.mark.parametrize("m", [0, 1, 2])
def test_yee_dispersion(oracle_lib, kind, pol, axis, m):
    """In a uniform lossless medium the fixed point is a discrete plane wave
    whose z wave number obeys the textbook Yee dispersion relation at the
    lateral wave number 2 pi m / n (TE and TM, along x and y; m = 2 is
    evanescent).  Sources are divergence-free so no static charge remains."""
    eps, n, nz, npml, omega, tau = 2.0, 16, 140, 24, 0.5, 0.5
    nx, ny = (n, 2) if axis == "x" else (2, n)
    e = np.full((nz, ny, nx), eps + 0j)
    sig_e, sig_h = inputs.pml_profiles(nz, npml, npml, eps, eps)
    src = inputs.plane_source(e.shape, npml + 5, pol=pol,
                              kx=m if axis == "x" else 0,
                              ky=m if axis == "y" else 0, field_kind=kind)
    xs = dense.fixed_point(e, sig_e, sig_h, src, omega, tau)
    coef = oracle.coeffs(e, sig_e, sig_h, src, omega, tau)
    assert _rel(oracle.phi(coef, xs), xs) < 1e-13
    ph = P(xs)
    comp = ph[np.argmax([np.linalg.norm(c) for c in ph])]
    col = comp[:, 0, 0]
    k_s = npml + 5
    ks = np.arange(k_s + 3, k_s + (15 if m == 2 else 60))
    ratio = col[ks + 1] / col[ks]
    kz = np.mean(1j * np.log(ratio))
    pred = _yee_kz(eps, omega, tau, 2 * np.pi * m / n)
    assert abs(kz - pred) < 2e-5 * abs(pred)


# --------------------------------------------------------------------------
# Component updates: index shifts and signs fixed by Listings 1 and 2
# --------------------------------------------------------------------------
def _update_ref(F, t, c, src, g1, g2, sign, here, nbr, backward):
    """F <- t F + Src + s c D in explicit real arithmetic (one rounding per
    numpy operation, so no fused multiply-add): G = G1 + G2 at the cell
    (index ``here``) and at its neighbour (``nbr``); D = G(p) - G(p - e) for a
    backward (H) and G(p + e) - G(p) for a forward (E) difference."""
    gr = g1[here].real + g2[here].real
    gi = g1[here].imag + g2[here].imag
    nr = g1[nbr].real + g2[nbr].real
    ni = g1[nbr].imag + g2[nbr].imag
    dr, di = (gr - nr, gi - ni) if backward else (nr - gr, ni - gi)
    tfr = t.real * F.real - t.imag * F.imag
    tfi = t.real * F.imag + t.imag * F.real
    cdr = c.real * dr - c.imag * di
    cdi = c.real * di + c.imag * dr
    re = tfr + cdr if sign > 0 else tfr - cdr
    im = tfi + cdi if sign > 0 else tfi - cdi
    if src is not None:
        re = re + src.real
        im = im + src.imag
    return re + 1j * im


def test_listing_components_bitwise(oracle_lib):
    """The two components the paper prints fix their shifts, signs and
    source arrays: H_yx (Listing 1) is driven by E_x = E_xy + E_xz through the
    difference over the outer (z) dimension, E_x(k) - E_x(k-1), subtracted
    after scaling by c, with the source array SrcHy; H_zx (Listing 2) by E_x
    through the middle (y) dimension, E_x(j) - E_x(j-1) added after scaling,
    without a source.  The E parts with the same shapes use the forward
    difference and read the new H (Fig. 3).  Checked bit for bit against the
    update evaluated in explicit real arithmetic on random data (interior
    cells, where no wrap or wall is involved)."""
    g = inputs.rng(11)
    nz, ny, nx = 5, 6, 7

    def crand(*s):
        return g.standard_normal(s) + 1j * g.standard_normal(s)

    coef = crand(28, nz, ny, nx)
    x0 = crand(12, nz, ny, nx)
    x1 = oracle.iterate(coef, x0.copy(), 1)
    k_hi, k_lo = (slice(1, None),), (slice(0, -1),)
    j_hi, j_lo = (slice(None), slice(1, None)), (slice(None), slice(0, -1))
    # H_yx (2): -c (E_x(k) - E_x(k-1)) + SrcHy (array 25)
    ref = _update_ref(x0[2][1:], coef[2][1:], coef[14][1:], coef[25][1:], x0[6], x0[7],
                      -1, k_hi, k_lo, True)
    assert np.array_equal(x1[2][1:], ref)
    # H_zx (4): +c (E_x(j) - E_x(j-1)), no source
    ref = _update_ref(x0[4][:, 1:], coef[4][:, 1:], coef[16][:, 1:], None, x0[6], x0[7],
                      +1, j_hi, j_lo, True)
    assert np.array_equal(x1[4][:, 1:], ref)
    # E_xy (6): -c (H_y(k+1) - H_y(k)) with the new H_y = H_yx + H_yz, SrcEx (26)
    ref = _update_ref(x0[6][:-1], coef[6][:-1], coef[18][:-1], coef[26][:-1], x1[2], x1[3],
                      -1, k_lo, k_hi, False)
    assert np.array_equal(x1[6][:-1], ref)
    # E_xz (7): +c (H_z(j+1) - H_z(j)), no source
    ref = _update_ref(x0[7][:, :-1], coef[7][:, :-1], coef[19][:, :-1], None, x1[4], x1[5],
                      +1, j_lo, j_hi, False)
    assert np.array_equal(x1[7][:, :-1], ref)


def test_flop_counts_match_paper(oracle_lib):
    """Sec. III-A: 22 flops for a Listing-1 update, 20 for Listing 2, 248 per
    lattice-site update (4 with a source array, 8 without)."""
    f1, f2 = oracle.flops_per_update(True), oracle.flops_per_update(False)
    assert (f1, f2) == (22, 20)
    assert 4 * f1 + 8 * f2 == 248


# --------------------------------------------------------------------------
# Structural invariants
# --------------------------------------------------------------------------
def test_linearity_in_source(oracle_lib):
    """Each iterate from x0 = 0 is linear in the sources (every step is affine
    in them and x0 = 0)."""
    pb1 = inputs.random_problem(6, 5, 10, seed=21)
    pb2 = inputs.random_problem(6, 5, 10, seed=22)
    a, b = 0.7 - 0.3j, -1.1 + 0.4j
    mix = {k: a * pb1.sources[k] + b * pb2.sources[k] for k in pb1.sources}
    c1 = _coef(pb1)
    c2 = oracle.coeffs(pb1.eps, pb1.sig_e, pb1.sig_h, pb2.sources, pb1.omega, pb1.tau)
    c3 = oracle.coeffs(pb1.eps, pb1.sig_e, pb1.sig_h, mix, pb1.omega, pb1.tau)
    x1, x2, x3 = (oracle.zero_fields(pb1.shape) for _ in range(3))
    for step in (1, 1, 1, 7, 15):
        oracle.iterate(c1, x1, step)
        oracle.iterate(c2, x2, step)
        oracle.iterate(c3, x3, step)
        assert _rel(x3, a * x1 + b * x2) < 1e-13


def test_zero_source_stays_zero(oracle_lib):
    pb = inputs.solar_cell(8, 8, 20, seed=3, npml=4)
    pb.sources = {}
    coef = _coef(pb)
    assert not np.any(coef[24:])
    x = oracle.iterate(coef, oracle.zero_fields(pb.shape), 40)
    assert not np.any(x)


def test_flat_stack_xy_invariance(oracle_lib):
    """Flat layers + uniform x-polarised source: every column is identical,
    only E_xy and H_yx are non-zero, the other 10 split arrays stay exactly 0,
    and a 2 x 2 grid gives bit-identical columns (1D reduction)."""
    pb = inputs.solar_cell(6, 5, 24, seed=5, npml=4, flat=True)
    coef = _coef(pb)
    x = oracle.iterate(coef, oracle.zero_fields(pb.shape), 60)
    for q in range(12):
        if q in (2, 6):
            assert np.any(x[q])
        else:
            assert not np.any(x[q]), q
    col = x[:, :, :1, :1]
    assert np.array_equal(x, np.broadcast_to(col, x.shape))
    small = inputs.solar_cell(2, 2, 24, seed=5, npml=4, flat=True)
    assert np.array_equal(small.eps[:, 0, 0], pb.eps[:, 0, 0])
    xs = oracle.iterate(_coef(small), oracle.zero_fields(small.shape), 60)
    assert np.array_equal(xs[:, :, :1, :1], col)


def test_mirror_symmetry_xy(oracle_lib):
    """Swapping x <-> y in the geometry and the source polarisation maps
    E_x <-> E_y, E_z -> E_z (polar) and H_x <-> -H_y, H_z -> -H_z (axial)."""
    pb = inputs.solar_cell(8, 8, 20, seed=9, npml=4, texture_amp=2)
    g = inputs.rng(99)
    pb.eps = pb.eps + 0.3 * g.random(pb.eps.shape)  # break every residual symmetry
    sx = pb.sources["Ex"] * (1 + 0.2 * g.standard_normal(pb.shape))
    pb.sources = {"Ex": sx}
    sw = lambda a: np.ascontiguousarray(np.swapaxes(a, -1, -2))  # noqa: E731
    pbm = inputs.Problem(eps=sw(pb.eps), sig_e=pb.sig_e, sig_h=pb.sig_h,
                         sources={"Ey": sw(sx)}, omega=pb.omega, tau=pb.tau)
    n = 30
    x = oracle.iterate(_coef(pb), oracle.zero_fields(pb.shape), n)
    xm = oracle.iterate(_coef(pbm), oracle.zero_fields(pb.shape), n)
    # index map and sign: mirrored component q' = perm[q], value sign[q] * sw(x[q])
    perm = {0: 2, 1: 3, 2: 0, 3: 1, 4: 5, 5: 4, 6: 8, 7: 9, 8: 6, 9: 7, 10: 11, 11: 10}
    scale = np.linalg.norm(x)
    for q in range(12):
        s = -1.0 if q < 6 else 1.0
        assert np.linalg.norm(xm[perm[q]] - s * sw(x[q])) <= 1e-13 * scale, q


# --------------------------------------------------------------------------
# Coefficients: closed forms for sigma = 0
# --------------------------------------------------------------------------
def test_coefficients_lossless_closed_form(oracle_lib):
    nz, ny, nx = 6, 3, 4
    w, tau, h = 0.37, 0.45, 1.0
    eps = np.full((nz, ny, nx), 2.5 + 0j)
    eps[2] = -3.0 + 0j  # back iteration plane, Eq. (5)
    S = np.ones((nz, ny, nx), dtype=complex)
    coef = oracle.coeffs(eps, np.zeros(nz), np.zeros(nz),
                         {"Hx": S, "Hy": S, "Ex": S, "Ey": S}, w, tau, h)
    e1, e2 = np.exp(-1j * w * tau), np.exp(-1j * w * tau / 2)
    fwd = np.ones(nz, bool)
    fwd[2] = False
    for q in range(6):
        assert np.allclose(coef[q], e1, rtol=0, atol=1e-15)
        assert np.allclose(coef[12 + q], tau / h * e2, rtol=0, atol=1e-15)
    for q in range(6, 12):
        assert np.allclose(coef[q][fwd], e1, rtol=0, atol=1e-15)
        assert np.allclose(coef[12 + q][fwd], tau / (2.5 * h) * e2, rtol=0, atol=1e-15)
        assert np.allclose(coef[q][~fwd], np.conj(e1), rtol=0, atol=1e-15)
        assert np.allclose(coef[12 + q][~fwd], tau / (3.0 * h) * np.conj(e2), rtol=0, atol=1e-15)
    assert np.allclose(coef[24], tau * e2, atol=1e-15)      # tau S / e^{iwt/2}
    assert np.allclose(coef[26][fwd], tau * e1, atol=1e-15)  # tau e^{-iwt} S
    assert np.allclose(coef[26][~fwd], -tau, atol=1e-15)     # -tau S (Eq. 5)


def test_pml_and_loss_damp(oracle_lib):
    """With sigma > 0 every t has modulus < 1 (passive update)."""
    pb = inputs.solar_cell(4, 4, 20, seed=2, npml=5, loss_range=(0.1, 0.5))
    coef = _coef(pb)
    pml = np.r_[0:5, 15:20]
    for q in (0, 2):  # H z-difference parts damped inside the PML
        assert np.all(np.abs(coef[q][pml]) < 1 - 1e-6)
    for q in range(6, 12):  # E damped by the material loss everywhere
        assert np.all(np.abs(coef[q]) < 1)
    assert np.all(np.abs(coef[:12]) <= 1 + 1e-15)


# --------------------------------------------------------------------------
# The undamped modes (R16, R17): one iteration multiplies a curl-free H with
# no E, and (in lossless cells) a curl-free E with no H, by exactly
# e^{-i w tau}.  These are the modes the mixed solver's window averaging
# targets; the pin checks the claim against the oracle's iteration.
# --------------------------------------------------------------------------
def _grad_field(phi, backward):
    """Components (x, y, z) of the discrete gradient of phi (nz, ny, nx),
    periodic in x/y: forward differences phi(p + e) - phi(p), or backward."""
    out = []
    for ax in (2, 1, 0):  # x, y, z axes of the array
        if backward:
            out.append(phi - np.roll(phi, 1, axis=ax))
        else:
            out.append(np.roll(phi, -1, axis=ax) - phi)
    return out


@pytest.mark.parametrize("field", ["H", "E"])
def test_curl_free_fields_rotate_by_exp_minus_i_omega_tau(oracle_lib, field):
    pb = inputs.random_problem(8, 7, 16, seed=17, npml=3)
    if field == "E":
        pb.eps = pb.eps.real + 0j  # lossless cells
    coef = oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, {}, pb.omega, pb.tau, pb.h)
    g = inputs.rng(18)
    phi = g.standard_normal(pb.shape) + 1j * g.standard_normal(pb.shape)
    phi[:5] = 0.0  # zero in and next to the PML planes and the z walls
    phi[-5:] = 0.0
    comps = _grad_field(phi, backward=(field == "E"))
    x = oracle.zero_fields(pb.shape)
    base = 0 if field == "H" else 6
    for a in range(3):
        split = g.uniform(0, 1, pb.shape)  # any division between the two parts
        x[base + 2 * a] = split * comps[a]
        x[base + 2 * a + 1] = (1 - split) * comps[a]
    lam = np.exp(-1j * pb.omega * pb.tau)
    # physical fields: the other field's split parts become equal and opposite
    # (a split-difference mode, invisible in P), the curl-free field rotates
    y = P(oracle.phi(coef, x))
    assert np.linalg.norm(y - lam * P(x)) <= 1e-14 * np.linalg.norm(P(x))
    # a gradient that reaches into the PML decays there instead
    if field == "H":
        phi2 = g.standard_normal(pb.shape) + 0j
        comps = _grad_field(phi2, backward=False)
        x2 = oracle.zero_fields(pb.shape)
        for a in range(3):
            x2[2 * a] = comps[a]
        y2 = P(oracle.phi(coef, x2))
        assert np.linalg.norm(y2 - lam * P(x2)) > 1e-3 * np.linalg.norm(P(x2))


@pytest.mark.parametrize("bcx,bcy", [(0, 0), (1, 1)])
def test_memory_light_mode_bitwise(oracle_lib, bcx, bcy):
    """The memory-light iteration (coefficients evaluated per cell) equals the
    stored-coefficient iteration bit for bit: all four sources, a graded PML,
    back-iteration cells."""
    pb = inputs.random_problem(7, 6, 12, seed=23, bcx=bcx, bcy=bcy)
    g = inputs.rng(24)
    mask = g.random(pb.shape) < 0.1
    pb.eps[mask] = -g.uniform(1, 4, mask.sum()) + 1j * g.uniform(0.1, 1, mask.sum())
    coef = _coef(pb)
    a = oracle.iterate(coef, oracle.zero_fields(pb.shape), 9, bcx, bcy)
    b = oracle.iterate_light(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h,
                             oracle.zero_fields(pb.shape), 9, bcx, bcy)
    assert np.array_equal(a, b)


def test_spectral_radius_of_the_iteration(oracle_lib):
    """Convergence of the iteration matrix M = Phi(.) - Phi(0) by power
    iteration from a random split state on a lossy stack with PML: the
    dominant eigenvalue is exactly e^{-i w tau} (the curl-free H and the split
    differences that one iteration only rotates, R16/R17), so rho(M) = 1 on
    the split space rather than < 1, and that eigenvalue is defective: the
    norm ratio approaches 1 like 1 + O(1/n) (polynomial, not exponential,
    growth of the split differences it drives).  The physical residual and
    divergence-free sources keep the solver off this subspace; convergence of
    the physical fields is pinned by test_iteration_converges_to_fixed_point."""
    pb = inputs.random_problem(6, 5, 12, seed=31, npml=3, loss_range=(0.3, 0.8))
    coef = oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, {}, pb.omega, pb.tau, pb.h)
    g = inputs.rng(32)
    x = g.standard_normal((12,) + pb.shape) + 1j * g.standard_normal((12,) + pb.shape)
    x /= np.linalg.norm(x)
    lam_ref = np.exp(-1j * pb.omega * pb.tau)
    ratio = {}
    for n in range(1, 3001):
        y = oracle.phi(coef, x)
        r = np.linalg.norm(y)
        if n in (1000, 3000):
            ratio[n] = r
            lam = np.vdot(x, y) / np.vdot(x, x)
        x = y / r
    assert abs(lam - lam_ref) < 1e-3
    assert 1.0 <= ratio[3000] < 1.0 + 1e-3
    # an eigenvalue of modulus > 1 would hold the ratio above 1 at a constant
    assert ratio[3000] - 1.0 < 0.6 * (ratio[1000] - 1.0)


def test_split_difference_of_symmetric_pairs_is_invisible(oracle_lib):
    """The reading behind the pair-sum form of the complex64 inner sweeps:
    where both parts of a split pair have identical coefficients (the z pairs
    everywhere, the x and y pairs on planes without a PML term), moving a
    value from one part to the other changes no physical field after an
    iteration -- one iteration maps the pair's sum on its own and the other
    field reads only sums.  On a PML plane the same move of an x pair is
    visible (control)."""
    pb = inputs.random_problem(7, 6, 14, seed=41, npml=3)
    coef = oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h)
    g = inputs.rng(42)
    shape = (12,) + pb.shape
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    ref = P(oracle.phi(coef, x))
    nz = pb.shape[0]
    hsym = np.asarray(pb.sig_h) == 0.0
    esym = np.asarray(pb.sig_e) == 0.0
    assert hsym.any() and esym.any() and not hsym.all() and not esym.all()
    y = x.copy()
    for c in range(6):
        a, b = 2 * c, 2 * c + 1
        sym = np.ones(nz, bool) if c in (2, 5) else (hsym if c < 3 else esym)
        d = (g.standard_normal(pb.shape) + 1j * g.standard_normal(pb.shape)) * sym[:, None, None]
        y[a] += d
        y[b] -= d
    out = P(oracle.phi(coef, y))
    assert np.linalg.norm(out - ref) <= 1e-13 * np.linalg.norm(ref)
    # control: the same move of the H_x pair on a PML plane is seen
    k = int(np.nonzero(~hsym)[0][0])
    z = x.copy()
    z[0, k] += 1.0
    z[1, k] -= 1.0
    assert np.linalg.norm(P(oracle.phi(coef, z)) - ref) > 1e-6 * np.linalg.norm(ref)
