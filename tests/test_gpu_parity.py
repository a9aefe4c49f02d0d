"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Tolerances: coefficient arrays elementwise 2e-15 relative (both sides round
the same closed forms in different operation orders); iterates 1e-12 in the
relative 2-norm over all 12 split arrays and, part by part, every value
within 1e-12 of the largest field magnitude (so an error confined to one
part or a few cells cannot hide in the global norm); the naive, fused and
blocked sweeps bit-identical to each other (same per-element operation
sequence)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1510_05218_amd import inputs  # noqa: E402
from paper_1510_05218_amd import thiim  # noqa: E402


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle_run(pb, n):
    coef = oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h)
    x = oracle.iterate(coef, oracle.zero_fields(pb.shape), n, pb.bcx, pb.bcy)
    return coef, x


def _gpu_run(pb, n, **kw):
    s = thiim.Solver(pb, **kw)
    s.iterate(n)
    x = s.fields()
    torch.cuda.synchronize()
    return s, x


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _assert_parity(xg, xo, tol=1e-12, what=None):
    """GPU iterate against the oracle's: relative 2-norm over all parts, and
    the largest absolute error of each of the 12 parts against the largest
    magnitude of the whole field."""
    xg = np.asarray(xg.cpu().numpy() if hasattr(xg, "cpu") else xg)
    xo = np.asarray(xo)
    assert _rel(xg, xo) < tol, what
    scale = float(np.max(np.abs(xo)))
    for q in range(12):
        err = float(np.max(np.abs(xg[q] - xo[q])))
        assert err <= tol * scale, (what, q, err, scale)


def _with_back_cells(pb, seed):
    g = inputs.rng(seed)
    mask = g.random(pb.eps.shape) < 0.1
    pb.eps[mask] = -g.uniform(1, 4, mask.sum()) + 1j * g.uniform(0.1, 1, mask.sum())
    return pb


@pytest.mark.parametrize("storage", ["full", "compact"])
def test_coefficients_match_oracle(storage):
    _require_gpu()
    pb = _with_back_cells(inputs.random_problem(17, 13, 11, seed=3), 5)
    s = thiim.Solver(pb, kernel="naive", storage=storage)
    cg = s.coeffs().cpu().numpy()
    co = oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau)
    for q in range(28):
        err = np.abs(cg[q] - co[q])
        assert np.all(err <= 2e-15 * np.abs(co[q]) + 1e-300), q


@pytest.mark.parametrize("kernel,storage", [("naive", "full"), ("fused", "full"),
                                            ("blocked", "full"), ("fused", "compact"),
                                            ("blocked", "compact")])
def test_c1_layered_textured_200_iterations(kernel, storage):
    """24 x 24 interior cells + 2 x 6 PML planes, three textured layers,
    normal-incidence x-polarised source, 200 iterations."""
    _require_gpu()
    pb = inputs.solar_cell(24, 24, 36, seed=1, npml=6)
    _, xo = _oracle_run(pb, 200)
    _, xg = _gpu_run(pb, 200, kernel=kernel, storage=storage)
    _assert_parity(xg, xo)


def test_128cubed_random_media_20_iterations():
    """128^3 cells of per-cell random media with back-iteration cells and
    random sources on all four source arrays (every cell and part active from
    the first iteration), 20 iterations: every sweep form against the oracle
    (1e-12) and bit-identical to each other."""
    _require_gpu()
    pb = _with_back_cells(inputs.random_problem(128, 128, 128, seed=29, npml=6), 30)
    _, xo = _oracle_run(pb, 20)
    _, xn = _gpu_run(pb, 20, kernel="naive", storage="full")
    _assert_parity(xn, xo)
    for kernel, storage in (("fused", "compact"), ("blocked", "compact"), ("blocked", "full")):
        s, x = _gpu_run(pb, 20, kernel=kernel, storage=storage)
        s.close()
        assert torch.equal(x, xn), (kernel, storage)


@pytest.mark.parametrize("bcx,bcy", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_random_ragged_problem(bcx, bcy):
    """Per-cell random materials with back-iteration cells, random sources on
    all four source arrays, sizes that leave ragged tiles in x, y and z."""
    _require_gpu()
    pb = _with_back_cells(inputs.random_problem(37, 29, 23, seed=11, bcx=bcx, bcy=bcy), 12)
    _, xo = _oracle_run(pb, 25)
    _, xn = _gpu_run(pb, 25, kernel="naive")
    _assert_parity(xn, xo)
    for tile in [(64, 8), (32, 8), (64, 4), (16, 16)]:
        for zc in (0, 5, 64):
            _, xf = _gpu_run(pb, 25, kernel="fused", tile=tile, z_chunk=zc)
            assert torch.equal(xf, xn), (tile, zc)
    # temporally blocked: 12 two-iteration passes + 1 fused remainder
    for storage in ("full", "compact"):
        for tile in [(64, 8), (64, 6), (32, 16)]:
            for zc in (0, 3, 5, 64):
                _, xb = _gpu_run(pb, 25, kernel="blocked", tile=tile, z_chunk=zc,
                                 storage=storage)
                assert torch.equal(xb, xn), ("blocked", storage, tile, zc)
    # compact storage: the same iterates from derived coefficients
    _, xnc = _gpu_run(pb, 25, kernel="naive", storage="compact")
    assert torch.equal(xnc, xn)
    for tile in [(64, 8), (32, 8), (64, 4), (16, 16)]:
        _, xf = _gpu_run(pb, 25, kernel="fused", tile=tile, storage="compact")
        assert torch.equal(xf, xn), ("fused compact", tile)


def test_tiny_grids_wrap_many_times():
    """nx, ny far below the tile width: periodic wrap inside one tile."""
    _require_gpu()
    for shape in [(6, 2, 2), (9, 3, 5), (12, 7, 2)]:
        nz, ny, nx = shape
        pb = inputs.random_problem(nx, ny, nz, seed=sum(shape), npml=1)
        _, xo = _oracle_run(pb, 15)
        _, xn = _gpu_run(pb, 15, kernel="naive")
        _, xf = _gpu_run(pb, 15, kernel="fused")
        _, xb = _gpu_run(pb, 15, kernel="blocked")
        _, xbc = _gpu_run(pb, 15, kernel="blocked", storage="compact")
        _assert_parity(xn, xo)
        assert torch.equal(xf, xn)
        assert torch.equal(xb, xn)
        assert torch.equal(xbc, xn)


def test_smallest_grid_and_zero_iterations():
    """Degenerate cases: the smallest legal grid (2 x 2 x 2: every cell is a
    boundary cell on all three axes; periodic and Dirichlet x/y, back-
    iteration cells included) on every kernel and storage, and zero
    iterations, which leave the fields bit for bit as they were (zero at
    create, the current iterate later)."""
    _require_gpu()
    for bcx, bcy in [(0, 0), (1, 1)]:
        pb = inputs.random_problem(2, 2, 2, seed=5, npml=0, bcx=bcx, bcy=bcy)
        pb.eps[0, 1, 0] = -2.5 + 0.3j
        _, xo = _oracle_run(pb, 30)
        assert np.linalg.norm(xo) > 0
        for kernel in ("naive", "fused", "blocked"):
            for storage in ("full", "compact"):
                s, xg = _gpu_run(pb, 30, kernel=kernel, storage=storage)
                s.close()
                _assert_parity(xg, xo, what=(bcx, kernel, storage))
    pb = inputs.solar_cell(24, 24, 36, seed=1, npml=6)
    s = thiim.Solver(pb, kernel="blocked", storage="compact")
    s.iterate(0)
    assert not torch.any(s.fields() != 0)
    s.iterate(7)
    x7 = s.fields().clone()
    s.iterate(0)
    assert torch.equal(s.fields(), x7)
    assert s.iterations == 7
    s.close()


def test_zero_source_stays_zero():
    _require_gpu()
    pb = inputs.solar_cell(24, 20, 30, seed=2, npml=4)
    pb.sources = {}
    for kernel in ("naive", "fused", "blocked"):
        _, x = _gpu_run(pb, 30, kernel=kernel)
        assert not torch.any(x != 0)


def test_residual_matches_oracle():
    _require_gpu()
    pb = inputs.solar_cell(24, 24, 36, seed=4, npml=6)
    coef, xo = _oracle_run(pb, 80)
    s, _ = _gpu_run(pb, 80, kernel="fused")
    r_gpu = s.residual()
    r_or = oracle.residual(coef, xo)
    assert abs(r_gpu - r_or) <= 1e-10 * r_or
    # the residual call does not advance the state
    assert s.iterations == 80


def test_checkpoint_resume_bitwise():
    _require_gpu()
    pb = inputs.solar_cell(32, 24, 30, seed=6, npml=5)
    s_full, x_full = _gpu_run(pb, 40, kernel="fused")
    s1, x1 = _gpu_run(pb, 17, kernel="fused")
    s2 = thiim.Solver(pb, kernel="naive")
    s2.set_fields(x1)
    s2.iterate(23)
    assert torch.equal(s2.fields(), x_full)


def test_solve_reaches_tolerance():
    _require_gpu()
    pb = inputs.solar_cell(16, 16, 30, seed=8, npml=6, loss_range=(0.3, 0.6),
                           eps_range=(1.0, 3.0), texture_amp=2)
    pb.omega = 0.8
    s = thiim.Solver(pb, kernel="fused")
    rc, it, r = s.solve(1e-6, 20000, 100)
    assert rc == thiim.THIIM_OK and r <= 1e-6
    coef = oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau)
    assert abs(oracle.residual(coef, s.fields().cpu().numpy()) - r) <= 1e-8 * r + 1e-15


def test_full_size_flat_stack_512():
    """512^3 (the production-size workload) with flat layers: every column
    equals the oracle's 2 x 2 x 512 run (x/y invariance), 100 iterations, in
    the launch configuration of the benchmark."""
    _require_gpu()
    if torch.cuda.get_device_properties(0).total_memory < 150e9:
        pytest.skip("needs the 288 GB of an MI355X")
    n = 512
    pb = inputs.solar_cell(n, n, n, seed=3, npml=6, flat=True)
    s = thiim.Solver(pb, kernel="blocked", storage="compact")
    s.iterate(100)
    x = s.fields()
    small = inputs.solar_cell(2, 2, n, seed=3, npml=6, flat=True)
    _, xo = _oracle_run(small, 100)
    col = torch.from_numpy(xo[:, :, 0, 0]).to(x.device)
    for q in range(12):
        xq = x[q]
        ref = col[q][:, None, None]
        err = torch.linalg.vector_norm(xq - ref)
        assert float(err) <= 1e-12 * float(torch.linalg.vector_norm(x)), q
        # every column identical
        assert torch.equal(xq, xq[:, :1, :1].expand_as(xq)), q
    s.close()
    del x
    torch.cuda.empty_cache()


def _window(a, j0, i0, w):
    """[..., ny, nx] array -> the w x w window starting at (j0, i0), wrapped."""
    ny, nx = a.shape[-2:]
    jj = (j0 + np.arange(w)) % ny
    ii = (i0 + np.arange(w)) % nx
    return np.ascontiguousarray(np.take(np.take(a, jj, axis=-2), ii, axis=-1))


def test_full_size_textured_512_sampled_columns():
    """The 512^3 benchmark workload itself (textured interface, 200 spheres,
    graded PML, periodic x/y), 20 iterations in the benchmark's launch
    configuration, checked on sampled columns: after n iterations a cell
    depends only on cells at most n (+1) steps away in x and y, so the oracle
    run on a full-depth window of width W + 2m (m = n + 2 > light cone)
    reproduces the W x W centre columns exactly.  Windows: one on a sphere,
    one across the periodic corner (wrap), one on the textured interface."""
    _require_gpu()
    if torch.cuda.get_device_properties(0).total_memory < 150e9:
        pytest.skip("needs the 288 GB of an MI355X")
    n, it, w = 512, 20, 8
    m = it + 2
    pb = inputs.solar_cell(n, n, n, seed=3, npml=6, n_spheres=200)
    sph = np.argwhere(pb.eps == 2.1 + 0j)
    assert len(sph) > 0
    k_s, j_s, i_s = sph[len(sph) // 2]
    s = thiim.Solver(pb, kernel="blocked", storage="compact")
    s.iterate(it)
    x = s.fields()
    corners = [(int(j_s) - w // 2, int(i_s) - w // 2), (n - w // 2, n - w // 2), (200, 300)]
    for j0, i0 in corners:
        print(f"[512 sampled] window at ({j0}, {i0})", flush=True)
        wj, wi = j0 - m, i0 - m
        big = w + 2 * m
        sub = inputs.Problem(**{**pb.__dict__})
        sub.eps = _window(pb.eps, wj, wi, big)
        sub.sources = {k: _window(v, wj, wi, big) for k, v in pb.sources.items()}
        sub.bcx = sub.bcy = 1  # the window edge is outside the light cone of the centre
        _, xo = _oracle_run(sub, it)
        ref = xo[:, :, m:m + w, m:m + w]
        jj = torch.tensor((j0 + np.arange(w)) % n, device=x.device)
        ii = torch.tensor((i0 + np.arange(w)) % n, device=x.device)
        got = x.index_select(2, jj).index_select(3, ii).cpu().numpy()
        err = np.linalg.norm(got - ref)
        assert err <= 1e-12 * np.linalg.norm(ref), (j0, i0, err)
    s.close()
    del x
    torch.cuda.empty_cache()


def test_full_size_textured_512_every_cell(capsys):
    """The 512^3 benchmark workload (textured, 200 spheres, PML, periodic
    x/y), 200 iterations in the benchmark's launch configuration -- enough for
    the field to pass the textured interface around plane 170, so that all
    twelve parts are non-zero -- against the oracle's memory-light mode on
    the host (bit-identical to its stored mode): every value of the 12 split
    arrays, each part's error within 1e-12 of the norm of all fields (parts
    born at the wave front are ~1e-110 and carry cancellation noise relative
    to themselves), and the whole within 1e-12 relative.

    The source sits on plane k_s and one iteration moves influence by at most
    one plane, so after n iterations every plane above k_s + n + 1 is still
    exactly zero; the oracle runs on planes [0, k_s + n + 32) only (the planes
    it drops would only ever feed it zeros) and the GPU's planes above must be
    exactly zero.  The oracle's own top 16 planes staying zero checks that
    the cut was never reached."""
    _require_gpu()
    if torch.cuda.get_device_properties(0).total_memory < 150e9:
        pytest.skip("needs the 288 GB of an MI355X")
    n, it, chunk = 512, 200, 20
    pb = inputs.solar_cell(n, n, n, seed=3, npml=6, n_spheres=200)
    s = thiim.Solver(pb, kernel="blocked", storage="compact")
    s.iterate(it)
    x = s.fields().cpu().numpy()
    s.close()
    torch.cuda.empty_cache()
    nzc = pb.meta["k_s"] + it + 32
    assert not np.any(x[:, nzc:])
    src = {k: v[:nzc] for k, v in pb.sources.items()}
    xo = oracle.zero_fields((nzc, n, n))
    for done in range(0, it, chunk):
        oracle.iterate_light(pb.eps[:nzc], pb.sig_e[:nzc], pb.sig_h[:nzc], src, pb.omega,
                             pb.tau, pb.h, xo, chunk)
        with capsys.disabled():
            print(f"[512 every cell] oracle at {done + chunk} iterations", flush=True)
    assert not np.any(xo[:, nzc - 16:])
    x = x[:, :nzc]
    total = np.linalg.norm(xo)
    for q in range(12):
        err = np.linalg.norm(x[q] - xo[q])
        ref = np.linalg.norm(xo[q])
        print(f"[512 every cell] part {q}: norm {ref:.3e}, error {err:.2e}", flush=True)
        assert ref > 0 and err <= 1e-12 * total
    assert np.linalg.norm(x - xo) <= 1e-12 * np.linalg.norm(xo)


def test_invalid_material_rejected_at_create():
    """eps' = 0 (neither Eq. 3 nor Eq. 5 applies) and non-finite eps are
    found by the coefficient kernel and reported as THIIM_EINVAL by
    thiim_create; a valid problem on the same device still works after."""
    _require_gpu()
    for bad in (0.0 + 0.3j, complex(float("nan"), 0.0), complex(2.0, float("inf"))):
        for storage in ("full", "compact"):
            pb = inputs.random_problem(9, 7, 6, seed=4)
            pb.eps[3, 2, 5] = bad
            with pytest.raises(thiim.ThiimError) as e:
                thiim.Solver(pb, storage=storage)
            assert e.value.status == thiim.THIIM_EINVAL, (bad, storage)
            assert "eps" in thiim.last_error()
    pb = inputs.random_problem(9, 7, 6, seed=4)
    s, x = _gpu_run(pb, 5, kernel="blocked", storage="compact")
    s.close()
    _, xo = _oracle_run(pb, 5)
    _assert_parity(x, xo)
