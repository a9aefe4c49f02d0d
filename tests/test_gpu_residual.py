"""GPU checks of the residual that the fused pass forms while it iterates.

thiim_create computes ||P Phi(0)|| and thiim_residual computes
||P(Phi(x) - x)|| / ||P Phi(0)|| (P the sum of each split pair, the physical
fields) inside one fused pass, from the old and new values of every cell,
with one partial sum per workgroup.  Here both are recomputed from fields
that the library returns: Phi(0) and Phi(x) by one plain iteration, the norms
in torch.  The grids are chosen so that one launch holds more workgroups
than the partial-sum buffer (the pass then coarsens its z chunking) and so
that it does not."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1510_05218_amd import inputs  # noqa: E402
from paper_1510_05218_amd import thiim  # noqa: E402


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pnorm(f):
    return torch.linalg.vector_norm(f[0::2] + f[1::2]).item()


# (grid, fused tile, z chunk): 16 x 16 tiles in 4-plane chunks on 128 x 128 x 80
# make 64 x 20 = 1280 workgroups, more than the 1024 partial sums that grid
# gets, so the residual pass runs 5-plane chunks
CASES = [((37, 29, 23), (64, 8), 0, "periodic"),
         ((80, 128, 128), (16, 16), 4, "periodic"),
         ((24, 20, 18), (32, 8), 5, "dirichlet")]


@pytest.mark.parametrize("storage", ["compact", "full"])
@pytest.mark.parametrize("shape,tile,zc,bc", CASES)
def test_residual_matches_fields(shape, tile, zc, bc, storage):
    _require_gpu()
    print(f"[residual] {shape} tile {tile} z chunk {zc} {bc} {storage}", flush=True)
    nz, ny, nx = shape
    d = 1 if bc == "dirichlet" else 0
    pb = inputs.random_problem(nx, ny, nz, seed=41, npml=2, bcx=d, bcy=d)
    kw = dict(kernel="fused", tile=tile, z_chunk=zc, storage=storage)
    # Phi(0): one iteration from the state thiim_create leaves
    s0 = thiim.Solver(pb, **kw)
    s0.iterate(1)
    s0.stream.synchronize()
    phi0 = _pnorm(s0.fields())
    s0.close()
    assert phi0 > 0
    s = thiim.Solver(pb, **kw)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    x = torch.complex(torch.randn((12, nz, ny, nx), dtype=torch.float64, device="cuda",
                                  generator=g),
                      torch.randn((12, nz, ny, nx), dtype=torch.float64, device="cuda",
                                  generator=g))
    s.set_fields(x)
    rel = s.residual()
    assert torch.equal(s.fields(), x)  # the residual does not advance x
    s.iterate(1)
    s.stream.synchronize()
    ref = _pnorm(s.fields() - x) / phi0
    s.close()
    assert abs(rel - ref) <= 1e-12 * ref, (rel, ref)


@pytest.mark.parametrize("storage", ["compact", "full"])
@pytest.mark.parametrize("bc", [0, 1])
def test_phi0_of_a_plane_source(bc, storage):
    """thiim_create forms ||P Phi(0)|| on the planes that a source can reach
    in one iteration (here the plane source and the plane below it) as a grid
    of its own: it must equal the norm over the whole Phi(0)."""
    _require_gpu()
    print(f"[residual] plane source, bc {bc}, {storage}", flush=True)
    pb = inputs.solar_cell(40, 36, 48, seed=5, npml=6)
    pb.bcx = pb.bcy = bc
    srcs = [v for v in pb.sources.values()]
    planes = sorted({int(k) for v in srcs for k in np.nonzero(np.abs(v).sum(axis=(1, 2)))[0]})
    assert 0 < len(planes) < 4  # a plane source, far from the walls
    s = thiim.Solver(pb, kernel="fused", storage=storage)
    x = torch.zeros((12, 48, 36, 40), dtype=torch.complex128, device="cuda")
    s.set_fields(x)
    s.iterate(1)
    s.stream.synchronize()
    phi = s.fields().clone()
    phi0 = _pnorm(phi)
    nz_planes = sorted({int(k) for k in torch.nonzero(
        (phi[0::2] + phi[1::2]).abs().sum(dim=(0, 2, 3))).flatten().tolist()})
    assert nz_planes and nz_planes[0] >= planes[0] - 1 and nz_planes[-1] <= planes[-1]
    # residual of x = Phi(0) is ||P(Phi(Phi(0)) - Phi(0))|| / ||P Phi(0)||
    s.iterate(1)
    s.stream.synchronize()
    ref = _pnorm(s.fields() - phi) / phi0
    s.set_fields(phi)
    rel = s.residual()
    s.close()
    assert abs(rel - ref) <= 1e-12 * ref, (rel, ref)


@pytest.mark.parametrize("where", ["first", "last", "first_and_last"])
def test_phi0_of_sources_at_the_z_walls(where):
    """The range of planes a source reaches in one iteration, clipped at the
    z walls: a source only on plane 0, only on the last plane, or on both
    (the range is then the whole grid)."""
    _require_gpu()
    print(f"[residual] source at the z walls: {where}", flush=True)
    nx, ny, nz = 20, 18, 14
    pb = inputs.random_problem(nx, ny, nz, seed=47, npml=2)
    planes = {"first": [0], "last": [nz - 1], "first_and_last": [0, nz - 1]}[where]
    for key in pb.sources:
        v = np.zeros_like(pb.sources[key])
        for k in planes:
            v[k] = pb.sources[key][k]
        pb.sources[key] = v
    s = thiim.Solver(pb, kernel="fused", storage="compact")
    s.iterate(1)
    s.stream.synchronize()
    phi = s.fields().clone()
    phi0 = _pnorm(phi)
    assert phi0 > 0
    s.iterate(1)
    s.stream.synchronize()
    ref = _pnorm(s.fields() - phi) / phi0
    s.set_fields(phi)
    rel = s.residual()
    s.close()
    assert abs(rel - ref) <= 1e-12 * ref, (rel, ref)


def test_residual_after_iterations_matches_blocked_and_naive():
    """The same residual from contexts whose iterations run the blocked and
    the naive sweeps: their iterates are bit-identical and the residual pass
    is the fused one in every case (its z chunking, and so the order of the
    partial sums, may differ: 1e-13)."""
    _require_gpu()
    print("[residual] blocked / naive / fused contexts agree", flush=True)
    pb = inputs.random_problem(40, 36, 30, seed=43, npml=3)
    vals = []
    for kern in ("naive", "fused", "blocked"):
        s = thiim.Solver(pb, kernel=kern, storage="compact")
        s.iterate(12)
        vals.append(s.residual())
        s.close()
    assert max(vals) - min(vals) <= 1e-13 * max(vals), vals
    assert np.isfinite(vals[0]) and vals[0] > 0
