"""GPU checks of the solver's guards: divergence detection and the
auto-tuner on the thinnest legal grids.

A medium with gain (eps'' < 0, so sigma = w eps'' < 0) makes |t_E| > 1 and the
THIIM iteration grow without bound; every solver form must stop with
THIIM_EDIVERGED once the residual exceeds 1e6 times the smallest one it
reached, long before any value overflows (every kernel still runs to its
normal end: the values are merely large).  The auto-tuner must accept
grids of 2 and 3 planes (one z chunk) and keep the iterates bit-identical."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1510_05218_amd import inputs  # noqa: E402
from paper_1510_05218_amd import thiim  # noqa: E402


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gain_problem():
    pb = inputs.random_problem(12, 10, 16, seed=71, npml=2)
    pb.eps = np.abs(pb.eps.real) + 1.0 - 1.5j  # eps' in [1, ...], eps'' = -1.5: gain
    return pb


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gain_medium_is_reported_as_diverging(precision):
    _require_gpu()
    print(f"[guards] gain medium, {precision}", flush=True)
    kw = {"precision": "mixed", "t_block": 3} if precision == "mixed" else {}
    s = thiim.Solver(_gain_problem(), storage="compact", **kw)
    with pytest.raises(thiim.ThiimError) as ei:
        s.solve(1e-8, 200000, 20 if precision == "fp64" else 0)
    assert ei.value.status == thiim.THIIM_EDIVERGED
    s.close()


def test_gain_medium_batch_is_reported_as_diverging():
    _require_gpu()
    print("[guards] gain medium, batched FP64 solve", flush=True)
    b = thiim.Batch([_gain_problem(), inputs.random_problem(8, 8, 12, seed=72)])
    with pytest.raises(thiim.ThiimError) as ei:
        b.solve(1e-8, 20000, 20)
    assert ei.value.status == thiim.THIIM_EDIVERGED
    b.close()


@pytest.mark.parametrize("nz", [2, 3])
def test_autotune_on_thin_grids(nz):
    """4 x 4 x nz: the only z chunk is the whole grid."""
    _require_gpu()
    print(f"[guards] autotune 4x4x{nz}", flush=True)
    pb = inputs.random_problem(4, 4, nz, seed=73 + nz, npml=0)
    ref = thiim.Solver(pb, kernel="naive", storage="compact")
    ref.iterate(9)
    xr = ref.fields()
    s = thiim.Solver(pb, storage="compact")
    tun = s.autotune(3)
    assert tun["z_chunk"] == nz and tun["timed"] >= 1
    s.iterate(9)
    assert torch.equal(s.fields(), xr)
    ref.close()
    s.close()


def test_tuner_cache_applies_without_timing(tmp_path):
    """The first autotune on a grid times and stores its choice; a second
    context of the same grid takes it from the cache (no timing) and
    iterates bit-identically; invalid configurations are rejected."""
    _require_gpu()
    print("[guards] tuner cache", flush=True)
    pb = inputs.random_problem(40, 30, 24, seed=79)
    cache = thiim.TunerCache(str(tmp_path / "tune.json"))
    s1 = thiim.Solver(pb, storage="compact")
    t1 = s1.autotune(3, cache=cache)
    assert not t1.get("cached") and t1["timed"] >= 1
    s2 = thiim.Solver(pb, storage="compact")
    t2 = s2.autotune(3, cache=thiim.TunerCache(str(tmp_path / "tune.json")))
    assert t2["cached"] and (t2["kernel"], t2["tile_x"], t2["tile_y"], t2["z_chunk"]) == \
        (t1["kernel"], t1["tile_x"], t1["tile_y"], t1["z_chunk"])
    ref = thiim.Solver(pb, kernel="naive", storage="compact")
    for s in (s1, s2, ref):
        s.iterate(11)
    assert torch.equal(s2.fields(), ref.fields()) and torch.equal(s1.fields(), ref.fields())
    for bad in ({"kernel": 1, "tile_x": 64, "tile_y": 8, "z_chunk": 4},
                {"kernel": 3, "tile_x": 48, "tile_y": 8, "z_chunk": 4},
                {"kernel": 2, "tile_x": 64, "tile_y": 8, "z_chunk": 0}):
        with pytest.raises(thiim.ThiimError) as e:
            thiim.thiim_apply_tuning(s2.ctx, bad)
        assert e.value.status == thiim.THIIM_EINVAL
    for s in (s1, s2, ref):
        s.close()
