"""The allocation-free batch (thiim_batch_create_static): item tables and
queue counters in the library's static device scratch instead of a caller
workspace.  Checked against the workspace batch (thiim_batch_create) bit for
bit on two calls in a row, the second with fewer and smaller problems, and
the scratch's guards (size limit, one static batch per device)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1510_05218_amd import inputs  # noqa: E402
from paper_1510_05218_amd import thiim  # noqa: E402


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _first_set():
    return [
        (inputs.random_problem(37, 19, 14, seed=81), dict(kernel="blocked", tile=(32, 16))),
        (inputs.solar_cell(24, 24, 36, seed=1, npml=6), dict(kernel="blocked", tile=(64, 8),
                                                             z_chunk=7)),
        (inputs.random_problem(17, 30, 21, seed=82, bcx=1, bcy=1), dict(kernel="fused",
                                                                        tile=(16, 16))),
        (inputs.random_problem(70, 9, 12, seed=83, bcy=1), dict(kernel="blocked", tile=(64, 6))),
        (inputs.random_problem(20, 20, 16, seed=84), dict(kernel="fused", tile=(32, 8))),
    ]


def _second_set():
    return [
        (inputs.random_problem(9, 7, 6, seed=85), dict(kernel="blocked", tile=(32, 16))),
        (inputs.random_problem(12, 5, 8, seed=86, bcx=1), dict(kernel="fused", tile=(64, 8))),
    ]


def _run(probs, n, static):
    stream = torch.cuda.Stream()
    solvers = [thiim.Solver(pb, storage="compact", stream=stream, **kw) for pb, kw in probs]
    ws = None
    if static:
        b = thiim.thiim_batch_create_static([s.ctx for s in solvers])
    else:
        with torch.cuda.stream(stream):
            ws = torch.empty(thiim.thiim_batch_workspace_bytes(len(solvers)),
                             dtype=torch.uint8, device="cuda")
        b = thiim.thiim_batch_create([s.ctx for s in solvers], ws.data_ptr(), ws.numel())
    thiim.thiim_batch_iterate(b, n)
    res = thiim.thiim_batch_residual(b, len(solvers))
    xs = [s.fields() for s in solvers]
    stream.synchronize()
    thiim.thiim_batch_destroy(b)
    for s in solvers:
        s.close()
    return xs, res


@pytest.mark.parametrize("n", [64 + 7])
def test_static_batch_matches_workspace_batch_twice(n):
    _require_gpu()
    for name, probs, iters in (("first", _first_set(), n), ("second, smaller", _second_set(),
                                                            37)):
        print(f"[no-alloc] {name} call: {len(probs)} problems, {iters} iterations",
              flush=True)
        xw, rw = _run(probs, iters, static=False)
        xs, rs = _run(probs, iters, static=True)
        assert np.array_equal(rw, rs), name
        for a, b in zip(xw, xs):
            assert torch.equal(a, b), name


def test_static_batch_guards():
    _require_gpu()
    print("[no-alloc] guards", flush=True)
    pb = inputs.random_problem(8, 8, 8, seed=87)
    stream = torch.cuda.Stream()
    s1 = thiim.Solver(pb, storage="compact", stream=stream)
    s2 = thiim.Solver(pb, storage="compact", stream=stream)
    b1 = thiim.thiim_batch_create_static([s1.ctx])
    with pytest.raises(thiim.ThiimError) as e:
        thiim.thiim_batch_create_static([s2.ctx])  # the device's scratch is held
    assert e.value.status == thiim.THIIM_EINVAL
    thiim.thiim_batch_destroy(b1)
    b2 = thiim.thiim_batch_create_static([s2.ctx])  # released by destroy
    thiim.thiim_batch_iterate(b2, 4)
    stream.synchronize()
    thiim.thiim_batch_destroy(b2)
    s1.close()
    s2.close()


def test_static_batch_size_limit():
    """More problems than the static scratch holds: refused before any
    device work (the contexts are not even looked at)."""
    arr = (ctypes.c_void_p * 129)()
    out = ctypes.c_void_p()
    rc = thiim.lib().thiim_batch_create_static(arr, 129, ctypes.byref(out))
    assert rc == thiim.THIIM_EINVAL and not out.value
    assert "at most 128" in thiim.last_error()
