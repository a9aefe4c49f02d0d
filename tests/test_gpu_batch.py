"""GPU checks of the batched solver and the auto-tuner.

Every sweep configuration produces bit-identical iterates, so a batch (one
launch per configuration and pass over the concatenated tiles of all its
problems, replayed from a captured HIP graph) must reproduce, bit for bit,
each problem iterated on its own -- for uneven grids, mixed configurations,
both boundary types and iteration counts that are not multiples of the
graph or of the blocked pass.  One batched problem is also compared with
the oracle (1e-12), tying the batched path to it directly."""
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


def _problems():
    return [
        (inputs.random_problem(37, 19, 14, seed=51), dict(kernel="blocked", tile=(32, 16))),
        (inputs.solar_cell(24, 24, 36, seed=1, npml=6), dict(kernel="blocked", tile=(64, 8),
                                                             z_chunk=7)),
        (inputs.random_problem(17, 30, 21, seed=52, bcx=1, bcy=1), dict(kernel="fused",
                                                                        tile=(16, 16))),
        (inputs.random_problem(70, 9, 12, seed=53, bcy=1), dict(kernel="blocked", tile=(64, 6))),
        (inputs.random_problem(20, 20, 16, seed=54), dict(kernel="fused", tile=(32, 8),
                                                          z_chunk=5)),
        (inputs.random_problem(33, 12, 10, seed=55), dict(kernel="blocked", tile=(32, 16))),
    ]


def _solo(pb, kw, n):
    s = thiim.Solver(pb, storage="compact", **kw)
    s.iterate(n)
    x = s.fields()
    torch.cuda.synchronize()
    s.close()
    return x


@pytest.mark.parametrize("n,default_stream", [(64 * 2 + 5, False), (64 + 2, False),
                                              (37, True)])
def test_batch_equals_individual(n, default_stream):
    _require_gpu()
    print(f"[batch] n={n} default_stream={default_stream}", flush=True)
    probs = _problems()
    stream = torch.cuda.default_stream() if default_stream else torch.cuda.Stream()
    solvers = [thiim.Solver(pb, storage="compact", stream=stream, **kw) for pb, kw in probs]
    ws = torch.empty(thiim.thiim_batch_workspace_bytes(len(solvers)), dtype=torch.uint8,
                     device="cuda")
    b = thiim.thiim_batch_create([s.ctx for s in solvers], ws.data_ptr(), ws.numel())
    thiim.thiim_batch_iterate(b, n)
    stream.synchronize()
    for s, (pb, kw) in zip(solvers, probs):
        assert s.iterations == n
        assert torch.equal(s.fields(), _solo(pb, kw, n)), kw
    thiim.thiim_batch_destroy(b)
    for s in solvers:
        s.close()


def test_batch_matches_oracle():
    _require_gpu()
    pb = inputs.random_problem(37, 19, 14, seed=61)
    others = [inputs.random_problem(20, 20, 16, seed=62)]
    bt = thiim.Batch([pb] + others)
    bt.iterate(70)
    bt.synchronize()
    x = bt.solvers[0].fields().cpu().numpy()
    coef = oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau, pb.h)
    xo = oracle.iterate(coef, oracle.zero_fields(pb.shape), 70)
    assert np.linalg.norm(x - xo) <= 1e-12 * np.linalg.norm(xo)
    bt.close()


def test_batch_solve_matches_individual_solves():
    _require_gpu()
    probs = [inputs.random_problem(12, 10, 16, seed=71, all_sources=False),
             inputs.random_problem(20, 14, 12, seed=72, all_sources=False, omega=0.5),
             inputs.random_problem(9, 9, 20, seed=73, all_sources=False, bcx=1)]
    tol, every = 1e-9, 128
    bt = thiim.Batch(probs)
    rc, its, res = bt.solve(tol, 200000, every)
    assert rc == thiim.THIIM_OK, (its, res)
    assert np.all(res <= tol)
    for i, pb in enumerate(probs):
        s = thiim.Solver(pb, storage="compact")
        rc1, it1, r1 = s.solve(tol, 200000, every)
        assert rc1 == thiim.THIIM_OK
        assert it1 == its[i] and r1 == res[i]
        assert torch.equal(s.fields(), bt.solvers[i].fields())
        s.close()
    # problems converged at different iteration counts
    assert len(set(its.tolist())) > 1
    bt.close()


def test_autotune_keeps_iterates_and_reports_choice():
    _require_gpu()
    pb = inputs.solar_cell(48, 40, 64, seed=2, npml=6)
    s = thiim.Solver(pb, storage="compact")
    s.iterate(3)
    t = s.autotune(trial_iters=4)
    assert t["kernel"] in (thiim.KERNELS["fused"], thiim.KERNELS["blocked"])
    assert 1 <= t["timed"] <= 8 and t["candidates"] >= t["timed"]
    assert t["ms_per_iteration"] > 0 and t["z_chunk"] >= 4
    assert s.iterations == 3  # tuning did not advance the state
    s.iterate(17)
    ref = _solo(pb, {}, 20)
    assert torch.equal(s.fields(), ref)
    s.close()


def test_batch_rejects_full_storage_and_duplicates():
    _require_gpu()
    pb = inputs.random_problem(8, 8, 8, seed=5)
    s_full = thiim.Solver(pb, storage="full")
    s_c = thiim.Solver(pb, storage="compact")
    ws = torch.empty(thiim.thiim_batch_workspace_bytes(2), dtype=torch.uint8, device="cuda")
    for ctxs in ([s_full.ctx, s_c.ctx], [s_c.ctx, s_c.ctx]):
        with pytest.raises(thiim.ThiimError) as e:
            thiim.thiim_batch_create(ctxs, ws.data_ptr(), ws.numel())
        assert e.value.status == thiim.THIIM_EINVAL
    s_full.close()
    s_c.close()


@pytest.mark.parametrize("t_block", [0, 3])
def test_batch_mixed_solve_matches_individual_mixed_solves(t_block):
    """With a fixed inner count m above every averaging window, each batched
    problem runs exactly the defect-correction steps of its own mixed solve:
    same sweep counts, same residuals, bit-identical fields (two sweeps per
    inner pass on 32 x 32 regions, and three on 32 x 16)."""
    _require_gpu()
    print(f"[batch mixed] t_block={t_block}", flush=True)
    probs = [inputs.random_problem(12, 10, 16, seed=81, all_sources=False),
             inputs.random_problem(20, 14, 12, seed=82, all_sources=False, omega=0.5),
             inputs.random_problem(9, 9, 20, seed=83, all_sources=False, bcx=1),
             inputs.random_problem(40, 33, 10, seed=84, all_sources=False, omega=0.2)]
    tol, m = 1e-9, 300
    bt = thiim.Batch(probs, precision="mixed", t_block=t_block)
    rc, its, res = bt.solve(tol, 400000, m)
    assert rc == thiim.THIIM_OK, (its, res)
    for i, pb in enumerate(probs):
        s = thiim.Solver(pb, storage="compact", precision="mixed", t_block=t_block)
        rc1, it1, r1 = s.solve(tol, 400000, m)
        assert rc1 == thiim.THIIM_OK
        assert it1 == its[i] and r1 == res[i], (i, it1, its[i], r1, res[i])
        assert torch.equal(s.fields(), bt.solvers[i].fields())
        s.close()
    bt.close()


def test_batch_mixed_adaptive_reaches_tolerance():
    _require_gpu()
    probs = [inputs.solar_cell(24, 24, 36, seed=s, npml=6, loss_range=(0.1, 0.5),
                               wavelength_nm=wl)
             for s, wl in ((10, 400.0), (11, 700.0), (12, 1000.0))]
    bt = thiim.Batch(probs, precision="mixed")
    rc, its, res = bt.solve(1e-8, 400000, 0)
    assert rc == thiim.THIIM_OK and np.all(res <= 1e-8), (its, res)
    # the FP64 residual recomputed from scratch agrees
    assert np.all(bt.residual() <= 1e-8)
    bt.close()


def test_batch_autotune_keeps_iterates():
    _require_gpu()
    probs = [inputs.random_problem(40, 36, 20, seed=91), inputs.random_problem(70, 20, 30, seed=92)]
    bt = thiim.Batch(probs, autotune=True, trial_iters=4)
    t = bt.tuning
    assert t["kernel"] in (thiim.KERNELS["fused"], thiim.KERNELS["blocked"]) and t["timed"] == 14
    # both ways were timed and the faster applied
    assert t["one_for_all_ms"] > 0 and t["per_grid_ms"] > 0
    assert t["ms_per_iteration"] == min(t["one_for_all_ms"], t["per_grid_ms"])
    assert t["per_grid"] == int(t["per_grid_ms"] < t["one_for_all_ms"])
    bt.iterate(70)
    bt.synchronize()
    for s, pb in zip(bt.solvers, probs):
        assert s.iterations == 70
        assert torch.equal(s.fields(), _solo(pb, {}, 70))
    bt.close()
