"""Host-side checks of the C-ABI library (no GPU, no compute calls): it loads,
exports every symbol the header declares, sizes workspaces and rejects bad
arguments before touching the device."""
import os
import re

import pytest

from paper_1510_05218_amd import thiim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "thiim.h")).read()
    return sorted(set(re.findall(r"\b(thiim_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    L = thiim.lib()
    declared = _declared_symbols()
    assert set(declared) == set(thiim.SYMBOLS)
    for name in declared:
        assert hasattr(L, name), name


def test_workspace_bytes_layout():
    g = thiim.make_grid((36, 24, 24))
    n = 24 * 24 * 36
    b = thiim.thiim_workspace_bytes(g)
    assert b >= 52 * 16 * n          # 28 coefficient + 2 x 12 field arrays
    assert b < 52 * 16 * n + 2 ** 20
    g512 = thiim.make_grid((512, 512, 512))
    b512 = thiim.thiim_workspace_bytes(g512)
    assert abs(b512 - 52 * 16 * 512 ** 3) < 2 ** 20  # 111.7 GB
    c512 = thiim.thiim_workspace_bytes(thiim.make_grid((512, 512, 512), storage="compact"))
    assert abs(c512 - 29 * 16 * 512 ** 3) < 2 ** 20  # eps + 4 Src + 24 fields


@pytest.mark.parametrize("field,value", [("nx", 1), ("nz", 0), ("tau", 0.6), ("tau", 0.0),
                                         ("h", -1.0), ("bc_x", 2), ("kernel", 9),
                                         ("tile_x", 48), ("z_chunk", -1), ("t_block", 99),
                                         ("storage", 2), ("precision", 2), ("adjoint", 2)])
def test_invalid_grid_rejected(field, value):
    g = thiim.make_grid((10, 10, 10))
    setattr(g, field, value)
    with pytest.raises(thiim.ThiimError) as e:
        thiim.thiim_workspace_bytes(g)
    assert e.value.status == thiim.THIIM_EINVAL
    assert thiim.last_error()


def test_adjoint_workspace():
    g = thiim.make_grid((36, 24, 24), storage="compact")
    ga = thiim.make_grid((36, 24, 24), storage="compact", adjoint=True)
    n = 24 * 24 * 36
    extra = thiim.thiim_workspace_bytes(ga) - thiim.thiim_workspace_bytes(g)
    # 4 x 12 adjoint buffers + 3 source arrays, each of a padded stride
    assert 51 * 16 * n <= extra < 51 * 16 * (n + 1024)
    with pytest.raises(thiim.ThiimError) as e:
        thiim.thiim_workspace_bytes(thiim.make_grid((8, 8, 8), storage="full", adjoint=True))
    assert e.value.status == thiim.THIIM_EINVAL


def test_batch_workspace_bytes():
    b1 = thiim.thiim_batch_workspace_bytes(1)
    b100 = thiim.thiim_batch_workspace_bytes(100)
    assert b1 >= 256 and b100 > b1 and b100 % 256 == 0
    with pytest.raises(thiim.ThiimError) as e:
        thiim.thiim_batch_workspace_bytes(0)
    assert e.value.status == thiim.THIIM_EINVAL


def test_create_rejects_missing_inputs_without_device():
    g = thiim.make_grid((8, 8, 8))
    with pytest.raises(thiim.ThiimError) as e:
        thiim.thiim_create(g, thiim.Coeffs(), 0.3, 0, 0)
    assert e.value.status == thiim.THIIM_EINVAL


def test_status_strings():
    for code, name in [(0, "THIIM_OK"), (-1, "THIIM_EINVAL"), (-2, "THIIM_ENOMEM"),
                       (-3, "THIIM_EDEVICE"), (-4, "THIIM_EDIVERGED"),
                       (-5, "THIIM_ENOTCONV")]:
        assert thiim.status_str(code) == name


def test_solver_refuses_cpu():
    from paper_1510_05218_amd import inputs

    pb = inputs.solar_cell(8, 8, 16, seed=1, npml=3)
    with pytest.raises(RuntimeError):
        thiim.Solver(pb, device="cpu")


def test_missing_library_fails_loudly():
    """Without the built HIP library the binding raises at first use: there
    is no CPU fallback."""
    import subprocess
    import sys

    code = ("import paper_1510_05218_amd.thiim as t\n"
            "try:\n"
            "    t.lib()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n")
    env = dict(os.environ, THIIM_LIBRARY="/nonexistent/libthiim.so")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "no CPU fallback" in r.stdout


def test_tuner_cache_round_trip(tmp_path):
    """The tuner cache persists entries keyed by grid, boundaries, storage,
    precision and device, and survives a reload."""
    path = str(tmp_path / "tune.json")
    g = thiim.make_grid((36, 24, 24), storage="compact")
    g2 = thiim.make_grid((36, 24, 24), storage="full")
    c = thiim.TunerCache(path)
    k = thiim.TunerCache.key(g, "dev")
    assert c.get(k) is None
    c.put(k, {"kernel": 3, "tile_x": 32, "tile_y": 16, "t_block": 2, "z_chunk": 36,
              "ms_per_iteration": 0.1, "model_ms": 0.0})
    c2 = thiim.TunerCache(path)
    assert c2.get(k)["tile_y"] == 16 and "model_ms" not in c2.get(k)
    assert c2.get(thiim.TunerCache.key(g2, "dev")) is None
    assert c2.get(thiim.TunerCache.key(g, "other device")) is None


def test_apply_tuning_rejects_null():
    with pytest.raises(thiim.ThiimError) as e:
        thiim.thiim_apply_tuning(None, {"kernel": 3, "tile_x": 32, "tile_y": 16,
                                        "z_chunk": 4})
    assert e.value.status == thiim.THIIM_EINVAL
