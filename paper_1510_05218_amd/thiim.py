"""Python binding of the THIIM C-ABI (``include/thiim.h``): ctypes argument
marshalling only.  Every step of the iteration runs in the HIP kernels of
``libthiim.so``; torch provides device memory and the stream.  There is no
fallback: without the built library (or without a GPU) the calls raise.

Module-level functions carry the C names (``thiim_create``, ``thiim_iterate``
...); :class:`Solver` bundles them with the torch-owned buffers.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# THIIM_LIBRARY may name another build of the same C-ABI (e.g. a tuning build)
LIB_PATH = os.environ.get("THIIM_LIBRARY") or os.path.join(_HERE, "libthiim.so")

THIIM_OK = 0
THIIM_EINVAL = -1
THIIM_ENOMEM = -2
THIIM_EDEVICE = -3
THIIM_EDIVERGED = -4
THIIM_ENOTCONV = -5
PERIODIC, DIRICHLET = 0, 1
KERNELS = {"auto": 0, "naive": 1, "fused": 2, "blocked": 3}
STORAGES = {"full": 0, "compact": 1}
PRECISIONS = {"fp64": 0, "mixed": 1}

SYMBOLS = ("thiim_workspace_bytes", "thiim_create", "thiim_iterate",
           "thiim_residual", "thiim_solve", "thiim_get_fields",
           "thiim_set_fields", "thiim_get_coeffs", "thiim_iterations",
           "thiim_adjoint_grad", "thiim_autotune", "thiim_batch_workspace_bytes",
           "thiim_batch_create", "thiim_batch_iterate", "thiim_batch_residual",
           "thiim_batch_solve", "thiim_batch_autotune", "thiim_batch_destroy",
           "thiim_batch_create_static", "thiim_stream_probe", "thiim_apply_tuning",
           "thiim_destroy",
           "thiim_last_error", "thiim_status_str")


class ThiimError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_str(status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
                ("h", ctypes.c_double), ("tau", ctypes.c_double),
                ("kernel", ctypes.c_int), ("t_block", ctypes.c_int),
                ("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int),
                ("z_chunk", ctypes.c_int), ("storage", ctypes.c_int),
                ("precision", ctypes.c_int), ("adjoint", ctypes.c_int),
                ("stream", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int),
                ("t_block", ctypes.c_int), ("z_chunk", ctypes.c_int),
                ("ms_per_iteration", ctypes.c_double), ("model_ms", ctypes.c_double),
                ("candidates", ctypes.c_int), ("timed", ctypes.c_int),
                ("one_for_all_ms", ctypes.c_double), ("per_grid_ms", ctypes.c_double),
                ("per_grid", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Coeffs(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_void_p),
                ("sigma_e", ctypes.POINTER(ctypes.c_double)),
                ("sigma_h", ctypes.POINTER(ctypes.c_double)),
                ("src", ctypes.c_void_p * 4)]


_lib = None


def lib():
    """The loaded ``libthiim.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1510_05218_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.thiim_workspace_bytes.argtypes = [P(Grid), P(ctypes.c_size_t)]
        L.thiim_create.argtypes = [P(Grid), P(Coeffs), d, vp, ctypes.c_size_t, P(vp)]
        L.thiim_iterate.argtypes = [vp, i]
        L.thiim_residual.argtypes = [vp, P(d)]
        L.thiim_solve.argtypes = [vp, d, i, i, P(i), P(d)]
        L.thiim_get_fields.argtypes = [vp, vp]
        L.thiim_set_fields.argtypes = [vp, vp]
        L.thiim_get_coeffs.argtypes = [vp, vp]
        L.thiim_iterations.argtypes = [vp, P(ctypes.c_longlong)]
        L.thiim_adjoint_grad.argtypes = [vp, vp, d, i, i, vp, P(d), P(i), P(d)]
        L.thiim_autotune.argtypes = [vp, i, P(Tuning)]
        L.thiim_apply_tuning.argtypes = [vp, P(Tuning)]
        L.thiim_batch_workspace_bytes.argtypes = [i, P(ctypes.c_size_t)]
        L.thiim_batch_create.argtypes = [P(vp), i, vp, ctypes.c_size_t, P(vp)]
        L.thiim_batch_create_static.argtypes = [P(vp), i, P(vp)]
        L.thiim_stream_probe.argtypes = [vp, vp, ctypes.c_longlong, ctypes.c_longlong, i, i,
                                         vp]
        L.thiim_batch_iterate.argtypes = [vp, i]
        L.thiim_batch_residual.argtypes = [vp, P(d)]
        L.thiim_batch_solve.argtypes = [vp, d, i, i, P(i), P(d)]
        L.thiim_batch_autotune.argtypes = [vp, i, P(Tuning)]
        L.thiim_batch_destroy.argtypes = [vp]
        L.thiim_batch_destroy.restype = None
        L.thiim_destroy.argtypes = [vp]
        L.thiim_destroy.restype = None
        L.thiim_last_error.restype = ctypes.c_char_p
        L.thiim_status_str.argtypes = [i]
        L.thiim_status_str.restype = ctypes.c_char_p
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().thiim_status_str(int(status)).decode()


def last_error() -> str:
    return lib().thiim_last_error().decode()


def _check(rc):
    if rc != THIIM_OK:
        raise ThiimError(rc, last_error())
    return rc


# ---------------------------------------------------------------------------
# the C calls, one wrapper each
# ---------------------------------------------------------------------------
def thiim_workspace_bytes(grid: Grid) -> int:
    n = ctypes.c_size_t()
    _check(lib().thiim_workspace_bytes(ctypes.byref(grid), ctypes.byref(n)))
    return n.value


def thiim_create(grid: Grid, coeffs: Coeffs, omega: float, workspace_ptr: int,
                 workspace_bytes: int):
    ctx = ctypes.c_void_p()
    _check(lib().thiim_create(ctypes.byref(grid), ctypes.byref(coeffs), float(omega),
                              ctypes.c_void_p(workspace_ptr), workspace_bytes,
                              ctypes.byref(ctx)))
    return ctx


def thiim_iterate(ctx, n: int):
    _check(lib().thiim_iterate(ctx, int(n)))


def thiim_residual(ctx) -> float:
    r = ctypes.c_double()
    _check(lib().thiim_residual(ctx, ctypes.byref(r)))
    return r.value


def thiim_solve(ctx, tol: float, max_it: int, check_every: int = 50):
    """Returns (status, iterations, rel_res); ENOTCONV is returned, not raised."""
    it, r = ctypes.c_int(), ctypes.c_double()
    rc = lib().thiim_solve(ctx, float(tol), int(max_it), int(check_every),
                           ctypes.byref(it), ctypes.byref(r))
    if rc not in (THIIM_OK, THIIM_ENOTCONV):
        _check(rc)
    return rc, it.value, r.value


def thiim_get_fields(ctx, dst_ptr: int):
    _check(lib().thiim_get_fields(ctx, ctypes.c_void_p(dst_ptr)))


def thiim_set_fields(ctx, src_ptr: int):
    _check(lib().thiim_set_fields(ctx, ctypes.c_void_p(src_ptr)))


def thiim_get_coeffs(ctx, dst_ptr: int):
    _check(lib().thiim_get_coeffs(ctx, ctypes.c_void_p(dst_ptr)))


def thiim_iterations(ctx) -> int:
    n = ctypes.c_longlong()
    _check(lib().thiim_iterations(ctx, ctypes.byref(n)))
    return n.value


def thiim_adjoint_grad(ctx, weight_ptr: int, tol: float, max_it: int, check_every: int,
                       grad_ptr: int):
    """Returns (status, J, iterations, rel_res); ENOTCONV is returned, not raised."""
    J, it, r = ctypes.c_double(), ctypes.c_int(), ctypes.c_double()
    rc = lib().thiim_adjoint_grad(ctx, ctypes.c_void_p(weight_ptr), float(tol), int(max_it),
                                  int(check_every), ctypes.c_void_p(grad_ptr), ctypes.byref(J),
                                  ctypes.byref(it), ctypes.byref(r))
    if rc not in (THIIM_OK, THIIM_ENOTCONV):
        _check(rc)
    return rc, J.value, it.value, r.value


def thiim_autotune(ctx, trial_iters: int = 10) -> Tuning:
    out = Tuning()
    _check(lib().thiim_autotune(ctx, int(trial_iters), ctypes.byref(out)))
    return out


def thiim_apply_tuning(ctx, tuning: dict):
    t = Tuning(**{k: tuning[k] for k, _ in Tuning._fields_ if k in tuning})
    _check(lib().thiim_apply_tuning(ctx, ctypes.byref(t)))


class TunerCache:
    """Persisted thiim_autotune choices, a JSON file keyed by what decides the
    choice: grid shape, boundaries, storage, precision and the device (name,
    architecture, compute units).  ``Solver.autotune(cache=...)`` applies a
    cached entry (thiim_apply_tuning) instead of timing, and stores what it
    times.  Writes go to a temporary file that replaces the old one."""

    def __init__(self, path):
        import json

        self.path = path
        self.entries = {}
        if os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    @staticmethod
    def key(grid: Grid, device: str) -> str:
        return (f"{grid.nx}x{grid.ny}x{grid.nz}|bc{grid.bc_x}{grid.bc_y}|s{grid.storage}"
                f"|p{grid.precision}|{device}")

    def get(self, key):
        return self.entries.get(key)

    def put(self, key, tuning: dict):
        import json

        self.entries[key] = {k: tuning[k] for k in ("kernel", "tile_x", "tile_y", "t_block",
                                                    "z_chunk", "ms_per_iteration")}
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def device_key(device) -> str:
    """Name, architecture and compute units of a torch device."""
    import torch

    p = torch.cuda.get_device_properties(device)
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}cu"


def thiim_batch_workspace_bytes(n: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().thiim_batch_workspace_bytes(int(n), ctypes.byref(b)))
    return b.value


def thiim_batch_create(ctxs, workspace_ptr: int, workspace_bytes: int):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    out = ctypes.c_void_p()
    _check(lib().thiim_batch_create(arr, len(ctxs), ctypes.c_void_p(workspace_ptr),
                                    workspace_bytes, ctypes.byref(out)))
    return out


def thiim_batch_create_static(ctxs):
    """The allocation-free batch: item tables and queue counters in the
    library's static device scratch (at most 128 problems, one such batch per
    device at a time)."""
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    out = ctypes.c_void_p()
    _check(lib().thiim_batch_create_static(arr, len(ctxs), ctypes.byref(out)))
    return out


def thiim_stream_probe(src_ptr: int, dst_ptr: int, n: int, stride: int, nin: int, nout: int,
                       stream_ptr: int):
    _check(lib().thiim_stream_probe(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), int(n),
                                    int(stride), int(nin), int(nout),
                                    ctypes.c_void_p(stream_ptr)))


def thiim_batch_iterate(batch, n: int):
    _check(lib().thiim_batch_iterate(batch, int(n)))


def thiim_batch_residual(batch, n: int):
    r = (ctypes.c_double * n)()
    _check(lib().thiim_batch_residual(batch, r))
    return np.array(r[:])


def thiim_batch_solve(batch, n: int, tol: float, max_it: int, check_every: int = 200):
    """Returns (status, iterations[n], rel_res[n]); ENOTCONV is returned."""
    it, r = (ctypes.c_int * n)(), (ctypes.c_double * n)()
    rc = lib().thiim_batch_solve(batch, float(tol), int(max_it), int(check_every), it, r)
    if rc not in (THIIM_OK, THIIM_ENOTCONV):
        _check(rc)
    return rc, np.array(it[:]), np.array(r[:])


def thiim_batch_autotune(batch, trial_iters: int = 8) -> Tuning:
    out = Tuning()
    _check(lib().thiim_batch_autotune(batch, int(trial_iters), ctypes.byref(out)))
    return out


def thiim_batch_destroy(batch):
    lib().thiim_batch_destroy(batch)


def thiim_destroy(ctx):
    lib().thiim_destroy(ctx)


# ---------------------------------------------------------------------------
# convenience wrapper owning the torch buffers
# ---------------------------------------------------------------------------
def make_grid(shape, tau=0.5, h=1.0, bcx=PERIODIC, bcy=PERIODIC, kernel="auto",
              t_block=0, tile=(0, 0), z_chunk=0, stream=None, storage="full",
              precision="fp64", adjoint=False) -> Grid:
    nz, ny, nx = shape
    return Grid(nx, ny, nz, bcx, bcy, h, tau, KERNELS[kernel], t_block,
                tile[0], tile[1], z_chunk, STORAGES[storage], PRECISIONS[precision],
                int(bool(adjoint)), stream)


class Solver:
    """One THIIM problem resident on the GPU.

    ``problem`` is an :class:`paper_1510_05218_amd.inputs.Problem` (material
    data, PML profiles, sources, omega, tau).  Its ``eps`` and source arrays
    may be numpy arrays (copied to the device for ``thiim_create`` and
    released afterwards) or complex128 device tensors (used in place)."""

    def __init__(self, problem, kernel="auto", t_block=0, tile=(0, 0), z_chunk=0,
                 device="cuda", stream=None, storage="full", precision="fp64",
                 adjoint=False):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("the THIIM library needs an MI355X GPU (no CPU path)")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.shape = tuple(problem.eps.shape)
        nz, ny, nx = self.shape
        self.N = nx * ny * nz
        self.grid = make_grid(self.shape, problem.tau, problem.h, problem.bcx,
                              problem.bcy, kernel, t_block, tile, z_chunk,
                              self.stream.cuda_stream, storage, precision, adjoint)
        self.ws_bytes = thiim_workspace_bytes(self.grid)
        # allocated on the stream the library runs on, so that torch's caching
        # allocator never hands the memory to another stream while kernels of
        # this context may still use it (and after the caller's pending work)
        with self._lib_stream():
            self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            eps = self._to_dev(problem.eps)
            srcs = [self._to_dev(problem.sources[k]) if k in problem.sources else None
                    for k in ("Hx", "Hy", "Ex", "Ey")]
        self._sig_e = np.ascontiguousarray(problem.sig_e, dtype=np.float64)
        self._sig_h = np.ascontiguousarray(problem.sig_h, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        co = Coeffs(eps.data_ptr(), self._sig_e.ctypes.data_as(dp),
                    self._sig_h.ctypes.data_as(dp),
                    (ctypes.c_void_p * 4)(*[s.data_ptr() if s is not None else None
                                            for s in srcs]))
        self.omega = float(problem.omega)
        self.ctx = thiim_create(self.grid, co, self.omega, self.workspace.data_ptr(),
                                self.ws_bytes)
        del eps, srcs

    def _to_dev(self, a):
        """Device complex128 tensor for an input array (no copy if it is one)."""
        if isinstance(a, self.torch.Tensor):
            return a.to(self.device, self.torch.complex128).contiguous()
        t = self.torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))
        return t.to(self.device, non_blocking=False)

    # -- calls
    def iterate(self, n):
        thiim_iterate(self.ctx, n)

    def residual(self):
        return thiim_residual(self.ctx)

    def solve(self, tol, max_it, check_every=50):
        """FP64: residual every check_every iterations.  MIXED: check_every
        inner sweeps per correction, 0 = adaptive."""
        return thiim_solve(self.ctx, tol, max_it, check_every)

    def autotune(self, trial_iters=10, cache=None):
        """Chooses this context's sweep configuration (thiim_autotune).  With
        a :class:`TunerCache`, a configuration cached for the same grid,
        storage, precision and device is applied without timing (the result
        then carries ``"cached": True``); otherwise the timed choice is
        stored in the cache."""
        if cache is not None:
            key = TunerCache.key(self.grid, device_key(self.device))
            hit = cache.get(key)
            if hit is not None:
                thiim_apply_tuning(self.ctx, hit)
                return {**hit, "cached": True}
        out = thiim_autotune(self.ctx, trial_iters).as_dict()
        if cache is not None:
            cache.put(key, out)
        return out

    def _lib_stream(self):
        """Context for torch work whose results the library reads or writes:
        the library's stream first waits for the caller's current stream (so
        inputs produced there are complete), then the conversions and
        allocations run on the library's stream, ordered before the C call."""
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        return self.torch.cuda.stream(self.stream)

    def adjoint_grad(self, weight, tol=1e-10, max_it=100000, check_every=50):
        """Gradient of J = sum w eps'' |E|^2 at the current state.  Returns
        (status, J, grad, iterations, rel_res) with grad a complex128 tensor
        (nz, ny, nx) holding dJ/deps' + 1j dJ/deps''."""
        with self._lib_stream():
            w = self._to_dev_real(weight)
            grad = self.torch.empty(self.shape, dtype=self.torch.complex128,
                                    device=self.device)
        rc, J, it, r = thiim_adjoint_grad(self.ctx, w.data_ptr(), tol, max_it, check_every,
                                          grad.data_ptr())
        return rc, J, grad, it, r

    def _to_dev_real(self, a):
        if isinstance(a, self.torch.Tensor):
            t = a.to(self.device, self.torch.float64).contiguous()
        else:
            t = self.torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)
        assert tuple(t.shape) == self.shape
        return t

    def fields(self):
        """The 12 split fields, complex128 tensor (12, nz, ny, nx) on the GPU."""
        with self._lib_stream():
            out = self.torch.empty((12,) + self.shape, dtype=self.torch.complex128,
                                   device=self.device)
        thiim_get_fields(self.ctx, out.data_ptr())
        return out

    def set_fields(self, x):
        with self._lib_stream():
            x = x.to(self.device, self.torch.complex128).contiguous()
        assert tuple(x.shape) == (12,) + self.shape
        thiim_set_fields(self.ctx, x.data_ptr())
        self.stream.synchronize()

    def coeffs(self):
        with self._lib_stream():
            out = self.torch.empty((28,) + self.shape, dtype=self.torch.complex128,
                                   device=self.device)
        thiim_get_coeffs(self.ctx, out.data_ptr())
        return out

    @property
    def iterations(self):
        return thiim_iterations(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            self.stream.synchronize()  # no kernel of this context still runs
            thiim_destroy(self.ctx)
            self.ctx = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many problems advanced together (thiim_batch_*): ``problems`` is a list
    of ``inputs.Problem``; each gets a compact-storage :class:`Solver` on one
    shared non-default stream (so that the batch can capture HIP graphs);
    ``autotune`` picks the batch's sweep configuration (thiim_batch_autotune)."""

    def __init__(self, problems, autotune=False, trial_iters=8, device="cuda", stream=None,
                 **solver_kw):
        import torch

        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.solvers = [Solver(p, storage="compact", device=device, stream=self.stream,
                               **solver_kw) for p in problems]
        self.n = len(self.solvers)
        self.ws_bytes = thiim_batch_workspace_bytes(self.n)
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.batch = thiim_batch_create([s.ctx for s in self.solvers],
                                        self.workspace.data_ptr(), self.ws_bytes)
        self.tuning = (thiim_batch_autotune(self.batch, trial_iters).as_dict() if autotune
                       else None)

    def iterate(self, n):
        thiim_batch_iterate(self.batch, n)

    def residual(self):
        return thiim_batch_residual(self.batch, self.n)

    def solve(self, tol, max_it, check_every=200):
        return thiim_batch_solve(self.batch, self.n, tol, max_it, check_every)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "batch", None) is not None:
            self.stream.synchronize()
            thiim_batch_destroy(self.batch)
            self.batch = None
        for s in getattr(self, "solvers", []):
            s.close()
        self.solvers = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
