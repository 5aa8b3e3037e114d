"""ctypes binding of libdode.so: the C ABI of include/dode.h with the same names.

Only argument marshalling happens here (shape/dtype/device checks, pointers,
the current HIP stream); every step of the computation runs in the library's
kernels.  Tensors are torch tensors on the GPU; the library reads and writes
their memory in place.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdode.so")

DODE_OK, DODE_ERR_ARG, DODE_ERR_SHAPE, DODE_ERR_DTYPE, DODE_ERR_NONFINITE, DODE_ERR_OOM, \
    DODE_ERR_HIP, DODE_ERR_UNSUPPORTED = range(8)
STATUS_NAMES = ["DODE_OK", "DODE_ERR_ARG", "DODE_ERR_SHAPE", "DODE_ERR_DTYPE",
                "DODE_ERR_NONFINITE", "DODE_ERR_OOM", "DODE_ERR_HIP", "DODE_ERR_UNSUPPORTED"]
DODE_F64, DODE_F32, DODE_BF16, DODE_FP8_E4M3 = range(4)
STORAGE = {"f64": DODE_F64, "f32": DODE_F32, "bf16": DODE_BF16, "fp8": DODE_FP8_E4M3}

# Every symbol include/dode.h declares (checked by the CPU test suite).
EXPORTS = ["dode_last_error", "dode_spgd_defaults", "dar_create", "dar_create_ex", "dar_destroy",
           "dar_info",
           "dar_set_values", "dode_apply", "dode_loss", "dode_loss_noalloc", "dode_grad",
           "dode_metrics", "spgd_step",
           "spgd_solve", "spgd_plan_create", "spgd_plan_destroy", "spgd_plan_load",
           "spgd_plan_store", "spgd_run", "spgd_plan_timing", "spgd_plan_info",
           "spgd_plan_schedule",
           "dode_loss_bwd", "dode_routes_create", "dode_routes_destroy", "dar_from_logits",
           "dar_logits_bwd", "dode_dar_from_speeds", "dode_path_costs", "dar_from_costs",
           "dense_spgd_run", "dode_dar_costs_from_speeds", "dode_dar_patterns_from_speeds"]


class DodeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")


class Dims(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("L", ctypes.c_int32), ("T", ctypes.c_int32),
                ("H", ctypes.c_int32), ("K", ctypes.c_int32)]


class SpgdParams(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch_rows", ctypes.c_int32), ("eta", ctypes.c_double),
                ("eps", ctypes.c_double), ("optimizer", ctypes.c_int32),
                ("check_finite", ctypes.c_int32), ("kernel_path", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("day_tile", ctypes.c_int32),
                ("refine_steps", ctypes.c_int32), ("adj_order", ctypes.c_int32),
                ("slabs", ctypes.c_int32)]


_lib = None


def lib():
    """Load libdode.so; raise if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1901_09266_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        L.dode_last_error.restype = ctypes.c_char_p
        L.dode_spgd_defaults.argtypes = [P(SpgdParams)]
        L.dode_spgd_defaults.restype = None
        L.dar_create.argtypes = [P(Dims), i32, P(i32), P(i32), P(P(dbl)), i32, vp, P(vp)]
        L.dar_create_ex.argtypes = [P(Dims), i32, P(i32), P(i32), P(P(dbl)), i32, i32, vp, P(vp)]
        L.dode_dar_from_speeds.argtypes = [i32, vp, vp, i64, i32, vp, vp, i32, i32, dbl, i32, i32,
                                           i32, vp, vp]
        L.dode_dar_costs_from_speeds.argtypes = [i32, vp, vp, i64, i32, vp, vp, i32, i32, dbl, i32,
                                                 i32, i32, vp, vp, vp]
        L.dode_dar_patterns_from_speeds.argtypes = [i32, vp, vp, i64, i32, vp, vp, i32, P(i32), i32,
                                                    dbl, i32, i32, i32, vp, vp, vp]
        L.dode_path_costs.argtypes = [i32, vp, vp, i64, i32, vp, vp, i32, i32, dbl, i32, i32, vp, vp]
        L.dar_from_costs.argtypes = [vp, i32, vp, vp, dbl, vp, vp, vp]
        L.dense_spgd_run.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, i32, i32, i32, dbl, dbl,
                                     P(dbl), vp]
        L.dar_destroy.argtypes = [vp]
        L.dar_info.argtypes = [vp, P(Dims), P(i32), P(i64), P(i32), P(i64)]
        L.dar_set_values.argtypes = [vp, i32, vp, vp]
        L.dode_apply.argtypes = [vp, i32, vp, i32, vp, vp]
        L.dode_loss.argtypes = [vp, i32, vp, vp, i32, vp, vp]
        L.dode_loss_noalloc.argtypes = [vp, i32, vp, vp, i32, vp, vp]
        L.dode_grad.argtypes = [vp, i32, vp, vp, i32, vp, vp]
        L.dode_metrics.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, vp]
        L.spgd_step.argtypes = [vp, i32, P(i32), i32, vp, vp, vp, i32, P(SpgdParams), vp]
        L.spgd_solve.argtypes = [vp, P(i32), i32, vp, vp, vp, P(SpgdParams), P(i32), ctypes.c_uint64,
                                 P(dbl), vp]
        L.spgd_plan_create.argtypes = [vp, P(i32), i32, P(SpgdParams), P(i32), ctypes.c_uint64, vp,
                                       P(vp)]
        L.spgd_plan_destroy.argtypes = [vp]
        L.spgd_run.argtypes = [vp, i32, i32, vp, vp]
        L.spgd_plan_load.argtypes = [vp, vp, vp, vp, vp]
        L.spgd_plan_store.argtypes = [vp, vp, vp, vp]
        L.spgd_plan_timing.argtypes = [vp, i32, P(dbl), P(i64)]
        L.spgd_plan_info.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
        L.spgd_plan_schedule.argtypes = [vp, P(i32), P(i32), P(i32), P(i32), P(dbl)]
        L.dode_loss_bwd.argtypes = [vp, i32, vp, vp, i32, dbl, vp, vp, vp]
        L.dode_routes_create.argtypes = [P(Dims), i64, i32, P(i32), P(i32), P(i32), P(i32), vp, P(vp)]
        L.dode_routes_destroy.argtypes = [vp]
        L.dar_from_logits.argtypes = [vp, i32, vp, vp, vp, vp]
        L.dar_logits_bwd.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        for name in EXPORTS:
            if name not in ("dode_last_error", "dode_spgd_defaults"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != DODE_OK:
        raise DodeError(status, lib().dode_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, name, dtype=None, shape=None):
    import torch
    if t is None:
        return ctypes.c_void_p(0)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def spgd_defaults() -> SpgdParams:
    p = SpgdParams()
    lib().dode_spgd_defaults(ctypes.byref(p))
    return p


def make_params(epochs=300, batch_rows=8192, eta=5.0, eps=1e-10, optimizer=0, check_finite=1,
                kernel_path=0, use_graph=1, day_tile=32, refine_steps=0, adj_order=1, slabs=1):
    """kernel_path 0 = fastest for the storage type, 1 = sparse pattern kernels,
    2 = matrix-core tiles with one launch per minibatch, 3 = one cooperative
    launch per epoch with grid barriers (day_tile given); use_graph 1 = replay
    one captured hipGraph per epoch; day_tile = days per matrix-core wave (16,
    32 or 64, or 0 to choose the schedule by timing at load); refine_steps =
    full-batch steps per epoch on corrected FP8 values; adj_order = item order
    of the matrix-core adjoint (0, 1, or 2 for runs of consecutive reached
    intervals per wave) and slabs = day slabs per epoch when day_tile is
    given."""
    return SpgdParams(int(epochs), int(batch_rows), float(eta), float(eps), int(optimizer),
                      int(check_finite), int(kernel_path), int(use_graph), int(day_tile),
                      int(refine_steps), int(adj_order), int(slabs))


class Dar:
    """Owner of a dode_dar handle (freed by dar_destroy on close / garbage collection)."""

    def __init__(self, handle, dims, C, storage):
        self.handle = handle
        self.dims = dims
        self.C = C
        self.storage = storage

    @property
    def state_dtype(self):
        import torch
        return torch.float64 if self.storage == DODE_F64 else torch.float32

    def close(self):
        if self.handle:
            lib().dar_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


DAR_CORRECTION = 1


def dar_create(P, L, T, H, K, row_ptr, col_idx, values, storage="f32", correction=False,
               stream=None) -> Dar:
    """values: list of C float64 arrays [K][T][nnz] (host).  correction (FP8
    storage): also keep the bf16 correction tiles used by refinement steps."""
    st = STORAGE[storage] if isinstance(storage, str) else int(storage)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    vals = [np.ascontiguousarray(v, dtype=np.float64) for v in values]
    nnz = int(rp[-1]) if rp.size else 0
    for v in vals:
        if v.size != K * T * nnz:
            raise ValueError(f"values must be [K][T][nnz] = {K * T * nnz} entries, got {v.size}")
    ptrs = (ctypes.POINTER(ctypes.c_double) * len(vals))(
        *[v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for v in vals])
    dims = Dims(P, L, T, H, K)
    out = ctypes.c_void_p()
    _check(lib().dar_create_ex(ctypes.byref(dims), len(vals),
                               rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ptrs, st,
                               DAR_CORRECTION if correction else 0, _stream(stream),
                               ctypes.byref(out)))
    return Dar(out, (P, L, T, H, K), len(vals), st)


def dar_info(dar: Dar):
    dims, C, nnz, st, nb = Dims(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().dar_info(dar.handle, ctypes.byref(dims), ctypes.byref(C), ctypes.byref(nnz),
                          ctypes.byref(st), ctypes.byref(nb)))
    return dict(P=dims.P, L=dims.L, T=dims.T, H=dims.H, K=dims.K, C=C.value, nnz=nnz.value,
                storage=st.value, device_bytes=nb.value)


def dar_set_values(dar: Dar, cluster: int, W, stream=None):
    P, L, T, H, K = dar.dims
    _check(lib().dar_set_values(dar.handle, cluster, _ptr(W, "W", dar.state_dtype), _stream(stream)))


def dode_apply(dar: Dar, cluster: int, Q, Xhat, stream=None):
    P, L, T, H, K = dar.dims
    n = Q.shape[0]
    _check(lib().dode_apply(dar.handle, cluster, _ptr(Q, "Q", dar.state_dtype, (n, T, P)), n,
                            _ptr(Xhat, "Xhat", dar.state_dtype, (n, H, L)), _stream(stream)))


def dode_loss(dar: Dar, cluster: int, Q, X, loss, stream=None):
    import torch
    P, L, T, H, K = dar.dims
    n = Q.shape[0]
    _check(lib().dode_loss(dar.handle, cluster, _ptr(Q, "Q", dar.state_dtype, (n, T, P)),
                           _ptr(X, "X", dar.state_dtype, (n, H, L)), n,
                           _ptr(loss, "loss", torch.float64, (n,)), _stream(stream)))


def dode_loss_noalloc(dar: Dar, cluster: int, Q, X, loss, stream=None):
    """dode_loss without any allocation (library scratch of 4 MiB per GPU)."""
    import torch
    P, L, T, H, K = dar.dims
    n = Q.shape[0]
    _check(lib().dode_loss_noalloc(dar.handle, cluster, _ptr(Q, "Q", dar.state_dtype, (n, T, P)),
                                   _ptr(X, "X", dar.state_dtype, (n, H, L)), n,
                                   _ptr(loss, "loss", torch.float64, (n,)), _stream(stream)))


def dode_grad(dar: Dar, cluster: int, Q, X, G, stream=None):
    P, L, T, H, K = dar.dims
    n = Q.shape[0]
    _check(lib().dode_grad(dar.handle, cluster, _ptr(Q, "Q", dar.state_dtype, (n, T, P)),
                           _ptr(X, "X", dar.state_dtype, (n, H, L)), n,
                           _ptr(G, "G", dar.state_dtype, (n, T, P)), _stream(stream)))


def dode_metrics(dar: Dar, cluster: int, Q, X, loss=None, kkt=None, r2=None, stream=None):
    import torch
    P, L, T, H, K = dar.dims
    n = Q.shape[0]
    _check(lib().dode_metrics(dar.handle, cluster, _ptr(Q, "Q", dar.state_dtype, (n, T, P)),
                              _ptr(X, "X", dar.state_dtype, (n, H, L)), n,
                              _ptr(loss, "loss", torch.float64, (n,)),
                              _ptr(kkt, "kkt", torch.float64, (n,)),
                              _ptr(r2, "r2", torch.float64, (n,)), _stream(stream)))


def spgd_step(dar: Dar, cluster: int, chunk_h, X, Q, A, params: SpgdParams, stream=None):
    P, L, T, H, K = dar.dims
    n = Q.shape[0]
    ch = np.ascontiguousarray(chunk_h, dtype=np.int32)
    _check(lib().spgd_step(dar.handle, cluster, ch.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           ch.size, _ptr(X, "X", dar.state_dtype, (n, H, L)),
                           _ptr(Q, "Q", dar.state_dtype, (n, T, P)),
                           _ptr(A, "A", dar.state_dtype, (n, T, P)), n, ctypes.byref(params),
                           _stream(stream)))


def spgd_solve(dar: Dar, day_cluster, X, Q, A, params: SpgdParams, perm=None, seed=0,
               loss_hist=False, stream=None):
    """Runs Algorithm 1 on all days; returns loss history [D][E] (numpy) if asked."""
    P, L, T, H, K = dar.dims
    dc = np.ascontiguousarray(day_cluster, dtype=np.int32)
    D = dc.size
    pp = ctypes.POINTER(ctypes.c_int32)()
    if perm is not None:
        perm = np.ascontiguousarray(perm, dtype=np.int32)
        if perm.shape != (params.epochs, dar.C, H):
            raise ValueError(f"perm must be [E][C][H] = {(params.epochs, dar.C, H)}")
        pp = perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    hist = np.zeros((D, params.epochs)) if loss_hist else None
    hp = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if loss_hist else \
        ctypes.POINTER(ctypes.c_double)()
    _check(lib().spgd_solve(dar.handle, dc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), D,
                            _ptr(X, "X", dar.state_dtype, (D, H, L)),
                            _ptr(Q, "Q", dar.state_dtype, (D, T, P)),
                            _ptr(A, "A", dar.state_dtype, (D, T, P)), ctypes.byref(params), pp,
                            ctypes.c_uint64(seed), hp, _stream(stream)))
    return hist


class Plan:
    """Owner of a dode_plan handle; keeps its Dar alive."""

    def __init__(self, handle, dar, D, E):
        self.handle = handle
        self.dar = dar
        self.D = D
        self.E = E

    def close(self):
        if self.handle:
            lib().spgd_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spgd_plan_create(dar: Dar, day_cluster, params: SpgdParams, perm=None, seed=0, stream=None) -> Plan:
    P, L, T, H, K = dar.dims
    dc = np.ascontiguousarray(day_cluster, dtype=np.int32)
    pp = ctypes.POINTER(ctypes.c_int32)()
    if perm is not None:
        perm = np.ascontiguousarray(perm, dtype=np.int32)
        if perm.shape != (params.epochs, dar.C, H):
            raise ValueError(f"perm must be [E][C][H] = {(params.epochs, dar.C, H)}")
        pp = perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    out = ctypes.c_void_p()
    _check(lib().spgd_plan_create(dar.handle, dc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  dc.size, ctypes.byref(params), pp, ctypes.c_uint64(seed),
                                  _stream(stream), ctypes.byref(out)))
    return Plan(out, dar, dc.size, params.epochs)


def spgd_plan_load(plan: Plan, X, Q, A=None, stream=None):
    """Copy X [D][H][L], Q and A [D][T][P] (A None = zeros) into the plan's state."""
    P, L, T, H, K = plan.dar.dims
    D = plan.D
    dt = plan.dar.state_dtype
    _check(lib().spgd_plan_load(plan.handle, _ptr(X, "X", dt, (D, H, L)), _ptr(Q, "Q", dt, (D, T, P)),
                                _ptr(A, "A", dt, (D, T, P)), _stream(stream)))


def spgd_plan_store(plan: Plan, Q, A=None, stream=None):
    P, L, T, H, K = plan.dar.dims
    D = plan.D
    dt = plan.dar.state_dtype
    _check(lib().spgd_plan_store(plan.handle, _ptr(Q, "Q", dt, (D, T, P)), _ptr(A, "A", dt, (D, T, P)),
                                 _stream(stream)))


def spgd_run(plan: Plan, epoch_begin, n_epochs, loss=None, stream=None):
    """Epochs of the plan's schedule on its state; loss (optional) is dev float64 [n_epochs][D]."""
    import torch
    _check(lib().spgd_run(plan.handle, int(epoch_begin), int(n_epochs),
                          _ptr(loss, "loss", torch.float64, (n_epochs, plan.D)) if loss is not None
                          else ctypes.c_void_p(0), _stream(stream)))


def spgd_plan_info(plan: Plan) -> dict:
    """day_tile (0 on the sparse kernels), minibatches per epoch, intervals per
    minibatch and day groups of a plan."""
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().spgd_plan_info(plan.handle, *[ctypes.byref(x) for x in v]))
    return dict(zip(("day_tile", "n_minibatches", "minibatch_intervals", "n_day_groups"),
                    (x.value for x in v)))


def spgd_plan_schedule(plan: Plan) -> dict:
    """Matrix-core schedule in use: day tile, adjoint item order, day slabs,
    candidates timed at load and the chosen candidate's epoch time (ms)."""
    v = [ctypes.c_int32() for _ in range(4)]
    ms = ctypes.c_double()
    _check(lib().spgd_plan_schedule(plan.handle, *[ctypes.byref(x) for x in v], ctypes.byref(ms)))
    return dict(day_tile=v[0].value, adj_order=v[1].value, slabs=v[2].value, n_timed=v[3].value,
                best_ms=ms.value)


def spgd_plan_timing(plan: Plan, enable: bool):
    """Returns (ms[3], launches[3]) accumulated since the last call and switches timing."""
    ms = (ctypes.c_double * 3)()
    n = (ctypes.c_int64 * 3)()
    _check(lib().spgd_plan_timing(plan.handle, int(bool(enable)), ms, n))
    return list(ms), list(n)


def dode_loss_bwd(dar: Dar, cluster: int, Q, X, grad_out: float, dQ=None, dW=None, stream=None):
    P, L, T, H, K = dar.dims
    n = Q.shape[0]
    dt = dar.state_dtype
    nnz = dar_info(dar)["nnz"]
    _check(lib().dode_loss_bwd(dar.handle, cluster, _ptr(Q, "Q", dt, (n, T, P)),
                               _ptr(X, "X", dt, (n, H, L)), n, float(grad_out),
                               _ptr(dQ, "dQ", dt, (n, T, P)), _ptr(dW, "dW", dt, (K, T, nnz)),
                               _stream(stream)))


class Routes:
    """Owner of a dode_routes handle (path structure of the route-choice model)."""

    def __init__(self, handle, dims, nnz, n_paths, n_pairs):
        self.handle = handle
        self.dims = dims
        self.nnz = nnz
        self.n_paths = n_paths
        self.n_pairs = n_pairs

    def close(self):
        if self.handle:
            lib().dode_routes_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dode_routes_create(P, L, T, H, K, nnz, path_od, pair_ptr, pair_link, pair_nz, stream=None) -> Routes:
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (path_od, pair_ptr, pair_link, pair_nz)]
    ip = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for a in arrs]
    out = ctypes.c_void_p()
    dims = Dims(P, L, T, H, K)
    _check(lib().dode_routes_create(ctypes.byref(dims), int(nnz), arrs[0].size, *ip, _stream(stream),
                                    ctypes.byref(out)))
    return Routes(out, (P, L, T, H, K), int(nnz), arrs[0].size, int(arrs[1][-1]))


def _route_dtype(t):
    import torch
    if t.dtype not in (torch.float32, torch.float64):
        raise TypeError("route tensors must be float32 or float64")
    return 1 if t.dtype == torch.float64 else 0


def dar_from_logits(routes: Routes, Rr, z, W, stream=None):
    P, L, T, H, K = routes.dims
    f64 = _route_dtype(z)
    dt = z.dtype
    _check(lib().dar_from_logits(routes.handle, f64, _ptr(Rr, "Rr", dt, (K, T, routes.n_pairs)),
                                 _ptr(z, "z", dt, (routes.n_paths,)),
                                 _ptr(W, "W", dt, (K, T, routes.nnz)), _stream(stream)))


def dar_logits_bwd(routes: Routes, Rr, z, dW, dz, stream=None):
    P, L, T, H, K = routes.dims
    f64 = _route_dtype(z)
    dt = z.dtype
    _check(lib().dar_logits_bwd(routes.handle, f64, _ptr(Rr, "Rr", dt, (K, T, routes.n_pairs)),
                                _ptr(z, "z", dt, (routes.n_paths,)),
                                _ptr(dW, "dW", dt, (K, T, routes.nnz)),
                                _ptr(dz, "dz", dt, (routes.n_paths,)), _stream(stream)))


def dode_dar_from_speeds(path_ptr, path_link, link_len, speed, dt, H, K, Rr=None, stream=None):
    """Dynamic assignment ratios from link speeds (device tensors): path_ptr
    int32 [n_paths+1], path_link int32 [n_pairs] (links in traversal order),
    link_len [L], speed [n_days][L][H_speed] (float32 or float64, one dtype).
    Returns Rr [K][H][n_pairs], the day mean of the ratios."""
    Rr, _ = dode_dar_costs_from_speeds(path_ptr, path_link, link_len, speed, dt, H, K, Rr=Rr,
                                       with_costs=False, stream=stream)
    return Rr


def dode_dar_costs_from_speeds(path_ptr, path_link, link_len, speed, dt, H, K, Rr=None, cost=None,
                               with_costs=True, stream=None):
    """As dode_dar_from_speeds, and (with_costs) the mean path costs of the H
    departure intervals from the same trajectories.  Returns (Rr [K][H][n_pairs],
    cost [H][n_paths] or None)."""
    import torch
    if speed.dim() == 2:
        speed = speed.unsqueeze(0)
    n_days, L, H_speed = speed.shape
    f64 = speed.dtype == torch.float64
    n_paths = path_ptr.numel() - 1
    n_pairs = path_link.numel()
    if Rr is None:
        Rr = torch.empty((K, H, n_pairs), dtype=speed.dtype, device=speed.device)
    if with_costs and cost is None:
        cost = torch.empty((H, n_paths), dtype=speed.dtype, device=speed.device)
    if not with_costs:
        cost = None
    for t in (path_ptr, path_link, link_len, speed, Rr) + ((cost,) if cost is not None else ()):
        if not t.is_contiguous():
            raise ValueError("arrays must be contiguous")
    if link_len.dtype != speed.dtype or Rr.dtype != speed.dtype or (
            cost is not None and cost.dtype != speed.dtype):
        raise ValueError("link_len, speed, Rr and cost must share one dtype")
    if tuple(Rr.shape) != (K, H, n_pairs):
        raise ValueError(f"Rr must be [{K}][{H}][{n_pairs}]")
    if cost is not None and tuple(cost.shape) != (H, n_paths):
        raise ValueError(f"cost must be [{H}][{n_paths}]")
    _check(lib().dode_dar_costs_from_speeds(
        n_paths, path_ptr.data_ptr(), path_link.data_ptr(), n_pairs, L, link_len.data_ptr(),
        speed.data_ptr(), n_days, H_speed, float(dt), H, K, int(f64), Rr.data_ptr(),
        cost.data_ptr() if cost is not None else None, _stream(stream)))
    return Rr, cost


def dode_dar_patterns_from_speeds(path_ptr, path_link, link_len, speed, pattern_ptr, dt, H, K,
                                  Rr=None, cost=None, with_costs=False, stream=None):
    """The ratios (and with_costs the mean path costs) of several traffic
    patterns in one call: pattern q holds days pattern_ptr[q] ..
    pattern_ptr[q+1]-1 of speed [D][L][H_speed].  Returns (Rr [n_patterns][K][H]
    [n_pairs], cost [n_patterns][H][n_paths] or None)."""
    import torch
    n_days, L, H_speed = speed.shape
    f64 = speed.dtype == torch.float64
    n_paths = path_ptr.numel() - 1
    n_pairs = path_link.numel()
    pp = np.ascontiguousarray(pattern_ptr, dtype=np.int32)
    nq = pp.size - 1
    if nq < 1 or pp[-1] != n_days:
        raise ValueError(f"pattern_ptr must run from 0 to the {n_days} days of speed")
    if Rr is None:
        Rr = torch.empty((nq, K, H, n_pairs), dtype=speed.dtype, device=speed.device)
    if with_costs and cost is None:
        cost = torch.empty((nq, H, n_paths), dtype=speed.dtype, device=speed.device)
    if not with_costs:
        cost = None
    for t in (path_ptr, path_link, link_len, speed, Rr) + ((cost,) if cost is not None else ()):
        if not t.is_contiguous():
            raise ValueError("arrays must be contiguous")
    if link_len.dtype != speed.dtype or Rr.dtype != speed.dtype or (
            cost is not None and cost.dtype != speed.dtype):
        raise ValueError("link_len, speed, Rr and cost must share one dtype")
    if tuple(Rr.shape) != (nq, K, H, n_pairs):
        raise ValueError(f"Rr must be [{nq}][{K}][{H}][{n_pairs}]")
    if cost is not None and tuple(cost.shape) != (nq, H, n_paths):
        raise ValueError(f"cost must be [{nq}][{H}][{n_paths}]")
    _check(lib().dode_dar_patterns_from_speeds(
        n_paths, path_ptr.data_ptr(), path_link.data_ptr(), n_pairs, L, link_len.data_ptr(),
        speed.data_ptr(), nq, pp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), H_speed,
        float(dt), H, K, int(f64), Rr.data_ptr(), cost.data_ptr() if cost is not None else None,
        _stream(stream)))
    return Rr, cost


def dode_path_costs(path_ptr, path_link, link_len, speed, dt, T, cost=None, stream=None):
    """Mean path travel times of a pattern's days (device tensors, as for
    dode_dar_from_speeds).  Returns cost [T][n_paths]: for departures at t*dt,
    the day mean of the time to cross the whole path."""
    import torch
    if speed.dim() == 2:
        speed = speed.unsqueeze(0)
    n_days, L, H_speed = speed.shape
    f64 = speed.dtype == torch.float64
    n_paths = path_ptr.numel() - 1
    n_pairs = path_link.numel()
    if cost is None:
        cost = torch.empty((T, n_paths), dtype=speed.dtype, device=speed.device)
    for t in (path_ptr, path_link, link_len, speed, cost):
        if not t.is_contiguous():
            raise ValueError("arrays must be contiguous")
    if link_len.dtype != speed.dtype or cost.dtype != speed.dtype:
        raise ValueError("link_len, speed and cost must share one dtype")
    if tuple(cost.shape) != (T, n_paths):
        raise ValueError(f"cost must be [{T}][{n_paths}]")
    _check(lib().dode_path_costs(n_paths, path_ptr.data_ptr(), path_link.data_ptr(), n_pairs, L,
                                 link_len.data_ptr(), speed.data_ptr(), n_days, H_speed, float(dt),
                                 T, int(f64), cost.data_ptr(), _stream(stream)))
    return cost


def dar_from_costs(routes: Routes, Rr, cost, theta, W, portions=None, stream=None):
    """W [K][T][nnz] of eq. "assign" from ratios Rr [K][T][n_pairs] and logit
    portions of the path costs cost [T][n_paths] (eqs. "logit", "rt"); the
    portions are also written to `portions` [T][n_paths] when given."""
    P, L, T, H, K = routes.dims
    f64 = _route_dtype(cost)
    dt = cost.dtype
    pp = None if portions is None else _ptr(portions, "portions", dt, (T, routes.n_paths))
    _check(lib().dar_from_costs(routes.handle, f64, _ptr(Rr, "Rr", dt, (K, T, routes.n_pairs)),
                                _ptr(cost, "cost", dt, (T, routes.n_paths)), float(theta), pp,
                                _ptr(W, "W", dt, (K, T, routes.nnz)), _stream(stream)))


def dense_spgd_run(B, y, q, A, perms, chunk, eta, eps=1e-10, optimizer=0, loss_hist=False,
                   stream=None):
    """Algorithm 1 on a dense B [m][n] (device tensors, float32, float64, or
    bfloat16 with float32 y, q, A): q, A [n] are updated in place; perms int32
    [E][m] on the device.  Returns the per-epoch losses (numpy, FP64) when
    loss_hist is set, else None."""
    import torch
    m, n = B.shape
    if B.dtype not in (torch.float32, torch.float64, torch.bfloat16):
        raise TypeError("B must be float32, float64 or bfloat16")
    dt = torch.float32 if B.dtype == torch.bfloat16 else B.dtype
    prec = 2 if B.dtype == torch.bfloat16 else int(dt == torch.float64)
    E = perms.shape[0] if perms.numel() else 0
    bp = _ptr(B, "B", B.dtype, (m, n))
    yp = _ptr(y, "y", dt, (m,))
    qp = _ptr(q, "q", dt, (n,))
    ap = _ptr(A, "A", dt, (n,))
    pp = _ptr(perms, "perms", torch.int32, (E, m))
    hist = np.zeros(max(E, 1)) if loss_hist else None
    hp = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if loss_hist else None
    _check(lib().dense_spgd_run(m, n, prec, bp, yp, qp, ap, pp, E, int(chunk),
                                int(optimizer), float(eta), float(eps), hp, _stream(stream)))
    return hist[:E] if loss_hist else None
