"""Python front end of the FP64 CPU oracle in dode_oracle.c.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the GPU library or its binding.

What each entry point follows in the paper (arXiv 1901.09266):
  apply       eq. "finalobj" / eq. "assign": xhat = rho q
  loss        eq. "nnls": ||rho q - x||^2 (no 1/2, no mean)
  grad        Algorithm 1's g = rho^T (rho q - x)
  spgd        Algorithm 1 (permute, minibatch, Adagrad or fixed step, max(q, 0))
  kkt, r2     end-of-solve checks (Step 6 "Quality check")
  rho_from_logits, loss_backward, logits_backward
              eqs. "logit", "flow", "assign" with free logits per path
  dar_from_speeds
              eqs. "dar2"/"dar", "cost": ratios from link speeds
  path_costs, logit_portions, rho_from_portions
              eqs. "cost", "logit", "rt", "assign": route portions from the
              mean path travel time of a pattern's days, and the assignment
              matrix they give
  dense_spgd, dense_loss
              Algorithm 1 on a dense B (section "Algorithm efficiency")

Pins (tests/test_oracle_pins.py): brute-force active-set enumeration, scipy's
Lawson-Hanson NNLS, planted noiseless recovery, KKT conditions, the adjoint
identity <rho q, r> = <q, rho^T r>, the paper's global matrix indexing
(Table "DODE framework variable vectorization") against a dense product,
central finite differences, closed forms (identity assignment, first Adagrad
step), torch.optim.Adagrad driving the same minibatches, scale invariance of
Adagrad, day independence and row/block equivalence for a single minibatch.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dode_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

__all__ = ["build_oracle", "Dims", "apply", "adjoint", "loss", "grad", "kkt", "r2", "spgd_day",
           "spgd_step", "spgd", "metrics", "route_softmax", "rho_from_logits", "loss_backward",
           "logits_backward", "fixed_step_eta", "dar_from_speeds", "path_costs", "logit_portions",
           "rho_from_portions", "dense_loss", "dense_spgd", "lib"]


def build_oracle(force: bool = True) -> str:
    """Compile dode_oracle.c into liboracle.so with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unused-parameter",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build_oracle(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dptr, iptr = P(ctypes.c_double), P(ctypes.c_int32)
        dims = P(Dims)
        L.orc_apply.argtypes = [dims, iptr, iptr, dptr, dptr, dptr]
        L.orc_adjoint.argtypes = [dims, iptr, iptr, dptr, dptr, dptr]
        L.orc_loss.argtypes = [dims, iptr, iptr, dptr, dptr, dptr]
        L.orc_loss.restype = ctypes.c_double
        L.orc_grad.argtypes = [dims, iptr, iptr, dptr, dptr, dptr, dptr]
        L.orc_kkt.argtypes = [dims, iptr, iptr, dptr, dptr, dptr]
        L.orc_kkt.restype = ctypes.c_double
        L.orc_r2.argtypes = [dims, iptr, iptr, dptr, dptr, dptr]
        L.orc_r2.restype = ctypes.c_double
        L.orc_spgd_day.argtypes = [dims, iptr, iptr, dptr, dptr, dptr, dptr, iptr, ctypes.c_int64,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_double, ctypes.c_double, dptr]
        L.orc_spgd_step.argtypes = [dims, iptr, iptr, dptr, dptr, dptr, dptr, iptr, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        L.orc_spgd.argtypes = [dims, ctypes.c_int32, iptr, iptr, iptr, P(dptr), dptr, dptr, dptr,
                               iptr, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                               dptr, ctypes.c_int32]
        L.orc_metrics.argtypes = [dims, ctypes.c_int32, iptr, iptr, iptr, P(dptr), dptr, dptr,
                                  dptr, dptr, dptr, ctypes.c_int32]
        L.orc_metrics.restype = None
        L.orc_route_softmax.argtypes = [ctypes.c_int32, ctypes.c_int32, iptr, dptr, dptr]
        L.orc_rho_from_logits.argtypes = [dims, ctypes.c_int32, iptr, iptr, iptr, dptr, dptr, iptr,
                                          iptr, dptr]
        L.orc_loss_backward.argtypes = [dims, iptr, iptr, dptr, ctypes.c_int32, dptr, dptr, dptr, dptr]
        L.orc_loss_backward.restype = None
        L.orc_logits_backward.argtypes = [dims, ctypes.c_int32, iptr, iptr, iptr, dptr, dptr, iptr,
                                          iptr, dptr, dptr]
        i32 = ctypes.c_int32
        L.orc_dar_from_speeds.argtypes = [i32, iptr, iptr, i32, dptr, dptr, i32, i32,
                                          ctypes.c_double, i32, i32, i32, dptr]
        L.orc_path_costs.argtypes = [i32, iptr, iptr, i32, dptr, dptr, i32, i32, ctypes.c_double,
                                     i32, i32, dptr]
        L.orc_logit_portions.argtypes = [i32, i32, iptr, i32, ctypes.c_double, dptr, dptr]
        L.orc_logit_portions.restype = None
        L.orc_dense_loss.argtypes = [i32, i32, dptr, dptr, dptr]
        L.orc_dense_loss.restype = ctypes.c_double
        L.orc_dense_spgd.argtypes = [i32, i32, dptr, dptr, dptr, dptr, iptr, i32, i32, i32,
                                     ctypes.c_double, ctypes.c_double, dptr]
        L.orc_rho_from_portions.argtypes = [dims, i32, iptr, iptr, iptr, dptr, dptr, iptr, iptr,
                                            dptr]
        _lib = L
    return _lib


class Dims(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("L", ctypes.c_int32), ("T", ctypes.c_int32),
                ("H", ctypes.c_int32), ("K", ctypes.c_int32)]


class _DimsRef:
    def __init__(self, P, L, T, H, K):
        self.obj = Dims(P, L, T, H, K)
        self.ref = ctypes.byref(self.obj)


def _dims(P, L, T, H, K):
    return _DimsRef(P, L, T, H, K).ref


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _null_d():
    return ctypes.POINTER(ctypes.c_double)()


class _Pattern:
    def __init__(self, P, L, T, H, K, row_ptr, col_idx):
        self._d = Dims(P, L, T, H, K)
        self.dims = ctypes.byref(self._d)
        self.shape = (P, L, T, H, K)
        self.rp, self.rp_p = _i(row_ptr)
        self.ci, self.ci_p = _i(col_idx)


def _pat(inst_or_tuple):
    if isinstance(inst_or_tuple, _Pattern):
        return inst_or_tuple
    i = inst_or_tuple
    return _Pattern(i.P, i.L, i.T, i.H, i.K, i.row_ptr, i.col_idx)


def apply(inst, W, q):
    """xhat[h][a] of one day (q is [T][P])."""
    pt = _pat(inst)
    P, L, T, H, K = pt.shape
    W, Wp = _d(W)
    q, qp = _d(q)
    out = np.zeros((H, L))
    _, op = _d(out)
    lib().orc_apply(pt.dims, pt.rp_p, pt.ci_p, Wp, qp, op)
    return out


def adjoint(inst, W, r):
    pt = _pat(inst)
    P, L, T, H, K = pt.shape
    W, Wp = _d(W)
    r, rp = _d(r)
    out = np.zeros((T, P))
    _, op = _d(out)
    lib().orc_adjoint(pt.dims, pt.rp_p, pt.ci_p, Wp, rp, op)
    return out


def loss(inst, W, q, x):
    pt = _pat(inst)
    W, Wp = _d(W)
    q, qp = _d(q)
    x, xp = _d(x)
    return lib().orc_loss(pt.dims, pt.rp_p, pt.ci_p, Wp, qp, xp)


def grad(inst, W, q, x):
    pt = _pat(inst)
    P, L, T, H, K = pt.shape
    W, Wp = _d(W)
    q, qp = _d(q)
    x, xp = _d(x)
    out = np.zeros((T, P))
    _, op = _d(out)
    lib().orc_grad(pt.dims, pt.rp_p, pt.ci_p, Wp, qp, xp, op)
    return out


def kkt(inst, W, q, x):
    pt = _pat(inst)
    W, Wp = _d(W)
    q, qp = _d(q)
    x, xp = _d(x)
    return lib().orc_kkt(pt.dims, pt.rp_p, pt.ci_p, Wp, qp, xp)


def r2(inst, W, q, x):
    pt = _pat(inst)
    W, Wp = _d(W)
    q, qp = _d(q)
    x, xp = _d(x)
    return lib().orc_r2(pt.dims, pt.rp_p, pt.ci_p, Wp, qp, xp)


def spgd_day(inst, W, x, perm, E, chunk, q0=None, A0=None, granularity=0, optimizer=0,
             eta=5.0, eps=1e-10, record_loss=True):
    """Algorithm 1 on one day. perm is [E][units]. Returns (q, A, loss_hist)."""
    pt = _pat(inst)
    P, L, T, H, K = pt.shape
    W, Wp = _d(W)
    x, xp = _d(x)
    q = np.zeros((T, P)) if q0 is None else np.array(q0, dtype=np.float64, copy=True)
    A = np.zeros((T, P)) if A0 is None else np.array(A0, dtype=np.float64, copy=True)
    _, qp = _d(q)
    _, Ap = _d(A)
    perm, pp = _i(perm)
    hist = np.zeros(E) if record_loss else None
    hp = _d(hist)[1] if record_loss else _null_d()
    rc = lib().orc_spgd_day(pt.dims, pt.rp_p, pt.ci_p, Wp, xp, qp, Ap, pp, perm.shape[-1], E, chunk,
                            granularity, optimizer, eta, eps, hp)
    if rc != 0:
        raise RuntimeError(f"orc_spgd_day failed ({rc})")
    return q, A, hist


def spgd_step(inst, W, x, q, A, hblocks, optimizer=0, eta=5.0, eps=1e-10):
    """One minibatch on the rows of the listed observation intervals; returns (q, A)."""
    pt = _pat(inst)
    W, Wp = _d(W)
    x, xp = _d(x)
    q = np.array(q, dtype=np.float64, copy=True)
    A = np.array(A, dtype=np.float64, copy=True)
    hb, hbp = _i(hblocks)
    rc = lib().orc_spgd_step(pt.dims, pt.rp_p, pt.ci_p, Wp, xp, _d(q)[1], _d(A)[1], hbp, hb.size,
                             optimizer, eta, eps)
    if rc != 0:
        raise RuntimeError("orc_spgd_step failed")
    return q, A


def spgd(inst, x, perm, E, chunk, days=None, q0=None, A0=None, granularity=0, optimizer=0,
         eta=5.0, eps=1e-10, record_loss=True, nthreads=None, W=None):
    """Algorithm 1 on many days of `inst` (all, or the index list `days`), OpenMP over days.
    perm is [E][C][units].  Returns (Q, A, loss_hist[D][E])."""
    pt = _pat(inst)
    P, L, T, H, K = pt.shape
    days = np.arange(inst.D) if days is None else np.asarray(days)
    D = days.shape[0]
    dc, dcp = _i(inst.day_cluster[days])
    Ws = [np.ascontiguousarray(w, dtype=np.float64) for w in (inst.W if W is None else W)]
    Wptrs = (ctypes.POINTER(ctypes.c_double) * len(Ws))(
        *[w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for w in Ws])
    X, Xp = _d(np.asarray(x)[days])
    Q = np.zeros((D, T, P)) if q0 is None else np.array(q0, dtype=np.float64, copy=True)
    A = np.zeros((D, T, P)) if A0 is None else np.array(A0, dtype=np.float64, copy=True)
    _, Qp = _d(Q)
    _, Ap = _d(A)
    perm, pp = _i(perm)
    hist = np.zeros((D, E)) if record_loss else None
    hp = _d(hist)[1] if record_loss else _null_d()
    nthreads = nthreads or os.cpu_count() or 1
    rc = lib().orc_spgd(pt.dims, D, dcp, pt.rp_p, pt.ci_p, Wptrs, Xp, Qp, Ap, pp,
                        perm.shape[1] * perm.shape[2], perm.shape[2], E, chunk, granularity,
                        optimizer, eta, eps, hp, nthreads)
    if rc != 0:
        raise RuntimeError(f"orc_spgd failed ({rc})")
    return Q, A, hist


def metrics(inst, x, Q, days=None, nthreads=None, W=None):
    """Per-day (loss, kkt, r2) arrays for the days `days` (default all) with demand Q."""
    pt = _pat(inst)
    days = np.arange(inst.D) if days is None else np.asarray(days)
    D = days.shape[0]
    dc, dcp = _i(inst.day_cluster[days])
    Ws = [np.ascontiguousarray(w, dtype=np.float64) for w in (inst.W if W is None else W)]
    Wptrs = (ctypes.POINTER(ctypes.c_double) * len(Ws))(
        *[w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for w in Ws])
    X, Xp = _d(np.asarray(x)[days])
    Q, Qp = _d(Q)
    out = [np.zeros(D) for _ in range(3)]
    ptrs = [_d(o)[1] for o in out]
    lib().orc_metrics(pt.dims, D, dcp, pt.rp_p, pt.ci_p, Wptrs, Xp, Qp, *ptrs,
                      nthreads or os.cpu_count() or 1)
    return tuple(out)


def route_softmax(P, path_od, z):
    path_od, pp = _i(path_od)
    z, zp = _d(z)
    pi = np.zeros(z.shape[0])
    lib().orc_route_softmax(P, z.shape[0], pp, zp, _d(pi)[1])
    return pi


def rho_from_logits(ri, c, z):
    """W[l][t][nz] of cluster c of a RouteInstance under logits z."""
    dims = _dims(ri.P, ri.L, ri.T, ri.H, ri.K)
    po, pop = _i(ri.path_od)
    pp_, ppp = _i(ri.pair_ptr)
    pl, plp = _i(ri.pair_link)
    R, Rp = _d(ri.R[c])
    z, zp = _d(z)
    rp, rpp = _i(ri.row_ptr)
    ci, cip = _i(ri.col_idx)
    W = np.zeros((ri.K, ri.T, ri.nnz))
    rc = lib().orc_rho_from_logits(dims, ri.n_paths, pop, ppp, plp, Rp, zp, rpp, cip, _d(W)[1])
    if rc != 0:
        raise RuntimeError("pair not in pattern")
    return W


def loss_backward(inst, W, X, Q, want_W=True, want_Q=True):
    """(dW [K][T][nnz], dQ [n][T][P]) of sum_d ||rho q_d - x_d||^2 over the n days given."""
    pt = _pat(inst)
    P, L, T, H, K = pt.shape
    W, Wp = _d(W)
    X, Xp = _d(X)
    Q, Qp = _d(Q)
    n = Q.shape[0]
    dW = np.zeros_like(W) if want_W else None
    dQ = np.zeros_like(Q) if want_Q else None
    lib().orc_loss_backward(pt.dims, pt.rp_p, pt.ci_p, Wp, n, Xp, Qp,
                            _d(dW)[1] if want_W else _null_d(), _d(dQ)[1] if want_Q else _null_d())
    return dW, dQ


def logits_backward(ri, c, z, dW):
    dims = _dims(ri.P, ri.L, ri.T, ri.H, ri.K)
    po, pop = _i(ri.path_od)
    pp_, ppp = _i(ri.pair_ptr)
    pl, plp = _i(ri.pair_link)
    R, Rp = _d(ri.R[c])
    z, zp = _d(z)
    rp, rpp = _i(ri.row_ptr)
    ci, cip = _i(ri.col_idx)
    dW, dWp = _d(dW)
    dz = np.zeros(ri.n_paths)
    rc = lib().orc_logits_backward(dims, ri.n_paths, pop, ppp, plp, Rp, zp, rpp, cip, dWp, _d(dz)[1])
    if rc != 0:
        raise RuntimeError("pair not in pattern")
    return dz


def fixed_step_eta(inst, c=0, iters=200):
    """Fixed step 1/lambda_max(rho^T rho) for cluster c: lambda_max from `iters`
    FP64 power-iteration steps on g = rho^T rho v starting at all ones."""
    W = inst.W[c]
    v = np.ones((inst.T, inst.P))
    lam = 0.0
    zero = np.zeros((inst.H, inst.L))
    for _ in range(iters):
        w = grad(inst, W, v, zero)          # rho^T (rho v - 0)
        lam = float(np.sqrt(np.sum(w * w)) / np.sqrt(np.sum(v * v)))
        v = w / np.sqrt(np.sum(w * w))
    return 1.0 / lam


def _walk_flag(walk):
    if walk not in ("f64", "f32"):
        raise ValueError(f"walk must be 'f64' or 'f32', not {walk!r}")
    return 1 if walk == "f32" else 0


def dar_from_speeds(path_ptr, path_link, link_len, speed, dt, H, K, walk="f64"):
    """Dynamic assignment ratios from link speeds (eqs. "dar", "cost"; see
    orc_dar_from_speeds): speed is [n_days][L][H_speed] (or [L][H_speed] for
    one day), link_len [L] in the same distance unit, dt in the time unit of
    length/speed.  Returns Rr[K][H][n_pairs], the mean over the days.

    walk="f32" decides which interval's speed each link is crossed at in
    binary32 (lengths and speeds rounded to binary32, travel times summed in
    binary32), as a single-precision run does; the rest stays FP64."""
    path_ptr, pp = _i(np.asarray(path_ptr))
    path_link, plp = _i(np.asarray(path_link))
    sp = np.asarray(speed, dtype=np.float64)
    if sp.ndim == 2:
        sp = sp[None]
    n_days, L, H_speed = sp.shape
    ln, lnp = _d(np.asarray(link_len, dtype=np.float64))
    sp, spp = _d(sp)
    n_paths = path_ptr.shape[0] - 1
    n_pairs = int(path_ptr[-1])
    out = np.zeros((K, H, n_pairs))
    _, op = _d(out)
    rc = lib().orc_dar_from_speeds(n_paths, pp, plp, L, lnp, spp, n_days, H_speed,
                                   ctypes.c_double(dt), H, K, _walk_flag(walk), op)
    if rc != 0:
        raise RuntimeError(f"orc_dar_from_speeds failed ({rc})")
    return out


def path_costs(path_ptr, path_link, link_len, speed, dt, T, walk="f64"):
    """Mean path travel time per departure interval (eqs. "cost", "logit",
    "rt"; see orc_path_costs): speed [n_days][L][H_speed] (or [L][H_speed]),
    departures at t*dt for t < T.  Returns cost[T][n_paths].  walk as for
    dar_from_speeds (each day's travel time walked in binary32)."""
    path_ptr, pp = _i(np.asarray(path_ptr))
    path_link, plp = _i(np.asarray(path_link))
    sp = np.asarray(speed, dtype=np.float64)
    if sp.ndim == 2:
        sp = sp[None]
    n_days, L, H_speed = sp.shape
    ln, lnp = _d(np.asarray(link_len, dtype=np.float64))
    sp, spp = _d(sp)
    n_paths = path_ptr.shape[0] - 1
    out = np.zeros((T, n_paths))
    _, op = _d(out)
    rc = lib().orc_path_costs(n_paths, pp, plp, L, lnp, spp, n_days, H_speed, ctypes.c_double(dt),
                              T, _walk_flag(walk), op)
    if rc != 0:
        raise RuntimeError(f"orc_path_costs failed ({rc})")
    return out


def logit_portions(P, path_od, theta, cost):
    """Route portions p[T][n_paths] = per-OD softmax of -theta * cost[T][n_paths]
    (eqs. "logit", "rt")."""
    path_od, pop = _i(path_od)
    cost, cp = _d(cost)
    T, n_paths = cost.shape
    out = np.zeros((T, n_paths))
    lib().orc_logit_portions(P, n_paths, pop, T, ctypes.c_double(theta), cp, _d(out)[1])
    return out


def rho_from_portions(P, L, T, H, K, path_od, pair_ptr, pair_link, row_ptr, col_idx, Rr, p):
    """W[K][T][nnz] of eq. "assign" from ratios Rr[K][T][n_pairs] and
    time-dependent portions p[T][n_paths]."""
    dims = _dims(P, L, T, H, K)
    po, pop = _i(path_od)
    pp_, ppp = _i(pair_ptr)
    pl, plp = _i(pair_link)
    R, Rp = _d(Rr)
    pv, pvp = _d(p)
    rp, rpp = _i(row_ptr)
    ci, cip = _i(col_idx)
    W = np.zeros((K, T, ci.shape[0]))
    rc = lib().orc_rho_from_portions(dims, po.shape[0], pop, ppp, plp, Rp, pvp, rpp, cip, _d(W)[1])
    if rc != 0:
        raise RuntimeError("pair not in pattern")
    return W


def dense_loss(B, y, q):
    """||B q - y||^2 of a dense B [m][n]."""
    B, Bp = _d(B)
    y, yp = _d(y)
    q, qp = _d(q)
    return lib().orc_dense_loss(B.shape[0], B.shape[1], Bp, yp, qp)


def dense_spgd(B, y, perms, chunk, eta, eps=1e-10, optimizer=0, q0=None, A0=None):
    """Algorithm 1 on a dense B [m][n] (see orc_dense_spgd); perms [E][m] row
    orders.  Returns (q, A, loss_hist [E])."""
    B, Bp = _d(B)
    y, yp = _d(y)
    m, n = B.shape
    perms, pp = _i(np.asarray(perms).reshape(-1, m) if m else np.zeros((0, 0)))
    E = perms.shape[0]
    q = np.zeros(n) if q0 is None else np.array(q0, dtype=np.float64)
    A = np.zeros(n) if A0 is None else np.array(A0, dtype=np.float64)
    q, qp = _d(q)
    A, Ap = _d(A)
    hist = np.zeros(E)
    rc = lib().orc_dense_spgd(m, n, Bp, yp, qp, Ap, pp, E, chunk, optimizer, ctypes.c_double(eta),
                              ctypes.c_double(eps), _d(hist)[1])
    if rc != 0:
        raise RuntimeError(f"orc_dense_spgd failed ({rc})")
    return q, A, hist
