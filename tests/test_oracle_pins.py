"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the part of the oracle it pins and the fact it uses.  None of
them calls the HIP library.
"""
import itertools

import numpy as np
import pytest
import scipy.optimize
import torch

import oracle as orc
from synth import make_config, make_instance, make_perms, make_route_instance
from synth.instances import make_row_perms


def dense_rho(inst, W):
    """The assignment matrix in the paper's global layout (Table "DODE framework
    variable vectorization"): link-interval row (h2-1)|A|+a, OD-interval column
    (h1-1)|K|+k, written 0-based as row h*L + a, column t*P + p."""
    P, L, T, H, K = inst.P, inst.L, inst.T, inst.H, inst.K
    M = np.zeros((H * L, T * P))
    rows = np.repeat(np.arange(L), np.diff(inst.row_ptr))
    for l in range(K):
        for t in range(T):
            h = t + l
            if h >= H:
                continue
            for j in range(inst.nnz):
                M[h * L + rows[j], t * P + inst.col_idx[j]] = W[l, t, j]
    return M


def tiny(seed, P=2, L=4, T=6, K=3, inc=0.6, days=1, noise="add1", zero_frac=0.0):
    return make_instance(P=P, L=L, T=T, K=K, sizes=(days,), inc=inc, pattern="bernoulli",
                         demand="uniform50", noise=noise, x_dtype="f64", seed=seed,
                         planted_zero_frac=zero_frac)


def full_batch_fixed(inst, x, E, eta, q0=None):
    perm = np.tile(np.arange(inst.H, dtype=np.int32), (E, 1))
    q, _, hist = orc.spgd_day(inst, inst.W[0], x, perm, E, inst.H, q0=q0, optimizer=1, eta=eta)
    return q, hist


def lam_max(M):
    return float(np.linalg.eigvalsh(M.T @ M)[-1])


# ---------------------------------------------------------------- O1 / O3 --
@pytest.mark.parametrize("cid_shape", [dict(P=4, L=6, T=12, K=3, inc=0.5),
                                       dict(P=7, L=9, T=10, K=4, inc=0.3),
                                       dict(P=5, L=8, T=9, K=3, inc=0.4, H=7)])
def test_apply_and_grad_match_global_matrix(cid_shape):
    """O1/O3 against the paper's global vectorised matrix and a library matmul."""
    kw = dict(cid_shape)
    H = kw.pop("H", None)
    inst = make_instance(sizes=(2,), pattern="bernoulli", demand="uniform50", noise="add1",
                         x_dtype="f64", seed=11, H=H, **kw)
    M = dense_rho(inst, inst.W[0])
    rng = np.random.default_rng(0)
    q = rng.uniform(0, 10, (inst.T, inst.P))
    x = inst.x[0]
    xh = orc.apply(inst, inst.W[0], q)
    np.testing.assert_allclose(xh.ravel(), M @ q.ravel(), rtol=1e-13, atol=1e-12)
    g = orc.grad(inst, inst.W[0], q, x)
    np.testing.assert_allclose(g.ravel(), M.T @ (M @ q.ravel() - x.ravel()), rtol=1e-12, atol=1e-10)
    L = orc.loss(inst, inst.W[0], q, x)
    assert abs(L - np.sum((M @ q.ravel() - x.ravel()) ** 2)) <= 1e-12 * L


def test_adjoint_identity_corridor():
    """O1 vs O3: <rho q, r> = <q, rho^T r> at a full corridor day (T=H=288)."""
    inst = make_instance(P=50, L=200, T=288, K=6, sizes=(1,), inc=0.1, pattern="corridor",
                         demand="gamma", noise="mult5", seed=3)
    rng = np.random.default_rng(1)
    q = rng.standard_normal((inst.T, inst.P))
    r = rng.standard_normal((inst.H, inst.L))
    lhs = np.sum(orc.apply(inst, inst.W[0], q) * r)
    rhs = np.sum(q * orc.adjoint(inst, inst.W[0], r))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.sqrt(np.sum(q * q) * np.sum(r * r)))


def test_generator_observation_matches_apply():
    """O1 against the generator's noiseless counts (built with sparse library products)."""
    inst = make_instance(P=50, L=200, T=288, K=6, sizes=(2,), inc=0.1, pattern="corridor",
                         demand="gamma", noise="mult5", seed=4, keep_x0=True)
    for d in range(2):
        np.testing.assert_allclose(orc.apply(inst, inst.W[0], inst.qstar[d]), inst.x0[d],
                                   rtol=1e-12, atol=1e-9)


def test_lag_ratios_sum_to_one():
    """DAR fractions of one departure interval sum to one over arrival intervals
    (eq. "dar"); blocks past the last interval are dropped."""
    inst = make_config(1)
    W = inst.W[0]
    full = W.sum(axis=0)[: inst.T - inst.K + 1]
    np.testing.assert_allclose(full, 1.0, rtol=1e-14)
    assert np.all(W[2, inst.T - 2:] == 0) and np.all(W[1, inst.T - 1:] == 0)


def test_finite_differences_of_loss():
    """O2/O3: g = (1/2) grad of the loss, by central differences."""
    inst = make_config(1)
    rng = np.random.default_rng(2)
    q = rng.uniform(1, 20, (inst.T, inst.P))
    x = inst.x[0]
    g = orc.grad(inst, inst.W[0], q, x)
    h = 1e-4
    for i in rng.choice(inst.T * inst.P, 12, replace=False):
        e = np.zeros(inst.T * inst.P)
        e[i] = h
        e = e.reshape(q.shape)
        fd = (orc.loss(inst, inst.W[0], q + e, x) - orc.loss(inst, inst.W[0], q - e, x)) / (2 * h)
        assert abs(fd - 2 * g.ravel()[i]) <= 1e-6 * (1 + abs(fd))


# ------------------------------------------------------------ O4 optimum --
def brute_force_nnls(M, y):
    """Exact NNLS by enumerating every support and keeping the KKT point."""
    n = M.shape[1]
    best = None
    for mask in itertools.product([0, 1], repeat=n):
        S = np.nonzero(mask)[0]
        q = np.zeros(n)
        if S.size:
            qs, *_ = np.linalg.lstsq(M[:, S], y, rcond=None)
            if np.any(qs < -1e-12):
                continue
            q[S] = np.maximum(qs, 0)
        g = M.T @ (M @ q - y)
        free = np.setdiff1d(np.arange(n), S)
        if free.size and np.any(g[free] < -1e-9 * (1 + np.abs(M.T @ y).max())):
            continue
        val = np.sum((M @ q - y) ** 2)
        if best is None or val < best[0]:
            best = (val, q)
    return best


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_brute_force_active_set(seed):
    """P1: a long full-batch fixed-step run reaches the enumerated NNLS optimum."""
    inst = tiny(seed)
    M = dense_rho(inst, inst.W[0])
    y = inst.x[0].ravel().copy()
    y[::3] *= 0.2          # push some constraints active
    Lstar, qstar = brute_force_nnls(M, y)
    ev = np.linalg.eigvalsh(M.T @ M)
    E = int(min(400000, 40 * ev[-1] / max(ev[0], 1e-12)))
    q, hist = full_batch_fixed(inst, y.reshape(inst.H, inst.L), E, 1.0 / ev[-1])
    assert abs(hist[-1] - Lstar) <= 1e-10 * max(Lstar, 1.0)
    np.testing.assert_allclose(M @ q.ravel(), M @ qstar, rtol=1e-8, atol=1e-8)


def test_scipy_nnls_config1():
    """P2: Lawson-Hanson (scipy.optimize.nnls) on the config-1 days (72 x 48)."""
    inst = make_config(1)
    M = dense_rho(inst, inst.W[0])
    eta = 1.0 / lam_max(M)
    ev = np.linalg.eigvalsh(M.T @ M)
    E = int(min(300000, 40 * ev[-1] / ev[0]))
    for d in range(inst.D):
        y = inst.x[d].ravel()
        qs, rn = scipy.optimize.nnls(M, y, maxiter=5000)
        q, hist = full_batch_fixed(inst, inst.x[d], E, eta)
        assert abs(hist[-1] - rn ** 2) <= 1e-8 * rn ** 2
        np.testing.assert_allclose(M @ q.ravel(), M @ qs, rtol=1e-6, atol=1e-6)
        assert orc.kkt(inst, inst.W[0], q, inst.x[d]) <= 1e-6 * np.abs(M.T @ y).max()


@pytest.mark.parametrize("zero_frac", [0.0, 0.3])
def test_planted_recovery(zero_frac):
    """P3: noiseless data from a planted q* with full column rank is recovered."""
    inst = tiny(21, P=3, L=8, T=8, K=3, inc=0.6, noise="none", zero_frac=zero_frac)
    M = dense_rho(inst, inst.W[0])
    s = np.linalg.svd(M, compute_uv=False)
    assert s[-1] > 1e-3 * s[0]
    ev = s ** 2
    E = int(min(400000, 60 * ev[0] / ev[-1]))
    q, hist = full_batch_fixed(inst, inst.x0[0], E, 1.0 / ev[0])
    np.testing.assert_allclose(q, inst.qstar[0], rtol=1e-7, atol=1e-6)
    assert hist[-1] <= 1e-12 * np.sum(inst.x0[0] ** 2)
    # Adagrad from zero also drives the loss down on the same data
    perm = make_perms(9, 3000, 1, inst.H)[:, 0]
    _, _, h2 = orc.spgd_day(inst, inst.W[0], inst.x0[0], perm, 3000, 2, eta=1.0)
    assert h2[-1] < 1e-3 * h2[0]


def test_kkt_at_zero_is_max_back_projection():
    """P4 closed form: at q = 0 and x >= 0, g = -rho^T x <= 0 and the KKT residual is max(rho^T x)."""
    inst = make_config(1)
    M = dense_rho(inst, inst.W[0])
    q0 = np.zeros((inst.T, inst.P))
    for d in range(3):
        assert abs(orc.kkt(inst, inst.W[0], q0, inst.x[d]) - (M.T @ inst.x[d].ravel()).max()) <= 1e-12 * 1e3


def test_r2_against_sklearn():
    """Step 6 R^2 against sklearn's r2_score."""
    from sklearn.metrics import r2_score
    inst = make_config(1)
    rng = np.random.default_rng(5)
    q = rng.uniform(0, 30, (inst.T, inst.P))
    xh = orc.apply(inst, inst.W[0], q)
    for d in range(2):
        assert abs(orc.r2(inst, inst.W[0], q, inst.x[d]) - r2_score(inst.x[d].ravel(), xh.ravel())) < 1e-12


# ----------------------------------------------------- O4 closed forms --
def identity_instance(P=5, T=4):
    """K=1, L=P, rho = I: every row is its own coordinate."""
    inst = make_instance(P=P, L=P, T=T, K=1, sizes=(1,), inc=1.0, pattern="bernoulli",
                         demand="uniform50", noise="add1", x_dtype="f64", seed=1)
    inst.row_ptr = np.arange(P + 1, dtype=np.int32)
    inst.col_idx = np.arange(P, dtype=np.int32)
    inst.W = [np.ones((1, T, P))]
    return inst


def test_identity_fixed_step_closed_form():
    """P7(i): rho = I, one full-batch fixed step with eta = 1 from any q0 gives max(x, 0)."""
    inst = identity_instance()
    rng = np.random.default_rng(3)
    x = rng.standard_normal((inst.H, inst.L)) * 5
    q0 = rng.uniform(-3, 3, (inst.T, inst.P))
    q, _ = full_batch_fixed(inst, x, 1, 1.0, q0=q0)
    np.testing.assert_allclose(q, np.maximum(x, 0), rtol=1e-15, atol=1e-14)


def test_first_adagrad_step_closed_form():
    """P7(ii): from q0 = 0 the first Adagrad step is eta |g| / (|g| + eps) where g < 0, else 0."""
    inst = make_config(1)
    eta, eps = 0.7, 1e-10
    perm = np.tile(np.arange(inst.H, dtype=np.int32), (1, 1))
    for d in range(3):
        g = orc.grad(inst, inst.W[0], np.zeros((inst.T, inst.P)), inst.x[d])
        q, A, _ = orc.spgd_day(inst, inst.W[0], inst.x[d], perm, 1, inst.H, optimizer=0, eta=eta, eps=eps)
        expect = np.where(g < 0, eta * np.abs(g) / (np.abs(g) + eps), 0.0)
        np.testing.assert_allclose(q, expect, rtol=1e-15, atol=0)
        np.testing.assert_array_equal(A, g * g)


def test_identity_adagrad_scalar_recursion():
    """Separable special case: with rho = I and minibatches of whole intervals,
    each coordinate sees exactly one 1-D Adagrad step per epoch on (q - x)^2/2."""
    inst = identity_instance(P=3, T=6)
    rng = np.random.default_rng(8)
    x = rng.uniform(0, 4, (inst.H, inst.L))
    E, eta, eps = 7, 0.9, 1e-10
    perm = make_perms(12, E, 1, inst.H)[:, 0]
    q, A, _ = orc.spgd_day(inst, inst.W[0], x, perm, E, 2, optimizer=0, eta=eta, eps=eps)
    for i in range(inst.T * inst.P):
        qi, ai, xi = 0.0, 0.0, x.ravel()[i]
        for _ in range(E):
            g = qi - xi
            ai += g * g
            qi = max(qi - eta * g / (np.sqrt(ai) + eps), 0.0)
        assert abs(q.ravel()[i] - qi) <= 1e-13 * (1 + abs(qi))


def dense_spgd_torch(M, y, perms, chunk_rows_fn, E, eta, L):
    """Algorithm 1 written with torch's Adagrad (the paper's implementation
    platform) on the dense global matrix: per minibatch set x.grad = B_o^T(B_o x - y_o),
    take optimizer.step(), then clamp at zero."""
    Mt = torch.from_numpy(M)
    yt = torch.from_numpy(y)
    xv = torch.zeros(M.shape[1], dtype=torch.float64, requires_grad=False)
    opt = torch.optim.Adagrad([xv], lr=eta, eps=1e-10)
    for e in range(E):
        for rows in chunk_rows_fn(perms[e]):
            Bo = Mt[rows]
            g = Bo.T @ (Bo @ xv - yt[rows])
            xv.grad = g
            opt.step()
            with torch.no_grad():
                xv.clamp_(min=0.0)
    return xv.numpy()


@pytest.mark.parametrize("granularity", [0, 1])
def test_spgd_matches_torch_adagrad(granularity):
    """O4 end to end (permutation use, minibatch slicing incl. the short tail,
    Adagrad constants, projection) against torch.optim.Adagrad."""
    inst = make_config(1)
    M = dense_rho(inst, inst.W[0])
    E, eta = 6, 2.0
    L, H = inst.L, inst.H
    if granularity == 0:
        chunk = 5    # 12 blocks -> minibatches of 5, 5, 2
        perms = make_perms(77, E, 1, H)[:, 0]
        fn = lambda pe: [np.concatenate([np.arange(h * L, (h + 1) * L) for h in pe[s:s + chunk]])
                         for s in range(0, H, chunk)]
    else:
        chunk = 17   # 72 rows -> 17, 17, 17, 17, 4
        perms = make_row_perms(78, E, H * L)
        fn = lambda pe: [pe[s:s + chunk] for s in range(0, H * L, chunk)]
    for d in range(2):
        ref = dense_spgd_torch(M, inst.x[d].ravel(), perms, fn, E, eta, L)
        q, _, _ = orc.spgd_day(inst, inst.W[0], inst.x[d], perms, E, chunk, granularity=granularity,
                               optimizer=0, eta=eta)
        np.testing.assert_allclose(q.ravel(), ref, rtol=1e-10, atol=1e-10)


def test_adagrad_gradient_scale_invariance():
    """P8: scaling rho and x by 2 multiplies g by 4; the Adagrad iterates are
    unchanged up to eps (a wrong accumulator or missing square root fails)."""
    inst = make_config(1)
    E = 20
    perm = make_perms(31, E, 1, inst.H)[:, 0]
    q1, _, _ = orc.spgd_day(inst, inst.W[0], inst.x[0], perm, E, 4, eta=3.0)
    q2, _, _ = orc.spgd_day(inst, 2 * inst.W[0], 2 * inst.x[0], perm, E, 4, eta=3.0)
    np.testing.assert_allclose(q1, q2, rtol=1e-9, atol=1e-9)
    # and the fixed step scales its rate by 1/4 instead
    q3, _, _ = orc.spgd_day(inst, inst.W[0], inst.x[0], perm, E, 4, optimizer=1, eta=0.01)
    q4, _, _ = orc.spgd_day(inst, 2 * inst.W[0], 2 * inst.x[0], perm, E, 4, optimizer=1, eta=0.0025)
    np.testing.assert_allclose(q3, q4, rtol=1e-12, atol=1e-12)


def test_day_independence_bitwise():
    """P9: solving days jointly equals solving them one at a time, bit for bit."""
    inst = make_instance(P=6, L=10, T=16, K=3, sizes=(3, 2), inc=0.4, pattern="bernoulli",
                         demand="uniform50", noise="add1", x_dtype="f64", seed=44)
    E = 5
    perms = make_perms(45, E, inst.C, inst.H)
    Q, A, hist = orc.spgd(inst, inst.x, perms, E, 3, nthreads=4)
    for d in range(inst.D):
        c = inst.day_cluster[d]
        q, a, h = orc.spgd_day(inst, inst.W[c], inst.x[d], perms[:, c], E, 3)
        np.testing.assert_array_equal(Q[d], q)
        np.testing.assert_array_equal(hist[d], h)


def test_single_minibatch_rows_equal_blocks():
    """P10: with one minibatch per epoch, row and block minibatches coincide."""
    inst = make_config(1)
    E = 4
    pb = make_perms(50, E, 1, inst.H)[:, 0]
    pr = make_row_perms(51, E, inst.H * inst.L)
    q1, _, h1 = orc.spgd_day(inst, inst.W[0], inst.x[0], pb, E, inst.H, granularity=0, eta=2.0)
    q2, _, h2 = orc.spgd_day(inst, inst.W[0], inst.x[0], pr, E, inst.H * inst.L, granularity=1, eta=2.0)
    np.testing.assert_allclose(q1, q2, rtol=1e-12, atol=1e-12)


def test_loss_history_decreases_config1_fixed_step():
    inst = make_config(1)
    M = dense_rho(inst, inst.W[0])
    perm = make_perms(inst.seed + 1, 200, 1, inst.H)[:, 0]
    _, _, h = orc.spgd_day(inst, inst.W[0], inst.x[0], perm, 200, inst.H, optimizer=1,
                           eta=1.0 / lam_max(M))
    assert np.all(np.diff(h) <= 1e-9 * h[:-1])


# ------------------------------------------------------------------ O6 --
def test_route_softmax_against_scipy():
    from scipy.special import softmax
    ri = make_route_instance()
    pi = orc.route_softmax(ri.P, ri.path_od, ri.z0[0])
    for p in range(ri.P):
        ks = ri.path_od == p
        np.testing.assert_allclose(pi[ks], softmax(ri.z0[0][ks]), rtol=1e-14)


def test_rho_from_uniform_logits_closed_form():
    """With equal logits, sum over lags of rho(z) at (a, p) is (#paths of p
    through a) / (#paths of p), since each path's lag ratios sum to one."""
    ri = make_route_instance()
    W = orc.rho_from_logits(ri, 0, np.zeros(ri.n_paths))
    rows = np.repeat(np.arange(ri.L), np.diff(ri.row_ptr))
    tsafe = ri.T - ri.K + 1
    for j in range(ri.nnz):
        a, p = rows[j], ri.col_idx[j]
        ks = np.nonzero(ri.path_od == p)[0]
        through = sum(1 for k in ks if a in ri.pair_link[ri.pair_ptr[k]:ri.pair_ptr[k + 1]])
        np.testing.assert_allclose(W[:, :tsafe, j].sum(axis=0), through / ks.size, rtol=1e-13)


def test_route_and_rho_gradients_by_finite_differences():
    """O6: dL/dW, dL/dQ and dL/dz against central differences of the loss."""
    ri = make_route_instance()
    z = ri.z0[0]
    W = orc.rho_from_logits(ri, 0, z)
    Q = ri.qstar * 0.9
    X = ri.x

    def total(Wv, Qv):
        return sum(orc.loss(ri, Wv, Qv[d], X[d]) for d in range(ri.D))

    dW, dQ = orc.loss_backward(ri, W, X, Q)
    rng = np.random.default_rng(9)
    h = 1e-5
    for _ in range(6):
        l, t, j = rng.integers(ri.K), rng.integers(ri.T - ri.K), rng.integers(ri.nnz)
        Wp, Wm = W.copy(), W.copy()
        Wp[l, t, j] += h
        Wm[l, t, j] -= h
        fd = (total(Wp, Q) - total(Wm, Q)) / (2 * h)
        assert abs(fd - dW[l, t, j]) <= 1e-5 * (1 + abs(fd))
        d, t2, p = rng.integers(ri.D), rng.integers(ri.T), rng.integers(ri.P)
        Qp, Qm = Q.copy(), Q.copy()
        Qp[d, t2, p] += h
        Qm[d, t2, p] -= h
        fd = (total(W, Qp) - total(W, Qm)) / (2 * h)
        assert abs(fd - dQ[d, t2, p]) <= 1e-5 * (1 + abs(fd))
    dz = orc.logits_backward(ri, 0, z, dW)
    for k in rng.choice(ri.n_paths, 8, replace=False):
        zp, zm = z.copy(), z.copy()
        zp[k] += h
        zm[k] -= h
        fd = (total(orc.rho_from_logits(ri, 0, zp), Q) - total(orc.rho_from_logits(ri, 0, zm), Q)) / (2 * h)
        assert abs(fd - dz[k]) <= 1e-5 * (1 + abs(fd))


def test_oracle_resume_is_bitwise():
    """Stopping the oracle after E1 epochs and continuing from its (Q, A) with
    the remaining epochs' permutations gives the uninterrupted run bit for bit."""
    from synth import make_instance, make_perms, chunk_h_blocks
    inst = make_instance(P=6, L=10, T=16, K=3, sizes=(3, 2), inc=0.4, pattern="bernoulli",
                         demand="uniform50", noise="add1", x_dtype="f64", seed=71)
    E, E1 = 9, 4
    perms = make_perms(72, E, inst.C, inst.H)
    bh = chunk_h_blocks(inst.L, inst.H, 25)
    Qa, Aa, _ = orc.spgd(inst, inst.x, perms, E, bh, optimizer=0, eta=2.0)
    Q1, A1, _ = orc.spgd(inst, inst.x, perms[:E1], E1, bh, optimizer=0, eta=2.0)
    Qb, Ab, _ = orc.spgd(inst, inst.x, perms[E1:], E - E1, bh, optimizer=0, eta=2.0, q0=Q1, A0=A1)
    np.testing.assert_array_equal(Qa, Qb)
    np.testing.assert_array_equal(Aa, Ab)


# ------------------------------------------- helpers the GPU tests rely on --
@pytest.mark.parametrize("shape", [dict(P=4, L=6, T=12, K=3, inc=0.5, bh=5),
                                   dict(P=7, L=9, T=10, K=4, inc=0.3, bh=3, H=8)])
def test_spgd_step_chain_equals_spgd_day(shape):
    """orc_spgd_step against the pinned orc_spgd_day (Algorithm 1): running
    spgd_step on the consecutive b_h-interval slices of each epoch's permutation
    (the last one shorter) reproduces spgd_day bit for bit, for both optimizers."""
    kw = dict(shape)
    bh = kw.pop("bh")
    H = kw.pop("H", None)
    inst = make_instance(sizes=(1,), pattern="bernoulli", demand="uniform50", noise="add1",
                         x_dtype="f64", seed=31, H=H, **kw)
    E = 4
    perm = make_perms(77, E, 1, inst.H)[:, 0]
    x = inst.x[0]
    for optimizer, eta in ((0, 2.0), (1, 0.02)):
        q_day, A_day, _ = orc.spgd_day(inst, inst.W[0], x, perm, E, bh, optimizer=optimizer,
                                       eta=eta, record_loss=False)
        q = np.zeros((inst.T, inst.P))
        A = np.zeros((inst.T, inst.P))
        for e in range(E):
            for s in range(0, inst.H, bh):
                q, A = orc.spgd_step(inst, inst.W[0], x, q, A, perm[e, s:s + bh],
                                     optimizer=optimizer, eta=eta)
        assert np.array_equal(q, q_day) and np.array_equal(A, A_day)


def test_spgd_step_against_dense_minibatch():
    """orc_spgd_step on the rows of the listed intervals, against the minibatch
    written with the paper's global matrix (Table "DODE framework variable
    vectorization") and a library matmul: r = M_S q - x_S, g = M_S^T r, then
    Adagrad (eps after the square root) and max(q, 0) (Algorithm 1)."""
    inst = make_config(1)
    M = dense_rho(inst, inst.W[0])
    rng = np.random.default_rng(12)
    q = rng.uniform(0, 20, (inst.T, inst.P))
    A = rng.uniform(0, 5, (inst.T, inst.P))
    x = inst.x[0]
    hb = np.array([7, 2, 10], dtype=np.int32)
    rows = (hb[:, None] * inst.L + np.arange(inst.L)[None, :]).ravel()
    MS = M[rows]
    g = MS.T @ (MS @ q.ravel() - x.ravel()[rows])
    eta, eps = 3.0, 1e-10
    A_ref = A.ravel() + g * g
    q_ref = np.maximum(q.ravel() - eta * g / (np.sqrt(A_ref) + eps), 0.0)
    q1, A1 = orc.spgd_step(inst, inst.W[0], x, q, A, hb, optimizer=0, eta=eta, eps=eps)
    np.testing.assert_allclose(A1.ravel(), A_ref, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(q1.ravel(), q_ref, rtol=1e-12, atol=1e-11)
    # untouched coordinates (g = 0) keep their value
    untouched = np.abs(g) == 0
    assert untouched.any()
    assert np.array_equal(q1.ravel()[untouched], q.ravel()[untouched])
    q2, _ = orc.spgd_step(inst, inst.W[0], x, q, A, hb, optimizer=1, eta=0.01)
    np.testing.assert_allclose(q2.ravel(), np.maximum(q.ravel() - 0.01 * g, 0.0), rtol=1e-12,
                               atol=1e-11)


@pytest.mark.parametrize("cid_seed", [(1, None), (1, 5), (4, None)])
def test_fixed_step_eta_is_inverse_lambda_max(cid_seed):
    """The fixed step of the config-1 reading: 1/lambda_max(rho^T rho), against a
    library symmetric eigensolver on the global matrix."""
    cid, seed = cid_seed
    if cid == 1:
        inst = make_config(1, seed=seed) if seed else make_config(1)
    else:
        inst = make_instance(P=5, L=7, T=9, K=3, sizes=(1,), inc=0.5, pattern="bernoulli",
                             demand="uniform50", noise="add1", x_dtype="f64", seed=44)
    M = dense_rho(inst, inst.W[0])
    lam = float(np.linalg.eigvalsh(M.T @ M)[-1])
    assert abs(orc.fixed_step_eta(inst) * lam - 1.0) <= 1e-10


def test_metrics_interleaved_clusters():
    """orc_metrics with the days of three clusters interleaved: every day takes
    its own cluster's matrix.  Loss, KKT residual and R^2 (Step 6 "Quality
    check") against the global matrix of that cluster, written out with numpy,
    and R^2 against a library routine."""
    from sklearn.metrics import r2_score
    inst = make_instance(P=4, L=6, T=12, K=3, sizes=(3, 2, 2), inc=0.5, pattern="bernoulli",
                         demand="uniform50", noise="add1", x_dtype="f64", seed=52)
    days = np.array([0, 3, 5, 1, 6, 2, 4])
    assert len(set(inst.day_cluster[days][:3])) == 3
    rng = np.random.default_rng(3)
    Q = rng.uniform(0, 30, (days.size, inst.T, inst.P))
    Q[:, :, 0] = 0.0
    loss, kkt, r2 = orc.metrics(inst, inst.x, Q, days=days, nthreads=2)
    for i, d in enumerate(days):
        c = int(inst.day_cluster[d])
        M = dense_rho(inst, inst.W[c])
        y = inst.x[d].ravel()
        r = M @ Q[i].ravel() - y
        g = M.T @ r
        assert abs(loss[i] - r @ r) <= 1e-12 * (r @ r)
        assert abs(kkt[i] - np.max(np.abs(np.minimum(Q[i].ravel(), g)))) <= 1e-12 * np.abs(g).max()
        assert abs(r2[i] - r2_score(y, M @ Q[i].ravel())) <= 1e-12
        # a different cluster's matrix gives a different loss: the pick matters
        other = dense_rho(inst, inst.W[(c + 1) % inst.C])
        ro = other @ Q[i].ravel() - y
        assert abs(ro @ ro - loss[i]) > 1e-6 * loss[i]
