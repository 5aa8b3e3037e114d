"""GPU parity: the HIP library through its C ABI against the FP64 oracle.

Bars (element by element unless stated):
  FP64 storage  kernels 1e-12 relative to the largest entry; solve loss <= 1e-6
                relative (final and history), demand 1e-8
  FP32 storage  kernels 2e-6 (ratios rounded to float on both sides); solve
                final loss <= 1e-3 relative per day
  BF16 / FP8    the library's kernels against the oracle run on the same
                rounded ratios (values computed independently in the test);
                solve final loss <= 1e-3 relative per day
"""
import numpy as np
import pytest

import oracle as orc
import paper_1901_09266_amd as dode
from synth import make_config, make_instance, make_perms, chunk_h_blocks
from gpu_helpers import say, make_dar, dev, rel, dequantized_values

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = {
    "config1": dict(P=4, L=6, T=12, K=3, sizes=(7,), inc=0.5, pattern="bernoulli"),
    "ragged": dict(P=37, L=300, T=20, H=17, K=4, sizes=(3,), inc=0.1, pattern="bernoulli"),
    "wideP": dict(P=70, L=5, T=9, H=12, K=3, sizes=(2,), inc=0.5, pattern="bernoulli"),
    "corridor": dict(P=50, L=200, T=40, K=6, sizes=(4,), inc=0.1, pattern="corridor"),
    "Tlt K": dict(P=3, L=4, T=2, H=5, K=4, sizes=(2,), inc=0.6, pattern="bernoulli"),
}


def inst_of(name, seed=1234, noise="add1"):
    kw = dict(SHAPES[name])
    return make_instance(demand="uniform50", noise=noise, x_dtype="f64", seed=seed, **kw)


def oracle_rows(inst, Wl, Q):
    xh = np.stack([orc.apply(inst, Wl[inst.day_cluster[d]], Q[d]) for d in range(Q.shape[0])])
    g = np.stack([orc.grad(inst, Wl[inst.day_cluster[d]], Q[d], inst.x[d]) for d in range(Q.shape[0])])
    ls = np.array([orc.loss(inst, Wl[inst.day_cluster[d]], Q[d], inst.x[d]) for d in range(Q.shape[0])])
    return xh, g, ls


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "fp8"])
def test_kernels_match_oracle(name, storage):
    inst = inst_of(name)
    say("kernels", name, storage)
    Wq = dequantized_values(inst, storage)
    dt = torch.float64 if storage == "f64" else torch.float32
    rng = np.random.default_rng(5)
    Q = rng.uniform(0, 20, (inst.D, inst.T, inst.P))
    if storage != "f64":
        Q = Q.astype(np.float32).astype(np.float64)
    X = inst.x if storage == "f64" else inst.x.astype(np.float32).astype(np.float64)
    xh_o, g_o, l_o = oracle_rows(inst, Wq, Q) if storage == "f64" else (None, None, None)
    if storage != "f64":
        xh_o = np.stack([orc.apply(inst, Wq[0], Q[d]) for d in range(inst.D)])
        g_o = np.stack([orc.grad(inst, Wq[0], Q[d], X[d]) for d in range(inst.D)])
        l_o = np.array([orc.loss(inst, Wq[0], Q[d], X[d]) for d in range(inst.D)])
    dar = make_dar(inst, storage)
    Qd, Xd = dev(Q, dt), dev(X, dt)
    Xh = torch.empty((inst.D, inst.H, inst.L), dtype=dt, device="cuda")
    G = torch.empty((inst.D, inst.T, inst.P), dtype=dt, device="cuda")
    loss = torch.empty(inst.D, dtype=torch.float64, device="cuda")
    dode.dode_apply(dar, 0, Qd, Xh)
    dode.dode_grad(dar, 0, Qd, Xd, G)
    dode.dode_loss(dar, 0, Qd, Xd, loss)
    torch.cuda.synchronize()
    tol = 1e-12 if storage == "f64" else 2e-6
    assert rel(Xh.cpu().numpy(), xh_o) <= tol
    assert rel(G.cpu().numpy(), g_o) <= (tol if storage == "f64" else 1e-4)
    np.testing.assert_allclose(loss.cpu().numpy(), l_o, rtol=1e-12 if storage == "f64" else 1e-4)


@pytest.mark.parametrize("name", ["config1", "ragged", "corridor"])
def test_metrics_match_oracle(name):
    inst = inst_of(name)
    say("metrics", name)
    rng = np.random.default_rng(6)
    Q = rng.uniform(0, 20, (inst.D, inst.T, inst.P))
    lo, ko, ro = orc.metrics(inst, inst.x, Q)
    dar = make_dar(inst, "f64")
    out = [torch.empty(inst.D, dtype=torch.float64, device="cuda") for _ in range(3)]
    dode.dode_metrics(dar, 0, dev(Q, torch.float64), dev(inst.x, torch.float64), *out)
    torch.cuda.synchronize()
    np.testing.assert_allclose(out[0].cpu().numpy(), lo, rtol=1e-12)
    np.testing.assert_allclose(out[1].cpu().numpy(), ko, rtol=1e-10)
    np.testing.assert_allclose(out[2].cpu().numpy(), ro, rtol=1e-12)


def test_spgd_step_matches_oracle():
    inst = inst_of("ragged")
    say("spgd_step ragged")
    rng = np.random.default_rng(7)
    Q0 = rng.uniform(0, 5, (inst.D, inst.T, inst.P))
    A0 = rng.uniform(0, 2, (inst.D, inst.T, inst.P))
    chunk = np.array([16, 3, 9, 0, 4], dtype=np.int32)
    for opt in (0, 1):
        dar = make_dar(inst, "f64")
        Qd, Ad = dev(Q0, torch.float64), dev(A0, torch.float64)
        p = dode.make_params(eta=0.3 if opt == 0 else 1e-3, optimizer=opt)
        dode.spgd_step(dar, 0, chunk, dev(inst.x, torch.float64), Qd, Ad, p)
        torch.cuda.synchronize()
        for d in range(inst.D):
            q, A = orc.spgd_step(inst, inst.W[0], inst.x[d], Q0[d], A0[d], chunk, optimizer=opt,
                                 eta=p.eta)
            assert rel(Qd[d].cpu().numpy(), q) <= 1e-12
            if opt == 0:
                assert rel(Ad[d].cpu().numpy(), A) <= 1e-12


def run_solve(inst, storage, E, batch_rows, eta, optimizer, perms, loss_hist=True, days=None,
              seed=0):
    dt = torch.float64 if storage == "f64" else torch.float32
    dar = make_dar(inst, storage)
    D = inst.D
    Xd = dev(inst.x, dt)
    Qd = torch.zeros((D, inst.T, inst.P), dtype=dt, device="cuda")
    Ad = torch.zeros_like(Qd)
    p = dode.make_params(epochs=E, batch_rows=batch_rows, eta=eta, optimizer=optimizer)
    hist = dode.spgd_solve(dar, inst.day_cluster, Xd, Qd, Ad, p, perm=perms, seed=seed,
                           loss_hist=loss_hist)
    torch.cuda.synchronize()
    return Qd.cpu().numpy().astype(np.float64), Ad.cpu().numpy().astype(np.float64), hist


def splitmix64_perms(seed, E, C, H):
    """The permutations the library draws when none are passed: one SplitMix64
    stream (Steele, Lea and Flood, "Fast splittable pseudorandom number
    generators", 2014) started at `seed`; for each (epoch, cluster) in order,
    a Fisher-Yates shuffle of 0..H-1 from the top, element i swapping with
    element (next draw mod (i + 1)) for i = H-1 down to 1."""
    M = (1 << 64) - 1
    s = seed & M
    out = np.empty((E, C, H), dtype=np.int32)
    for e in range(E):
        for c in range(C):
            p = list(range(H))
            for i in range(H - 1, 0, -1):
                s = (s + 0x9E3779B97F4A7C15) & M
                z = ((s ^ (s >> 30)) * 0xBF58476D1CE4E5B9) & M
                z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
                z ^= z >> 31
                j = z % (i + 1)
                p[i], p[j] = p[j], p[i]
            out[e, c] = p
    return out


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_library_drawn_permutations(storage):
    """perm = NULL: the library draws its permutations from the seed.  They
    are the SplitMix64 + Fisher-Yates draw above (so valid permutations): the
    solve equals the one given those permutations bit for bit, the same seed
    repeats, another seed differs, and the FP64 run matches the oracle."""
    inst = make_instance(P=20, L=40, T=24, K=4, sizes=(5, 3), inc=0.2, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f64", seed=56)
    say("library permutations", storage)
    E, seed, rows = 6, 0x5EED1901, 200
    perms = splitmix64_perms(seed, E, inst.C, inst.H)
    for e in range(E):
        for c in range(inst.C):
            assert sorted(perms[e, c]) == list(range(inst.H))
    drawn = run_solve(inst, storage, E, rows, 5.0, 0, None, seed=seed)
    given = run_solve(inst, storage, E, rows, 5.0, 0, perms)
    again = run_solve(inst, storage, E, rows, 5.0, 0, None, seed=seed)
    other = run_solve(inst, storage, E, rows, 5.0, 0, None, seed=seed + 1)
    for a, b in zip(drawn, given):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(drawn, again):
        np.testing.assert_array_equal(a, b)
    assert not np.array_equal(drawn[0], other[0])
    if storage == "f64":
        bh = chunk_h_blocks(inst.L, inst.H, rows)
        Qo, _, ho = orc.spgd(inst, inst.x, perms, E, bh, optimizer=0, eta=5.0)
        assert rel(drawn[0], Qo) <= 1e-8
        assert np.max(np.abs(drawn[2] - ho) / ho) <= 1e-9


def test_solve_config1_fixed_step_f64():
    """Config 1: FP64, fixed step 1/lambda_max, 200 epochs, full batch."""
    inst = make_config(1)
    say("solve config1 f64")
    E = 200
    eta = orc.fixed_step_eta(inst)
    perms = make_perms(inst.seed + 1, E, inst.C, inst.H)
    bh = chunk_h_blocks(inst.L, inst.H, 8192)
    Qo, Ao, ho = orc.spgd(inst, inst.x, perms, E, bh, optimizer=1, eta=eta)
    Qg, Ag, hg = run_solve(inst, "f64", E, 8192, eta, 1, perms)
    assert np.max(np.abs(hg - ho) / ho) <= 1e-6
    assert np.max(np.abs(hg[:, -1] - ho[:, -1]) / ho[:, -1]) <= 1e-10
    assert rel(Qg, Qo) <= 1e-8


@pytest.mark.parametrize("batch_rows", [35, 8192])
def test_solve_adagrad_multicluster_f64(batch_rows):
    """Several clusters of uneven size, several minibatches with a short tail."""
    inst = make_instance(P=6, L=10, T=16, K=3, sizes=(3, 2, 1), inc=0.4, pattern="bernoulli",
                         demand="uniform50", noise="add1", x_dtype="f64", seed=44)
    say("solve multicluster f64", batch_rows)
    E, eta = 25, 2.0
    perms = make_perms(45, E, inst.C, inst.H)
    bh = chunk_h_blocks(inst.L, inst.H, batch_rows)
    Qo, Ao, ho = orc.spgd(inst, inst.x, perms, E, bh, optimizer=0, eta=eta)
    Qg, Ag, hg = run_solve(inst, "f64", E, batch_rows, eta, 0, perms)
    assert np.max(np.abs(hg - ho) / ho) <= 1e-6
    assert rel(Qg, Qo) <= 1e-8
    assert rel(Ag, Ao) <= 1e-8


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_solve_is_deterministic(storage):
    inst = make_instance(P=20, L=40, T=24, K=4, sizes=(5, 3), inc=0.2, pattern="corridor",
                         demand="gamma", noise="mult5", seed=46)
    say("determinism", storage)
    perms = make_perms(47, 10, inst.C, inst.H)
    a = run_solve(inst, storage, 10, 200, 5.0, 0, perms)
    b = run_solve(inst, storage, 10, 200, 5.0, 0, perms)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[2], b[2])


@pytest.mark.parametrize("storage", ["f32", "bf16", "fp8"])
def test_solve_config2_shape_reduced_precision(storage):
    """Config-2 shapes (50 OD, 200 links, 288 intervals, K=6), 12 days, Adagrad
    eta 5, b 8192 (40 intervals per minibatch), 300 epochs."""
    inst = make_config(2, sizes=(12,))
    say("solve config2-shape", storage)
    E = 300
    perms = make_perms(inst.seed + 1, E, inst.C, inst.H)
    bh = chunk_h_blocks(inst.L, inst.H, 8192)
    Wq = dequantized_values(inst, storage)
    x64 = inst.x.astype(np.float64)
    Qo, _, ho = orc.spgd(inst, x64, perms, E, bh, optimizer=0, eta=5.0, W=Wq)
    Qg, _, hg = run_solve(inst, storage, E, 8192, 5.0, 0, perms)
    # final loss of the GPU demand, evaluated in FP64 with the library's ratios
    lg, _, _ = orc.metrics(inst, x64, Qg, W=Wq)
    lo = ho[:, -1]
    assert np.max(np.abs(lg - lo) / lo) <= 1e-3
    # and the history the library reports
    assert np.max(np.abs(hg[:, -1] - lo) / lo) <= 1e-3


def test_nonfinite_observations_rejected():
    inst = inst_of("config1")
    say("nonfinite")
    x = inst.x.copy()
    x[2, 3, 1] = np.nan
    dar = make_dar(inst, "f64")
    Q = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float64, device="cuda")
    A = torch.zeros_like(Q)
    with pytest.raises(dode.DodeError, match="NONFINITE"):
        dode.spgd_solve(dar, inst.day_cluster, dev(x, torch.float64), Q, A, dode.make_params(epochs=2))


MFMA_SHAPES = {
    # 16-row tiles with ragged ends on both sides, a 3-day, a 33-day and a
    # 17-day cluster (every cluster has more than 2 days, so each one-cluster
    # minibatch runs on the matrix-core tiles)
    "ragged": dict(P=37, L=50, T=20, H=23, K=4, sizes=(3, 33, 17), inc=0.2, pattern="bernoulli"),
    "corridor": dict(P=150, L=500, T=24, K=6, sizes=(40, 5), inc=0.08, pattern="corridor"),
    "wide": dict(P=70, L=9, T=10, K=3, sizes=(20,), inc=0.5, pattern="bernoulli"),
}


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
@pytest.mark.parametrize("name", list(MFMA_SHAPES))
@pytest.mark.parametrize("opt", [0, 1])
def test_mfma_step_matches_oracle(name, opt, storage):
    """One minibatch through the matrix-core kernels (bf16 or E4M3 values, split
    FP32 operands) against the oracle on the same rounded values."""
    kw = dict(MFMA_SHAPES[name])
    inst = make_instance(demand="uniform50", noise="add1", x_dtype="f32", seed=77, **kw)
    say("mfma step", name, opt, storage)
    Wq = dequantized_values(inst, storage)
    rng = np.random.default_rng(8)
    Q0 = rng.uniform(0, 5, (inst.D, inst.T, inst.P)).astype(np.float32).astype(np.float64)
    A0 = rng.uniform(0, 2, (inst.D, inst.T, inst.P)).astype(np.float32).astype(np.float64)
    X = inst.x.astype(np.float64)
    chunk = rng.choice(inst.H, size=min(inst.H, 7), replace=False).astype(np.int32)
    eta = 0.3 if opt == 0 else 1e-4
    dar = make_dar(inst, storage)
    for c in range(inst.C):
        days = inst.days_of(c)
        Qd, Ad = dev(Q0[days], torch.float32), dev(A0[days], torch.float32)
        p = dode.make_params(eta=eta, optimizer=opt)
        dode.spgd_step(dar, c, chunk, dev(X[days], torch.float32), Qd, Ad, p)
        torch.cuda.synchronize()
        Qg, Ag = Qd.cpu().numpy(), Ad.cpu().numpy()
        for k, d in enumerate(days):
            q, A = orc.spgd_step(inst, Wq[c], X[d], Q0[d], A0[d], chunk, optimizer=opt, eta=eta)
            assert rel(Qg[k], q) <= 1e-4, (c, d)
            if opt == 0:
                assert rel(Ag[k], A) <= 1e-4, (c, d)


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
@pytest.mark.parametrize("name", list(MFMA_SHAPES))
def test_mfma_solve_matches_oracle(name, storage):
    kw = dict(MFMA_SHAPES[name])
    inst = make_instance(demand="gamma", noise="mult5", x_dtype="f32", seed=78, **kw)
    say("mfma solve", name, storage)
    E = 40
    perms = make_perms(79, E, inst.C, inst.H)
    batch_rows = 5 * inst.L
    bh = chunk_h_blocks(inst.L, inst.H, batch_rows)
    Wq = dequantized_values(inst, storage)
    x64 = inst.x.astype(np.float64)
    Qo, _, ho = orc.spgd(inst, x64, perms, E, bh, optimizer=0, eta=5.0, W=Wq)
    Qg, _, hg = run_solve(inst, storage, E, batch_rows, 5.0, 0, perms)
    lg, _, _ = orc.metrics(inst, x64, Qg, W=Wq)
    assert np.max(np.abs(lg - ho[:, -1]) / ho[:, -1]) <= 1e-3
    assert np.max(np.abs(hg - ho) / ho) <= 1e-3


@pytest.mark.parametrize("storage", ["f64", "bf16", "fp8"])
def test_plan_with_interleaved_clusters(storage):
    """Days of different clusters interleaved in the caller's order; the plan's
    cluster-grouped copy, its loss history and the stored state must map back."""
    inst = make_instance(P=20, L=40, T=24, K=4, sizes=(7, 5, 3), inc=0.2, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f64", seed=48)
    say("plan interleaved", storage)
    rng = np.random.default_rng(11)
    order = rng.permutation(inst.D)
    inst.x = inst.x[order]
    inst.day_cluster = inst.day_cluster[order].copy()
    E = 12
    perms = make_perms(49, E, inst.C, inst.H)
    bh = chunk_h_blocks(inst.L, inst.H, 200)
    W = inst.W if storage == "f64" else dequantized_values(inst, storage)
    Qo, Ao, ho = orc.spgd(inst, inst.x, perms, E, bh, optimizer=0, eta=5.0, W=W)
    dt = torch.float64 if storage == "f64" else torch.float32
    dar = make_dar(inst, storage)
    p = dode.make_params(epochs=E, batch_rows=200, eta=5.0)
    plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=dt, device="cuda")
    dode.spgd_plan_load(plan, dev(inst.x, dt), Q0)
    loss = torch.zeros((E, inst.D), dtype=torch.float64, device="cuda")
    dode.spgd_run(plan, 0, 5, loss=loss[:5])
    dode.spgd_run(plan, 5, E - 5, loss=loss[5:])
    Q = torch.empty_like(Q0)
    A = torch.empty_like(Q0)
    dode.spgd_plan_store(plan, Q, A)
    torch.cuda.synchronize()
    tol = 1e-9 if storage == "f64" else 1e-3
    assert np.max(np.abs(loss.cpu().numpy().T - ho) / ho) <= tol
    assert rel(Q.cpu().numpy(), Qo) <= (1e-8 if storage == "f64" else 2e-2)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_epoch_graph_replays_match_eager(storage):
    """The captured per-epoch graph, replayed in several runs with eager work and
    synchronisations in between, gives the eager result bit for bit after each run."""
    inst = make_instance(P=30, L=60, T=48, K=5, sizes=(20, 13), inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5", seed=52)
    say("graph replay", storage)
    E = 9
    perms = make_perms(53, E, inst.C, inst.H)
    dt = torch.float32
    dar = make_dar(inst, storage)
    X = dev(inst.x, dt)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=dt, device="cuda")
    plans = []
    for g in (1, 0):
        p = dode.make_params(epochs=E, batch_rows=10 * inst.L, eta=5.0, use_graph=g)
        plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
        dode.spgd_plan_load(plan, X, Q0)
        plans.append(plan)
    for e0 in range(0, E, 3):
        outs = []
        for plan in plans:
            dode.spgd_run(plan, e0, 3)
            junk = torch.randn(1000, device="cuda").sum()   # eager work between replays
            torch.cuda.synchronize()
            Q = torch.empty_like(Q0)
            dode.spgd_plan_store(plan, Q)
            torch.cuda.synchronize()
            outs.append(Q.cpu().numpy())
        np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
def test_day_tile_gives_identical_results(storage):
    """Each day is its own matrix-core column with the same summation order, so
    16-, 32- and 64-day waves give the same bits; clusters of 70, 33 and 1 days
    leave ragged groups at every tile width.  A tuned plan (day_tile 0) runs
    trial minibatches at load and must reload the state: same bits again.  The
    64-day run is also checked against the oracle."""
    inst = make_instance(P=45, L=70, T=24, K=5, sizes=(70, 33, 1), inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f32", seed=61)
    say("day tile", storage)
    E = 8
    perms = make_perms(62, E, inst.C, inst.H)
    batch_rows = 6 * inst.L
    dar = make_dar(inst, storage)
    X = dev(inst.x, torch.float32)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    outs = {}
    for tile, order, slabs in ((16, 1, 1), (32, 1, 1), (64, 1, 1), (16, 0, 1), (32, 0, 1),
                               (64, 0, 1), (16, 2, 1), (32, 2, 1), (16, 1, 4), (32, 0, 2),
                               (32, 1, 3), (32, 2, 2), (0, 1, 1)):
        p = dode.make_params(epochs=E, batch_rows=batch_rows, eta=5.0, day_tile=tile,
                             adj_order=order, slabs=slabs)
        plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
        dode.spgd_plan_load(plan, X, Q0)
        info = dode.spgd_plan_info(plan)
        sch = dode.spgd_plan_schedule(plan)
        assert info["day_tile"] == tile if tile else info["day_tile"] in (16, 32, 64)
        assert sch["day_tile"] == info["day_tile"]
        assert sch["adj_order"] == order if tile else sch["adj_order"] in (0, 1, 2)
        assert sch["slabs"] == slabs if tile else sch["slabs"] in (1, 2, 4)
        groups = sum(-(-n // info["day_tile"]) for n in (70, 33, 1))
        assert info["n_day_groups"] == groups and info["minibatch_intervals"] == 6
        loss = torch.zeros((E, inst.D), dtype=torch.float64, device="cuda")
        dode.spgd_run(plan, 0, E, loss=loss)
        Q = torch.empty_like(Q0)
        A = torch.empty_like(Q0)
        dode.spgd_plan_store(plan, Q, A)
        torch.cuda.synchronize()
        outs[(tile, order, slabs)] = (Q.cpu().numpy(), A.cpu().numpy(), loss.cpu().numpy())
    for key in outs:
        for a, b in zip(outs[key], outs[(32, 1, 1)]):
            np.testing.assert_array_equal(a, b)
    Wq = dequantized_values(inst, storage)
    bh = chunk_h_blocks(inst.L, inst.H, batch_rows)
    _, _, ho = orc.spgd(inst, inst.x.astype(np.float64), perms, E, bh, optimizer=0, eta=5.0, W=Wq)
    assert np.max(np.abs(outs[(64, 1, 1)][2].T - ho) / ho) <= 1e-3


def test_schedule_tuner_times_every_candidate_and_remembers():
    """day_tile 0: the first plan of a shape times an epoch of every schedule
    candidate (3 day tiles x 3 adjoint orders x 1, 2 or 4 day slabs; the
    chunked order has no 64-day waves, and slab counts above the number of day
    groups are skipped) and keeps the fastest; a second plan of the same
    shapes, storage and cluster sizes reuses that choice without timing;
    another storage type is a new key."""
    inst = make_instance(P=41, L=66, T=30, K=4, sizes=(50, 20), inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f32", seed=64)
    say("schedule tuner")
    perms = make_perms(65, 4, inst.C, inst.H)
    X = dev(inst.x, torch.float32)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    seen = []
    for storage in ("bf16", "bf16", "fp8"):
        dar = make_dar(inst, storage)
        p = dode.make_params(epochs=4, batch_rows=5 * inst.L, eta=5.0, day_tile=0)
        plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
        dode.spgd_plan_load(plan, X, Q0)
        seen.append(dode.spgd_plan_schedule(plan))
    groups = {t: sum(-(-n // t) for n in (50, 20)) for t in (16, 32, 64)}
    want = sum((3 if t < 64 else 2) * sum(1 for k in (1, 2, 4) if k <= groups[t]) for t in groups)
    assert want == 19
    assert seen[0]["n_timed"] == want and seen[0]["best_ms"] > 0
    assert seen[1]["n_timed"] == 0
    pick = ("day_tile", "adj_order", "slabs")
    assert [seen[1][k] for k in pick] == [seen[0][k] for k in pick]
    assert seen[2]["n_timed"] == want


def test_schedule_file_is_read_and_appended(tmp_path, monkeypatch):
    """DODE_SCHEDULE_CACHE: a plan whose key has a valid line in the file takes
    that schedule without timing (the last valid line wins, invalid ones are
    skipped); a plan of a new key tunes and appends its choice, which the file
    then holds under the same key."""
    inst = make_instance(P=37, L=54, T=24, K=3, sizes=(41, 23), inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f32", seed=66)
    say("schedule file")
    perms = make_perms(67, 3, inst.C, inst.H)
    X = dev(inst.x, torch.float32)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    arch = torch.cuda.get_device_properties(0).gcnArchName
    bh = 4
    sizes = "".join(f"{n}," for n in np.bincount(inst.day_cluster))

    def key(storage_code):
        return f"{arch}|{inst.P},{inst.L},{inst.T},{inst.H},{inst.K}|{bh}|{storage_code}|0|{sizes}"

    path = tmp_path / "schedules.txt"
    # DODE_BF16 = 2, DODE_FP8_E4M3 = 3
    path.write_text(f"{key(2)}\t32 1 1 0.5\n"
                    f"{key(2)}\t64 2 1 0.1\n"       # invalid: no chunked 64-day waves
                    f"{key(2)}\tgarbage\n"
                    f"{key(2)}\t16 2 2 0.4\n"
                    f"other-key\t64 0 1 0.2\n")
    monkeypatch.setenv("DODE_SCHEDULE_CACHE", str(path))
    got = []
    for storage in ("bf16", "fp8"):
        dar = make_dar(inst, storage)
        p = dode.make_params(epochs=3, batch_rows=bh * inst.L, eta=5.0, day_tile=0)
        plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
        dode.spgd_plan_load(plan, X, Q0)
        got.append(dode.spgd_plan_schedule(plan))
    pick = ("day_tile", "adj_order", "slabs")
    assert got[0]["n_timed"] == 0 and [got[0][k] for k in pick] == [16, 2, 2]
    assert got[1]["n_timed"] > 0
    lines = [ln.split("\t") for ln in path.read_text().splitlines()]
    mine = [v.split() for k, v in lines if k == key(3)]
    assert len(mine) == 1
    assert [int(v) for v in mine[0][:3]] == [got[1][k] for k in pick]
    assert abs(float(mine[0][3]) - got[1]["best_ms"]) <= 1e-5 * got[1]["best_ms"] + 1e-6


def test_day_tile_rejected():
    inst = make_instance(P=10, L=12, T=6, K=2, sizes=(3,), inc=0.3, pattern="bernoulli", seed=63)
    dar = make_dar(inst, "bf16")
    with pytest.raises(dode.DodeError, match="day_tile"):
        dode.spgd_plan_create(dar, inst.day_cluster, dode.make_params(day_tile=48), stream=0)
    with pytest.raises(dode.DodeError, match="adj_order 2 needs day_tile"):
        dode.spgd_plan_create(dar, inst.day_cluster, dode.make_params(day_tile=64, adj_order=2),
                              stream=0)


@pytest.mark.parametrize("name", ["ragged", "corridor"])
def test_refinement_steps_match_oracle(name):
    """FP8 plan with 2 refinement steps per epoch: each epoch is the minibatches
    of Algorithm 1 on the FP8 values, then 2 full-batch steps (all H intervals
    as one minibatch) on the corrected values h + c.  The oracle runs the same
    composition in FP64; the plan's per-epoch losses (FP8 values) and final
    demand must match, and the corrected values must beat plain FP8 on the
    exact loss."""
    kw = dict(MFMA_SHAPES[name])
    inst = make_instance(demand="gamma", noise="mult5", x_dtype="f32", seed=91, **kw)
    say("refinement", name)
    E, R = 6, 2
    perms = make_perms(92, E, inst.C, inst.H)
    batch_rows = 4 * inst.L
    bh = chunk_h_blocks(inst.L, inst.H, batch_rows)
    Wq = dequantized_values(inst, "fp8")
    Wr = dequantized_values(inst, "fp8corr")
    # corrected values are far closer to the exact ones than the FP8 values
    for c in range(inst.C):
        assert np.max(np.abs(Wr[c] - inst.W[c])) <= 2.0 ** -12 * np.max(np.abs(inst.W[c]))
        assert np.max(np.abs(Wr[c] - inst.W[c])) < 0.1 * np.max(np.abs(Wq[c] - inst.W[c]))
    x64 = inst.x.astype(np.float64)
    ident = np.tile(np.arange(inst.H, dtype=np.int32), (1, inst.C, 1))
    Q = A = None
    hist = []
    for e in range(E):
        Q, A, _ = orc.spgd(inst, x64, perms[e:e + 1], 1, bh, q0=Q, A0=A, W=Wq, record_loss=False)
        for _ in range(R):
            Q, A, _ = orc.spgd(inst, x64, ident, 1, inst.H, q0=Q, A0=A, W=Wr, record_loss=False)
        hist.append(orc.metrics(inst, x64, Q, W=Wq)[0])
    ho = np.stack(hist, axis=1)
    dar = make_dar(inst, "fp8", correction=True)
    p = dode.make_params(epochs=E, batch_rows=batch_rows, eta=5.0, refine_steps=R)
    plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    dode.spgd_plan_load(plan, dev(inst.x, torch.float32), Q0)
    loss = torch.zeros((E, inst.D), dtype=torch.float64, device="cuda")
    dode.spgd_run(plan, 0, E, loss=loss)
    Qg = torch.empty_like(Q0)
    dode.spgd_plan_store(plan, Qg)
    torch.cuda.synchronize()
    assert np.max(np.abs(loss.cpu().numpy().T - ho) / ho) <= 1e-3
    lg, _, _ = orc.metrics(inst, x64, Qg.cpu().numpy().astype(np.float64))
    lo, _, _ = orc.metrics(inst, x64, Q)
    assert np.max(np.abs(lg - lo) / lo) <= 1e-3


def test_refinement_needs_correction_tiles():
    inst = make_instance(P=10, L=12, T=6, K=2, sizes=(3,), inc=0.3, pattern="bernoulli", seed=93)
    for storage, corr in (("fp8", False), ("bf16", False)):
        dar = make_dar(inst, storage, correction=corr)
        with pytest.raises(dode.DodeError, match="refine_steps"):
            dode.spgd_plan_create(dar, inst.day_cluster, dode.make_params(refine_steps=1), stream=0)
    with pytest.raises(dode.DodeError, match="FP8"):
        make_dar(inst, "bf16", correction=True)
    dar = make_dar(inst, "fp8", correction=True)
    with pytest.raises(dode.DodeError, match="correction"):
        dode.dar_set_values(dar, 0, torch.zeros((inst.K, inst.T, len(inst.col_idx)), device="cuda"))


ONE_LAUNCH_SHAPES = {
    # 40 intervals per minibatch: long components of neighbouring intervals
    "long components": dict(P=50, L=200, T=288, K=6, sizes=(20, 3), inc=0.1, pattern="corridor"),
    # H > T + K: the last intervals reach no departure interval
    "H past T": dict(P=37, L=50, T=20, H=30, K=4, sizes=(3, 33, 17), inc=0.2, pattern="bernoulli"),
    # one lag: every interval is its own component
    "K=1": dict(P=24, L=40, T=30, K=1, sizes=(17,), inc=0.3, pattern="bernoulli"),
    "corridor": dict(P=150, L=500, T=48, K=6, sizes=(40, 5), inc=0.08, pattern="corridor"),
}


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
@pytest.mark.parametrize("name", list(ONE_LAUNCH_SHAPES))
def test_one_launch_minibatch_equals_two_launches(name, storage):
    """kernel_path 2 runs each minibatch as one launch (forward, residual,
    adjoint and step per component of the minibatch); kernel_path 0 runs the
    forward and the adjoint as separate launches.  Same arithmetic per item:
    the demand, the accumulator and the loss history agree bit for bit, for
    every day tile, and the one-launch run matches the oracle on the same
    rounded values."""
    kw = dict(ONE_LAUNCH_SHAPES[name])
    inst = make_instance(demand="gamma", noise="mult5", x_dtype="f32", seed=95, **kw)
    say("one launch vs two", name, storage)
    E = 5
    perms = make_perms(96, E, inst.C, inst.H)
    batch_rows = 8192 if inst.L >= 200 else 7 * inst.L
    dar = make_dar(inst, storage)
    X = dev(inst.x, torch.float32)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    outs = {}
    for path, tile in ((0, 32), (2, 32), (2, 16), (2, 64)):
        p = dode.make_params(epochs=E, batch_rows=batch_rows, eta=5.0, kernel_path=path,
                             day_tile=tile)
        plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
        dode.spgd_plan_load(plan, X, Q0)
        loss = torch.zeros((E, inst.D), dtype=torch.float64, device="cuda")
        dode.spgd_run(plan, 0, E, loss=loss)
        Q = torch.empty_like(Q0)
        A = torch.empty_like(Q0)
        dode.spgd_plan_store(plan, Q, A)
        torch.cuda.synchronize()
        outs[(path, tile)] = (Q.cpu().numpy(), A.cpu().numpy(), loss.cpu().numpy())
    for key in ((2, 32), (2, 16), (2, 64)):
        for a, b in zip(outs[key], outs[(0, 32)]):
            np.testing.assert_array_equal(a, b)
    Wq = dequantized_values(inst, storage)
    bh = chunk_h_blocks(inst.L, inst.H, batch_rows)
    _, _, ho = orc.spgd(inst, inst.x.astype(np.float64), perms, E, bh, optimizer=0, eta=5.0, W=Wq)
    assert np.max(np.abs(outs[(2, 32)][2].T - ho) / ho) <= 1e-3


def run_paths(inst, storage, E, perms, batch_rows, configs, refine=0):
    """Q, A and the loss history of one plan per (kernel_path, day_tile,
    adj_order) in `configs`."""
    dar = make_dar(inst, storage, correction=refine > 0)
    X = dev(inst.x, torch.float32)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    outs = {}
    for path, tile, order in configs:
        p = dode.make_params(epochs=E, batch_rows=batch_rows, eta=5.0, kernel_path=path,
                             day_tile=tile, adj_order=order, refine_steps=refine)
        plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
        dode.spgd_plan_load(plan, X, Q0)
        loss = torch.zeros((E, inst.D), dtype=torch.float64, device="cuda")
        dode.spgd_run(plan, 0, 2, loss=loss[:2])
        dode.spgd_run(plan, 2, E - 2, loss=loss[2:])
        Q = torch.empty_like(Q0)
        A = torch.empty_like(Q0)
        dode.spgd_plan_store(plan, Q, A)
        torch.cuda.synchronize()
        outs[(path, tile, order)] = (Q.cpu().numpy(), A.cpu().numpy(), loss.cpu().numpy())
    return outs


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
@pytest.mark.parametrize("name", ["long components", "H past T", "corridor"])
def test_persistent_epoch_equals_separate_launches(name, storage):
    """kernel_path 3 runs every minibatch of an epoch in one cooperative launch
    with grid barriers between the forward and adjoint phases; the items are
    those of the separate launches, so the demand, the accumulator and the
    loss history agree bit for bit, for each adjoint order and day tile (the
    run is split over two spgd_run calls, so the epoch argument is exercised)."""
    kw = dict(ONE_LAUNCH_SHAPES[name])
    inst = make_instance(demand="gamma", noise="mult5", x_dtype="f32", seed=97, **kw)
    say("persistent epoch vs separate launches", name, storage)
    E = 5
    perms = make_perms(98, E, inst.C, inst.H)
    batch_rows = 8192 if inst.L >= 200 else 7 * inst.L
    configs = [(0, 32, 2), (3, 32, 1), (3, 16, 2), (3, 16, 0), (3, 64, 1)]
    outs = run_paths(inst, storage, E, perms, batch_rows, configs)
    for key in configs[1:]:
        for a, b in zip(outs[key], outs[configs[0]]):
            np.testing.assert_array_equal(a, b)


def test_persistent_epoch_with_refinement():
    """kernel_path 3 with 2 refinement steps per epoch (run as separate launches
    after the persistent minibatch launch) gives the bits of kernel_path 0."""
    inst = make_instance(P=40, L=120, T=36, K=4, sizes=(30, 9), inc=0.12, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f32", seed=99)
    say("persistent epoch with refinement")
    E = 4
    perms = make_perms(100, E, inst.C, inst.H)
    configs = [(0, 32, 1), (3, 32, 1), (3, 16, 2)]
    outs = run_paths(inst, "fp8", E, perms, 6 * inst.L, configs, refine=2)
    for key in configs[1:]:
        for a, b in zip(outs[key], outs[configs[0]]):
            np.testing.assert_array_equal(a, b)


def test_persistent_epoch_barrier_error_is_reported(monkeypatch):
    """The grid barrier's wait is bounded: with a spin limit of zero polls every
    waiting block gives up at once, the launch ends, and spgd_run reports the
    error instead of hanging."""
    inst = make_instance(P=20, L=40, T=24, K=4, sizes=(40,), inc=0.2, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f32", seed=101)
    say("persistent epoch barrier error path")
    perms = make_perms(102, 2, inst.C, inst.H)
    dar = make_dar(inst, "bf16")
    p = dode.make_params(epochs=2, batch_rows=4 * inst.L, eta=5.0, kernel_path=3, day_tile=32)
    plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    dode.spgd_plan_load(plan, dev(inst.x, torch.float32), Q0)
    monkeypatch.setenv("DODE_PERSIST_SPIN_LIMIT", "0")
    with pytest.raises(dode.DodeError, match="grid barrier"):
        dode.spgd_run(plan, 0, 1)
    monkeypatch.delenv("DODE_PERSIST_SPIN_LIMIT")
    torch.cuda.synchronize()


def test_persistent_epoch_rejected_without_a_fixed_schedule():
    inst = make_instance(P=10, L=12, T=6, K=2, sizes=(5,), inc=0.3, pattern="bernoulli", seed=103)
    dar = make_dar(inst, "bf16")
    for kw in (dict(day_tile=0), dict(day_tile=32, slabs=2), dict(day_tile=32, adj_order=2)):
        with pytest.raises(dode.DodeError, match="kernel_path 3"):
            dode.spgd_plan_create(dar, inst.day_cluster, dode.make_params(kernel_path=3, **kw),
                                  stream=0)


def test_refinement_orders_give_identical_results():
    """An FP8 plan with 2 refinement steps per epoch: with the chunked adjoint
    (order 2) the refinement steps also run chunked over every departure
    interval; the results are the bits of the interval-major adjoint (order 0)
    for both day tiles, and the one-launch minibatch path agrees too."""
    inst = make_instance(P=45, L=70, T=24, K=5, sizes=(70, 33, 3), inc=0.15, pattern="corridor",
                         demand="gamma", noise="mult5", x_dtype="f32", seed=66)
    say("refinement orders")
    E = 4
    perms = make_perms(67, E, inst.C, inst.H)
    dar = make_dar(inst, "fp8", correction=True)
    X = dev(inst.x, torch.float32)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    outs = {}
    for tile, order, path in ((32, 0, 0), (32, 2, 0), (16, 2, 0), (16, 0, 0), (32, 2, 2)):
        p = dode.make_params(epochs=E, batch_rows=6 * inst.L, eta=5.0, refine_steps=2,
                             day_tile=tile, adj_order=order, kernel_path=path)
        plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
        dode.spgd_plan_load(plan, X, Q0)
        loss = torch.zeros((E, inst.D), dtype=torch.float64, device="cuda")
        dode.spgd_run(plan, 0, E, loss=loss)
        Q = torch.empty_like(Q0)
        A = torch.empty_like(Q0)
        dode.spgd_plan_store(plan, Q, A)
        torch.cuda.synchronize()
        outs[(tile, order, path)] = (Q.cpu().numpy(), A.cpu().numpy(), loss.cpu().numpy())
    for key in outs:
        for a, b in zip(outs[key], outs[(32, 0, 0)]):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("slabs", [1, 2])
def test_kernel_timing_keeps_the_bits(slabs):
    """With kernel timing on, every launch gets an event pair (and day slabs
    run one after another on the run's stream); the demand, the accumulator
    and the loss history are the same bits as without timing, and the launch
    counts are those of the schedule."""
    inst = make_instance(demand="gamma", noise="mult5", x_dtype="f32", seed=131,
                         **ONE_LAUNCH_SHAPES["corridor"])
    say("kernel timing keeps the bits", slabs)
    E = 5
    perms = make_perms(132, E, inst.C, inst.H)
    dar = make_dar(inst, "bf16")
    X = dev(inst.x, torch.float32)
    Q0 = torch.zeros((inst.D, inst.T, inst.P), dtype=torch.float32, device="cuda")
    outs = []
    for timing in (False, True):
        p = dode.make_params(epochs=E, batch_rows=8192, eta=5.0, day_tile=32, adj_order=2,
                             slabs=slabs)
        plan = dode.spgd_plan_create(dar, inst.day_cluster, p, perm=perms, stream=0)
        dode.spgd_plan_load(plan, X, Q0)
        assert dode.spgd_plan_schedule(plan)["slabs"] == slabs
        loss = torch.zeros((E, inst.D), dtype=torch.float64, device="cuda")
        dode.spgd_run(plan, 0, 2, loss=loss[:2])
        if timing:
            dode.spgd_plan_timing(plan, True)
        dode.spgd_run(plan, 2, E - 2, loss=loss[2:])
        if timing:
            ms, n = dode.spgd_plan_timing(plan, False)
            nch = dode.spgd_plan_info(plan)["n_minibatches"]
            assert n[0] == n[1] == (E - 2) * nch * slabs
            assert ms[0] > 0 and ms[1] > 0
        Q = torch.empty_like(Q0)
        A = torch.empty_like(Q0)
        dode.spgd_plan_store(plan, Q, A)
        torch.cuda.synchronize()
        outs.append((Q.cpu().numpy(), A.cpu().numpy(), loss.cpu().numpy()))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
