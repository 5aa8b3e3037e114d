"""Route portions from mean path costs and the assignment they give, on the
GPU (dode_path_costs, dar_from_costs) against the FP64 oracle: FP64 and FP32
(FP32 path costs against the oracle's binary32 walk), ragged routes, day counts that are not multiples of the 4-day groups, slices
of more than 4 days, the whole speeds -> ratios -> costs -> assignment chain,
and the argument checks."""
import numpy as np
import pytest

import oracle as orc
import paper_1901_09266_amd as dode
from synth import make_choice_instance
from gpu_helpers import say, dev, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

THETA = 0.6   # 0.01 per second, costs in minutes


def small(seed=0, days=(9,)):
    return make_choice_instance(L=48, P=7, H=36, K=4, m=5, sizes=days, ragged=True,
                                seed=2000 + seed)


def costs(ci, speed, f64, T=None):
    t = torch.float64 if f64 else torch.float32
    return dode.dode_path_costs(dev(ci.path_ptr, torch.int32), dev(ci.path_link, torch.int32),
                                dev(ci.link_len, t), dev(speed, t), ci.dt, ci.T if T is None else T)


def routes(ci):
    return dode.dode_routes_create(ci.P, ci.L, ci.T, ci.H, ci.K, ci.nnz, ci.path_od, ci.path_ptr,
                                   ci.path_link, ci.pair_nz)


@pytest.mark.parametrize("f64", [True, False])
def test_path_costs_match_oracle(f64):
    ci = small(seed=1)
    say("path costs", f64, ci.n_paths, ci.speed.shape)
    for days in (slice(0, 9), slice(2, 3), slice(0, 4), slice(1, 7)):
        sp = ci.speed[days]
        got = costs(ci, sp, f64).cpu().numpy()
        ref = orc.path_costs(ci.path_ptr, ci.path_link, ci.link_len, sp.astype(np.float64), ci.dt,
                             ci.T, walk="f64" if f64 else "f32")
        err = np.abs(got - ref) / ref
        if f64:
            assert err.max() <= 1e-13
        else:
            # the same binary32 day travel times on both sides (the oracle
            # walks in binary32 too), FP64 day sums in another order, and one
            # rounding of the mean to FP32
            assert err.max() <= 2e-7


def test_path_costs_partial_horizon():
    """T below the speed horizon: only the first T departure intervals."""
    ci = small(seed=2, days=(5,))
    say("path costs T<H")
    got = costs(ci, ci.speed, True, T=20).cpu().numpy()
    ref = orc.path_costs(ci.path_ptr, ci.path_link, ci.link_len, ci.speed.astype(np.float64), ci.dt, 20)
    assert got.shape == (20, ci.n_paths)
    assert rel(got, ref) <= 1e-13


def test_path_costs_slices_of_eight_days():
    """1100 days of 450 routes over 288 intervals pass the 256 MiB slice
    budget at 4 days per slice, so slices hold 8 days; checked on sampled
    routes, which the oracle computes alone."""
    ci = make_choice_instance(sizes=(1100,), seed=2100)
    say("path costs 1100 days", ci.n_paths)
    got = costs(ci, ci.speed, False).cpu().numpy()
    rng = np.random.default_rng(0)
    for k in rng.choice(ci.n_paths, 6, replace=False):
        pp = np.array([0, ci.path_ptr[k + 1] - ci.path_ptr[k]])
        pl = ci.path_link[ci.path_ptr[k]:ci.path_ptr[k + 1]]
        ref = orc.path_costs(pp, pl, ci.link_len, ci.speed.astype(np.float64), ci.dt, ci.T,
                             walk="f32")[:, 0]
        err = np.abs(got[:, k] - ref) / ref
        # binary32 day times on both sides, FP64 sums of 1100 days in slices
        assert err.max() <= 2e-7


@pytest.mark.parametrize("f64", [True, False])
def test_assignment_from_costs_matches_oracle(f64):
    ci = small(seed=3)
    t = torch.float64 if f64 else torch.float32
    rng = np.random.default_rng(3)
    Rr = rng.uniform(0, 1, size=(ci.K, ci.T, ci.n_pairs))
    cost = rng.uniform(5, 25, size=(ci.T, ci.n_paths))
    if not f64:
        Rr = Rr.astype(np.float32).astype(np.float64)
        cost = cost.astype(np.float32).astype(np.float64)
    p_ref = orc.logit_portions(ci.P, ci.path_od, THETA, cost)
    W_ref = orc.rho_from_portions(ci.P, ci.L, ci.T, ci.H, ci.K, ci.path_od, ci.path_ptr, ci.path_link,
                                  ci.row_ptr, ci.col_idx, Rr, p_ref)
    r = routes(ci)
    say("assign from costs", f64)
    W = torch.full((ci.K, ci.T, ci.nnz), -1.0, dtype=t, device="cuda")
    p = torch.full((ci.T, ci.n_paths), -1.0, dtype=t, device="cuda")
    dode.dar_from_costs(r, dev(Rr, t), dev(cost, t), THETA, W, portions=p)
    torch.cuda.synchronize()
    tol = 1e-14 if f64 else 1e-6     # FP64 sums; FP32: one rounding of the result
    assert rel(p.cpu().numpy(), p_ref) <= tol
    got = W.cpu().numpy()
    assert np.all(np.abs(got - W_ref) <= tol * np.abs(W_ref) + 1e-300)
    # without the portions output
    W2 = torch.zeros_like(W)
    dode.dar_from_costs(r, dev(Rr, t), dev(cost, t), THETA, W2)
    torch.cuda.synchronize()
    assert torch.equal(W, W2)


def test_speeds_to_assignment_chain_fp64():
    """speeds -> ratios (dode_dar_from_speeds) and mean costs (dode_path_costs)
    -> portions and assignment (dar_from_costs), against the oracle's chain,
    for each pattern of a two-pattern instance."""
    ci = make_choice_instance(L=64, P=8, H=48, K=5, m=6, sizes=(6, 3), ragged=True, seed=2200)
    r = routes(ci)
    t = torch.float64
    pp, pl, ln = dev(ci.path_ptr, torch.int32), dev(ci.path_link, torch.int32), dev(ci.link_len, t)
    for c in range(2):
        sp = ci.speed[ci.day_cluster == c].astype(np.float64)
        say("chain pattern", c)
        Rr = dode.dode_dar_from_speeds(pp, pl, ln, dev(sp, t), ci.dt, ci.H, ci.K)
        cost = dode.dode_path_costs(pp, pl, ln, dev(sp, t), ci.dt, ci.T)
        W = torch.empty((ci.K, ci.T, ci.nnz), dtype=t, device="cuda")
        dode.dar_from_costs(r, Rr, cost, THETA, W)
        torch.cuda.synchronize()
        Rr_o = orc.dar_from_speeds(ci.path_ptr, ci.path_link, ci.link_len, sp, ci.dt, ci.H, ci.K)
        c_o = orc.path_costs(ci.path_ptr, ci.path_link, ci.link_len, sp, ci.dt, ci.T)
        W_o = orc.rho_from_portions(ci.P, ci.L, ci.T, ci.H, ci.K, ci.path_od, ci.path_ptr,
                                    ci.path_link, ci.row_ptr, ci.col_idx, Rr_o,
                                    orc.logit_portions(ci.P, ci.path_od, THETA, c_o))
        assert rel(cost.cpu().numpy(), c_o) <= 1e-13
        assert np.max(np.abs(W.cpu().numpy() - W_o)) <= 1e-12


@pytest.mark.parametrize("f64", [True, False])
def test_costs_from_ratio_trajectories(f64):
    """The combined call returns the ratios of dode_dar_from_speeds bit for bit
    and the path costs of dode_path_costs up to the order of the FP64 day sums."""
    ci = small(seed=5)
    t = torch.float64 if f64 else torch.float32
    pp, pl, ln = dev(ci.path_ptr, torch.int32), dev(ci.path_link, torch.int32), dev(ci.link_len, t)
    sp = dev(ci.speed, t)
    say("ratios + costs", f64)
    Rr2, c2 = dode.dode_dar_costs_from_speeds(pp, pl, ln, sp, ci.dt, ci.H, ci.K)
    Rr1 = dode.dode_dar_from_speeds(pp, pl, ln, sp, ci.dt, ci.H, ci.K)
    c1 = dode.dode_path_costs(pp, pl, ln, sp, ci.dt, ci.T)
    torch.cuda.synchronize()
    assert torch.equal(Rr1, Rr2)
    assert rel(c2.cpu().numpy(), c1.cpu().numpy()) <= (1e-12 if f64 else 1e-6)
    if f64:
        ref = orc.path_costs(ci.path_ptr, ci.path_link, ci.link_len, ci.speed.astype(np.float64),
                             ci.dt, ci.T)
        assert rel(c2.cpu().numpy(), ref) <= 1e-13


def test_costs_from_ratio_trajectories_chunks(monkeypatch):
    """160 days of 450 routes with the trajectory scratch capped at 1 GiB need
    two chunks: the running FP64 sums across chunks give dode_path_costs'
    means."""
    monkeypatch.setenv("DODE_DAR_SCRATCH_BYTES", str(1 << 30))
    ci = make_choice_instance(sizes=(160,), seed=2300)
    t = torch.float32
    pp, pl, ln = dev(ci.path_ptr, torch.int32), dev(ci.path_link, torch.int32), dev(ci.link_len, t)
    sp = dev(ci.speed, t)
    say("ratios + costs, 160 days")
    _, c2 = dode.dode_dar_costs_from_speeds(pp, pl, ln, sp, ci.dt, ci.H, ci.K)
    c1 = dode.dode_path_costs(pp, pl, ln, sp, ci.dt, ci.T)
    torch.cuda.synchronize()
    # same FP32 day travel times on both sides; FP64 sums in another order
    assert rel(c2.cpu().numpy(), c1.cpu().numpy()) <= 1e-6


def test_chunking_does_not_change_bits(monkeypatch):
    """40 days in one trajectory chunk, and in chunks of 2 days (the scratch
    capped at 24 MiB, 10.9 MB per day): the days are summed in the same order
    either way, so ratios and costs are equal bit for bit; a cap that is not a
    positive byte count is an argument error."""
    ci = make_choice_instance(sizes=(40,), seed=2400)
    t = torch.float32
    pp, pl, ln = dev(ci.path_ptr, torch.int32), dev(ci.path_link, torch.int32), dev(ci.link_len, t)
    sp = dev(ci.speed, t)
    say("chunking bits, 40 days")
    monkeypatch.delenv("DODE_DAR_SCRATCH_BYTES", raising=False)
    r1, c1 = dode.dode_dar_costs_from_speeds(pp, pl, ln, sp, ci.dt, ci.H, ci.K)
    monkeypatch.setenv("DODE_DAR_SCRATCH_BYTES", str(24 << 20))
    r2, c2 = dode.dode_dar_costs_from_speeds(pp, pl, ln, sp, ci.dt, ci.H, ci.K)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2) and torch.equal(c1, c2)
    for bad in ("0", "-5", "12x", ""):
        monkeypatch.setenv("DODE_DAR_SCRATCH_BYTES", bad)
        with pytest.raises(dode.DodeError, match="DODE_DAR_SCRATCH_BYTES"):
            dode.dode_dar_costs_from_speeds(pp, pl, ln, sp, ci.dt, ci.H, ci.K)


def test_theta_zero_gives_equal_portions():
    """theta = 0: every route of an OD gets 1 / (its number of routes), whatever
    the costs (eq. "logit"); single-route ODs get 1."""
    ci = small(seed=6)
    t = torch.float64
    rng = np.random.default_rng(6)
    cost = dev(rng.uniform(5, 25, size=(ci.T, ci.n_paths)), t)
    Rr = dev(rng.uniform(0, 1, size=(ci.K, ci.T, ci.n_pairs)), t)
    W = torch.empty((ci.K, ci.T, ci.nnz), dtype=t, device="cuda")
    p = torch.empty((ci.T, ci.n_paths), dtype=t, device="cuda")
    say("theta 0")
    dode.dar_from_costs(routes(ci), Rr, cost, 0.0, W, portions=p)
    torch.cuda.synchronize()
    n_routes = np.bincount(ci.path_od, minlength=ci.P)[ci.path_od]
    np.testing.assert_array_equal(p.cpu().numpy(), np.broadcast_to(1.0 / n_routes, (ci.T, ci.n_paths)))


def test_argument_checks():
    ci = small(seed=4, days=(2,))
    say("choice checks")
    t = torch.float64
    bad = ci.path_link.copy()
    bad[0] = ci.L
    with pytest.raises(dode.DodeError, match="path_link"):
        dode.dode_path_costs(dev(ci.path_ptr, torch.int32), dev(bad, torch.int32),
                             dev(ci.link_len, t), dev(ci.speed, t), ci.dt, ci.T)
    sp = ci.speed.astype(np.float64).copy()
    sp[1, 2, 3] = np.nan
    with pytest.raises(dode.DodeError, match="positive"):
        costs(ci, sp, True)
    with pytest.raises(dode.DodeError, match="dt"):
        dode.dode_path_costs(dev(ci.path_ptr, torch.int32), dev(ci.path_link, torch.int32),
                             dev(ci.link_len, t), dev(ci.speed, t), 0.0, ci.T)
    r = routes(ci)
    Rr = torch.zeros((ci.K, ci.T, ci.n_pairs), dtype=t, device="cuda")
    cost = torch.ones((ci.T, ci.n_paths), dtype=t, device="cuda")
    W = torch.empty((ci.K, ci.T, ci.nnz), dtype=t, device="cuda")
    with pytest.raises(dode.DodeError, match="theta"):
        dode.dar_from_costs(r, Rr, cost, float("inf"), W)
    with pytest.raises(ValueError, match="cost"):
        dode.dar_from_costs(r, Rr, cost[:, :-1].contiguous(), THETA, W)


@pytest.mark.parametrize("f64", [True, False])
def test_patterns_in_one_call_equal_one_call_per_pattern(f64):
    """dode_dar_patterns_from_speeds on three patterns of 4, 1 and 6 days
    gives, pattern by pattern, the bits of dode_dar_costs_from_speeds on that
    pattern's days (ratios and costs), also with a scratch cap that splits the
    largest pattern; malformed pattern offsets are shape errors."""
    ci = small(seed=5, days=(11,))
    say("patterns in one call", f64)
    t = torch.float64 if f64 else torch.float32
    pp, pl = dev(ci.path_ptr, torch.int32), dev(ci.path_link, torch.int32)
    ln, sp = dev(ci.link_len, t), dev(ci.speed, t)
    ptr = np.array([0, 4, 5, 11], dtype=np.int32)
    Rr, cost = dode.dode_dar_patterns_from_speeds(pp, pl, ln, sp, ptr, ci.dt, ci.H, ci.K,
                                                  with_costs=True)
    Rr_only, none = dode.dode_dar_patterns_from_speeds(pp, pl, ln, sp, ptr, ci.dt, ci.H, ci.K)
    assert none is None
    torch.cuda.synchronize()
    for q in range(3):
        r1, c1 = dode.dode_dar_costs_from_speeds(pp, pl, ln, sp[ptr[q]:ptr[q + 1]], ci.dt, ci.H,
                                                 ci.K)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(Rr[q].cpu().numpy(), r1.cpu().numpy())
        np.testing.assert_array_equal(Rr_only[q].cpu().numpy(), r1.cpu().numpy())
        np.testing.assert_array_equal(cost[q].cpu().numpy(), c1.cpu().numpy())
    for bad in ([0, 4, 4, 11], [1, 4, 5, 11], [0, 6, 5, 11]):
        with pytest.raises((dode.DodeError, ValueError)):
            dode.dode_dar_patterns_from_speeds(pp, pl, ln, sp, np.array(bad, np.int32), ci.dt,
                                               ci.H, ci.K)


def test_patterns_in_one_call_with_a_scratch_cap(monkeypatch):
    """With the trajectory scratch capped at two days the patterns are split
    into chunks: the same ratios as without the cap (days summed in order)."""
    ci = small(seed=6, days=(9,))
    say("patterns with scratch cap")
    pp, pl = dev(ci.path_ptr, torch.int32), dev(ci.path_link, torch.int32)
    ln, sp = dev(ci.link_len, torch.float64), dev(ci.speed, torch.float64)
    ptr = np.array([0, 5, 9], dtype=np.int32)
    full, _ = dode.dode_dar_patterns_from_speeds(pp, pl, ln, sp, ptr, ci.dt, ci.H, ci.K)
    n_pairs = ci.path_link.shape[0]
    monkeypatch.setenv("DODE_DAR_SCRATCH_BYTES", str(2 * n_pairs * (ci.H + 1) * 8))
    capped, _ = dode.dode_dar_patterns_from_speeds(pp, pl, ln, sp, ptr, ci.dt, ci.H, ci.K)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(full.cpu().numpy(), capped.cpu().numpy())
