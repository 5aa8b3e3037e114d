"""Pins of the oracle's route portions from mean path costs (eqs. "cost",
"logit", "rt") and of the assignment matrix they give (eq. "assign"), CPU only."""
import numpy as np
import pytest

import oracle as orc
from synth import make_choice_instance


def two_link_day(v0, v1):
    """Speeds [2 links][H_speed] from per-interval lists."""
    return np.array([v0, v1], dtype=np.float64)


def test_constant_speed_closed_form():
    """At constant speeds a path takes sum(len / v) whatever the departure."""
    lens = np.array([1.3, 4.1, 0.7, 6.2, 2.0])
    v = np.array([0.9, 1.1, 0.4, 0.8, 1.3])
    H = 20
    sp = np.repeat(v[:, None], H, axis=1)
    pp = np.array([0, 5, 8])
    pl = np.array([0, 1, 2, 3, 4, 4, 2, 0])
    c = orc.path_costs(pp, pl, lens, np.stack([sp, sp, sp]), 5.0, H)
    assert c.shape == (H, 2)
    np.testing.assert_allclose(c[:, 0], np.sum(lens / v), rtol=1e-14)
    np.testing.assert_allclose(c[:, 1], lens[4] / v[4] + lens[2] / v[2] + lens[0] / v[0], rtol=1e-14)


def test_hand_computed_step_speeds():
    """A 2-link path (3 mi, 2 mi), dt = 5 min, speeds in mi/min per interval:
    link 0: 0.5, 0.5, 1; link 1: 0.5, 0.25, 1.  Each link is crossed at the
    speed of the interval in which it is entered (eq. "cost"):
      depart 0:  6 min on link 0, enter link 1 at 6 (interval 1): 8 min  -> 14
      depart 5:  6 min, enter link 1 at 11 (interval 2): 2 min           -> 8
      depart 10: 3 min, enter link 1 at 13 (interval 2): 2 min           -> 5
      depart 15: after the day the last interval's speeds hold           -> 5
    A second day at 1 mi/min everywhere takes 5 min; c~ is the mean."""
    day1 = two_link_day([0.5, 0.5, 1.0], [0.5, 0.25, 1.0])
    day2 = np.ones((2, 3))
    pp, pl, ln = np.array([0, 2]), np.array([0, 1]), np.array([3.0, 2.0])
    c1 = orc.path_costs(pp, pl, ln, day1, 5.0, 4)[:, 0]
    np.testing.assert_allclose(c1, [14.0, 8.0, 5.0, 5.0], rtol=1e-15)
    c = orc.path_costs(pp, pl, ln, np.stack([day1, day2]), 5.0, 4)[:, 0]
    np.testing.assert_allclose(c, [9.5, 6.5, 5.0, 5.0], rtol=1e-15)


def test_zero_days_gives_zero():
    c = orc.path_costs(np.array([0, 1]), np.array([0]), np.array([1.0]), np.ones((0, 1, 3)), 5.0, 3)
    assert np.all(c == 0)


def test_logit_two_paths_closed_form():
    """Two routes of one OD: p_1 = 1 / (1 + exp(-theta (c_2 - c_1))); with
    theta = 0.01 per second and costs of 300 s and 400 s, p_1 = 1/(1 + e^-1)."""
    cost = np.array([[300.0, 400.0], [500.0, 500.0], [400.0, 300.0]])
    p = orc.logit_portions(1, np.array([0, 0]), 0.01, cost)
    e = 1.0 / (1.0 + np.exp(-1.0))
    np.testing.assert_allclose(p, [[e, 1 - e], [0.5, 0.5], [1 - e, e]], rtol=1e-15)


def test_logit_invariants():
    """Per (OD, interval): portions sum to 1, a cheaper route gets the larger
    portion, adding a constant to an OD's costs changes nothing, theta = 0
    gives equal portions and a single route gets 1; large theta * cost stays
    finite (the maximum is subtracted before exp)."""
    rng = np.random.default_rng(5)
    path_od = np.array([0, 0, 0, 1, 2, 2])
    P, T = 3, 7
    cost = rng.uniform(200, 900, size=(T, 6))
    p = orc.logit_portions(P, path_od, 0.01, cost)
    for od in range(P):
        sel = path_od == od
        np.testing.assert_allclose(p[:, sel].sum(axis=1), 1.0, rtol=1e-14)
        for t in range(T):
            order_c = np.argsort(cost[t, sel], kind="stable")
            assert np.all(np.diff(p[t, sel][order_c]) <= 0)
    np.testing.assert_allclose(p[:, 3], 1.0)
    shift = cost.copy()
    shift[:, :3] += 1234.5
    np.testing.assert_allclose(orc.logit_portions(P, path_od, 0.01, shift), p, rtol=1e-12)
    u = orc.logit_portions(P, path_od, 0.0, cost)
    np.testing.assert_allclose(u, np.array([1 / 3] * 3 + [1.0] + [0.5] * 2)[None, :].repeat(T, 0),
                               rtol=1e-15)
    big = orc.logit_portions(P, path_od, 50.0, cost)
    assert np.all(np.isfinite(big))
    np.testing.assert_allclose(big[:, path_od == 0].sum(axis=1), 1.0, rtol=1e-14)


def small_choice(ragged=True, seed=0):
    return make_choice_instance(L=24, P=5, H=12, K=3, m=3, sizes=(3,), ragged=ragged,
                                seed=1000 + seed)


def test_assign_constant_portions_match_free_logits():
    """Portions that do not depend on the interval give the assignment of the
    time-independent logit form with the same softmax."""
    ci = small_choice(seed=1)
    rng = np.random.default_rng(3)
    Rr = rng.uniform(0, 1, size=(ci.K, ci.T, ci.n_pairs))
    z = rng.standard_normal(ci.n_paths)
    pi = orc.route_softmax(ci.P, ci.path_od, z)

    class RI:   # the fields rho_from_logits reads
        pass
    ri = RI()
    for f in ("P", "L", "T", "H", "K", "n_paths", "nnz", "path_od", "row_ptr", "col_idx"):
        setattr(ri, f, getattr(ci, f))
    ri.pair_ptr, ri.pair_link, ri.R = ci.path_ptr, ci.path_link, [Rr]
    W1 = orc.rho_from_logits(ri, 0, z)
    W2 = orc.rho_from_portions(ci.P, ci.L, ci.T, ci.H, ci.K, ci.path_od, ci.path_ptr, ci.path_link,
                               ci.row_ptr, ci.col_idx, Rr, np.tile(pi, (ci.T, 1)))
    np.testing.assert_allclose(W2, W1, rtol=1e-14, atol=0)


def test_assign_conservation():
    """When every pair's ratios sum to 1 over the lags, the lag sum of entry
    (a, p) at interval t is the portion of OD p's interval-t demand whose
    route crosses link a: the sum of p[t][k] over those routes."""
    for seed in range(3):
        ci = small_choice(seed=seed)
        rng = np.random.default_rng(seed)
        Rr = rng.uniform(0, 1, size=(ci.K, ci.T, ci.n_pairs))
        Rr /= Rr.sum(axis=0, keepdims=True)
        p = rng.uniform(0, 1, size=(ci.T, ci.n_paths))
        W = orc.rho_from_portions(ci.P, ci.L, ci.T, ci.H, ci.K, ci.path_od, ci.path_ptr,
                                  ci.path_link, ci.row_ptr, ci.col_idx, Rr, p)
        lagsum = W.sum(axis=0)                                   # [T][nnz]
        expect = np.zeros((ci.T, ci.nnz))
        rows = np.repeat(np.arange(ci.L), np.diff(ci.row_ptr))
        for j in range(ci.nnz):
            a, od = rows[j], ci.col_idx[j]
            for k in np.nonzero(ci.path_od == od)[0]:
                if a in ci.path_link[ci.path_ptr[k]:ci.path_ptr[k + 1]]:
                    expect[:, j] += p[:, k]
        np.testing.assert_allclose(lagsum, expect, rtol=1e-13)
        assert np.all(expect > 0)


def test_pipeline_single_route_is_delta_rho():
    """With one route per OD every portion is 1 (any theta), and the
    assignment is the path's ratios placed at its pattern entries."""
    ci = make_choice_instance(L=24, P=3, H=12, K=3, m=3, sizes=(2,), ragged=False, seed=1100)
    keep = np.array([i % 3 == 0 for i in range(ci.n_paths)])   # freeway route of each OD
    pp = np.concatenate([[0], np.cumsum(np.diff(ci.path_ptr)[keep])])
    pl = np.concatenate([ci.path_link[ci.path_ptr[k]:ci.path_ptr[k + 1]] for k in np.nonzero(keep)[0]])
    od = ci.path_od[keep]
    sp = ci.speed.astype(np.float64)
    Rr = orc.dar_from_speeds(pp, pl, ci.link_len, sp, ci.dt, ci.H, ci.K)
    c = orc.path_costs(pp, pl, ci.link_len, sp, ci.dt, ci.T)
    p = orc.logit_portions(ci.P, od, 0.6, c)
    np.testing.assert_array_equal(p, 1.0)
    rows = np.repeat(np.arange(ci.L), np.diff(ci.row_ptr))
    S = np.zeros((ci.L, ci.P), dtype=bool)
    S[pl, np.repeat(od, np.diff(pp))] = True
    rp = np.concatenate([[0], np.cumsum(S.sum(axis=1))]).astype(np.int32)
    col = np.nonzero(S)[1].astype(np.int32)
    W = orc.rho_from_portions(ci.P, ci.L, ci.T, ci.H, ci.K, od, pp, pl, rp, col, Rr, p)
    rows = np.repeat(np.arange(ci.L), np.diff(rp))
    for m in range(pl.shape[0]):
        k = np.searchsorted(pp, m, side="right") - 1
        j = np.nonzero((rows == pl[m]) & (col == od[k]))[0][0]
        np.testing.assert_array_equal(W[:, :, j], Rr[:, :, m])


def test_costs_order_follows_congestion():
    """In the deepest-congestion pattern the freeway route costs more than the
    arterial one in the AM peak on inbound corridors and less at night, so the
    logit moves demand to the arterial in the peak."""
    ci = make_choice_instance(L=160, P=6, H=288, K=6, m=10, sizes=(3, 2), seed=1200)
    sel = ci.day_cluster == 0
    c = orc.path_costs(ci.path_ptr, ci.path_link, ci.link_len, ci.speed[sel].astype(np.float64),
                       ci.dt, ci.T)
    p = orc.logit_portions(ci.P, ci.path_od, 0.6, c)   # 0.01 per second in minutes
    seg = ci.L // 8
    for od in range(ci.P):
        ks = np.nonzero(ci.path_od == od)[0]
        first = ci.path_link[ci.path_ptr[ks[0]]]
        if (first // seg) % 2 != 0:
            continue   # outbound: AM peak is light
        f, a = ks[0], ks[1]
        night, peak = 2 * 12, 8 * 12        # 02:00 and 08:00
        assert c[night, f] < c[night, a] and p[night, f] > p[night, a]
        assert c[peak, f] > c[peak, a] and p[peak, f] < p[peak, a]
