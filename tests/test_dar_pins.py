"""Pins of the oracle's dynamic assignment ratios from link speeds (eqs.
"dar2"/"dar", Example "DAR matrix computation", eq. "cost"), CPU only."""
import numpy as np
import pytest

import oracle as orc
from synth import make_speed_instance


def one_path(lengths):
    n = len(lengths)
    return np.array([0, n]), np.arange(n), np.asarray(lengths, dtype=np.float64)


def test_constant_speed_closed_form():
    """Constant speeds shift every interval by the travel time o to the link:
    the window [h dt + o, (h+1) dt + o] puts 1 - f in lag floor(o/dt) and f in
    the next, f = o/dt - floor(o/dt)."""
    dt, H, K = 5.0, 24, 6
    lens = [1.3, 4.1, 0.7, 6.2, 2.0]
    pp, pl, ln = one_path(lens)
    v = 0.9
    sp = np.full((len(lens), H), v)
    R = orc.dar_from_speeds(pp, pl, ln, sp, dt, H, K)
    offs = np.concatenate([[0.0], np.cumsum(np.array(lens) / v)[:-1]])
    for i, o in enumerate(offs):
        l0 = int(np.floor(o / dt))
        f = o / dt - l0
        for h in range(H - K):
            expect = np.zeros(K)
            expect[l0] += 1 - f
            if l0 + 1 < K:
                expect[l0 + 1] += f
            np.testing.assert_allclose(R[:, h, i], expect, atol=1e-13)


def test_worked_example_fractions():
    """Example "DAR matrix computation": a path over three links; the DARs of
    departure interval H_1 follow from the boundary trajectories departing at
    t^1 and t^2.  Link 1 gives 1; link 2's window straddles H_1 / H_2
    (omega_1 + omega_2); link 3's starts in H_1, covers H_2 and ends in H_3
    (omega_3 + |H_2| + omega_4)."""
    dt, H, K = 5.0, 6, 4
    L1, L2 = 1.0, 2.0
    # link speeds per interval: the t^1 = 0 departure crosses links 1 and 2
    # inside H_1 at slopes zeta_1 = zeta_2 = 1; the t^2 = dt departure meets
    # zeta_1' = 0.5 on link 1 and zeta_2' = 0.4 on link 2 (entered in H_2)
    sp = np.ones((3, H))
    sp[0, 1] = 0.5
    sp[1, 1] = 0.4
    pp, pl, ln = one_path([L1, L2, 1.0])
    R = orc.dar_from_speeds(pp, pl, ln, sp, dt, H, K)
    t1, t2 = 0.0, dt
    c1 = L1 / sp[0, 0]
    e2, e2p = t1 + c1, t2 + L1 / sp[0, 1]           # entry times at link 2
    e3, e3p = e2 + L2 / sp[1, 0], e2p + L2 / sp[1, 1]   # entry times at link 3
    assert e2 < dt <= e2p < 2 * dt and e3 < dt and 2 * dt <= e3p < 3 * dt
    w1 = t2 - (t1 + c1)        # the example's omega_1 = t^2 - (t^1 + c_1(t^1))
    w2 = e2p - t2
    w3 = dt - e3
    w4 = e3p - 2 * dt
    assert R[0, 0, 0] == pytest.approx(1.0)
    assert R[0, 0, 1] == pytest.approx(w1 / (w1 + w2), rel=1e-14)
    assert R[1, 0, 1] == pytest.approx(w2 / (w1 + w2), rel=1e-14)
    total = w3 + dt + w4
    assert R[0, 0, 2] == pytest.approx(w3 / total, rel=1e-14)
    assert R[1, 0, 2] == pytest.approx(dt / total, rel=1e-14)
    assert R[2, 0, 2] == pytest.approx(w4 / total, rel=1e-14)
    assert (w1, w2, w3, w4) == pytest.approx((4.0, 2.0, 2.0, 2.0))


def test_shares_sum_to_one_inside_the_band():
    si = make_speed_instance(L=64, P=12, H=48, sizes=(3, 2), inc=0.1, seed=7)
    R = orc.dar_from_speeds(si.path_ptr, si.path_link, si.link_len, si.speed, si.dt, si.H, 8)
    assert R.min() >= 0 and R.max() <= 1 + 1e-12
    tot = R.sum(axis=0)                       # [H][n_pairs]
    # every window ends well before lag 8 and the last hour: all mass kept
    np.testing.assert_allclose(tot[: si.H - 12], 1.0, atol=1e-12)


def test_day_mean_is_the_mean_of_single_days():
    si = make_speed_instance(L=48, P=8, H=36, sizes=(4,), inc=0.15, seed=8)
    R = orc.dar_from_speeds(si.path_ptr, si.path_link, si.link_len, si.speed, si.dt, si.H, 6)
    each = [orc.dar_from_speeds(si.path_ptr, si.path_link, si.link_len, si.speed[d], si.dt, si.H, 6)
            for d in range(4)]
    np.testing.assert_allclose(R, np.mean(each, axis=0), atol=1e-14)


def test_entry_times_follow_eq_cost():
    """The window of departure interval h at the i-th link runs between the
    entry times of the departures at h dt and (h+1) dt, each the composition of
    the link travel times (eq. "cost"); checked against a step-by-step
    simulation of the two vehicles at 1e-4 minute resolution."""
    dt, H, K = 5.0, 20, 8
    rng = np.random.default_rng(3)
    lens = rng.uniform(0.5, 2.0, size=6)
    sp = rng.uniform(0.3, 1.2, size=(6, H))
    pp, pl, ln = one_path(lens)
    R = orc.dar_from_speeds(pp, pl, ln, sp, dt, H, K)

    def simulate(t0):
        t, out, step = t0, [t0], 1e-4
        for a in range(6):
            v = sp[a, min(int(np.floor(t / dt)), H - 1)]   # speed fixed at entry
            x = 0.0
            while x < lens[a]:
                x += v * step
                t += step
            out.append(t)
        return out

    for h in (0, 3, 7):
        s, e = simulate(h * dt), simulate((h + 1) * dt)
        for i in range(6):
            lo, hi = min(s[i], e[i]), max(s[i], e[i])
            for l in range(K):
                a, b = max(lo, (h + l) * dt), min(hi, (h + l + 1) * dt)
                want = max(b - a, 0.0) / (hi - lo)
                assert abs(R[l, h, i] - want) <= 2e-4, (h, i, l)


def test_fifo_violation_and_zero_window():
    """A sharp speed-up lets the later departure overtake: the end points are
    swapped (the window between them).  Equal entry times give a zero window:
    all the interval's share goes to the interval of that instant."""
    dt, H, K = 5.0, 6, 4
    pp, pl, ln = one_path([4.0, 1.0])
    sp = np.ones((2, H))
    sp[0, 0] = 1.0 / 3.0  # departures at 0 cross link 1 in 12 minutes
    sp[0, 1] = 4.0        # those at 5 in 1 minute: entry times 12 and 6, swapped
    R = orc.dar_from_speeds(pp, pl, ln, sp, dt, H, K)
    assert R[1, 0, 1] == pytest.approx((10.0 - 6.0) / 6.0)
    assert R[2, 0, 1] == pytest.approx((12.0 - 10.0) / 6.0)
    assert R[0, 0, 1] == pytest.approx(0.0)
    # zero window: link 1 crossed by the departures at 0 and at 5 both at 8
    sp[0, 0], sp[0, 1] = 0.5, 4.0 / 3.0
    R = orc.dar_from_speeds(pp, pl, ln, sp, dt, H, K)
    assert R[1, 0, 1] == pytest.approx(1.0) and R[:, 0, 1].sum() == pytest.approx(1.0)


def binary32_boundary_path():
    """Three links; the first takes 5 - 1e-9 minutes at speed 1, which is
    5 exactly once rounded to binary32, so a binary32 walk enters the second
    link at the 5-minute boundary (interval 1, speed 0.5) and a binary64 walk
    just before it (interval 0, speed 1)."""
    dt, H, K = 5.0, 6, 4
    pp, pl, ln = one_path([5.0 - 1e-9, 1.0, 1.0])
    sp = np.ones((3, H))
    sp[1, 1] = 0.5
    assert np.float32(ln[0]) == np.float32(5.0) and ln[0] < 5.0
    return dt, H, K, pp, pl, ln, sp


def test_binary32_walk_decides_in_binary32():
    """walk="f32" takes the entry interval from the binary32 travel times.
    Departure interval 0 at the third link: the departure at 0 enters it at
    5 + 1/0.5 = 7 in binary32 (6 - 1e-9 in binary64), the one at 5 at
    5 + 5 + 1 = 11 (12 - 1e-9: link 1 entered at 10 - 1e-9, in interval 1).
    The windows [7, 11] and [6, 12] split over intervals 1 and 2 as 3:1 and
    4:2; the path costs of the departure at 0 (all three links) are 8 and
    7 - 1e-9."""
    dt, H, K, pp, pl, ln, sp = binary32_boundary_path()
    R32 = orc.dar_from_speeds(pp, pl, ln, sp, dt, H, K, walk="f32")
    R64 = orc.dar_from_speeds(pp, pl, ln, sp, dt, H, K)
    assert (R32[1, 0, 2], R32[2, 0, 2]) == (0.75, 0.25)
    assert R64[1, 0, 2] == pytest.approx(4.0 / 6.0, abs=1e-9)
    assert R64[2, 0, 2] == pytest.approx(2.0 / 6.0, abs=1e-9)
    c32 = orc.path_costs(pp, pl, ln, sp, dt, 2, walk="f32")
    c64 = orc.path_costs(pp, pl, ln, sp, dt, 2)
    assert c32[0, 0] == 8.0 and c64[0, 0] == pytest.approx(7.0, abs=1e-8)
    with pytest.raises(ValueError):
        orc.path_costs(pp, pl, ln, sp, dt, 2, walk="f16")


def test_binary32_walk_equals_binary64_when_exact():
    """Lengths in quarter units and speeds in {0.5, 1, 2, 4}: every travel
    time is a short binary fraction, exact in binary32, so both walks take the
    same decisions and give the same bits."""
    rng = np.random.default_rng(21)
    si = make_speed_instance(L=64, P=12, H=48, sizes=(3,), inc=0.1, seed=22)
    ln = rng.integers(1, 24, size=si.link_len.shape) * 0.25
    sp = np.array([0.5, 1.0, 2.0, 4.0])[rng.integers(0, 4, size=si.speed.shape)]
    R32 = orc.dar_from_speeds(si.path_ptr, si.path_link, ln, sp, si.dt, si.H, 8, walk="f32")
    R64 = orc.dar_from_speeds(si.path_ptr, si.path_link, ln, sp, si.dt, si.H, 8)
    assert np.array_equal(R32, R64) and R64.max() > 0
    c32 = orc.path_costs(si.path_ptr, si.path_link, ln, sp, si.dt, si.H, walk="f32")
    c64 = orc.path_costs(si.path_ptr, si.path_link, ln, sp, si.dt, si.H)
    assert np.array_equal(c32, c64)
