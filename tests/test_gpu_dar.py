"""Dynamic assignment ratios from link speeds on the GPU (dode_dar_from_speeds)
against the FP64 oracle: FP64 and FP32 (FP32 against the oracle's binary32
walk, so both sides take each link at the same interval's speed), ragged path
lengths, several day chunks, the FIFO / zero-window cases, and the argument
checks."""
import numpy as np
import pytest

import oracle as orc
import paper_1901_09266_amd as dode
from synth import make_speed_instance
from gpu_helpers import say, dev, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run(si, K, dt, speed, f64=True):
    t = torch.float64 if f64 else torch.float32
    return dode.dode_dar_from_speeds(dev(si.path_ptr, torch.int32), dev(si.path_link, torch.int32),
                                     dev(si.link_len, t), dev(speed, t), dt, si.H, K)


@pytest.mark.parametrize("f64", [True, False])
def test_matches_oracle_ragged_paths(f64):
    si = make_speed_instance(L=80, P=20, H=60, sizes=(5, 2), inc=0.1, seed=11)
    # ragged paths: cut every path to its own length (1 .. 8 links)
    lens = np.arange(20) % 8 + 1
    keep = np.concatenate([si.path_link[si.path_ptr[k]:si.path_ptr[k] + lens[k]] for k in range(20)])
    si.path_link = keep.astype(np.int32)
    si.path_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    say("dar ragged", f64)
    for days in (slice(0, 5), slice(5, 7)):
        R = run(si, 6, si.dt, si.speed[days], f64)
        torch.cuda.synchronize()
        Ro = orc.dar_from_speeds(si.path_ptr, si.path_link, si.link_len, si.speed[days].astype(np.float64),
                                 si.dt, si.H, 6, walk="f64" if f64 else "f32")
        got = R.cpu().numpy()
        if f64:
            assert np.max(np.abs(got - Ro)) <= 1e-12
        else:
            # both sides cross each link at the speed of the same interval
            # (the walk in binary32); what is left is the FP32 window
            # arithmetic: end points within a few ulps of 60 minutes on
            # windows of about 5 minutes
            assert np.max(np.abs(got - Ro)) <= 2e-5


@pytest.mark.parametrize("K", [3, 7, 8, 12, 16])
def test_lag_counts_fp64(K):
    """Every unrolled window instance (up to 6, 8 and 16 lags) against the oracle."""
    si = make_speed_instance(L=80, P=12, H=40, sizes=(3,), inc=0.15, seed=15)
    say("dar lags", K)
    R = run(si, K, si.dt, si.speed, True)
    torch.cuda.synchronize()
    Ro = orc.dar_from_speeds(si.path_ptr, si.path_link, si.link_len, si.speed.astype(np.float64),
                             si.dt, si.H, K)
    assert np.max(np.abs(R.cpu().numpy() - Ro)) <= 1e-12


def test_several_day_chunks_fp32(monkeypatch):
    """160 days of a 500-link corridor with the trajectory scratch capped at
    1 GiB need two chunks (154 days each); the chunked day mean must equal
    the oracle's."""
    monkeypatch.setenv("DODE_DAR_SCRATCH_BYTES", str(1 << 30))
    si = make_speed_instance(L=500, P=150, H=288, sizes=(160,), seed=12)
    say("dar chunks")
    R = run(si, 6, si.dt, si.speed, f64=False)
    torch.cuda.synchronize()
    # the oracle walks the trajectories in binary32 too, so both sides take
    # every link at the same interval's speed; the rest is the FP32 window
    # arithmetic and the FP32 running sum over 160 days
    Ro = orc.dar_from_speeds(si.path_ptr, si.path_link, si.link_len, si.speed.astype(np.float64),
                             si.dt, si.H, 6, walk="f32")
    err = np.abs(R.cpu().numpy() - Ro)
    assert err.mean() <= 1e-7 and err.max() <= 2e-5


def test_fifo_and_zero_window_fp64():
    si = make_speed_instance(L=8, P=1, H=6, sizes=(2,), inc=0.25, seed=13)
    si.path_ptr = np.array([0, 2], dtype=np.int32)
    si.path_link = np.array([0, 1], dtype=np.int32)
    si.link_len = np.array([4.0, 1.0] + [1.0] * 6)
    sp = np.ones((2, 8, 6))
    sp[0, 0, 0], sp[0, 0, 1] = 1.0 / 3.0, 4.0       # overtaking: swapped end points
    sp[1, 0, 0], sp[1, 0, 1] = 0.5, 4.0 / 3.0       # equal entry times: zero window
    say("dar fifo")
    for d in range(2):
        R = run(si, 4, 5.0, sp[d])
        torch.cuda.synchronize()
        Ro = orc.dar_from_speeds(si.path_ptr, si.path_link, si.link_len, sp[d], 5.0, 6, 4)
        assert np.max(np.abs(R.cpu().numpy() - Ro)) <= 1e-12


def test_argument_checks():
    si = make_speed_instance(L=16, P=2, H=12, sizes=(1,), inc=0.25, seed=14)
    say("dar checks")
    bad = si.path_link.copy()
    bad[1] = 99
    with pytest.raises(dode.DodeError, match="path_link"):
        dode.dode_dar_from_speeds(dev(si.path_ptr, torch.int32), dev(bad, torch.int32),
                                  dev(si.link_len, torch.float64), dev(si.speed, torch.float64), 5.0, 12, 4)
    sp = si.speed.astype(np.float64).copy()
    sp[0, 3, 4] = 0.0
    with pytest.raises(dode.DodeError, match="positive"):
        run(si, 4, 5.0, sp)
    with pytest.raises(dode.DodeError, match="K="):
        run(si, 17, 5.0, si.speed)
