"""Host logic of the measurement script (no GPU): the per-launch byte model
behind the roofline figures, checked against closed forms and invariants
that any correct count must meet, and the lookup of committed traffic
counter summaries, which must refuse a summary taken on other kernel
sources."""
import os
import sys
from types import SimpleNamespace

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from synth import make_perms  # noqa: E402


def tiny(K, day_cluster, C=2, H=12, L=5, P=3, nnz=7):
    return SimpleNamespace(P=P, L=L, T=H, H=H, K=K, nnz=nnz, C=C,
                           day_cluster=np.asarray(day_cluster, dtype=np.int64))


@pytest.mark.parametrize("bh", [1, 4, 5, 12])
def test_single_lag_epoch_is_closed_form(bh):
    """K = 1: a minibatch reaches exactly its own intervals, so one epoch
    moves every X row once, every residual row out and back, every Q (and A)
    row once and every ratio block once."""
    inst = tiny(1, [0, 0, 1, 1, 1])
    perms = make_perms(5, 2, inst.C, inst.H)
    s, esz, D = 4, 2, 5
    fwd, adj = bench.launch_bytes(inst, perms, bh, esz, [1], s_state=s)
    assert len(fwd) == len(adj) == -(-inst.H // bh)
    blocks = inst.C * inst.T * inst.nnz * esz
    assert fwd.sum() == D * (inst.H * inst.L * (4 + s) + inst.T * inst.P * s) + blocks
    assert adj.sum() == D * (inst.H * inst.L * s + inst.T * inst.P * 4 * s) + blocks


@pytest.mark.parametrize("K", [2, 3, 6])
def test_ratio_blocks_read_once_per_epoch(K):
    """With no days only the ratio values remain: each block (l, t) with
    t + l < H is read once per epoch by the forward and once by the adjoint,
    whatever the permutation and the minibatch size."""
    inst = tiny(K, [])
    perms = make_perms(7, 3, inst.C, inst.H)
    nblk = sum(min(K, inst.H - t) for t in range(inst.T))
    for bh in (1, 3, 12):
        fwd, adj = bench.launch_bytes(inst, perms, bh, 1, [0, 2])
        assert fwd.sum() == adj.sum() == 2 * inst.C * nblk * inst.nnz


def test_lags_only_add_reached_rows():
    """K > 1 reaches more demand rows than K = 1 (never fewer), and the X and
    residual rows, fixed by the minibatch alone, are unchanged."""
    perms = make_perms(9, 1, 2, 12)
    f1, a1 = bench.launch_bytes(tiny(1, [0, 1, 1], nnz=0), perms, 4, 2, [0])
    f3, a3 = bench.launch_bytes(tiny(3, [0, 1, 1], nnz=0), perms, 4, 2, [0])
    assert np.all(f3 >= f1) and np.all(a3 >= a1) and f3.sum() > f1.sum()
    # with P = 0 only the X and residual rows are left: equal for any K
    f1p, a1p = bench.launch_bytes(tiny(1, [0, 1, 1], P=0, nnz=0), perms, 4, 2, [0])
    f3p, a3p = bench.launch_bytes(tiny(3, [0, 1, 1], P=0, nnz=0), perms, 4, 2, [0])
    assert np.array_equal(f1p, f3p) and np.array_equal(a1p, a3p)


def test_refinement_steps_move_everything():
    """Each full-batch refinement step reads every row and every block, with
    the 3-byte corrected values."""
    inst = tiny(2, [0, 1])
    perms = make_perms(11, 1, inst.C, inst.H)
    f0, _ = bench.launch_bytes(inst, perms, 4, 1, [0], refine=0)
    f2, a2 = bench.launch_bytes(inst, perms, 4, 1, [0], refine=2)
    assert len(f2) == len(f0) + 2 and np.array_equal(f2[2:], f0)
    nblk = sum(min(2, inst.H - t) for t in range(inst.T))
    full_f = 2 * (inst.H * inst.L * 8 + inst.T * inst.P * 4) + inst.C * nblk * inst.nnz * 3
    assert f2[0] == f2[1] == full_f


def test_traffic_lookup_follows_the_source_hash(monkeypatch, tmp_path):
    """A counter summary is used while the kernel sources hash to its
    recorded value, and refused (None) once they do not; a missing summary or
    kernel gives None."""
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_spgd_config3_bf16.md").write_text(
        "# summary\n\nsource_sha256: " + "ab" * 32 + "\nfwd_bytes_per_launch: 123\n"
        "adj_bytes_per_launch: 456\n")
    (tmp_path / "profiles" / "traffic_spgd_config2_perday_f32.md").write_text(
        "source_sha256: " + "ab" * 32 + "\nfwd_bytes_per_launch: 7\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "ab" * 32)
    assert bench.counted_traffic(3, "bf16", "fwd") == 123
    assert bench.counted_traffic(3, "bf16", "adj") == 456
    assert bench.counted_traffic(2, "f32", "fwd", "_perday") == 7
    assert bench.counted_traffic(2, "f32", "adj", "_perday") is None
    assert bench.counted_traffic(3, "fp8", "adj") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "cd" * 32)
    assert bench.counted_traffic(3, "bf16", "adj") is None


def test_traffic_per_epoch_and_schedule(monkeypatch, tmp_path):
    """The per-epoch figures a summary records with the schedule it was taken
    at: the minibatch launches' bytes per epoch, one refinement step's bytes,
    and the schedule string; all refused once the sources change."""
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_spgd_config5_fp8.md").write_text(
        "source_sha256: " + "ab" * 32 + "\nfwd_bytes_per_launch: 10\nadj_bytes_per_launch: 20\n"
        "minibatch_bytes_per_epoch: 3480\nrefine_bytes_per_step: 77\nschedule: 64,1,2\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "ab" * 32)
    assert bench.counted_traffic(5, "fp8", "minibatch") == 3480
    assert bench.counted_traffic(5, "fp8", "refine") == 77
    assert bench.counted_traffic(5, "fp8", "schedule") == "64,1,2"
    assert bench.counted_traffic(5, "fp8", "refine_fwd") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "cd" * 32)
    assert bench.counted_traffic(5, "fp8", "minibatch") is None


def test_epoch_bytes_is_the_touch_once_floor():
    """The headline roofline's bytes per epoch: each cluster's ratio nonzeros
    once (the lag band has sum_t min(K, H - t) blocks) plus, per day, X read
    once, Q read and written at 2 bytes (bf16 copy) and A read and written in
    FP32.  At 150 OD, 500 links, T = H = 288, K = 6, 8 clusters of 6000
    nonzeros per block and 1095 days this is 1.362816 GB."""
    inst = SimpleNamespace(P=150, L=500, T=288, H=288, K=6, nnz=6000, C=8, D=1095)
    nblk = 6 * 288 - (1 + 2 + 3 + 4 + 5)
    assert nblk == 1713
    want = 8 * nblk * 6000 * 2 + 1095 * (288 * 500 * 4 + 2 * 288 * 150 * 2 + 2 * 288 * 150 * 4)
    assert want == 1_362_816_000
    assert bench.epoch_bytes(inst, "bf16") == want
    # FP32 demand and the plain FP32 form count 4 bytes per demand value
    q32 = want + 1095 * 2 * 288 * 150 * 2
    assert bench.epoch_bytes(inst, "bf16", s_q=4) == q32
    assert bench.epoch_bytes(inst, "f32") == q32 + 8 * nblk * 6000 * 2
    # FP8 values: one byte per nonzero
    assert bench.epoch_bytes(inst, "fp8") == want - 8 * nblk * 6000


def test_alu_roofline_follows_the_source_hash(monkeypatch, tmp_path):
    """The ratio legs report the ALU bound from a committed VALU count only
    while the kernel source hashes to the value recorded with it; otherwise
    they fall back to the HBM figure and say why."""
    import hashlib
    src = tmp_path / "k.hip"
    src.write_text("kernel text\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "p.md").write_text(f"# x\n\nsource_sha256: {digest}\n"
                               "valu_instructions_per_step: 614400000000\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "DAR_SOURCES", ("k.hip",))
    r = bench.alu_roofline("p.md", "kern", 1000.0, 8_000_000_000)
    # 614.4e9 instructions in one second: exactly the ceiling
    assert r["bound"] == "alu" and abs(r["frac"] - 1.0) < 1e-12
    assert r["hbm"]["achieved_GBs"] == 8.0
    src.write_text("kernel text, changed\n")
    r = bench.alu_roofline("p.md", "kern", 1000.0, 8_000_000_000)
    assert r["bound"] == "hbm" and "note" in r and r["achieved"] == 8.0


def test_refinement_step_bytes():
    """A full-batch refinement step touches every array once like an epoch,
    with the ratio nonzeros read as the FP8 code and its bf16 correction (3
    bytes).  At the config-5 shapes (400 OD, 1500 links, 12 clusters of 48000
    nonzeros per block, 1095 days): 2.96 GB of ratios + 1095 days x (1.728 MB
    of observations + 0.4608 MB of demand + 0.9216 MB of accumulator)."""
    inst = SimpleNamespace(P=400, L=1500, T=288, H=288, K=6, nnz=48000, C=12, D=1095)
    nblk = 1713
    want = 12 * nblk * 48000 * 3 + 1095 * (288 * 1500 * 4 + 2 * 288 * 400 * 2 + 2 * 288 * 400 * 4)
    assert bench.refine_step_bytes(inst) == want
    assert abs(want - 6.3656e9) < 1e6
    assert bench.refine_step_bytes(inst, s_q=4) == want + 1095 * 2 * 288 * 400 * 2
