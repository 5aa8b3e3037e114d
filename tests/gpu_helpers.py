"""Shared helpers of the GPU tests: move a synthetic instance into the library
and print the case before each GPU step."""
import sys

import numpy as np

import paper_1901_09266_amd as dode


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def make_dar(inst, storage="f64", W=None, correction=False):
    return dode.dar_create(inst.P, inst.L, inst.T, inst.H, inst.K, inst.row_ptr, inst.col_idx,
                           inst.W if W is None else W, storage=storage, correction=correction,
                           stream=0)


def dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def e4m3_table():
    """All non-negative finite OCP E4M3FN values, indexed by code 0..126."""
    vals = []
    for code in range(127):
        e, m = code >> 3, code & 7
        vals.append(m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7))
    return np.array(vals)


def quantize_e4m3(v):
    """Round |v| <= 448 to the nearest E4M3FN value, ties to the even code."""
    tab = e4m3_table()
    a = np.abs(v).ravel()
    idx = np.searchsorted(tab, a)
    idx = np.clip(idx, 1, len(tab) - 1)
    lo, hi = tab[idx - 1], tab[idx]
    pick_hi = (hi - a < a - lo) | ((hi - a == a - lo) & ((idx % 2) == 0))
    out = np.where(pick_hi, hi, lo)
    out = np.where(a >= 448, 448.0, out)
    return (np.sign(v).ravel() * out).reshape(v.shape)


def quantize_bf16(v):
    """Round to bfloat16 (8 significant bits), ties to even."""
    a = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(a)                      # a = m 2^e, |m| in [0.5, 1)
    return np.ldexp(np.round(m * 256.0), e - 8)   # np.round is round-half-even


def fp8_values(W, col_idx):
    """(FP8 values, corrected values) of one cluster's [K][T][nnz] values: one
    FP32 scale per (lag, interval, 64-OD group); the corrected value of
    refinement steps is h + c with h = bf16(fp32(scale * code)), c = bf16(w - h)."""
    tiles = col_idx // 64
    Wq, Wr = np.zeros_like(W), np.zeros_like(W)
    for tile in np.unique(tiles):
        sel = tiles == tile
        Ws = W[:, :, sel]
        amax = np.abs(Ws).max(axis=2, keepdims=True)
        sc = np.where(amax > 0, (amax / 448.0).astype(np.float32).astype(np.float64), 1.0)
        code = quantize_e4m3(Ws / sc)
        Wq[:, :, sel] = code * sc
        prod = (code.astype(np.float32) * sc.astype(np.float32)).astype(np.float64)
        h = quantize_bf16(prod)
        Wr[:, :, sel] = h + quantize_bf16(Ws - h)
    return Wq, Wr


def dequantized_values(inst, storage):
    """The values the library holds for each storage type, computed here from FP64
    ("fp8corr": the corrected values of refinement steps)."""
    out = []
    for W in inst.W:
        if storage in ("f64",):
            out.append(W.copy())
        elif storage == "f32":
            out.append(W.astype(np.float32).astype(np.float64))
        elif storage == "bf16":
            out.append(quantize_bf16(W))
        elif storage in ("fp8", "fp8corr"):
            out.append(fp8_values(W, inst.col_idx)[0 if storage == "fp8" else 1])
    return out


def rel_elem(a, b, floor_frac=1e-3):
    """Largest elementwise |a - b| / max(|b|, floor), floor = floor_frac * max|b|:
    every entry is held to its own size, down to a floor for entries near zero."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    floor = max(floor_frac * float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)))
