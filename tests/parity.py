"""Parity criteria between the HIP library and the FP64 oracle.

Same Philox streams on both sides, so differences come only from rare
branch flips of FP32 arithmetic (or none at all in FP64):
  * total detected weight: relative difference <= 0.5 %;
  * per bin: z_b = |W_gpu - W_ora| / sqrt(Var_gpu + Var_ora) <= 3 for every
    bin with weight, Var_b = W2_b - W_b^2 / N;
  * L1 spectrum error sum |W_gpu - W_ora| / sum W_ora <= 1 %;
  * GPU conservation exact in fixed point: sum of bins and sinks equals
    N * 2^32.
"""
from __future__ import annotations

import numpy as np

SCALE = 4294967296


def conservation_exact(g: dict, n_packets: int) -> bool:
    tot = int(np.sum(g["w_fx"], dtype=np.uint64)) + sum(int(v) for v in g["sinks_fx"].values())
    return tot == n_packets * SCALE


def metrics(g: dict, o: dict, n: int) -> dict:
    Wg, Wo = np.asarray(g["W"], dtype=np.float64), np.asarray(o["W"], dtype=np.float64)
    var = (g["W2"] - Wg**2 / n) + (o["W2"] - Wo**2 / n)
    use = (g["W2"] > 0) | (o["W2"] > 0)
    z = np.zeros_like(Wg)
    z[use] = np.abs(Wg[use] - Wo[use]) / np.sqrt(np.maximum(var[use], 1e-300))
    tot_o = Wo.sum()
    return {
        "total_rel": abs(Wg.sum() - tot_o) / tot_o if tot_o > 0 else abs(Wg.sum()),
        "z_max": float(z.max()) if z.size else 0.0,
        "l1": float(np.abs(Wg - Wo).sum() / tot_o) if tot_o > 0 else float(np.abs(Wg).sum()),
    }


def assert_parity(g: dict, o: dict, n: int, total_tol=5e-3, z_tol=3.0, l1_tol=1e-2):
    m = metrics(g, o, n)
    assert m["total_rel"] <= total_tol, m
    assert m["z_max"] <= z_tol, m
    assert m["l1"] <= l1_tol, m
    return m
