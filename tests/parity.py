"""Comparison of the HIP path (through the C ABI) with the FP64 oracle, pair by pair.

Protocol:
  masks   valid-correspondence sets must match exactly, except (a) points whose FP64
          projection lies within 1e-4 px of an integer coordinate (a cell decision) and
          (b) occlusion-gate near-ties (|margin| < 1e-5 m); both are counted.
  H, b    the oracle is re-run on the GPU's own correspondences ("mask-forced": same valid
          set, same integer cells); per 6x6 block max|dH| <= tol * max|H_block|, per
          component |db| <= tol * sum|terms|, F within tol relative.
"""
import numpy as np

import oracle

GPU_STATUS_FROM_ORACLE = np.array([0, 1, 2, 3, 4, 4, 6, 4], np.uint8)


def compare_pair_masks(ctx, prob, poses, k, band=1e-4, gate=1e-5, params=None, grad_mode=0):
    s, t = (int(v) for v in prob.pairs[k])
    sen = prob.sensors[prob.kf_sensor[s]]
    g = ctx.debug_pair(k, (sen["H"], sen["W"]))
    # status 5: the early depth-interval rejection would drop a point that passes the occlusion gate in
    # a cell it can reach (a band point's too, which the mask comparison below exempts)
    assert not np.any(g["status"] == 5), ("interval test drops a point", k, np.argwhere(g["status"] == 5)[:5])
    o = oracle.eval_pair(prob, poses, s, t, params or prob.params, pixels=True, grad_mode=grad_mode)
    gv = g["status"] == 0
    ov = o["status"] == 0
    mism = gv != ov
    uv = o["uv"]
    with np.errstate(invalid="ignore"):
        dist = np.nanmin(np.abs(uv - np.round(uv)), axis=-1)
    dist = np.where(np.isfinite(dist), dist, np.inf)
    near_int = dist < band
    near_gate = np.abs(np.nan_to_num(o["margin"], nan=np.inf)) < gate
    if (params or prob.params).get("occlusion_zbuffer", 0):
        # z-buffer variant: a point within the band of a cell boundary may enter either cell's
        # z-buffer, so the decisions of the points in the cells it can reach are ties as well
        Wt = prob.sensors[prob.kf_sensor[t]]["W"]
        fin = np.isfinite(uv).all(-1)
        bu = uv[near_int & fin]
        tied = set()
        for du in (-band, band):
            for dv in (-band, band):
                cx, cy = np.floor(bu[:, 0] + du).astype(np.int64), np.floor(bu[:, 1] + dv).astype(np.int64)
                tied.update((cy * Wt + cx).tolist())
        own = np.full(uv.shape[:2], -1, np.int64)
        own[fin] = (np.floor(uv[fin][:, 1]).astype(np.int64) * Wt + np.floor(uv[fin][:, 0]).astype(np.int64))
        near_gate = near_gate | np.isin(own, np.fromiter(tied, np.int64, len(tied)))
    bad = mism & ~near_int & ~near_gate
    code_mismatch = (GPU_STATUS_FROM_ORACLE[o["status"]] != g["status"]) & ~mism & ~near_int & ~near_gate
    return dict(gpu=g, orc=o, n_mismatch=int(mism.sum()), n_band=int((mism & near_int).sum()),
                n_gate=int((mism & near_gate & ~near_int).sum()), n_bad=int(bad.sum()),
                n_code=int(code_mismatch.sum()), n_valid=int(ov.sum()), bad_idx=np.argwhere(bad)[:10])


def forced_oracle(prob, poses, k, gpu_dbg, params=None, grad_mode=0):
    s, t = (int(v) for v in prob.pairs[k])
    fv = (gpu_dbg["status"] == 0).astype(np.uint8)
    fc = gpu_dbg["cell"].astype(np.int32)
    return oracle.eval_pair(prob, poses, s, t, params or prob.params, force_valid=fv, force_cell=fc,
                            grad_mode=grad_mode)


def compare_pair_sums(gpu_row, orc, tol):
    """Errors of one GPU pair record against the oracle's pair result, normalised as in the protocol."""
    Hg = gpu_row[:144].reshape(12, 12)
    bg = gpu_row[144:156]
    Ho = orc["H12"]
    worst = 0.0
    for r in (0, 6):
        for c in (0, 6):
            blk_o = Ho[r:r + 6, c:c + 6]
            scale = np.abs(blk_o).max()
            if scale == 0:
                continue
            worst = max(worst, np.abs(Hg[r:r + 6, c:c + 6] - blk_o).max() / scale)
    bscale = np.maximum(orc["babs12"], 1e-300)
    berr = float(np.max(np.abs(bg - orc["b12"]) / bscale)) if orc["n_valid"] else 0.0
    Ferr = abs(gpu_row[156] - orc["F"]) / max(abs(orc["F"]), 1e-300) if orc["n_valid"] else abs(gpu_row[156])
    counts_ok = int(gpu_row[157]) == orc["n_eval"] and int(gpu_row[158]) == orc["n_valid"]
    return dict(H=worst, b=berr, F=Ferr, counts_ok=counts_ok, ok=(worst <= tol and berr <= tol and Ferr <= tol
                                                                  and counts_ok))
