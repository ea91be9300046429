"""Oracle of the decision paths and chained warps (test infrastructure only).

What is computed (paper §IV-B, problem formulation, and Table V): between
rendered frames F_t and F_t+1 the frames P_1, P_2, P_3 are shown at t + i/4.
Decision d1 at t picks P_1: the warp W(F_t), or F_t again, in which case
the extrapolation E(F_t) is shown at t + 1/2. After d1 = warp, decision d2 at
t + 1/4 picks P_2 = W(P_1) or E(F_t). At t + 1/2 one more decision picks
P_3: after d1 = extrapolate, d3 picks W(P_2) or P_2 again; after d1 = warp,
d4 / d5 pick W(P_2) or E(P_1). The six paths are Table V's S1..S6.

Readings taken where the paper is silent:

* Of d4 and d5, d4 is the decision after d2 = warp and d5 the one after
  d2 = extrapolate (the text names them together).
* A warp of a predicted frame, W(P_i), advances it by one display interval:
  the forward warp of P_i with the motion of F_t (the only motion there is)
  at phase 1/4. P_i is used as an ordinary frame (its invalid pixels are 0).
* Frames are stored in the storage dtype between steps, as displayed frames
  are; ``store`` rounds each step's output before the next one.
* The fixed policy (a stand-in for the paper's learned predictor, which
  needs trained weights) warps at a decision node when the frame's motion
  variance Var_x + Var_y and the out-of-frame fraction of the warp that node
  would show are both at most given thresholds, else it extrapolates (or, at
  d3, shows P_2 again).

Nothing here is shared with, or imported by, the HIP path.
"""

from __future__ import annotations

import numpy as np

from . import warp_oracle

WARP, EXTRAPOLATE = 0, 1
REPEAT_KIND, WARP_KIND, EXTRAPOLATE_KIND = "repeat", "warp", "extrapolate"


def plan(d1: int, d2: int | None, d_last: int) -> dict:
    """Frames shown for decisions (d1, d2, the decision at t + 1/2).

    Returns ``{"scenario": "S1".."S6", "P1": (kind, source), "P2": ...,
    "P3": ..., "nodes": (1, 2 or None, 3/4/5), "new_frames": n}`` with kinds
    "repeat"/"warp"/"extrapolate" and sources "F", "P1", "P2".
    """
    if d1 not in (WARP, EXTRAPOLATE) or d_last not in (WARP, EXTRAPOLATE):
        raise ValueError("decisions are WARP (0) or EXTRAPOLATE (1)")
    if d1 == EXTRAPOLATE:
        # F_t again at t + 1/4, E(F_t) at t + 1/2 (no decision at t + 1/4)
        p1, p2 = (REPEAT_KIND, "F"), (EXTRAPOLATE_KIND, "F")
        if d_last == WARP:
            scen, p3 = "S2", (WARP_KIND, "P2")
        else:
            scen, p3 = "S1", (REPEAT_KIND, "P2")
        nodes = (1, None, 3)
    else:
        if d2 not in (WARP, EXTRAPOLATE):
            raise ValueError("d2 is needed after d1 = warp")
        p1 = (WARP_KIND, "F")
        if d2 == WARP:
            p2 = (WARP_KIND, "P1")
            scen, p3 = ("S6", (WARP_KIND, "P2")) if d_last == WARP else ("S5", (EXTRAPOLATE_KIND, "P1"))
            nodes = (1, 2, 4)
        else:
            p2 = (EXTRAPOLATE_KIND, "F")
            scen, p3 = ("S4", (WARP_KIND, "P2")) if d_last == WARP else ("S3", (EXTRAPOLATE_KIND, "P1"))
            nodes = (1, 2, 5)
    new = sum(1 for p in (p1, p2, p3) if p[0] != REPEAT_KIND)
    return {"scenario": scen, "P1": p1, "P2": p2, "P3": p3, "nodes": nodes, "new_frames": new}


def chained_warp(src, mv, phase: float, steps: int, store=None):
    """P_1 = W(src, phase), P_i = W(P_{i-1}, phase) with the same motion.

    ``src`` [N,C,H,W], ``mv`` [N,2,H,W]. Returns (out [S,N,C,H,W], mask
    [S,N,H,W], count [S,N]) in float64 / uint8 / int64. ``store`` (a function)
    rounds each step's frames to the storage dtype before the next step.
    """
    frames = np.asarray(src, dtype=np.float64)
    outs, masks, counts = [], [], []
    for _ in range(steps):
        out, mask, cnt = warp_oracle.forward(frames, mv, [phase])
        out = out[:, 0]
        if store is not None:
            out = np.asarray(store(out), dtype=np.float64)
        outs.append(out)
        masks.append(mask[:, 0])
        counts.append(cnt[:, 0])
        frames = out
    return np.stack(outs), np.stack(masks), np.stack(counts)


def threshold_policy(stats, invalid_fraction, max_variance: float, max_invalid: float):
    """Decisions (d1, d2, d_last) of the fixed policy for one frame.

    ``stats`` = (mean_x, var_x, mean_y, var_y) of the frame's motion;
    ``invalid_fraction`` = out-of-frame fraction of W(F_t) at phases 1/4,
    2/4, 3/4 (the warps shown at t + 1/4, t + 1/2 and t + 3/4). Node d1 looks
    at phase 1/4, d2 at 2/4, the last node at 3/4. Returns d2 = None when d1
    extrapolates.
    """
    var = float(stats[1]) + float(stats[3])
    calm = var <= max_variance

    def pick(k):
        return WARP if calm and float(invalid_fraction[k]) <= max_invalid else EXTRAPOLATE

    d1 = pick(0)
    d2 = pick(1) if d1 == WARP else None
    return d1, d2, pick(2)
