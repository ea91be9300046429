// Decision paths of the frames shown between two rendered frames (host code).
//
// Paper §IV-B (problem formulation) and Table V: between rendered frames F_t
// and F_t+1, P_1, P_2, P_3 are shown at t + 1/4, 2/4, 3/4. d1 (at t) shows
// W(F_t) at t + 1/4, or F_t again, after which E(F_t) is ready at t + 1/2.
// After d1 = warp, d2 (at t + 1/4) shows W(P_1) or E(F_t) at t + 1/2. At
// t + 1/2 one more decision picks P_3: d3 (after d1 = extrapolate) between
// W(P_2) and P_2 again; d4 (after d2 = warp) and d5 (after d2 = extrapolate)
// between W(P_2) and E(P_1). The six paths are Table V's S1..S6.
//
// The fixed policy stands in for the paper's learned predictor (which needs
// trained weights): warp at a node when the frame's motion variance and the
// out-of-frame fraction of the warp that node would show are both within
// given limits.
#include <cmath>

#include "exwarp.h"
#include "launch.h"

namespace {

void set_frame(exw_display_plan *p, int i, int32_t kind, int32_t source) {
    p->kind[i] = kind;
    p->source[i] = source;
}

}  // namespace

extern "C" {

exw_status exw_decision_plan(int32_t d1, int32_t d2, int32_t d_last, exw_display_plan *plan) {
    if (!plan) return exw::report(EXW_ERROR_INVALID_VALUE, "plan is NULL");
    const bool ok1 = d1 == EXW_DECIDE_WARP || d1 == EXW_DECIDE_EXTRAPOLATE;
    const bool ok3 = d_last == EXW_DECIDE_WARP || d_last == EXW_DECIDE_EXTRAPOLATE;
    if (!ok1 || !ok3)
        return exw::report(EXW_ERROR_INVALID_VALUE, "d1 and d_last must be warp or extrapolate");
    exw_display_plan p;
    if (d1 == EXW_DECIDE_EXTRAPOLATE) {
        // F_t again at t + 1/4; E(F_t) is ready at t + 1/2 (no node at t + 1/4)
        set_frame(&p, 0, EXW_SHOW_REPEAT, EXW_FROM_RENDERED);
        set_frame(&p, 1, EXW_SHOW_EXTRAPOLATE, EXW_FROM_RENDERED);
        if (d_last == EXW_DECIDE_WARP) {
            p.scenario = 2;
            set_frame(&p, 2, EXW_SHOW_WARP, EXW_FROM_P2);
        } else {
            p.scenario = 1;
            set_frame(&p, 2, EXW_SHOW_REPEAT, EXW_FROM_P2);
        }
        p.node[0] = 1;
        p.node[1] = 0;
        p.node[2] = 3;
    } else {
        if (d2 != EXW_DECIDE_WARP && d2 != EXW_DECIDE_EXTRAPOLATE)
            return exw::report(EXW_ERROR_INVALID_VALUE, "d2 must be warp or extrapolate after d1 = warp");
        set_frame(&p, 0, EXW_SHOW_WARP, EXW_FROM_RENDERED);
        p.node[0] = 1;
        p.node[1] = 2;
        if (d2 == EXW_DECIDE_WARP) {
            set_frame(&p, 1, EXW_SHOW_WARP, EXW_FROM_P1);
            p.node[2] = 4;
            p.scenario = d_last == EXW_DECIDE_WARP ? 6 : 5;
        } else {
            set_frame(&p, 1, EXW_SHOW_EXTRAPOLATE, EXW_FROM_RENDERED);
            p.node[2] = 5;
            p.scenario = d_last == EXW_DECIDE_WARP ? 4 : 3;
        }
        if (d_last == EXW_DECIDE_WARP)
            set_frame(&p, 2, EXW_SHOW_WARP, EXW_FROM_P2);
        else
            set_frame(&p, 2, EXW_SHOW_EXTRAPOLATE, EXW_FROM_P1);
    }
    p.new_frames = 0;
    for (int i = 0; i < 3; ++i) p.new_frames += p.kind[i] != EXW_SHOW_REPEAT ? 1 : 0;
    *plan = p;
    return exw::report(EXW_SUCCESS, "");
}

exw_status exw_threshold_policy(const double *motion_stats, const double *invalid_fraction,
                                double max_variance, double max_invalid, int32_t *decisions) {
    if (!motion_stats || !invalid_fraction || !decisions)
        return exw::report(EXW_ERROR_INVALID_VALUE, "NULL argument");
    if (std::isnan(max_variance) || std::isnan(max_invalid))
        return exw::report(EXW_ERROR_INVALID_VALUE, "thresholds must not be NaN");
    const double var = motion_stats[1] + motion_stats[3];
    const bool calm = var <= max_variance;  // false for a NaN variance
    auto pick = [&](int k) {
        return calm && invalid_fraction[k] <= max_invalid ? EXW_DECIDE_WARP
                                                          : EXW_DECIDE_EXTRAPOLATE;
    };
    decisions[0] = pick(0);
    decisions[1] = decisions[0] == EXW_DECIDE_WARP ? pick(1) : EXW_DECIDE_NONE;
    decisions[2] = pick(2);
    return exw::report(EXW_SUCCESS, "");
}

}  // extern "C"
