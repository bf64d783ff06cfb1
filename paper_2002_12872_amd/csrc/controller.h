// Step control shared by dpt_solve and the serving engine: precision phases,
// stopping rule and statuses (host code).
//
// delta_k = max |Z_k - Z_{k-1}| after the k-th application of the map, compared
// with tol directly or through the contraction bound (DPT_STOP_ESTIMATE).  The
// BF16 phase runs until that test passes or a stall and then always hands over to
// FP32 sweeps (its fixed point is biased by the BF16 product); FP32 ends with
// OK when delta_k < tol, optionally followed by FP64 sweeps to fp64_final_tol.
// A stall is a rounding floor: no progress by stall_ratio for stall_patience
// checks while delta already sits within ~1e4 ulps of the state's magnitude;
// larger non-decreasing deltas (cycles, chaos) run to the cap.
#pragma once

#include <algorithm>
#include <cmath>
#include <limits>

#include "dpt.h"
#include "dpt_internal.h"

namespace dpt {

struct Controller {
    enum Action { CONTINUE = 0, TO_FP32 = 1, TO_FP64 = 2, DONE = 3 };

    dpt_options o{};
    bool allow_fp64 = true;
    int phase = PH_FP32;
    int status = DPT_NOT_CONVERGED;
    int iters = 0;
    int it_phase[3] = {0, 0, 0};
    double best = std::numeric_limits<double>::infinity();
    int stall_run = 0;
    double last = std::numeric_limits<double>::quiet_NaN();
    // step ratios delta_k / delta_{k-1} inside one phase (r1 the most recent)
    double prev = std::numeric_limits<double>::quiet_NaN();
    double r1 = std::numeric_limits<double>::quiet_NaN(), r2 = std::numeric_limits<double>::quiet_NaN();

    // Distance-to-fixed-point proxy compared with tol.
    double error_measure(double dl) const {
        if (o.stop_rule != DPT_STOP_ESTIMATE || dl == 0.0) return dl;
        if (!(r1 < 0.5) || !(r2 < 0.5)) return dl;  // contraction not established: delta rule
        const double rho = std::max(r1, r2);
        return rho * dl / (1.0 - rho);
    }

    void start(const dpt_options &opt, int initial_phase, bool fp64_allowed) {
        o = opt;
        phase = initial_phase;
        allow_fp64 = fp64_allowed;
    }

    // Record one application of the map made in the current phase.
    void count_step() {
        ++iters;
        ++it_phase[phase];
    }

    bool capped() const { return iters >= o.max_iter; }

    // Decide after a step whose statistics are (dl, wm).  The caller applies
    // phase switches (TO_FP32 needs nothing; TO_FP64 needs the state upcast).
    Action update(double dl, double wm) {
        static const double kFloor[3] = {1.0, 1e4 * 5.96e-8, 1e4 * 1.11e-16};
        last = dl;
        if (!std::isfinite(dl) || !(wm <= o.blowup)) {
            status = DPT_DIVERGED;
            return DONE;
        }
        if (prev > 0.0 && std::isfinite(prev)) {
            r2 = r1;
            r1 = dl / prev;
        }
        prev = dl;
        const double err = error_measure(dl);
        bool stalled = false;
        if (dl == 0.0) {
            stalled = true;
        } else if (dl >= o.stall_ratio * best && dl <= kFloor[phase] * std::max(1.0, wm)) {
            stalled = ++stall_run >= o.stall_patience;
        } else {
            stall_run = 0;
        }
        best = std::min(best, dl);
        if (phase == PH_BF16) {
            if (err < o.tol || stalled) {
                phase = PH_FP32;
                reset_progress();
                return TO_FP32;
            }
        } else if (phase == PH_FP32) {
            if (err < o.tol) {
                if (o.fp64_final_tol > 0.0 && allow_fp64) {
                    phase = PH_FP64;
                    reset_progress();
                    return TO_FP64;
                }
                status = DPT_OK;
                return DONE;
            }
            if (stalled) {
                status = DPT_STALLED;
                return DONE;
            }
        } else {
            const double target = (o.precision == DPT_FP64) ? o.tol : o.fp64_final_tol;
            if (err < target) {
                status = DPT_OK;
                return DONE;
            }
            if (stalled) {
                status = DPT_STALLED;
                return DONE;
            }
        }
        return CONTINUE;
    }

    // A step of the coupling ramp (Supplement E): the map changes from step to
    // step, so neither convergence nor stall nor the contraction ratios are
    // judged; a non-finite or blown-up iterate still ends the solve.
    Action update_ramping(double dl, double wm) {
        last = dl;
        if (!std::isfinite(dl) || !(wm <= o.blowup)) {
            status = DPT_DIVERGED;
            return DONE;
        }
        return CONTINUE;
    }

    // Every row met its own stopping test (DPT_STOP_ROW).
    void finish_ok(double dl) {
        last = dl;
        status = DPT_OK;
    }

    void fill(dpt_result *r) const {
        if (!r) return;
        r->status = status;
        r->iters = iters;
        r->iters_bf16 = it_phase[PH_BF16];
        r->iters_fp32 = it_phase[PH_FP32];
        r->iters_fp64 = it_phase[PH_FP64];
        r->last_delta = last;
    }

  private:
    // New phase: restart stall tracking; the next delta measures the change of
    // fixed point (rounding bias), not contraction, so no ratio is formed with it
    // while the previous phase's ratios stay as the contraction estimate.
    void reset_progress() {
        best = std::numeric_limits<double>::infinity();
        stall_run = 0;
        prev = std::numeric_limits<double>::quiet_NaN();
    }
};

}  // namespace dpt
