// Stopping rule of the Krylov solvers at the rounding floor of an FP64 iterate (the
// test of eq. (4.3), ||b - A x|| <= tol ||b||, evaluated in FP64).  Host code, shared by
// the library and a host-compiled test.
//
// The solver replaces its recurrence's residual by the true residual at regular steps
// (each time the recurrence has halved since the last replacement: a full period) and
// whenever the recurrence reaches tol.  Far above the floor the true residual follows
// the recurrence; the iterations a full period takes measure how fast it converges.  The
// solver stops when the true residual has gone that many iterations without a 10 % gain
// over its best, twice in a row (progress is judged over the iterations in which a
// converging solve would have halved its residual, not from one check to the next: near
// tol the checks come every few iterations, and a solve still converging there shows
// small gains between them), and the true residual is at the rounding floor: at most
// kFloorFactor max(tol, rho), rho the floor of the iterate, u || |b| + sum_e |A_e| |x_e| ||
// / ||b||, a bound on how far one more FP64 rounding of x can move the residual
// (measured stagnation levels of PCG sit at a quarter to a third of it).  Near the floor
// the true residual of a replacement swings by a factor of a few around rho (it carries
// the rounding the iterate gathered since the last replacement, which the next step
// removes), so once stalled the solve keeps checking at every later replacement.  A
// solve that goes kGiveUpStalls windows without progress and never reaches the floor
// has stalled above it and is reported as not converged.
#pragma once

#include <cmath>

namespace agca {

constexpr double kReplaceEvery = 0.5;  // a full period: the recurrence halved since the last replacement
constexpr double kFloorFactor = 1.0;   // a floor stop needs rel_true <= max(tol, rho)
constexpr double kEndGain = 0.9;       // progress: 10 % below the best true residual so far
constexpr int kEndStalls = 2;          // windows in a row without progress: stop at the floor
constexpr int kGiveUpStalls = 6;       // ... stop above it (not converged)

struct EndChecks {
    double best = HUGE_VAL;
    int best_it = 0;    // iteration of the best true residual
    int mark = 0;       // iteration of the best, or of the last window without progress
    int stalls = 0;
    int last_full = 0;  // iteration of the last replacement after a full period
    int period = -1;    // iterations between the last two of them (-1: none measured yet)
    // record the true residual of a replacement at iteration it that is still above tol
    // (full: the recurrence had halved since the last replacement); true when the
    // iteration should stop.  Before any full period the window is the iteration count
    // at which the best was reached.
    bool stagnated(double rel_true, int it, bool full) {
        if (full) {
            period = it - last_full;
            last_full = it;
        }
        const int window = period > 0 ? period : (best_it > 1 ? best_it : 1);
        if (rel_true < kEndGain * best) {
            best = rel_true;
            best_it = mark = it;
            stalls = 0;
        } else if (it - mark >= window) {
            ++stalls;
            mark = it;
        }
        return stalls >= kEndStalls;
    }
    // after stagnated(): whether the solve has gone too long without progress to wait for
    // the floor any longer
    bool given_up() const { return stalls >= kGiveUpStalls; }
};

// whether a stop with true relative residual rel_true counts as the rounding floor
inline bool at_floor(double rel_true, double tol, double rho) {
    return rel_true <= kFloorFactor * std::fmax(tol, rho);
}

}  // namespace agca
