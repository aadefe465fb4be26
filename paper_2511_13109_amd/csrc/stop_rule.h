// Stopping rule of the Krylov solvers at the rounding floor of an FP64 iterate (the
// test of eq. (4.3), ||b - A x|| <= tol ||b||, evaluated in FP64).  Host code, shared by
// the library and a host-compiled test.
//
// The solver replaces its recurrence's residual by the true residual at regular steps
// (each time the recurrence has halved since the last replacement) and when the
// recurrence reaches tol.  Far above the floor the true residual follows the recurrence
// and halves between replacements; once it stops improving (no 10 % gain over the best
// earlier replacement, twice in a row) the solver stops, and so it does after
// kMaxEndChecks replacements made with the recurrence at tol.  The stop counts as the
// rounding floor only when the true residual is at most kFloorFactor max(tol, rho),
// rho the floor of the iterate: u || |b| + sum_e |A_e| |x_e| || / ||b||, a bound on how
// far one more FP64 rounding of x can move the residual (measured stagnation levels of
// PCG sit at a quarter to a third of it).  Otherwise the solve has stalled above the
// floor and is reported as not converged.
#pragma once

#include <cmath>

namespace agca {

constexpr double kFloorFactor = 1.0;   // a floor stop needs rel_true <= max(tol, rho)
constexpr double kEndGain = 0.9;       // a replacement improves when it is 10 % below the best
constexpr int kEndStalls = 2;          // replacements in a row without improvement that stop
constexpr int kMaxEndChecks = 8;       // replacements at tol after which the solver stops anyway

struct EndChecks {
    double best = HUGE_VAL;
    int end_checks = 0;
    int stalls = 0;
    // record the true residual of a replacement (at_end: the recurrence had reached tol)
    // that is still above tol; true when the iteration should stop
    bool stagnated(double rel_true, bool at_end) {
        if (at_end) ++end_checks;
        if (rel_true < kEndGain * best) {
            best = rel_true;
            stalls = 0;
        } else {
            ++stalls;
        }
        return stalls >= kEndStalls || end_checks >= kMaxEndChecks;
    }
};

// whether a stop with true relative residual rel_true counts as the rounding floor
inline bool at_floor(double rel_true, double tol, double rho) {
    return rel_true <= kFloorFactor * std::fmax(tol, rho);
}

}  // namespace agca
