// Stopping rule of the Krylov solvers at the rounding floor of an FP64 iterate (the
// test of eq. (4.3), ||b - A x|| <= tol ||b||, evaluated in FP64).  Host code, shared by
// the library and a host-compiled test.
//
// An "end check" happens when the recurrence's residual has reached tol and the true
// residual, recomputed from x, is still above it.  The solver then continues from the
// true residual; it gives up when the true residual has stopped improving, and the stop
// counts as the rounding floor only when the true residual is within kFloorFactor of
// max(tol, rho), rho the floor of the iterate: u || |b| + sum_e |A_e| |x_e| || / ||b||
// (a bound on how far one more FP64 rounding of x moves the residual).  Otherwise the
// solve has stalled above the floor and is reported as not converged.
#pragma once

#include <cmath>

namespace agca {

constexpr double kFloorFactor = 2.0;   // a floor stop needs rel_true <= 2 max(tol, rho)
constexpr double kEndGain = 0.9;       // an end check improves when it is 10 % below the best
constexpr int kEndStalls = 2;          // end checks in a row without improvement that stop
constexpr int kMaxEndChecks = 8;       // end checks after which the solver stops anyway

struct EndChecks {
    double best = HUGE_VAL;
    int checks = 0;
    int stalls = 0;
    // record the true residual of an end check; true when the iteration should stop
    bool stagnated(double rel_true) {
        ++checks;
        if (rel_true < kEndGain * best) {
            best = rel_true;
            stalls = 0;
        } else {
            ++stalls;
        }
        return stalls >= kEndStalls || checks >= kMaxEndChecks;
    }
};

// whether a stop with true relative residual rel_true counts as the rounding floor
inline bool at_floor(double rel_true, double tol, double rho) {
    return rel_true <= kFloorFactor * std::fmax(tol, rho);
}

}  // namespace agca
