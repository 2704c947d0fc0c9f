// hqr_refine_rule.hpp -- the stopping rule of the mixed-precision
// refinement, for one right-hand side.  Kept free of any runtime header so
// the host test suite compiles the same rule the device runs; the includer
// defines HQR_HD (the function's execution-space qualifiers).
#pragma once

namespace hqr {

struct RefineState {
    int first;    // 1-based step at which the column converged (0: not yet)
    int failed;   // the corrections stalled above the floor twice
    int stalls;   // consecutive steps whose ||dx|| did not halve
    int frozen;   // converged or failed: x no longer changes
    double prev;  // ||dx|| of the previous step
};

// One step (0-based `step`) with ndx = ||dx|| and nx = ||x + dx||:
//   * converged when ndx <= tol * nx;
//   * a correction that did not halve (ndx > prev / 2) is the rounding floor
//     of the iteration: accepted as converged when ndx <= floor * nx, else a
//     stall; two stalls in a row end the run as failed;
//   * a NaN correction never satisfies a test, so the column runs out of
//     steps unconverged.
HQR_HD inline void refine_rule_step(RefineState &st, int step, double ndx, double nx, double tol, double floor)
{
    if (st.frozen) return;
    if (ndx <= tol * nx) {
        st.first = step + 1;
        st.frozen = 1;
    } else if (step > 0 && ndx > 0.5 * st.prev) {
        if (ndx <= floor * nx) {
            st.first = step + 1;
            st.frozen = 1;
        } else if (++st.stalls >= 2) {
            st.failed = 1;
            st.frozen = 1;
        }
    } else {
        st.stalls = 0;
    }
    st.prev = ndx;
}

} // namespace hqr
