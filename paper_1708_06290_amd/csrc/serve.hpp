// Device-side pieces of the serving layer shared by the host scheduler and
// the work-item kernel.
#pragma once

#include "kernels.hpp"

namespace shs {

// One shift of one request: everything its wavefront needs.
struct ServeItem {
    const double *H;      // the system's H (column-major)
    int64_t ldh;
    const double *Rtop;   // m x m leading block of R
    double *refl;         // reflector store of this shift (FP64 sweep layout for m)
    double *Y;            // m x m scratch for the back substitution
    double *X;            // first column of this shift's n x m output block
    int64_t ldx;
    int32_t *status;
    double sr, si;        // the shift
    int n, m;
};

// Launch the work-item kernel over items[0 .. count) (device array); counter
// must be zero on entry.  Returns the launch error, if any.
hipError_t launch_serve(const ServeItem *items, int count, unsigned *counter, hipStream_t st);

}  // namespace shs
