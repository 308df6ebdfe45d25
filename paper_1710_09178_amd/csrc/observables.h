// Gauge observables of the handle's links.
#pragma once

#include "common.h"

namespace stag {

// Partial sums of Re and Im tr[U_t(x,0) ... U_t(x,Nt-1)] over the spatial
// sites, [2][nb] by block; returns nb.
int launch_polyakov(const Geom& g, const double2* links, double* part, hipStream_t s);

}  // namespace stag
