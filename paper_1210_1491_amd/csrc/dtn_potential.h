// The final potential's sources (eq. bw03), shared by the direct sum and the
// treecode.
#pragma once

#include "dtn_internal.h"

namespace dtn {

// One tile quadrature point: position, outward normal, single-layer weight
// w sigma (fitted Neumann data) and double-layer weight w phi.
struct TileSource {
    double x, y, z, nx, ny, nz, ws, wf;
};

// Writes the 16 sources of every tile of the plan: source q of patch i goes
// to src[slot[16 i + q]], or to src[16 i + q] when slot is NULL.
dtn_status launch_tile_sources(const Plan &p, const double *neumann, const int32_t *slot, TileSource *src,
                               hipStream_t s);

}  // namespace dtn
