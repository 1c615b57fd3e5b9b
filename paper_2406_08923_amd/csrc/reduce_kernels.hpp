// reduce_kernels.hpp -- deterministic FP64 diagnostics (internal).
#pragma once

#include "common.hpp"

namespace stn {

// Number of pass-1 workgroups for a geometry (fixed by the grid shape).
int reduce_nblocks(const Geo &g);

struct FieldPtrs {
    const void *p[8];
};

// nfields <= 8 device pointers; d_partial: 3 * nfields * reduce_nblocks(g)
// doubles; d_out: 3 * nfields doubles.
int launch_reduce(const FieldPtrs &d_fields, int nfields, int dtype, const Geo &g,
                  double *d_partial, double *d_out, hipStream_t s);

} // namespace stn
