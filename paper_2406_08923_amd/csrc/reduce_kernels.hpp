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

// Sixth-order first-derivative weights (unit spacing, offsets 1..3) and the
// inverse grid spacings.
struct EnergyCoef {
    double w1[3];
    double ids[3];
};

// Kinetic and magnetic sums of the 8 MHD fields (padded 3-D, periodic halos):
// d_out[0] = sum |u|^2, d_out[1] = sum |curl A|^2, d_out[2] = 0; d_partial: 3 *
// reduce_nblocks(g) doubles. Deterministic (fixed partition and tree).
int launch_energy(const FieldPtrs &d_fields, int dtype, const Geo &g, const EnergyCoef &ec,
                  double *d_partial, double *d_out, hipStream_t s);

} // namespace stn
