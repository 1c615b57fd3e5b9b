// filter_kernels.hpp -- launchers of the nonlinear window filters (internal).
#pragma once

#include "common.hpp"

namespace stn {

// op codes (the STENCIL_OP_* values of the public header)
constexpr int FILTER_OP_MAX = STENCIL_OP_MAX;
constexpr int FILTER_OP_MIN = STENCIL_OP_MIN;
constexpr int FILTER_OP_MEDIAN = STENCIL_OP_MEDIAN;
// largest window the median kernel selects from
constexpr int FILTER_MEDIAN_MAX = STENCIL_MEDIAN_MAX;

// One lane per output, window offsets listed (ntaps entries, element units).
template <typename S>
int launch_filter_gather(const S *in, S *out, const Geo &g, const int *offs, int ntaps, int op,
                         bool fuse, int bx, int by, hipStream_t s);

// 3-D box window of radius R (1..3), max or min, marching along z over lz
// planes per workgroup. dpp = false: LDS planes, ty lanes along y (4 or 8),
// ny and pf ignored. dpp = true: no LDS, x neighbours exchanged across lanes;
// ty waves per workgroup (4 or 8), ny rows per lane (2 or 4), pf planes in
// flight (1 or 3; 0 and 2 mean 1); xcd: XCD-aware order.
template <typename S>
int launch_filter_box3d(const S *in, S *out, const Geo &g, int R, int op, bool fuse, int ty,
                        int ny, int pf, int lz, bool dpp, int xcd, hipStream_t s);

} // namespace stn
