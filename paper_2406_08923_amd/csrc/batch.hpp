// batch.hpp -- device job table and launchers of the batched substep kernel
// (internal).
#pragma once

#include "rk_point.hpp"

namespace stn {

// One resident job of the batch: a scalar advection-diffusion field (2-D or
// 3-D, radius-3 periodic padding) integrated with the fused RK3 substep.
struct BatchJob {
    void *f[2];     // state buffers (storage type), used in ping-pong
    void *w;        // register (FP64 for POL_F64, FP32 otherwise)
    void *w2;       // second register (master policies)
    double *f64;    // FP64 master state (master policies)
    Geo g;
    FdWeights fd;
    double inv_ds[3], adv[3], nu, dt;
    int policy;     // RkPolicy
    int steps;      // RK steps to take in this tick
    int parity;     // index of the buffer holding the state when the tick starts
    int tiles_x, tiles_y; // per-point: tile_w x tile_h tiles; z march: 64 x 16 tiles
    int lz;               // z march: planes per tile
    int tile_w, tile_h;   // per-point: points per tile along x and y (product BT_X * BT_Y)
    int tile_begin; // first work item of the job (within its kind)
};

// Per-point work items are tiles of one plane, one lane per point: BT_X x
// BT_Y lanes per workgroup, shaped per job as tile_w x tile_h points
// (tile_w * tile_h = BT_X * BT_Y; 64 x 4 unless the server's search chose
// another shape for the job's class). The shape changes no result.
constexpr int BT_X = 64, BT_Y = 4;

// Table order: the n2d per-point jobs first (2-D jobs and small 3-D jobs:
// 64 x 4 tiles of one plane, total_tiles items), then the z-march jobs (3-D
// jobs of at least ZM_MIN_POINTS points: tiles of 64 x 16 points x lz
// planes, total3 items); each job's tile_begin counts within its own kind.
struct BatchTableHeader {
    int njobs;
    int total_tiles;
    int n2d;
    int total3;
};

// Table = header followed by njobs BatchJob records (device memory).
inline size_t batch_table_bytes(int njobs)
{
    return sizeof(BatchTableHeader) + sizeof(BatchJob) * (size_t)njobs;
}

// RK coefficients passed by value (alpha_i, beta_i of substeps 0..2).
struct RkCoeffs {
    double alpha[3], beta[3];
};

// The RK3 scheme's coefficients (defined with the C ABI of the fused substep).
RkCoeffs rk3_coeffs();

// One substep (sub = 3 * step + stage within the tick) of every job whose
// step < steps, by persistent grids of `blocks` workgroups walking the items
// (one launch for the 2-D jobs, one for the 3-D jobs).
int launch_batch_substep(const void *d_table, int sub, const RkCoeffs &rk, int blocks,
                         hipStream_t s);

// Copy a contiguous FP64 interior (x fastest) into a padded state buffer of
// storage type per policy (and into the FP64 master for master policies),
// then refresh the periodic halo of the state buffer.
int launch_job_upload(const double *src, const BatchJob &j, int which, hipStream_t s);

// Copy the interior of the job's state (the FP64 master for master policies)
// into a contiguous FP64 array.
int launch_job_download(const BatchJob &j, int which, double *dst, hipStream_t s);

} // namespace stn
