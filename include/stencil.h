/*
 * stencil.h -- C ABI of the MI355X (gfx950) stencil library, libstencil.so.
 *
 * Plain C types only: device pointers are void*, HIP streams are passed as
 * void* (a hipStream_t, or NULL for the default stream). Every entry point
 * returns a stencil_status; nothing throws or aborts across the ABI. On
 * failure stencil_last_error() returns a thread-local message.
 *
 * Array layout (paper Sec. 2.4, Eq. 2 and Fig. 1; row-wise scan order of
 * Sec. 4.4): a field with interior dims[0] x dims[1] x dims[2] (x fastest) is
 * stored padded by r cells on both sides of every active axis. Axis a < ndim
 * has extent dims[a] + 2r, unused axes have extent 1; the linear index of
 * padded cell (x, y, z) is x + Px*(y + Py*z), and padded coordinate q holds
 * interior point q - r. Buffers are caller-owned and must be aligned to their
 * element size; stencil_padded_elems() gives the element count.
 *
 * Asynchrony: apply/step calls enqueue work on the given stream and return;
 * errors detected at enqueue time are returned, device faults surface at the
 * next synchronising call. Plans are immutable after creation and may be used
 * from several host threads and streams at once (the caller keeps buffers in
 * flight on different streams disjoint).
 */
#ifndef STENCIL_H
#define STENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int stencil_status;
#define STENCIL_OK 0
#define STENCIL_EINVAL (-1)       /* bad descriptor, pointer, size or aliasing */
#define STENCIL_ENOMEM (-2)       /* device or host allocation failed */
#define STENCIL_EUNSUPPORTED (-3) /* valid request this build does not implement */
#define STENCIL_EDEVICE (-4)      /* HIP runtime error (sticky for the plan) */
#define STENCIL_EAGAIN (-5)       /* server queue full */
#define STENCIL_ESTATE (-6)       /* call not valid in the object's state */
#define STENCIL_ETIMEOUT (-7)     /* wait timed out */

/* Storage types. Arithmetic is FP64 for F64 storage and FP32 for F32 and BF16
 * storage (BF16 values are widened exactly and results rounded to nearest
 * even). */
typedef enum { STENCIL_F64 = 0, STENCIL_F32 = 1, STENCIL_BF16 = 2 } stencil_dtype;

/* Boundary function beta of Eq. 2. PERIODIC: the library keeps halos periodic.
 * USER_HALO: the caller fills the input halo; only the interior is written. */
typedef enum { STENCIL_BC_PERIODIC = 0, STENCIL_BC_USER_HALO = 1 } stencil_bc;

/* Kernel variants of the linear cross-correlation (STENCIL_VARIANT_AUTO lets
 * the plan choose, with timing when STENCIL_FLAG_AUTOTUNE is set).
 *  GENERIC : one lane per output, every tap read through the hardware caches
 *            (any ndim, radius and tap pattern).
 *  STAR3D  : 3-D axis-aligned stencils (radius 1..4): x-y plane tile staged in
 *            LDS, z taps from a per-lane register window marching along z.
 *  LINE1D  : 1-D stencils: block working set staged in LDS, several outputs
 *            per lane.
 *  BOX3D   : 3-D stencils with all (2R+1)^3 taps of their radius-R box
 *            nonzero, R = 1..8 (the multiply-add-bound regime of Sec. 5.2):
 *            a z march reading each plane once that keeps in registers the
 *            partial sums of the 2R + 1 output planes a plane feeds: the
 *            halo'd plane staged in LDS, several adjacent outputs per lane
 *            (the default, R = 1..8), or at R = 1 x neighbours moved across
 *            lanes (DPP) with the taps in scalar registers. Also 2-D
 *            stencils with all (2R+1)^2 taps nonzero, R = 1..8, on arrays
 *            below 4 GiB: the same LDS march over blocks of rows. */
#define STENCIL_VARIANT_AUTO (-1)
#define STENCIL_VARIANT_GENERIC 0
#define STENCIL_VARIANT_STAR3D 1
#define STENCIL_VARIANT_LINE1D 2
#define STENCIL_VARIANT_BOX3D 3

#define STENCIL_FLAG_AUTOTUNE 1u /* time the candidate variants at plan time */

/* Linear stencil descriptor (Eq. 3 generalised by Eq. 6-7):
 *   out_p = sum over s in [-r, r]^ndim of coeffs_s * in_{p+s}.
 * coeffs: host pointer to the dense (2r+1)^ndim tensor, x fastest, copied by
 * stencil_plan; zero taps are pruned. radius 0..1024 for ndim 1 (the
 * large-radius regime of Sec. 5, Fig. 8), 0..8 for ndim 2 and 3 (r = 0 is a
 * copy). Periodic plans need dims[a] >= r on every active axis. */
typedef struct stencil_desc {
    int ndim;             /* 1, 2 or 3 */
    int dims[3];          /* interior extents (unused axes ignored) */
    int radius;
    const double *coeffs; /* host, (2r+1)^ndim doubles */
    int dtype;            /* stencil_dtype */
    int bc;               /* stencil_bc */
    unsigned flags;       /* STENCIL_FLAG_* */
    int variant;          /* STENCIL_VARIANT_* */
    /* launch overrides (all zero = the plan's choice), per variant:
     *   STAR3D : {lanes along y, rows per lane, z planes per workgroup,
     *             flags: bit 0 XCD-aware workgroup order, bit 1 separate halo
     *             pass instead of writing periodic images, bit 2 tiles
     *             numbered fastest along y (else x), bit 3 hardware-cached
     *             z march (x/y taps through L1/L2, no LDS; 64-lane-wide
     *             tiles; (lanes, rows) one of (4,1) (4,2) (4,4) (2,4) (8,2)
     *             and prefetch/width ignored), bits 4..7 planes
     *             prefetched ahead (0 = default 2; only 2 is built), bits
     *             8..11 tile width in 64-lane waves (0 = 1), bits 12..15
     *             iterations per launch (0/1 = one; 2 = two chained
     *             iterations in one pass over HBM, periodic plans and the LDS
     *             variant only: the temporal blocking the paper's discussion
     *             asks for; results are bitwise those of one-iteration
     *             launches), bit 16 (two iterations, two rows per lane,
     *             r <= 4, at most 768 lanes) LDS planes stored y-fastest so
     *             a lane's two rows are one 2-wide read, bit 17 (one
     *             iteration) lane-exchange z march: no LDS, x taps moved
     *             across the 64 lanes of a wave by DPP shifts (a wave yields
     *             64 - 2r columns), y taps outside the lane's rows loaded;
     *             (lanes, rows) = (waves per workgroup, rows per lane) one of
     *             (4,2) (4,4) (8,2) (8,4), planes in flight 1 or 3 (bits
     *             4..7; 0 and 2 mean 1), width ignored; results bitwise
     *             those of the LDS march}; one-iteration
     *             (width, lanes, rows) one of
     *             (1,8,2) (1,4,4) (1,8,4) (1,16,2) (2,4,2) (2,4,4) (2,8,2)
     *             (4,2,2) (4,2,4) (4,4,2) (8,1,4) (8,2,2); two-iteration
     *             (1,8,2) (1,16,1) (1,16,2) (1,12,2) (2,8,2) (1,8,4), the
     *             lane grid 64*width x lanes*rows yielding (64*width - 2r) x
     *             (lanes*rows - 2r) outputs per tile
     *   BOX3D  : lane exchange (R = 1 only): {waves per workgroup 4 or 8,
     *             rows per lane 1 or 2, z planes per workgroup, flags: bit 0
     *             XCD-aware order, bits 4..7 planes in flight 1 or 3 (0 and 2
     *             mean 1)}; a wave yields 62 columns. LDS march, R = 1..8
     *             (and 2-D boxes, where the third
     *             entry counts blocks of 4 x (outputs per lane) rows per
     *             workgroup): {waves per workgroup 4,
     *             outputs per lane along x 4 or 8 (4 for 3-D R = 5..8), z
     *             planes per workgroup,
     *             flags: bit 0 XCD-aware order}; a wave yields 64 columns of
     *             (outputs per lane) rows
     *   GENERIC: {block x, block y} (a multiple of 64 lanes, at most 1024)
     *   LINE1D : {outputs per lane: 1, 2, 4 or 8, iterations fused per
     *             launch T (0/1 = none; T > 1 periodic only: the block
     *             loads its range plus r*T wrapped cells once and iterates in
     *             LDS, the temporal blocking the paper's discussion asks for),
     *             register blocking (nonzero: the lane's outputs are adjacent
     *             and each input read from LDS feeds all of them; outputs per
     *             lane 4, 8 or 16, needs 2r + 1 >= outputs - 1 and T <= 1;
     *             bitwise equal to the plain line)} */
    int tile[4];
    /* Field layout (both 0 = compact, the layout of Eq. 2 with rows of
     * dims[0] + 2r cells). x_offset: column of interior x = 0 (>= radius);
     * row_pitch: elements from one row to the next (>= x_offset + dims[0] +
     * radius; ndim >= 2 only). Cells outside [x_offset - r, x_offset +
     * dims[0] + r) of a row are never read or written. A field then holds
     * stencil_plan_padded_elems(plan) elements; y/z padding is unchanged.
     * Starting the interior of every row on a 128-byte boundary (x_offset *
     * element size and row_pitch * element size multiples of 128) makes the
     * star kernel's tile rows whole cache lines. */
    int row_pitch;
    int x_offset;
    /* What the stencil function zeta computes (STENCIL_OP_*). XCORR (0): the
     * cross-correlation above. MAX / MIN: the max filter of Sec. 2.3 (and its
     * min twin) over the window of offsets whose coeffs entry is nonzero (the
     * values only mark the window). MEDIAN: the median filter of Sec. 1 over
     * that window (at most STENCIL_MEDIAN_MAX cells; the lower median when
     * the count is even). Filters order values numerically with -0 below +0;
     * a window holding a NaN yields NaN; results are elements of the window
     * (no rounding). Filters run the GENERIC gather (any window) or, for 3-D
     * max/min over a full box of radius 1..3, the STAR3D z march (tile: {y
     * lanes 4 or 8, 0, z planes per workgroup, flags}: bit 0 XCD-aware order,
     * bit 17 the lane-exchange march, then {waves per workgroup 4 or 8, rows
     * per lane 2 or 4, z planes per workgroup, flags with planes in flight 1
     * or 3 in bits 4..7 (3 with four rows at radius 1 only)}; the default for
     * arrays below 4 GiB); LINE1D and fused iterations are cross-correlation
     * only. */
    int op;
} stencil_desc;

#define STENCIL_OP_XCORR 0
#define STENCIL_OP_MAX 1
#define STENCIL_OP_MIN 2
#define STENCIL_OP_MEDIAN 3
#define STENCIL_MEDIAN_MAX 27

typedef struct stencil_plan_s *stencil_plan_t;

/* Thread-local description of the last failure in this thread. */
const char *stencil_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int stencil_version(void);

/* Number of elements of a field with interior dims padded by r (compact
 * layout). */
size_t stencil_padded_elems(int ndim, const int dims[3], int radius);

/* Number of elements of one field in the plan's layout (linear plans with a
 * row pitch: pitch * padded rows * padded planes; otherwise as
 * stencil_padded_elems). Returns 0 for a NULL plan. */
size_t stencil_plan_padded_elems(stencil_plan_t plan);

/* Create a linear plan on the current HIP device. The plan owns a device copy
 * of the pruned taps. With STENCIL_FLAG_AUTOTUNE the candidate variants are
 * timed once on scratch buffers (synchronous) and the choice is cached per
 * process for the same shape class (and in the file STENCIL_TUNE_CACHE names,
 * if set). Arrays of any size are accepted; the STAR3D variant reads its
 * input plane by plane (one buffer resource per plane), except its
 * hardware-cached form (tile flag bit 3), which needs arrays below 4 GiB. */
stencil_status stencil_plan(const stencil_desc *desc, stencil_plan_t *out);

/* Release a plan (waits for nothing: the caller must not destroy a plan with
 * work in flight). NULL is accepted. */
stencil_status stencil_plan_destroy(stencil_plan_t plan);

/* Variant the plan will launch (after tuning), or a negative status. */
int stencil_plan_variant(stencil_plan_t plan);

/* Launch parameters the plan will use, in the layout of stencil_desc.tile for
 * its variant (passing them back in a descriptor reproduces the choice). */
stencil_status stencil_plan_tile(stencil_plan_t plan, int tile[4]);

/* iters chained applications on stream. d_a and d_b are caller-owned padded
 * device buffers of the plan's dtype and may not overlap. Iteration k reads
 * one and writes the other, starting d_a -> d_b, so the result is in d_b when
 * iters is odd and in d_a when even (iters = 0 does nothing).
 * PERIODIC: d_a's halo may be refreshed (its halo cells written) before the
 * first iteration, and the result carries a valid periodic halo; the other
 * buffer's contents are unspecified on return (launches of two iterations
 * never materialise the odd iterate, and only the last of them writes its
 * output's halo).
 * USER_HALO: iters must be 1; the caller's halo of d_a is read and only the
 * interior of d_b is written. */
stencil_status stencil_apply(stencil_plan_t plan, void *d_a, void *d_b, int iters,
                             void *stream);

/* stencil_apply with flags. STENCIL_APPLY_HALO_VALID: the caller guarantees
 * d_a's periodic halo is already valid (e.g. it is the result of an earlier
 * apply), so no halo refresh is launched and d_a is not written before the
 * first iteration. The launches are those of stencil_apply: a plan with two
 * iterations per launch issues a number of launches with the parity of iters
 * (e.g. iters = 2 runs as two one-iteration launches, iters = 4 as two
 * two-iteration launches). Other bits must be zero. */
#define STENCIL_APPLY_HALO_VALID 1u
stencil_status stencil_apply_ex(stencil_plan_t plan, void *d_a, void *d_b, int iters,
                                unsigned flags, void *stream);

/* Refresh the periodic halo of one padded buffer laid out as in a plan of
 * (ndim, dims, radius, dtype): every halo cell takes the value of the interior
 * cell congruent to it modulo dims (Eq. 2 with a periodic beta). */
stencil_status stencil_halo_periodic(int ndim, const int dims[3], int radius, int dtype,
                                     void *d_buf, void *stream);

/* The same periodic halo refresh for one field in a linear plan's layout
 * (its dims, radius, dtype, row_pitch and x_offset); d_buf holds
 * stencil_plan_padded_elems(plan) elements. Asynchronous on the stream. */
stencil_status stencil_plan_halo(stencil_plan_t plan, void *d_buf, void *stream);

/* Streaming copy of nbytes (multiple of 16, both pointers 16-byte aligned):
 * the r = 0 case used to measure achievable HBM bandwidth (Sec. 5.2). */
stencil_status stencil_copy(const void *d_src, void *d_dst, size_t nbytes, void *stream);

/* Central finite-difference weights on offsets -r..r for the derivative of
 * the given order (1 or 2), of accuracy order 2r, for unit spacing, computed
 * by solving the moment conditions. out receives 2r+1 doubles. */
stencil_status stencil_fd_weights(int order, int radius, double *out);


/* ------------------------------------------------------------------------ */
/* Fused nonlinear substep: derivative bank + right-hand side + RK3 update  */
/* ------------------------------------------------------------------------ */

/* Models (the nonlinear stencil function phi of Eq. 9 on the sixth-order,
 * radius-3 derivative bank gamma = AB of Eq. 8, Sec. 3.3):
 *  MHD8   : 8 fields (lnrho, u_x, u_y, u_z, s, A_x, A_y, A_z; Table A1), 3-D:
 *           R_lnrho = -u.grad lnrho - div u + nu lap lnrho
 *           R_u     = -(u.grad)u - cs2 grad(s + lnrho) + j x B
 *                     + nu [lap u + grad(div u)/3 + 2 S.grad lnrho]
 *           R_s     = -u.grad s + nu lap s + eta |j|^2 + 2 nu S:S
 *           R_A     = u x B + eta lap A
 *           with B = curl A, j = grad(div A) - lap A, S the traceless rate
 *           of shear: Eq. A1-A4 with rho, T, c_p, mu_0 = 1 and no heating,
 *           cooling, conduction or bulk viscosity.
 *  ADVDIFF: 1 field, 2-D or 3-D: R = -c.grad f + nu lap f.
 *  MHD_FULL: the same 8 fields, 3-D, the non-ideal MHD equations as written
 *           (Eq. A1-A4), closed by the ideal gas law (Sec. 3.3 names it
 *           but does not write it out; this form is chosen here):
 *           rho = exp(lnrho), cs2 = cs0^2 exp(gamma s / c_p
 *           + (gamma - 1)(lnrho - lnrho0)) with cs0^2 = desc.cs2,
 *           T = cs2 / ((gamma - 1) c_p), j = (grad div A - lap A) / mu_0,
 *           R_lnrho = -u.grad lnrho - div u
 *           R_u     = -(u.grad)u - cs2 grad(s / c_p + lnrho) + j x B / rho
 *                     + nu [lap u + grad(div u)/3 + 2 S.grad lnrho]
 *                     + zeta grad(div u)
 *           R_s     = -u.grad s + [H - C + K lap T + eta mu_0 |j|^2
 *                     + 2 rho nu S:S + zeta rho (div u)^2] / (rho T)
 *           R_A     = u x B + eta lap A
 *           with constant conductivity K, heating H and cooling C, and
 *           lap T = T [(gamma / c_p) lap s + (gamma - 1) lap lnrho + |g|^2],
 *           g = (gamma / c_p) grad s + (gamma - 1) grad lnrho (the chain
 *           rule on the bank's derivatives of s and lnrho).
 * Mixed derivatives are tensor products of the first-derivative stencil. */
#define STENCIL_MODEL_MHD8 0
#define STENCIL_MODEL_ADVDIFF 1
#define STENCIL_MODEL_MHD_FULL 2

/* Precision policies. F64: FP64 everywhere. F32_MASTER64 / BF16_MASTER64:
 * fields stored in FP32 / BF16, derivatives and RK registers in FP32, and an
 * FP64 master state that the last substep of every step recomputes as
 * master + b0 w1 + b1 w2 + b2 w3 in FP64 (so rounding does not accumulate in
 * the state across steps). F32_ONLY / BF16_ONLY: no master (ablation). */
#define STENCIL_PREC_F64 0
#define STENCIL_PREC_F32_MASTER64 1
#define STENCIL_PREC_BF16_MASTER64 2
#define STENCIL_PREC_F32_ONLY 3
#define STENCIL_PREC_BF16_ONLY 4

typedef struct stencil_rk_desc {
    int model;      /* STENCIL_MODEL_* */
    int ndim;       /* 3 for MHD8 and MHD_FULL, 2 or 3 for ADVDIFF */
    int dims[3];    /* interior extents, each >= 3 (periodic, radius 3) */
    int precision;  /* STENCIL_PREC_* */
    double ds[3];   /* grid spacing per axis (> 0) */
    double nu, eta, cs2;
    double adv[3];  /* ADVDIFF velocity */
    int block[3];   /* launch override (0 = plan's choice). CACHED: x lanes, y
                       lanes (x*y a multiple of 64, at most 256), block[2] 0
                       or 1 (one z plane per workgroup). LDS, MHD8 and
                       MHD_FULL: the brick of output points per workgroup,
                       one of 16x8x4 16x8x8 32x4x4 8x8x8. LDS, ADVDIFF:
                       {0, 0, z planes} */
    int variant;    /* STENCIL_RK_VARIANT_*: how the derivative bank reads its
                       taps */
    int row_pitch;  /* field layout, as in stencil_desc (both 0 = compact):  */
    int x_offset;   /* interior x = 0 at column x_offset >= 3 of rows of
                       row_pitch >= x_offset + dims[0] + 3 elements; every
                       buffer of the plan (f, w, w2, f64) uses this layout and
                       holds stencil_plan_padded_elems(plan) elements */
    /* MHD_FULL only (ignored otherwise; cs2 above is cs0^2 > 0): bulk
       viscosity zeta, vacuum permeability mu0 > 0, adiabatic index
       gamma > 1, specific heat c_p > 0, reference log density lnrho0,
       conductivity K, heating H and cooling C (all finite) */
    double zeta, mu0, gamma, cp, lnrho0, K, heat, cool;
    int mixed;      /* MHD8 and MHD_FULL: form of the bank's mixed derivatives
                       d_a d_b (a != b) in grad(div u) and grad(div A),
                       STENCIL_MIXED_*; must be 0 for ADVDIFF */
    unsigned flags; /* STENCIL_RK_FLAG_*; 0 = the plan's fixed defaults */
    int occupancy;  /* LDS bricks of MHD8 / MHD_FULL: waves per SIMD the
                       kernel is compiled for (0 = the compiler's choice; 4
                       with a 512-lane brick: at most 128 VGPRs, two
                       workgroups per CU); one of the built (brick, occupancy)
                       pairs, see block[]. Changes no result. */
} stencil_rk_desc;

/* Plan-time search (Sec. 5.1: the launch parameters are searched at runtime,
 * failed launches dropped; Sec. 5.4: register allocation is a tuning knob).
 * The plan times one RK3 step (three substeps, best of two after a warm-up)
 * of every candidate schedule on scratch buffers of the plan's shape and
 * keeps the fastest: MHD8 / MHD_FULL: the LDS bricks with their occupancy
 * targets and the CACHED variant's lane tiles; 3-D ADVDIFF: the z march with
 * 8, 16, 32 or 64 planes per tile and the CACHED tiles; 2-D ADVDIFF: the
 * CACHED tiles. Only block[] / occupancy / variant fields left at 0 (AUTO)
 * are searched. Every candidate computes the same arithmetic per point, so
 * results are bitwise those of the untuned plan. Choices are cached per
 * shape class in the process and, if the environment variable
 * STENCIL_TUNE_CACHE names a file, in that file across processes. Needs
 * scratch device memory of the plan's buffers for the search (released before
 * return). */
#define STENCIL_RK_FLAG_AUTOTUNE 1u

/* Mixed-derivative forms (the paper fixes sixth-order central differences,
 * Sec. 3.3, but not the mixed stencil). TENSOR: the product of the two
 * first-derivative stencils on the a-b plane (36 taps). DIAGONAL: the
 * second-derivative stencil along the two diagonals of the plane,
 * d_a d_b f = [D2 along (+a,+b) - D2 along (+a,-b)] / (4 h_a h_b) (12 taps,
 * also sixth-order). The two differ by O(h^6). */
#define STENCIL_MIXED_TENSOR 0
#define STENCIL_MIXED_DIAGONAL 1

/* Derivative-bank strategies (Sec. 4.1/4.4): AUTO = LDS for MHD8, MHD_FULL
 * and 3-D ADVDIFF grids of at least 2^20 points, CACHED otherwise. CACHED:
 * one lane per point, every tap a load through L1/L2. LDS, MHD8/MHD_FULL: a
 * workgroup owns a brick of points and streams the fields one at a time
 * through an LDS tile of the brick plus its halo. LDS, 3-D ADVDIFF: the
 * right-hand side is a radius-3 star, computed as a z march over 64 x 16
 * tiles (x-y plane in LDS, z taps in registers) with the RK update as its
 * epilogue; block[2] = z planes per tile (0 = chosen from the grid size:
 * 8..32, aiming at about 1024 tiles). */
#define STENCIL_RK_VARIANT_AUTO 0
#define STENCIL_RK_VARIANT_CACHED 1
#define STENCIL_RK_VARIANT_LDS 2

/* Buffers of one substep; all are caller-owned padded (radius 3) device
 * arrays of the plan's dims, one per field (entries beyond the model's field
 * count are ignored).
 *  f_in  : substep input (storage type; halo must be periodic-valid)
 *  f_out : substep output (storage type; interior and periodic halo written)
 *  w     : RK register, FP64 for PREC_F64, FP32 otherwise. Non-master
 *          policies update it in place (not read at substep 0, not written at
 *          substep 2). Master policies: written at substep 0, read at 1 and 2.
 *  w2    : master policies only: written at substep 1, read at substep 2.
 *  f64   : master policies only: FP64 state, read and written at substep 2
 *          (interior only). */
typedef struct stencil_fields {
    void *f_in[8];
    void *f_out[8];
    void *w[8];
    void *w2[8];
    double *f64[8];
} stencil_fields;

/* Plan of the fused substep of a model; RK coefficients are Williamson's
 * 2N-storage third-order scheme: alpha = (0, -5/9, -153/128), beta = (1/3,
 * 15/16, 8/15), substep i: w = alpha_i w + dt R(f), f = f + beta_i w.
 * STENCIL_EUNSUPPORTED if one padded FP64 buffer of the plan's layout would
 * reach 4 GiB (the substep kernels address each field with 32-bit offsets;
 * about 810^3 points per field). */
stencil_status stencil_plan_rk(const stencil_rk_desc *desc, stencil_plan_t *out);

/* Number of fields of the plan's model (8 for MHD8 and MHD_FULL, 1 for
 * ADVDIFF), or a negative status. */
int stencil_plan_nfields(stencil_plan_t plan);

/* The launch schedule an RK plan runs (after any search): out[0] = variant
 * (STENCIL_RK_VARIANT_CACHED or _LDS), out[1..3] = block (CACHED: x lanes, y
 * lanes, 1; LDS: the brick, or {64, 16, z planes} for the ADVDIFF z march),
 * out[4] = occupancy target (0 = compiler's choice). */
stencil_status stencil_plan_rk_schedule(stencil_plan_t plan, int out[5]);

/* One fused substep (substep = 0, 1, 2) as one kernel launch on stream. */
stencil_status stencil_step(stencil_plan_t plan, const stencil_fields *fields, int substep,
                            double dt, void *stream);

/* nsteps full RK3 steps (3 substeps each). f_in holds the initial state (its
 * halo is refreshed first) and f_in / f_out are used in ping-pong, so the
 * result is in f_out when nsteps is odd and in f_in when even. Registers and
 * the master (master policies: f64 must hold the FP64 copy of f_in) as in
 * stencil_step. A 2-D FP64 advection-diffusion plan created with the
 * automatic variant on an nx x ny grid with nx, ny >= 6, nx ny <= 5200 and
 * (nx + 6)(ny + 6) <= 7000 runs the whole call in one launch with its state
 * in LDS (temporal blocking of small grids); the buffers end as the substep
 * launches would leave them, bit for bit. */
stencil_status stencil_rk_run(stencil_plan_t plan, const stencil_fields *fields, int nsteps,
                              double dt, void *stream);

/* Global diagnostics in FP64 over the interior of nfields padded buffers of
 * the plan's geometry stored as dtype: host_out[3k..3k+2] = (sum, sum of
 * squares, max |f|) of field k. Deterministic (fixed two-level tree, no
 * floating-point atomics). Synchronises the stream. */
stencil_status stencil_reduce(stencil_plan_t plan, const void *const *fields, int nfields,
                              int dtype, double *host_out, void *stream);

/* stencil_reduce for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and partition, so the same results bit for bit, with the
 * partials in a fixed device array of the library (386 KiB per GPU, held until
 * the process ends) instead of memory allocated per call. Arguments, layout
 * and ownership as stencil_reduce; nfields <= 64 (more: STENCIL_EINVAL).
 * Every call on one GPU shares that array: calls that overlap in time on one
 * GPU (several host threads or streams) race and must be serialised by the
 * caller. Synchronises the stream. */
stencil_status stencil_reduce_noalloc(stencil_plan_t plan, const void *const *fields,
                                      int nfields, int dtype, double *host_out, void *stream);

/* Kinetic and magnetic energy of an MHD plan's state (MHD8 or MHD_FULL; the
 * fields of Eq. A1-A4 in Table A1 order): host_out[0] = 1/2 sum |u|^2 and
 * host_out[1] = 1/2 sum |B|^2 over the interior grid points, B = curl A by the
 * plan's sixth-order first-derivative stencil and spacing (plain sums over
 * points: multiply by the cell volume for integrals). fields: the 8 padded
 * buffers of the plan's layout stored as dtype, periodic halos valid (as
 * stencil_step and stencil_rk_run leave f_out). FP64 accumulation,
 * deterministic (fixed partition and tree, no floating-point atomics).
 * Synchronises the stream. */
stencil_status stencil_energy(stencil_plan_t plan, const void *const *fields, int dtype,
                              double *host_out, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched jobs and the serving loop                                        */
/* ------------------------------------------------------------------------ */

/* A stencil-integration job: the ADVDIFF model (R = -c.grad f + nu lap f,
 * sixth-order radius-3 derivatives, Sec. 3.2 with advection added) on a
 * periodic 2-D or 3-D grid of spacing 2 pi / dims[a], integrated for `steps`
 * RK3 steps of the fused substep. Jobs run batched: one persistent launch per
 * substep advances every resident job; a point is computed by the same code as
 * stencil_step, so a job's result does not depend on the batch it ran in. */
typedef struct stencil_job {
    int ndim;           /* 2 or 3 */
    int dims[3];        /* interior extents, each >= 3 */
    int steps;          /* RK3 steps, >= 1 */
    int precision;      /* STENCIL_PREC_F64, STENCIL_PREC_F32_MASTER64 or
                           STENCIL_PREC_F32_ONLY */
    double nu;          /* viscosity */
    double adv[3];      /* velocity c */
    double dt;          /* time step; <= 0 picks 0.1 ds_min / max(1, max |c|) */
    const double *init; /* host, interior initial state (x fastest); read when
                           the job is admitted: keep it valid while the job is
                           STENCIL_JOB_QUEUED */
    double *result;     /* host, interior final state in FP64 (the FP64 master
                           for master policies); written before the job turns
                           STENCIL_JOB_DONE */
} stencil_job;

#define STENCIL_JOB_QUEUED 0
#define STENCIL_JOB_RUNNING 1
#define STENCIL_JOB_DONE 2
#define STENCIL_JOB_FAILED 3
#define STENCIL_JOB_CANCELLED 4

typedef struct stencil_job_status {
    int state;           /* STENCIL_JOB_* */
    int error;           /* stencil_status of a FAILED job, else 0 */
    double t_submit;     /* seconds on the server clock; -1 if not reached */
    double t_admit;
    double t_first_tick; /* end of the first tick the job took part in */
    double t_done;
    long long steps_done;
} stencil_job_status;

typedef struct stencil_server_desc {
    size_t hbm_budget; /* device bytes for resident job state; 0 = 80% of free */
    int max_slots;     /* jobs resident at once, 1..4096 */
    int tick_steps;    /* RK steps per tick (>= 1); admission between ticks */
    int use_graph;     /* replay each tick from one captured hipGraph */
    int blocks;        /* persistent workgroups per launch; 0 = 8 per CU */
    int queue_cap;     /* jobs waiting for admission at most; 0 = unlimited */
    long long min_points; /* points per substep a tick gathers before it
                             stops adding resident jobs (0 = 4 Mi; a huge
                             value = every resident job every tick) */
    int policy;        /* order in which a tick takes resident jobs:
                          STENCIL_SERVE_OLDEST (0, default) oldest
                          submission first until min_points, then shorter
                          jobs while the tick grows by at most a quarter (no
                          job is passed by a later one: bounds the tail);
                          STENCIL_SERVE_SHORTEST (1) least remaining work
                          first, a job left out 16 ticks in a row taken
                          regardless (lowest median under overload) */
    int tune;          /* nonzero: search the batch schedule of every job class
                          (ndim, dims, precision) the first time it is
                          admitted (Sec. 5.1): z-march jobs 8/16/32/64 planes
                          per tile, per-point jobs 64x4/128x2/256x1/32x8
                          point tiles, each timed on one RK3 step of the
                          batched kernels between ticks; choices cached per
                          class (and in STENCIL_TUNE_CACHE's file). Changes no
                          result. 0: fixed schedule (depth from the grid size,
                          64x4 tiles) */
} stencil_server_desc;

#define STENCIL_SERVE_OLDEST 0
#define STENCIL_SERVE_SHORTEST 1

typedef struct stencil_server_s *stencil_server_t;

typedef struct stencil_server_stats {
    long long ticks, launches, admitted, completed, failed, cancelled;
    long long point_steps; /* sum over completed jobs of points x steps */
    size_t bytes_in_use, bytes_budget;
    int resident, queued;
    double busy_s;         /* wall time spent inside ticks */
    int tuned_classes;     /* job classes whose batch schedule was searched */
} stencil_server_stats;

/* Start a server on the current device: a host thread that admits queued jobs
 * (first fit, in arrival order) while their state fits the HBM budget and a
 * slot is free, keeps admitted jobs' fields resident on the device, advances
 * them tick by tick (tick_steps RK steps each; a tick takes resident jobs in
 * the order the policy sets until it holds min_points points) and retires
 * finished jobs (result copied out, memory freed). Jobs arriving while others
 * run are admitted at the next tick boundary. */
stencil_status stencil_server_create(const stencil_server_desc *desc, stencil_server_t *out);

/* Cancel queued and running jobs, stop the thread and free everything.
 * NULL is accepted. */
stencil_status stencil_server_destroy(stencil_server_t server);

/* Queue a job (descriptor copied; init and result pointers kept). Returns
 * STENCIL_EAGAIN when queue_cap jobs are already waiting, STENCIL_EINVAL for a
 * bad descriptor, STENCIL_EDEVICE after a device failure of the server. A job
 * larger than the whole budget fails at admission with STENCIL_ENOMEM. */
stencil_status stencil_submit(stencil_server_t server, const stencil_job *job, uint64_t *ticket);

/* Current status of a job (non-blocking). */
stencil_status stencil_poll(stencil_server_t server, uint64_t ticket, stencil_job_status *st);

/* Wait until the job is DONE, FAILED or CANCELLED, or timeout_ms passes
 * (negative: no limit; STENCIL_ETIMEOUT on expiry). */
stencil_status stencil_wait(stencil_server_t server, uint64_t ticket, stencil_job_status *st,
                            int timeout_ms);

/* Cancel a queued or running job (a running job stops at the next tick
 * boundary; its result is not written). */
stencil_status stencil_cancel(stencil_server_t server, uint64_t ticket);

/* Counters of the server. */
stencil_status stencil_server_stats_get(stencil_server_t server, stencil_server_stats *st);

/* Seconds since the server started, on the clock of the job timestamps. */
double stencil_server_clock(stencil_server_t server);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL_H */
