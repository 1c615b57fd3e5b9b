/*
 * stencil_oracle.c -- plain FP64 CPU oracle for the stencil hot path.
 *
 * TEST INFRASTRUCTURE ONLY. The product library never links, loads or calls
 * this file: only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do. It shares no code, header, table or constant with the GPU
 * path; every coefficient below is typed in here from the mathematics.
 *
 * Every routine is the textbook definition written out with plain loops. The
 * only concession to speed is an OpenMP "parallel for" over the slowest axis
 * of loops whose iterations are independent (each output point is computed by
 * the same sequential expression whatever the thread count); reductions stay
 * sequential. Build with -ffp-contract=off so no multiply-add is fused.
 *
 * Storage convention (paper Sec. 2.4, Eq. 2 and Fig. 1; row-wise scan order of
 * Sec. 4.4): a field with interior shape n[0] x n[1] x n[2] (x fastest) is
 * stored padded by r cells on both sides of every active axis. Axis a < ndim
 * has extent n[a] + 2r, an unused axis has extent 1. The linear index of
 * padded cell (x, y, z) is x + Px*(y + Py*z); padded coordinate q holds the
 * interior point q - r.
 *
 * Parity status: every function here is pinned by the CPU test-suite against
 * closed forms (moment conditions, polynomial exactness, Fourier symbols,
 * conservation, dense-matrix brute force, the RK3 stability polynomial and
 * term-by-term special cases of the right-hand side); the window filters
 * against scipy's rank filters with periodic wrap, a brute force over shifted
 * copies, max/min duality, signed-zero order and NaN confinement.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Indexing helpers                                                          */
/* ------------------------------------------------------------------------ */

static long ext(int ndim, int a, const long *n, int r)
{
    return a < ndim ? n[a] + 2L * r : 1L;
}

static size_t at(const long *P, long x, long y, long z)
{
    return (size_t)x + (size_t)P[0] * ((size_t)y + (size_t)P[1] * (size_t)z);
}

static long wrap(long i, long n)
{
    long m = i % n;
    return m < 0 ? m + n : m;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Padding psi with the periodic boundary function (Eq. 2, Fig. 1)           */
/* ------------------------------------------------------------------------ */

/* Every padded cell outside the interior takes the value of the interior cell
 * congruent to it modulo n on each active axis (edges and corners included). */
void oracle_fill_periodic(double *a, int ndim, const long *n, int r)
{
    long P[3] = {ext(ndim, 0, n, r), ext(ndim, 1, n, r), ext(ndim, 2, n, r)};
    for (long z = 0; z < P[2]; ++z)
        for (long y = 0; y < P[1]; ++y)
            for (long x = 0; x < P[0]; ++x) {
                long q[3] = {x, y, z};
                long s[3] = {0, 0, 0};
                int inside = 1;
                for (int d = 0; d < ndim; ++d) {
                    long i = q[d] - r;
                    if (i < 0 || i >= n[d])
                        inside = 0;
                    s[d] = r + wrap(i, n[d]);
                }
                if (!inside)
                    a[at(P, x, y, z)] = a[at(P, s[0], s[1], s[2])];
            }
}

/* ------------------------------------------------------------------------ */
/* Linear cross-correlation (Eq. 3; multi-dimensional form Eq. 6-7)          */
/* ------------------------------------------------------------------------ */

/* One output point: out_p = sum over offsets s in [-r, r]^ndim of
 * g_s * in_{p+s}. g is the dense (2r+1)^ndim coefficient tensor, x fastest.
 * Taps are visited in lexicographic (s_z, s_y, s_x) order. (x, y, z) are
 * interior coordinates. */
static double xcorr_point(const double *in, const long *P, int ndim, int r,
                          const double *g, long x, long y, long z)
{
    int K = 2 * r + 1;
    int rx = r, ry = ndim > 1 ? r : 0, rz = ndim > 2 ? r : 0;
    int Ky = ndim > 1 ? K : 1;
    double acc = 0.0;
    for (int sz = -rz; sz <= rz; ++sz)
        for (int sy = -ry; sy <= ry; ++sy)
            for (int sx = -rx; sx <= rx; ++sx) {
                double gs = g[(sx + r) + (size_t)K * ((sy + ry) + (size_t)Ky * (sz + rz))];
                acc += gs * in[at(P, x + rx + sx, y + ry + sy, z + rz + sz)];
            }
    return acc;
}

/* Interior of out receives the cross-correlation of in; out's halo is left
 * untouched. */
void oracle_xcorr(const double *in, double *out, int ndim, const long *n, int r,
                  const double *g)
{
    long P[3] = {ext(ndim, 0, n, r), ext(ndim, 1, n, r), ext(ndim, 2, n, r)};
    long nz = ndim > 2 ? n[2] : 1, ny = ndim > 1 ? n[1] : 1, nx = n[0];
    int ry = ndim > 1 ? r : 0, rz = ndim > 2 ? r : 0;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x)
                out[at(P, x + r, y + ry, z + rz)] = xcorr_point(in, P, ndim, r, g, x, y, z);
}

/* The same cross-correlation evaluated only at the listed interior points
 * (count triples x, y, z); used to check very large grids point by point. */
void oracle_xcorr_at(const double *in, int ndim, const long *n, int r, const double *g,
                     const long *pts, long count, double *out)
{
    long P[3] = {ext(ndim, 0, n, r), ext(ndim, 1, n, r), ext(ndim, 2, n, r)};
    for (long k = 0; k < count; ++k)
        out[k] = xcorr_point(in, P, ndim, r, g, pts[3 * k], pts[3 * k + 1], pts[3 * k + 2]);
}

/* ------------------------------------------------------------------------ */
/* Nonlinear window filters (Sec. 2.3: max filtering; Sec. 1: median)       */
/* ------------------------------------------------------------------------ */

/* The window is the set of offsets whose mask entry is nonzero (the dense
 * (2r+1)^ndim layout of the cross-correlation coefficients). Values are
 * ordered by IEEE totalOrder restricted to non-NaN numbers: numeric order,
 * with -0 below +0, so the maximum, minimum and median are unique elements of
 * the window whatever the order they are visited in. A window holding a NaN
 * yields NaN. The median of m values is the element of rank (m-1)/2 from the
 * bottom (the lower median when m is even). */
enum { FILTER_MAX = 1, FILTER_MIN = 2, FILTER_MEDIAN = 3 };

static int total_less(double a, double b)
{
    if (a == b)
        return a == 0.0 && signbit(a) && !signbit(b);
    return a < b;
}

static double filter_point(const double *in, const long *P, int ndim, int r, const double *mask,
                           int op, long x, long y, long z, double *scratch)
{
    int K = 2 * r + 1;
    int rx = r, ry = ndim > 1 ? r : 0, rz = ndim > 2 ? r : 0;
    int Ky = ndim > 1 ? K : 1;
    int m = 0, has_nan = 0;
    for (int sz = -rz; sz <= rz; ++sz)
        for (int sy = -ry; sy <= ry; ++sy)
            for (int sx = -rx; sx <= rx; ++sx) {
                if (mask[(sx + r) + (size_t)K * ((sy + ry) + (size_t)Ky * (sz + rz))] == 0.0)
                    continue;
                double v = in[at(P, x + rx + sx, y + ry + sy, z + rz + sz)];
                if (isnan(v))
                    has_nan = 1;
                scratch[m++] = v;
            }
    if (has_nan || m == 0)
        return NAN;
    if (op == FILTER_MAX || op == FILTER_MIN) {
        double best = scratch[0];
        for (int i = 1; i < m; ++i)
            if (op == FILTER_MAX ? total_less(best, scratch[i]) : total_less(scratch[i], best))
                best = scratch[i];
        return best;
    }
    /* median: insertion sort, then the element of rank (m - 1) / 2 */
    for (int i = 1; i < m; ++i) {
        double v = scratch[i];
        int j = i - 1;
        while (j >= 0 && total_less(v, scratch[j])) {
            scratch[j + 1] = scratch[j];
            --j;
        }
        scratch[j + 1] = v;
    }
    return scratch[(m - 1) / 2];
}

/* Interior of out receives the filter of in over the window; halo untouched.
 * Returns -1 for an unknown op. */
int oracle_filter(const double *in, double *out, int ndim, const long *n, int r,
                  const double *mask, int op)
{
    if (op < FILTER_MAX || op > FILTER_MEDIAN)
        return -1;
    long P[3] = {ext(ndim, 0, n, r), ext(ndim, 1, n, r), ext(ndim, 2, n, r)};
    long nz = ndim > 2 ? n[2] : 1, ny = ndim > 1 ? n[1] : 1, nx = n[0];
    int ry = ndim > 1 ? r : 0, rz = ndim > 2 ? r : 0;
    size_t K = 2 * (size_t)r + 1, cap = K;
    for (int a = 1; a < ndim; ++a)
        cap *= K;
#pragma omp parallel
    {
        double *scratch = malloc(cap * sizeof(double));
#pragma omp for schedule(static)
        for (long z = 0; z < nz; ++z)
            for (long y = 0; y < ny; ++y)
                for (long x = 0; x < nx; ++x)
                    out[at(P, x + r, y + ry, z + rz)] =
                        filter_point(in, P, ndim, r, mask, op, x, y, z, scratch);
        free(scratch);
    }
    return 0;
}

/* The same filter at listed interior points (count triples x, y, z). */
int oracle_filter_at(const double *in, int ndim, const long *n, int r, const double *mask,
                     int op, const long *pts, long count, double *out)
{
    if (op < FILTER_MAX || op > FILTER_MEDIAN)
        return -1;
    long P[3] = {ext(ndim, 0, n, r), ext(ndim, 1, n, r), ext(ndim, 2, n, r)};
    size_t K = 2 * (size_t)r + 1, cap = K;
    for (int a = 1; a < ndim; ++a)
        cap *= K;
    double *scratch = malloc(cap * sizeof(double));
    for (long k = 0; k < count; ++k)
        out[k] = filter_point(in, P, ndim, r, mask, op, pts[3 * k], pts[3 * k + 1], pts[3 * k + 2],
                              scratch);
    free(scratch);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sixth-order central differences (Sec. 3.3: radius-3 stencils)            */
/* ------------------------------------------------------------------------ */

/* The paper states the derivatives are 6th-order central differences but does
 * not print the weights. These are the standard centred weights on offsets
 * -3..3, i.e. the unique solution of the moment conditions
 * sum_m c_m m^k = k! [k = order] for k = 0..6. */
static const double C1[7] = {-1.0 / 60.0, 3.0 / 20.0, -3.0 / 4.0, 0.0,
                             3.0 / 4.0,   -3.0 / 20.0, 1.0 / 60.0};
static const double C2[7] = {1.0 / 90.0, -3.0 / 20.0, 3.0 / 2.0, -49.0 / 18.0,
                             3.0 / 2.0,  -3.0 / 20.0, 1.0 / 90.0};

void oracle_fd_weights(double *c1, double *c2)
{
    for (int i = 0; i < 7; ++i) {
        c1[i] = C1[i];
        c2[i] = C2[i];
    }
}

/* Derivative operators at padded cell (x, y, z) of a radius-3 padded field.
 * a, b are axes (0 = x, 1 = y, 2 = z); ds is the grid spacing per axis. */
static double d1(const double *f, const long *P, long x, long y, long z, int a,
                 const double *ds)
{
    double acc = 0.0;
    for (int m = -3; m <= 3; ++m)
        acc += C1[m + 3] * f[at(P, x + m * (a == 0), y + m * (a == 1), z + m * (a == 2))];
    return acc / ds[a];
}

static double d2(const double *f, const long *P, long x, long y, long z, int a,
                 const double *ds)
{
    double acc = 0.0;
    for (int m = -3; m <= 3; ++m)
        acc += C2[m + 3] * f[at(P, x + m * (a == 0), y + m * (a == 1), z + m * (a == 2))];
    return acc / (ds[a] * ds[a]);
}

/* Mixed derivative d_a d_b (a != b) as the tensor product of the first
 * derivative weights on the a-b plane through the point (36 nonzero taps). */
static double d11(const double *f, const long *P, long x, long y, long z, int a, int b,
                  const double *ds)
{
    double acc = 0.0;
    for (int i = -3; i <= 3; ++i)
        for (int j = -3; j <= 3; ++j) {
            long xx = x + i * (a == 0) + j * (b == 0);
            long yy = y + i * (a == 1) + j * (b == 1);
            long zz = z + i * (a == 2) + j * (b == 2);
            acc += C1[i + 3] * C1[j + 3] * f[at(P, xx, yy, zz)];
        }
    return acc / (ds[a] * ds[b]);
}

/* Mixed derivative d_a d_b (a != b) from the two diagonals of the a-b plane
 * through the point (12 nonzero taps). With h_a, h_b the spacings, the lines
 * g(s) = f(p + s h_a e_a + s h_b e_b) and k(s) = f(p + s h_a e_a - s h_b e_b)
 * satisfy g''(0) - k''(0) = 4 h_a h_b d_a d_b f; taking both second
 * derivatives with the sixth-order weights C2 (unit step in s), the centre
 * weights cancel, and the result is sixth-order accurate. */
static double d11_diag(const double *f, const long *P, long x, long y, long z, int a, int b,
                       const double *ds)
{
    double acc = 0.0;
    for (int m = 1; m <= 3; ++m) {
        long ax = m * (a == 0), ay = m * (a == 1), az = m * (a == 2);
        long bx = m * (b == 0), by = m * (b == 1), bz = m * (b == 2);
        double along = f[at(P, x + ax + bx, y + ay + by, z + az + bz)] +
                       f[at(P, x - ax - bx, y - ay - by, z - az - bz)];
        double across = f[at(P, x + ax - bx, y + ay - by, z + az - bz)] +
                        f[at(P, x - ax + bx, y - ay + by, z - az + bz)];
        acc += C2[m + 3] * (along - across);
    }
    return acc / (4.0 * ds[a] * ds[b]);
}

/* Operator codes for oracle_deriv: 0..2 first derivative along x, y, z;
 * 3..5 second derivative along x, y, z; 6 = xy, 7 = xz, 8 = yz mixed (tensor
 * product); 9 = xy, 10 = xz, 11 = yz mixed (diagonals). */
static double deriv_op(const double *f, const long *P, long x, long y, long z, int op,
                       const double *ds)
{
    switch (op) {
    case 0: case 1: case 2: return d1(f, P, x, y, z, op, ds);
    case 3: case 4: case 5: return d2(f, P, x, y, z, op - 3, ds);
    case 6: return d11(f, P, x, y, z, 0, 1, ds);
    case 7: return d11(f, P, x, y, z, 0, 2, ds);
    case 8: return d11(f, P, x, y, z, 1, 2, ds);
    case 9: return d11_diag(f, P, x, y, z, 0, 1, ds);
    case 10: return d11_diag(f, P, x, y, z, 0, 2, ds);
    case 11: return d11_diag(f, P, x, y, z, 1, 2, ds);
    }
    return NAN;
}

/* Apply one derivative operator over the interior of a radius-3 padded field
 * of dimension ndim (the operator's axes must be < ndim). Returns 0, or -1 for
 * an operator that does not exist in ndim dimensions. */
int oracle_deriv(const double *f, double *out, int ndim, const long *n, const double *ds,
                 int op)
{
    const int r = 3;
    int axes_needed = op < 3 ? op : op < 6 ? op - 3 : (op == 6 || op == 9) ? 1 : 2;
    if (op < 0 || op > 11 || axes_needed >= ndim)
        return -1;
    long P[3] = {ext(ndim, 0, n, r), ext(ndim, 1, n, r), ext(ndim, 2, n, r)};
    long nz = ndim > 2 ? n[2] : 1, ny = ndim > 1 ? n[1] : 1;
    int ry = ndim > 1 ? r : 0, rz = ndim > 2 ? r : 0;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < n[0]; ++x)
                out[at(P, x + r, y + ry, z + rz)] =
                    deriv_op(f, P, x + r, y + ry, z + rz, op, ds);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Nonlinear right-hand sides phi (Eq. 9; MHD form of Appendix A)           */
/* ------------------------------------------------------------------------ */

/* Field order of the 8-field system (Table A1): log density, velocity (3),
 * specific entropy, magnetic vector potential (3). */
enum { LNRHO = 0, UX = 1, UY = 2, UZ = 3, SS = 4, AX = 5, AY = 6, AZ = 7 };

/* The derivative bank gamma (Eq. 8) of the 8-field system at one padded cell:
 * values of u, gradients and Laplacians of lnrho and s, the velocity and
 * vector-potential Jacobians d_a v_b, their Laplacians and grad(div v), where
 * grad(div v)_a = sum_b d_a d_b v_b takes the pure second derivative when
 * a == b and the mixed derivative otherwise. */
typedef struct {
    double u[3], gl[3], gs[3], du[3][3], dA[3][3];
    double lapl, laps, lapu[3], lapA[3], gdivu[3], gdivA[3];
} mhd_bank;

static void mhd_bank_eval(const double *const *f, const long *P, long x, long y, long z,
                          const double *ds, int diag, mhd_bank *k)
{
    size_t p = at(P, x, y, z);
    k->lapl = 0.0;
    k->laps = 0.0;
    for (int b = 0; b < 3; ++b)
        k->u[b] = f[UX + b][p];
    for (int a = 0; a < 3; ++a) {
        k->gl[a] = d1(f[LNRHO], P, x, y, z, a, ds);
        k->gs[a] = d1(f[SS], P, x, y, z, a, ds);
        k->lapl += d2(f[LNRHO], P, x, y, z, a, ds);
        k->laps += d2(f[SS], P, x, y, z, a, ds);
        for (int b = 0; b < 3; ++b) {
            k->du[a][b] = d1(f[UX + b], P, x, y, z, a, ds); /* d_a u_b */
            k->dA[a][b] = d1(f[AX + b], P, x, y, z, a, ds); /* d_a A_b */
        }
    }
    for (int b = 0; b < 3; ++b) {
        k->lapu[b] = 0.0;
        k->lapA[b] = 0.0;
        for (int a = 0; a < 3; ++a) {
            k->lapu[b] += d2(f[UX + b], P, x, y, z, a, ds);
            k->lapA[b] += d2(f[AX + b], P, x, y, z, a, ds);
        }
    }
    for (int a = 0; a < 3; ++a) {
        k->gdivu[a] = 0.0;
        k->gdivA[a] = 0.0;
        for (int b = 0; b < 3; ++b) {
            if (a == b) {
                k->gdivu[a] += d2(f[UX + b], P, x, y, z, a, ds);
                k->gdivA[a] += d2(f[AX + b], P, x, y, z, a, ds);
            } else if (diag) {
                k->gdivu[a] += d11_diag(f[UX + b], P, x, y, z, a, b, ds);
                k->gdivA[a] += d11_diag(f[AX + b], P, x, y, z, a, b, ds);
            } else {
                k->gdivu[a] += d11(f[UX + b], P, x, y, z, a, b, ds);
                k->gdivA[a] += d11(f[AX + b], P, x, y, z, a, b, ds);
            }
        }
    }
}

/* Quantities shared by both MHD right-hand sides: div u, B = curl A, the
 * traceless rate of shear S_ab = (d_a u_b + d_b u_a)/2 - delta_ab div(u)/3,
 * (u.grad) u, S.grad(lnrho), S:S and u x B. */
typedef struct {
    double divu, B[3], S[3][3], adv[3], Sgl[3], SS2, uxB[3];
} mhd_derived;

static void mhd_derive(const mhd_bank *k, mhd_derived *d)
{
    d->divu = k->du[0][0] + k->du[1][1] + k->du[2][2];
    d->B[0] = k->dA[1][2] - k->dA[2][1];
    d->B[1] = k->dA[2][0] - k->dA[0][2];
    d->B[2] = k->dA[0][1] - k->dA[1][0];
    d->SS2 = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            d->S[a][b] = 0.5 * (k->du[a][b] + k->du[b][a]) - (a == b ? d->divu / 3.0 : 0.0);
            d->SS2 += d->S[a][b] * d->S[a][b];
        }
    for (int a = 0; a < 3; ++a) {
        d->adv[a] = 0.0;
        d->Sgl[a] = 0.0;
        for (int b = 0; b < 3; ++b) {
            d->adv[a] += k->u[b] * k->du[b][a]; /* (u.grad) u_a */
            d->Sgl[a] += d->S[a][b] * k->gl[b]; /* (S.grad lnrho)_a */
        }
    }
    d->uxB[0] = k->u[1] * d->B[2] - k->u[2] * d->B[1];
    d->uxB[1] = k->u[2] * d->B[0] - k->u[0] * d->B[2];
    d->uxB[2] = k->u[0] * d->B[1] - k->u[1] * d->B[0];
}

/* Eight-field proxy of the non-ideal MHD equations (Eq. A1-A4) with rho, T,
 * c_p and mu_0 set to one and heating, cooling, conduction and bulk viscosity
 * dropped, plus a nu-Laplacian on log density and entropy:
 *   R_lnrho = -u.grad(lnrho) - div u + nu lap(lnrho)
 *   R_u     = -(u.grad)u - cs2 grad(s + lnrho) + j x B
 *             + nu [lap u + grad(div u)/3 + 2 S.grad(lnrho)]
 *   R_s     = -u.grad(s) + nu lap(s) + eta |j|^2 + 2 nu S:S
 *   R_A     = u x B + eta lap(A)
 * with B = curl A and j = grad(div A) - lap A (curl curl A, mu_0 = 1).
 * f points at 8 radius-3 padded 3-D fields; (x, y, z) is a padded cell. */
static void mhd8_rhs_point(const double *const *f, const long *P, long x, long y, long z,
                           const double *ds, int diag, const double *prm, double *R)
{
    const double nu = prm[0], eta = prm[1], cs2 = prm[2];
    mhd_bank k;
    mhd_derived d;
    mhd_bank_eval(f, P, x, y, z, ds, diag, &k);
    mhd_derive(&k, &d);
    double j[3];
    for (int a = 0; a < 3; ++a)
        j[a] = k.gdivA[a] - k.lapA[a];
    double jxB[3] = {j[1] * d.B[2] - j[2] * d.B[1], j[2] * d.B[0] - j[0] * d.B[2],
                     j[0] * d.B[1] - j[1] * d.B[0]};
    double ugl = 0.0, ugs = 0.0, jj = 0.0;
    for (int a = 0; a < 3; ++a) {
        ugl += k.u[a] * k.gl[a];
        ugs += k.u[a] * k.gs[a];
        jj += j[a] * j[a];
    }
    R[LNRHO] = -ugl - d.divu + nu * k.lapl;
    for (int a = 0; a < 3; ++a)
        R[UX + a] = -d.adv[a] - cs2 * (k.gs[a] + k.gl[a]) + jxB[a] +
                    nu * (k.lapu[a] + k.gdivu[a] / 3.0 + 2.0 * d.Sgl[a]);
    R[SS] = -ugs + nu * k.laps + eta * jj + 2.0 * nu * d.SS2;
    for (int a = 0; a < 3; ++a)
        R[AX + a] = d.uxB[a] + eta * k.lapA[a];
}

/* The non-ideal MHD equations as written (Eq. A1-A4), closed by the ideal gas
 * law that Sec. 3.3 names without writing it out; the form taken here:
 *   rho = exp(lnrho)
 *   cs2 = cs0^2 exp(gamma s / c_p + (gamma - 1)(lnrho - lnrho0))
 *   T   = cs2 / ((gamma - 1) c_p)
 *   j   = mu_0^-1 curl B = mu_0^-1 (grad(div A) - lap A)
 *   R_lnrho = -u.grad(lnrho) - div u                                   (A1)
 *   R_u     = -(u.grad)u - cs2 grad(s / c_p + lnrho) + j x B / rho
 *             + nu [lap u + grad(div u)/3 + 2 S.grad(lnrho)]
 *             + zeta grad(div u)                                       (A2)
 *   R_s     = -u.grad(s) + [H - C + K lap T + eta mu_0 |j|^2
 *             + 2 rho nu S:S + zeta rho (div u)^2] / (rho T)           (A3)
 *   R_A     = u x B + eta lap(A)                                       (A4)
 * with constant conductivity K, heating H and cooling C, and lap T taken by
 * the chain rule from the bank's derivatives of s and lnrho:
 *   grad T = T g,  g = (gamma / c_p) grad s + (gamma - 1) grad lnrho,
 *   lap T  = T [(gamma / c_p) lap s + (gamma - 1) lap lnrho + |g|^2].
 * prm = {nu, eta, cs0^2, zeta, mu_0, gamma, c_p, lnrho0, K, H, C}. */
static void mhdfull_rhs_point(const double *const *f, const long *P, long x, long y, long z,
                              const double *ds, int diag, const double *prm, double *R)
{
    const double nu = prm[0], eta = prm[1], cs02 = prm[2], zeta = prm[3], mu0 = prm[4];
    const double gamma = prm[5], cp = prm[6], lnrho0 = prm[7], K = prm[8], H = prm[9],
                 C = prm[10];
    mhd_bank k;
    mhd_derived d;
    mhd_bank_eval(f, P, x, y, z, ds, diag, &k);
    mhd_derive(&k, &d);
    size_t p = at(P, x, y, z);
    const double lnrho = f[LNRHO][p], s = f[SS][p];
    const double rho = exp(lnrho);
    const double cs2 = cs02 * exp(gamma * s / cp + (gamma - 1.0) * (lnrho - lnrho0));
    const double T = cs2 / ((gamma - 1.0) * cp);
    double j[3], g[3], gg = 0.0;
    for (int a = 0; a < 3; ++a) {
        j[a] = (k.gdivA[a] - k.lapA[a]) / mu0;
        g[a] = gamma / cp * k.gs[a] + (gamma - 1.0) * k.gl[a];
        gg += g[a] * g[a];
    }
    const double lapT = T * (gamma / cp * k.laps + (gamma - 1.0) * k.lapl + gg);
    double jxB[3] = {j[1] * d.B[2] - j[2] * d.B[1], j[2] * d.B[0] - j[0] * d.B[2],
                     j[0] * d.B[1] - j[1] * d.B[0]};
    double ugl = 0.0, ugs = 0.0, jj = 0.0;
    for (int a = 0; a < 3; ++a) {
        ugl += k.u[a] * k.gl[a];
        ugs += k.u[a] * k.gs[a];
        jj += j[a] * j[a];
    }
    R[LNRHO] = -ugl - d.divu;
    for (int a = 0; a < 3; ++a)
        R[UX + a] = -d.adv[a] - cs2 * (k.gs[a] / cp + k.gl[a]) + jxB[a] / rho +
                    nu * (k.lapu[a] + k.gdivu[a] / 3.0 + 2.0 * d.Sgl[a]) + zeta * k.gdivu[a];
    R[SS] = -ugs + (H - C + K * lapT + eta * mu0 * jj + 2.0 * rho * nu * d.SS2 +
                    zeta * rho * d.divu * d.divu) / (rho * T);
    for (int a = 0; a < 3; ++a)
        R[AX + a] = d.uxB[a] + eta * k.lapA[a];
}

/* Scalar advection-diffusion: R = -c.grad f + nu lap f in ndim = 2 or 3
 * dimensions with radius-3 sixth-order operators (the diffusion case of
 * Sec. 3.2 with an advection term added). prm = {nu, c_x, c_y, c_z}. */
static void advdiff_rhs_point(const double *const *f, const long *P, int ndim, long x,
                              long y, long z, const double *ds, const double *prm,
                              double *R)
{
    double acc = 0.0;
    for (int a = 0; a < ndim; ++a)
        acc += -prm[1 + a] * d1(f[0], P, x, y, z, a, ds) + prm[0] * d2(f[0], P, x, y, z, a, ds);
    R[0] = acc;
}

enum { MODEL_MHD8 = 0, MODEL_ADVDIFF = 1, MODEL_MHD_FULL = 2 };

/* A model code may carry MIXED_DIAG (MHD models only): the bank then takes
 * its mixed derivatives from the diagonals (d11_diag) instead of the tensor
 * product (d11). */
enum { MIXED_DIAG = 0x100 };

static int model_nf(int model) { return (model & 0xff) == MODEL_ADVDIFF ? 1 : 8; }

static void rhs_point(int model, const double *const *f, const long *P, int ndim, long x,
                      long y, long z, const double *ds, const double *prm, double *R)
{
    const int base = model & 0xff, diag = (model & MIXED_DIAG) != 0;
    if (base == MODEL_MHD8)
        mhd8_rhs_point(f, P, x, y, z, ds, diag, prm, R);
    else if (base == MODEL_MHD_FULL)
        mhdfull_rhs_point(f, P, x, y, z, ds, diag, prm, R);
    else
        advdiff_rhs_point(f, P, ndim, x, y, z, ds, prm, R);
}

static int model_ok(int model, int ndim)
{
    const int base = model & 0xff;
    if (model & ~(0xff | MIXED_DIAG))
        return 0;
    if ((model & MIXED_DIAG) && base == MODEL_ADVDIFF)
        return 0;
    return ((base == MODEL_MHD8 || base == MODEL_MHD_FULL) && ndim == 3) ||
           (base == MODEL_ADVDIFF && (ndim == 2 || ndim == 3));
}

/* R over the whole interior (R's halos untouched). Returns -1 for an invalid
 * model / dimension combination. */
int oracle_rhs(int model, const double *const *f, double *const *R, int ndim, const long *n,
               const double *ds, const double *prm)
{
    const int r = 3;
    if (!model_ok(model, ndim))
        return -1;
    int nf = model_nf(model);
    long P[3] = {ext(ndim, 0, n, r), ext(ndim, 1, n, r), ext(ndim, 2, n, r)};
    long nz = ndim > 2 ? n[2] : 1;
    int rz = ndim > 2 ? r : 0;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < n[1]; ++y)
            for (long x = 0; x < n[0]; ++x) {
                double Rp[8];
                rhs_point(model, f, P, ndim, x + r, y + r, z + rz, ds, prm, Rp);
                size_t p = at(P, x + r, y + r, z + rz);
                for (int k = 0; k < nf; ++k)
                    R[k][p] = Rp[k];
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Low-storage (2N) third-order Runge-Kutta substep                         */
/* ------------------------------------------------------------------------ */

/* The paper integrates with a three-substep explicit third-order Runge-Kutta
 * scheme (Sec. 3.3) without printing its coefficients. This is Williamson's
 * 2N-storage scheme: for substep i = 0, 1, 2
 *     w <- alpha_i w + dt R(f),   f <- f + beta_i w,
 * with alpha = (0, -5/9, -153/128) and beta = (1/3, 15/16, 8/15). Because
 * alpha_0 = 0 the first substep sets w = dt R(f) and never reads the old w. */
static const double RK_ALPHA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double RK_BETA[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

void oracle_rk3_coeffs(double *alpha, double *beta)
{
    for (int i = 0; i < 3; ++i) {
        alpha[i] = RK_ALPHA[i];
        beta[i] = RK_BETA[i];
    }
}

static void rk_update(int stage, double R, double *w, double fin, double dt, double *fout)
{
    double wn = stage == 0 ? dt * R : RK_ALPHA[stage] * (*w) + dt * R;
    *w = wn;
    *fout = fin + RK_BETA[stage] * wn;
}

/* One substep over all nf fields of the model: reads fin (halos valid),
 * updates w in place on the interior, writes fout's interior and then refreshes
 * fout's periodic halo. fin and fout must be distinct arrays. */
int oracle_rk3_substep(int model, int stage, const double *const *fin, double *const *w,
                       double *const *fout, int ndim, const long *n, const double *ds,
                       const double *prm, double dt)
{
    const int r = 3;
    if (!model_ok(model, ndim) || stage < 0 || stage > 2)
        return -1;
    int nf = model_nf(model);
    long P[3] = {ext(ndim, 0, n, r), ext(ndim, 1, n, r), ext(ndim, 2, n, r)};
    long nz = ndim > 2 ? n[2] : 1;
    int rz = ndim > 2 ? r : 0;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < n[1]; ++y)
            for (long x = 0; x < n[0]; ++x) {
                double Rp[8];
                rhs_point(model, fin, P, ndim, x + r, y + r, z + rz, ds, prm, Rp);
                size_t p = at(P, x + r, y + r, z + rz);
                for (int k = 0; k < nf; ++k)
                    rk_update(stage, Rp[k], &w[k][p], fin[k][p], dt, &fout[k][p]);
            }
    for (int k = 0; k < nf; ++k)
        oracle_fill_periodic(fout[k], ndim, n, r);
    return 0;
}

/* The same substep evaluated only at listed interior points (count triples).
 * w_in[k*count + i] is the old w of field k at point i (ignored at stage 0);
 * w_out and f_out receive the new values in the same layout. */
int oracle_rk3_substep_at(int model, int stage, const double *const *fin, const double *w_in,
                          int ndim, const long *n, const double *ds, const double *prm,
                          double dt, const long *pts, long count, double *w_out,
                          double *f_out)
{
    const int r = 3;
    if (!model_ok(model, ndim) || stage < 0 || stage > 2)
        return -1;
    int nf = model_nf(model);
    long P[3] = {ext(ndim, 0, n, r), ext(ndim, 1, n, r), ext(ndim, 2, n, r)};
    int rz = ndim > 2 ? r : 0;
    for (long i = 0; i < count; ++i) {
        long x = pts[3 * i] + r, y = pts[3 * i + 1] + r, z = pts[3 * i + 2] + rz;
        double Rp[8];
        rhs_point(model, fin, P, ndim, x, y, z, ds, prm, Rp);
        size_t p = at(P, x, y, z);
        for (int k = 0; k < nf; ++k) {
            double wk = stage == 0 ? 0.0 : w_in[k * count + i];
            rk_update(stage, Rp[k], &wk, fin[k][p], dt, &f_out[k * count + i]);
            w_out[k * count + i] = wk;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Global diagnostics                                                        */
/* ------------------------------------------------------------------------ */

/* Sum, sum of squares and maximum magnitude over the interior, accumulated
 * sequentially in FP64 in storage order. */
void oracle_reduce(const double *f, int ndim, const long *n, int r, double *out)
{
    long P[3] = {ext(ndim, 0, n, r), ext(ndim, 1, n, r), ext(ndim, 2, n, r)};
    long nz = ndim > 2 ? n[2] : 1, ny = ndim > 1 ? n[1] : 1;
    int ry = ndim > 1 ? r : 0, rz = ndim > 2 ? r : 0;
    double s = 0.0, s2 = 0.0, mx = 0.0;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < n[0]; ++x) {
                double v = f[at(P, x + r, y + ry, z + rz)];
                s += v;
                s2 += v * v;
                if (fabs(v) > mx)
                    mx = fabs(v);
            }
    out[0] = s;
    out[1] = s2;
    out[2] = mx;
}

/* Kinetic and magnetic energy of the 8-field MHD state (Table A1 order), as
 * plain sums over the interior grid points, accumulated sequentially in FP64:
 *   out[0] = 1/2 sum |u|^2,
 *   out[1] = 1/2 sum |B|^2,  B = curl A with the sixth-order first derivatives
 *            (B_x = d_y A_z - d_z A_y, B_y = d_z A_x - d_x A_z,
 *             B_z = d_x A_y - d_y A_x).
 * f: 8 radius-3 padded 3-D fields with periodic halos. */
void oracle_energy(const double *const *f, const long *n, const double *ds, double *out)
{
    const int r = 3;
    long P[3] = {ext(3, 0, n, r), ext(3, 1, n, r), ext(3, 2, n, r)};
    double ek = 0.0, em = 0.0;
    for (long z = 0; z < n[2]; ++z)
        for (long y = 0; y < n[1]; ++y)
            for (long x = 0; x < n[0]; ++x) {
                const long X = x + r, Y = y + r, Z = z + r;
                size_t p = at(P, X, Y, Z);
                double u2 = 0.0;
                for (int a = 0; a < 3; ++a)
                    u2 += f[UX + a][p] * f[UX + a][p];
                const double B[3] = {
                    d1(f[AZ], P, X, Y, Z, 1, ds) - d1(f[AY], P, X, Y, Z, 2, ds),
                    d1(f[AX], P, X, Y, Z, 2, ds) - d1(f[AZ], P, X, Y, Z, 0, ds),
                    d1(f[AY], P, X, Y, Z, 0, ds) - d1(f[AX], P, X, Y, Z, 1, ds)};
                ek += u2;
                em += B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
            }
    out[0] = 0.5 * ek;
    out[1] = 0.5 * em;
}
