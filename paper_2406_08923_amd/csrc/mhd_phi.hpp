// mhd_phi.hpp -- the nonlinear stencil function phi (Eq. 9) of the two MHD
// models, evaluated from the sixth-order derivative bank of one point. Shared
// by the cached and the LDS-brick substep kernels, so both compute the same
// arithmetic on the same bank values.
//
// Field order (Table A1): lnrho, u_x, u_y, u_z, s, A_x, A_y, A_z.
//   MHD8 (proxy): Eq. A1-A4 with rho, T, c_p, mu_0 = 1, no heating, cooling,
//     conduction or bulk viscosity, plus a nu-Laplacian on lnrho and s.
//   MHD_FULL: Eq. A1-A4 as written, with an ideal-gas closure:
//     rho = exp(lnrho), cs2 = cs0^2 exp(gamma s / c_p + (gamma - 1)(lnrho - lnrho0)),
//     T = cs2 / ((gamma - 1) c_p), j = (grad div A - lap A) / mu_0,
//     R_u gains j x B / rho, -cs2 grad(s / c_p + lnrho) and zeta grad(div u);
//     R_s = -u.grad s + [H - C + K lap T + eta mu_0 |j|^2 + 2 rho nu S:S
//           + zeta rho (div u)^2] / (rho T), lap T by the chain rule:
//     lap T = T [(gamma / c_p) lap s + (gamma - 1) lap lnrho + |g|^2],
//     g = (gamma / c_p) grad s + (gamma - 1) grad lnrho.
#pragma once

#include "rk_kernels.hpp"

namespace stn {

constexpr int MHD_PROXY = 0; // STENCIL_MODEL_MHD8
constexpr int MHD_FULL = 2;  // STENCIL_MODEL_MHD_FULL

// The bank of one point, already scaled by the grid spacing: values, first
// derivatives (du[a][b] = d_a u_b), Laplacians, grad(div u), B = curl A and
// J = grad(div A) - lap A (curl curl A, before the 1/mu_0).
template <typename C> struct MhdBank {
    C l, s, gl[3], gs[3], lapl, laps;
    C u[3], du[3][3], lapu[3], gdivu[3];
    C A[3], B[3], J[3], lapA[3];
};

template <int MODEL, typename C>
__device__ __forceinline__ void mhd_phi(const MhdBank<C> &k, const MhdParams &m, C R[8])
{
    const C nu = C(m.nu), eta = C(m.eta);
    const C divu = k.du[0][0] + k.du[1][1] + k.du[2][2];
    C Sm[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Sm[i][j] = C(0.5) * (k.du[i][j] + k.du[j][i]) - (i == j ? divu / C(3) : C(0));
    C SS = 0, adv[3], Sgl[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        adv[i] = k.u[0] * k.du[0][i] + k.u[1] * k.du[1][i] + k.u[2] * k.du[2][i];
        Sgl[i] = Sm[i][0] * k.gl[0] + Sm[i][1] * k.gl[1] + Sm[i][2] * k.gl[2];
        SS += Sm[i][0] * Sm[i][0] + Sm[i][1] * Sm[i][1] + Sm[i][2] * Sm[i][2];
    }
    const C ugl = k.u[0] * k.gl[0] + k.u[1] * k.gl[1] + k.u[2] * k.gl[2];
    const C ugs = k.u[0] * k.gs[0] + k.u[1] * k.gs[1] + k.u[2] * k.gs[2];
    const C uxB[3] = {k.u[1] * k.B[2] - k.u[2] * k.B[1], k.u[2] * k.B[0] - k.u[0] * k.B[2],
                      k.u[0] * k.B[1] - k.u[1] * k.B[0]};
#pragma unroll
    for (int i = 0; i < 3; ++i)
        R[5 + i] = uxB[i] + eta * k.lapA[i];

    if constexpr (MODEL == MHD_PROXY) {
        const C cs2 = C(m.cs2);
        const C jxB[3] = {k.J[1] * k.B[2] - k.J[2] * k.B[1], k.J[2] * k.B[0] - k.J[0] * k.B[2],
                          k.J[0] * k.B[1] - k.J[1] * k.B[0]};
        R[0] = -ugl - divu + nu * k.lapl;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            R[1 + i] = -adv[i] - cs2 * (k.gs[i] + k.gl[i]) + jxB[i] +
                       nu * (k.lapu[i] + k.gdivu[i] / C(3) + C(2) * Sgl[i]);
        R[4] = -ugs + nu * k.laps + eta * (k.J[0] * k.J[0] + k.J[1] * k.J[1] + k.J[2] * k.J[2]) +
               C(2) * nu * SS;
    } else {
        static_assert(MODEL == MHD_FULL, "unknown MHD model");
        const C zeta = C(m.zeta), mu0 = C(m.mu0), gam = C(m.gamma), cp = C(m.cp);
        const C gm1 = gam - C(1), gcp = gam / cp;
        const C rho = exp(k.l);
        const C cs2 = C(m.cs2) * exp(gcp * k.s + gm1 * (k.l - C(m.lnrho0)));
        const C T = cs2 / (gm1 * cp);
        C j[3], gg = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            j[i] = k.J[i] / mu0;
            const C gi = gcp * k.gs[i] + gm1 * k.gl[i];
            gg += gi * gi;
        }
        const C lapT = T * (gcp * k.laps + gm1 * k.lapl + gg);
        const C jxB[3] = {j[1] * k.B[2] - j[2] * k.B[1], j[2] * k.B[0] - j[0] * k.B[2],
                          j[0] * k.B[1] - j[1] * k.B[0]};
        const C jj = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
        R[0] = -ugl - divu;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            R[1 + i] = -adv[i] - cs2 * (k.gs[i] / cp + k.gl[i]) + jxB[i] / rho +
                       nu * (k.lapu[i] + k.gdivu[i] / C(3) + C(2) * Sgl[i]) + zeta * k.gdivu[i];
        R[4] = -ugs + (C(m.heat) - C(m.cool) + C(m.K) * lapT + eta * mu0 * jj +
                       C(2) * rho * nu * SS + zeta * rho * divu * divu) /
                          (rho * T);
    }
}

} // namespace stn
