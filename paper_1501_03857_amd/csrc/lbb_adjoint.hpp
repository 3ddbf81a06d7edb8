// Device code of the discrete adjoint: gradient of the time-averaged bottom
// wall heat flux J = (1/N) sum_{n=1..N} q^n (Sec. 3.2) with respect to the
// bottom-wall temperatures T_b(x) (Sec. 3.1) and the wall strength G_w
// (Eq. (22)).  One reverse step transposes the forward step of
// lbb_device.hpp stage by stage, in reverse order, over whole-lattice FP64
// work arrays (one thread per node, 256 threads per block):
//   a_macro    rho, j, psi of the stored state (FP64), block mass partials
//   a_force    forces (Eqs. (7), (9), (22)), Q, velocity (Eq. (6)), grad rho
//   a_divv     div v seen by the temperature equation
//   a_stage    RK4 stage inputs T_2, T_3, T_4 (Eqs. (19)-(20))
//   a_tinit    adjoint of T^{t+1}: identity part and the RK4 weights
//   a_tstage   one RK4 stage transposed: the Eq. (18) stencils gathered from
//              the neighbours, pressure-work term differentiated in T and rho
//   a_tstencil stencil transposes of grad rho and div v
//   a_lb       push streaming transposed (gather), MRT collision transposed
//              in moment space, velocity transposed, per-node force parts
//   a_final    interaction-force stencil transposed (gather), EOS transposed,
//              rho = sum f, Zou-He completion transposed
//   a_hf       the heat-flux sample of a state transposed (source term)
// The state of a node is its stored populations: wall-row populations that
// arrive from outside are completions of the stored ones (Zou-He), so their
// adjoint is folded into the stored ones.
#pragma once

#include "lbb_device.hpp"

namespace lbb {

constexpr int NTA = 256;

struct AdjW {
    double *rho, *jx, *jy, *psi, *sx, *sy, *Fx, *Fy, *Q, *vx, *vy, *vTx, *vTy, *Drx, *Dry, *divv;
    double *Tk[4];   // RK4 stage inputs T_1 (= T^t) .. T_4
    double *gh[4];   // adjoints of the stage slopes h_1 .. h_4
    double *gDrx, *gDry, *gdiv, *grho, *gvx, *gvy, *gFx, *gFy, *gQ, *gsx, *gsy, *gpsi;
    double *part;    // block partials: [2b] d/d rho_ave, [2b+1] d/d G_w
    double *scal;    // [0] rho_ave, [1] dJ/d rho_ave of this step, [2] dJ/dG_w (accumulated)
};

__device__ __forceinline__ bool a_wall(const DevParams &P, int j) { return !P.periodic_y && (j == 0 || j == P.ny - 1); }

// neighbour of node (i, j) along e_a (false when beyond a wall)
__device__ __forceinline__ bool a_nbr(const DevParams &P, int i, int j, int dx, int dy, size_t &cn)
{
    int ii = i + dx, jj = j + dy;
    ii = ii < 0 ? ii + P.nx : (ii >= P.nx ? ii - P.nx : ii);
    if (P.periodic_y) jj = jj < 0 ? jj + P.ny : (jj >= P.ny ? jj - P.ny : jj);
    else if (jj < 0 || jj >= P.ny) return false;
    cn = (size_t)jj * P.nx + ii;
    return true;
}

__constant__ const double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
__constant__ const double kWpsi[9] = {0.0, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12};

// phi'(T) and phi''(T) of the Peng-Robinson alpha function (Eq. (21))
__device__ __forceinline__ void phi_derivs(const DevParams &P, double T, double &d1, double &d2)
{
    const double u = sqrt(T * P.inv_Tc);
    d1 = -P.kappa * (1.0 + P.kappa * (1.0 - u)) / (P.Tc * u);
    d2 = P.kappa * (1.0 + P.kappa) / (2.0 * P.Tc * P.Tc * u * u * u);
}

// (dp/drho)_T and (dp/dT)_rho of Eq. (21)
__device__ __forceinline__ void eos_derivs(const DevParams &P, double r, double T, double &dpdr, double &dpdT)
{
    const double u = sqrt(T * P.inv_Tc);
    const double s = 1.0 + P.kappa * (1.0 - u);
    const double phi = s * s;
    double d1, d2;
    phi_derivs(P, T, d1, d2);
    const double D1 = 1.0 - P.b * r, D2 = 1.0 + 2.0 * P.b * r - P.b * P.b * r * r;
    dpdr = P.R * T / (D1 * D1) - P.a * phi * 2.0 * r * (1.0 + P.b * r) / (D2 * D2);
    dpdT = r * P.R / D1 - P.a * r * r * d1 / D2;
}

// Zou-He completion transposed: the adjoint of the completed populations of
// a wall node folded onto the stored (known) ones; the others are zeroed.
__device__ __forceinline__ void zou_he_T(double g[9], int bottom)
{
    if (bottom) {
        g[4] += g[2];
        g[7] += g[5];
        g[8] += g[6];
        g[1] += -0.5 * g[5] + 0.5 * g[6];
        g[3] += 0.5 * g[5] - 0.5 * g[6];
        g[2] = g[5] = g[6] = 0.0;
    } else {
        g[2] += g[4];
        g[5] += g[7];
        g[6] += g[8];
        g[1] += 0.5 * g[7] - 0.5 * g[8];
        g[3] += -0.5 * g[7] + 0.5 * g[8];
        g[4] = g[7] = g[8] = 0.0;
    }
}

#define A_NODE                                                          \
    const size_t N = (size_t)P.nx * P.ny;                               \
    const size_t c = (size_t)blockIdx.x * NTA + threadIdx.x;            \
    const bool on = c < N;                                              \
    const int gi = on ? (int)(c % P.nx) : 0, gj = on ? (int)(c / P.nx) : 0; \
    (void)gi;

template <typename S>
__global__ __launch_bounds__(NTA) void a_macro(DevParams P, const S *__restrict__ f, const S *__restrict__ T, AdjW w)
{
    __shared__ double red[NTA / 64];
    A_NODE
    double m = 0.0;
    if (on) {
        double fl[9];
        load_node(P, f, N, c, gj, fl);
        double r = 0.0;
        for (int a = 0; a < 9; ++a) r += fl[a];
        w.rho[c] = r;
        w.jx[c] = fl[1] - fl[3] + fl[5] - fl[6] - fl[7] + fl[8];
        w.jy[c] = fl[2] - fl[4] + fl[5] + fl[6] - fl[7] - fl[8];
        const double Tv = P.T_ref + (double)T[c];
        w.Tk[0][c] = Tv;
        w.psi[c] = pseudopotential(P, r, Tv);
        m = r;
    }
    const double s = block_sum<NTA>(m, red);
    if (threadIdx.x == 0) w.part[blockIdx.x] = s;
}

__global__ void a_reduce_mass(DevParams P, AdjW w, int nb)
{
    __shared__ double red[NTA / 64];
    const double s = block_sum_array<NTA>(w.part, nb, red);
    if (threadIdx.x == 0) w.scal[0] = s / ((double)P.nx * (double)P.ny);
}

__global__ __launch_bounds__(NTA) void a_force(DevParams P, AdjW w)
{
    A_NODE
    if (!on) return;
    double sx = 0.0, sy = 0.0, Fx = 0.0, Fy = 0.0, Q = 0.0, rx = 0.0, ry = 0.0;
    const double r = w.rho[c];
    if (!a_wall(P, gj)) {
        for (int a = 1; a < 9; ++a) {
            size_t cn;
            a_nbr(P, gi, gj, kEX[a], kEY[a], cn);
            sx += kWpsi[a] * w.psi[cn] * kEX[a];
            sy += kWpsi[a] * w.psi[cn] * kEY[a];
            rx += 3.0 * kW[a] * kEX[a] * w.rho[cn];
            ry += 3.0 * kW[a] * kEY[a] * w.rho[cn];
        }
        const double ps = w.psi[c];
        Fx = -P.G * ps * sx;
        Fy = -P.G * ps * sy;
        Q = P.G * P.G * (sx * sx + sy * sy);
        if (!P.periodic_y && gj == 1) Fy += P.Gw_bottom * ps * ps / 6.0;
        if (!P.periodic_y && gj == P.ny - 2) Fy -= P.Gw_top * ps * ps / 6.0;
        Fy -= (r - w.scal[0]) * P.g;
    }
    w.sx[c] = sx;
    w.sy[c] = sy;
    w.Fx[c] = Fx;
    w.Fy[c] = Fy;
    w.Q[c] = Q;
    w.Drx[c] = rx;
    w.Dry[c] = ry;
    const double vx = (w.jx[c] + 0.5 * Fx) / r, vy = (w.jy[c] + 0.5 * Fy) / r;
    w.vx[c] = vx;
    w.vy[c] = vy;
    w.vTx[c] = a_wall(P, gj) ? 0.0 : vx;
    w.vTy[c] = a_wall(P, gj) ? 0.0 : vy;
}

__global__ __launch_bounds__(NTA) void a_divv(DevParams P, AdjW w)
{
    A_NODE
    if (!on) return;
    double d = 0.0;
    if (!a_wall(P, gj))
        for (int a = 1; a < 9; ++a) {
            size_t cn;
            a_nbr(P, gi, gj, kEX[a], kEY[a], cn);
            d += 3.0 * kW[a] * (kEX[a] * w.vTx[cn] + kEY[a] * w.vTy[cn]);
        }
    w.divv[c] = d;
}

// Eq. (18) at node c for the stage field Tf (with its stencils returned)
__device__ __forceinline__ double a_K(const DevParams &P, const AdjW &w, const double *Tf, int gi, int gj, size_t c,
                                      double &dTx, double &dTy, double &lap)
{
    dTx = dTy = lap = 0.0;
    const double tc = Tf[c];
    for (int a = 1; a < 9; ++a) {
        size_t cn;
        a_nbr(P, gi, gj, kEX[a], kEY[a], cn);
        dTx += 3.0 * kW[a] * kEX[a] * Tf[cn];
        dTy += 3.0 * kW[a] * kEY[a] * Tf[cn];
        lap += 6.0 * kW[a] * (Tf[cn] - tc);
    }
    const double r = w.rho[c];
    double d1, d2;
    phi_derivs(P, tc, d1, d2);
    const double Pt = r * P.R / (1.0 - P.b * r) - P.a * r * r * d1 / (1.0 + 2.0 * P.b * r - P.b * P.b * r * r);
    return -(w.vTx[c] * dTx + w.vTy[c] * dTy) + P.chi * (lap + (w.Drx[c] * dTx + w.Dry[c] * dTy) / r) -
           tc * Pt * w.divv[c] / (r * P.cv);
}

// T_{k+1} = T_1 + c_k K(T_k) on interior rows (T_1 on wall rows)
__global__ __launch_bounds__(NTA) void a_stage(DevParams P, AdjW w, int k, double ck)
{
    A_NODE
    if (!on) return;
    double h = 0.0;
    if (!a_wall(P, gj)) {
        double dx, dy, lp;
        h = a_K(P, w, w.Tk[k], gi, gj, c, dx, dy, lp);
    }
    w.Tk[k + 1][c] = w.Tk[0][c] + ck * h;
}

// Start of a reverse step: lT0 = lT1 (identity part of T^{t+1} = T^t + ...),
// slope adjoints from T^{t+1} = T^t + (h1 + 2 h2 + 2 h3 + h4)/6, the
// per-node accumulators cleared.
__global__ __launch_bounds__(NTA) void a_tinit(DevParams P, AdjW w, const double *__restrict__ lT1, double *__restrict__ lT0)
{
    A_NODE
    if (!on) return;
    const double g = a_wall(P, gj) ? 0.0 : lT1[c] / 6.0;
    w.gh[0][c] = g;
    w.gh[1][c] = 2.0 * g;
    w.gh[2][c] = 2.0 * g;
    w.gh[3][c] = g;
    lT0[c] = lT1[c];
    w.gDrx[c] = w.gDry[c] = w.gdiv[c] = w.grho[c] = w.gvx[c] = w.gvy[c] = 0.0;
}

// One RK4 stage transposed: gather the adjoint of T_k at c from the slope
// adjoints of c and its neighbours; accumulate the rho and v parts at c.
__global__ __launch_bounds__(NTA) void a_tstage(DevParams P, AdjW w, int k, double ck, double *__restrict__ lT0)
{
    A_NODE
    if (!on) return;
    const double *Tf = w.Tk[k];
    const double *gh = w.gh[k];
    double gT = 0.0;
    // neighbours c' = c - e_a whose stencils read T(c) with weight e_a
    for (int a = 1; a < 9; ++a) {
        size_t cp;
        if (!a_nbr(P, gi, gj, -kEX[a], -kEY[a], cp)) continue;
        const int jp = (int)(cp / P.nx);
        if (a_wall(P, jp)) continue;
        const double g = gh[cp];
        if (g == 0.0) continue;
        const double rp = w.rho[cp];
        const double ax = -w.vTx[cp] + P.chi * w.Drx[cp] / rp, ay = -w.vTy[cp] + P.chi * w.Dry[cp] / rp;
        gT += g * (3.0 * kW[a] * (ax * kEX[a] + ay * kEY[a]) + 6.0 * kW[a] * P.chi);
    }
    if (!a_wall(P, gj)) {
        const double g = gh[c];
        double dTx, dTy, lap;
        (void)a_K(P, w, Tf, gi, gj, c, dTx, dTy, lap);
        const double r = w.rho[c], Tv = Tf[c], dv = w.divv[c];
        double d1, d2;
        phi_derivs(P, Tv, d1, d2);
        const double D1 = 1.0 - P.b * r, D2 = 1.0 + 2.0 * P.b * r - P.b * P.b * r * r;
        const double Pt = r * P.R / D1 - P.a * r * r * d1 / D2;
        const double dPdT = -P.a * r * r * d2 / D2;
        gT += g * (-(10.0 / 3.0) * P.chi - dv / (r * P.cv) * (Pt + Tv * dPdT));
        w.gDrx[c] += g * P.chi * dTx / r;
        w.gDry[c] += g * P.chi * dTy / r;
        w.gvx[c] += -g * dTx;
        w.gvy[c] += -g * dTy;
        w.gdiv[c] += -g * Tv * Pt / (r * P.cv);
        const double dPr = P.R * P.b / (D1 * D1) - P.a * d1 * (1.0 + P.b * P.b * r * r) / (D2 * D2);
        w.grho[c] += g * (-P.chi * (w.Drx[c] * dTx + w.Dry[c] * dTy) / (r * r) - Tv * dv / P.cv * dPr);
        if (k > 0) w.gh[k - 1][c] += ck * gT;
    }
    lT0[c] += gT;
}

// Stencil transposes of grad rho and div v (the velocity seen by the
// temperature equation is zero on the wall rows, so only interior nodes
// receive the div v part); the temperature velocity adjoint joins v.
__global__ __launch_bounds__(NTA) void a_tstencil(DevParams P, AdjW w)
{
    A_NODE
    if (!on) return;
    double gr = 0.0, gu = 0.0, gv = 0.0;
    for (int a = 1; a < 9; ++a) {
        size_t cp;
        if (!a_nbr(P, gi, gj, -kEX[a], -kEY[a], cp)) continue;
        if (a_wall(P, (int)(cp / P.nx))) continue;
        gr += 3.0 * kW[a] * (kEX[a] * w.gDrx[cp] + kEY[a] * w.gDry[cp]);
        gu += 3.0 * kW[a] * kEX[a] * w.gdiv[cp];
        gv += 3.0 * kW[a] * kEY[a] * w.gdiv[cp];
    }
    w.grho[c] += gr;
    if (!a_wall(P, gj)) {
        w.gvx[c] += gu;
        w.gvy[c] += gv;
    } else {
        w.gvx[c] = 0.0;
        w.gvy[c] = 0.0;
    }
}

// Streaming and collision transposed at node c; writes the adjoint of the
// completed populations (before the density and completion parts), and the
// per-node force adjoints.
template <typename S>
__global__ __launch_bounds__(NTA) void a_lb(DevParams P, AdjW w, const S *__restrict__ f,
                                            const double *__restrict__ lf1, double *__restrict__ lf0)
{
    __shared__ double red[NTA / 64];
    A_NODE
    double pr = 0.0, pg = 0.0;
    if (on) {
        // push streaming transposed: f'(c + e_a, a) = f*(c, a)
        double gfs[9];
        for (int a = 0; a < 9; ++a) {
            size_t ct;
            gfs[a] = a_nbr(P, gi, gj, kEX[a], kEY[a], ct) ? lf1[(size_t)a * N + ct] : 0.0;
        }
        double fl[9];
        load_node(P, f, N, c, gj, fl);
        const double r = w.rho[c], vx = w.vx[c], vy = w.vy[c], Fx = w.Fx[c], Fy = w.Fy[c];
        // moments of f and the equilibrium (Eq. (5)), forcing (Eq. (8))
        const double s14 = fl[1] + fl[2] + fl[3] + fl[4], s58 = fl[5] + fl[6] + fl[7] + fl[8];
        double m[9];
        m[0] = r;
        m[1] = -4.0 * fl[0] - s14 + 2.0 * s58;
        m[2] = 4.0 * fl[0] - 2.0 * s14 + s58;
        m[3] = w.jx[c];
        m[4] = -2.0 * fl[1] + 2.0 * fl[3] + fl[5] - fl[6] - fl[7] + fl[8];
        m[5] = w.jy[c];
        m[6] = -2.0 * fl[2] + 2.0 * fl[4] + fl[5] + fl[6] - fl[7] - fl[8];
        m[7] = fl[1] - fl[2] + fl[3] - fl[4];
        m[8] = fl[5] - fl[6] + fl[7] - fl[8];
        const double v2 = vx * vx + vy * vy, vF = vx * Fx + vy * Fy;
        const double meq7 = r * (vx * vx - vy * vy), meq8 = r * vx * vy;
        const double S7 = 2.0 * (vx * Fx - vy * Fy), S8 = vx * Fy + vy * Fx;
        const double tau = P.tau_V + (r - P.rho_V) * P.tau_slope, s_nu = 1.0 / tau;
        const double L[9] = {P.s_rho, P.s_e, P.s_zeta, P.s_j, P.s_q, P.s_j, P.s_q, s_nu, s_nu};
        // f* = M^T diag(1/n) m*  ->  gm* = diag(1/n) M gf*
        double gms[9];
        {
            const double g14 = gfs[1] + gfs[2] + gfs[3] + gfs[4], g58 = gfs[5] + gfs[6] + gfs[7] + gfs[8];
            double a0 = 0.0;
            for (int a = 0; a < 9; ++a) a0 += gfs[a];
            gms[0] = a0 / 9.0;
            gms[1] = (-4.0 * gfs[0] - g14 + 2.0 * g58) / 36.0;
            gms[2] = (4.0 * gfs[0] - 2.0 * g14 + g58) / 36.0;
            gms[3] = (gfs[1] - gfs[3] + gfs[5] - gfs[6] - gfs[7] + gfs[8]) / 6.0;
            gms[4] = (-2.0 * gfs[1] + 2.0 * gfs[3] + gfs[5] - gfs[6] - gfs[7] + gfs[8]) / 12.0;
            gms[5] = (gfs[2] - gfs[4] + gfs[5] + gfs[6] - gfs[7] - gfs[8]) / 6.0;
            gms[6] = (-2.0 * gfs[2] + 2.0 * gfs[4] + gfs[5] + gfs[6] - gfs[7] - gfs[8]) / 12.0;
            gms[7] = (gfs[1] - gfs[2] + gfs[3] - gfs[4]) / 4.0;
            gms[8] = (gfs[5] - gfs[6] + gfs[7] - gfs[8]) / 4.0;
        }
        // m* = m - L (m - m_eq) + (1 - L/2) S
        double gm[9], gq[9], gS[9];
        for (int k = 0; k < 9; ++k) {
            gm[k] = (1.0 - L[k]) * gms[k];
            gq[k] = L[k] * gms[k];
            gS[k] = (1.0 - 0.5 * L[k]) * gms[k];
        }
        const double gsnu = gms[7] * (-(m[7] - meq7) - 0.5 * S7) + gms[8] * (-(m[8] - meq8) - 0.5 * S8);
        // m = M f  ->  gf += M^T gm
        double gf[9];
        gf[0] = gm[0] - 4.0 * gm[1] + 4.0 * gm[2];
        gf[1] = gm[0] - gm[1] - 2.0 * gm[2] + gm[3] - 2.0 * gm[4] + gm[7];
        gf[2] = gm[0] - gm[1] - 2.0 * gm[2] + gm[5] - 2.0 * gm[6] - gm[7];
        gf[3] = gm[0] - gm[1] - 2.0 * gm[2] - gm[3] + 2.0 * gm[4] + gm[7];
        gf[4] = gm[0] - gm[1] - 2.0 * gm[2] - gm[5] + 2.0 * gm[6] - gm[7];
        gf[5] = gm[0] + 2.0 * gm[1] + gm[2] + gm[3] + gm[4] + gm[5] + gm[6] + gm[8];
        gf[6] = gm[0] + 2.0 * gm[1] + gm[2] - gm[3] - gm[4] + gm[5] + gm[6] - gm[8];
        gf[7] = gm[0] + 2.0 * gm[1] + gm[2] - gm[3] - gm[4] - gm[5] - gm[6] + gm[8];
        gf[8] = gm[0] + 2.0 * gm[1] + gm[2] + gm[3] + gm[4] - gm[5] - gm[6] - gm[8];
        // m_eq(rho, v) of Eq. (5)
        double gr = gq[0] + gq[1] * (-2.0 + 3.0 * v2) + gq[2] * (1.0 - 3.0 * v2) + gq[3] * vx - gq[4] * vx +
                    gq[5] * vy - gq[6] * vy + gq[7] * (vx * vx - vy * vy) + gq[8] * vx * vy;
        double gvx = r * (6.0 * vx * (gq[1] - gq[2]) + gq[3] - gq[4] + 2.0 * vx * gq[7] + vy * gq[8]);
        double gvy = r * (6.0 * vy * (gq[1] - gq[2]) + gq[5] - gq[6] - 2.0 * vy * gq[7] + vx * gq[8]);
        // S(v, F, Q) of Eq. (8)
        const double a6 = gS[1] - gS[2];
        double gFx = 6.0 * a6 * vx + gS[3] - gS[4] + 2.0 * vx * gS[7] + vy * gS[8];
        double gFy = 6.0 * a6 * vy + gS[5] - gS[6] - 2.0 * vy * gS[7] + vx * gS[8];
        gvx += 6.0 * a6 * Fx + 2.0 * Fx * gS[7] + Fy * gS[8];
        gvy += 6.0 * a6 * Fy - 2.0 * Fy * gS[7] + Fx * gS[8];
        const double gQ = P.sig_e * gS[1] - P.sig_z * gS[2];
        (void)vF;
        // s_nu = 1 / tau(rho)
        gr += gsnu * (-P.tau_slope / (tau * tau));
        // v = (j + F/2)/rho, with what the temperature equation saw of v
        gvx += w.gvx[c];
        gvy += w.gvy[c];
        const double gjx = gvx / r, gjy = gvy / r;
        gFx += 0.5 * gvx / r;
        gFy += 0.5 * gvy / r;
        gr += -(gvx * vx + gvy * vy) / r;
        for (int a = 0; a < 9; ++a) lf0[(size_t)a * N + c] = gf[a] + kEX[a] * gjx + kEY[a] * gjy;
        // per-node force parts (no force on the wall rows)
        double gpsi = 0.0, gsx = 0.0, gsy = 0.0;
        if (!a_wall(P, gj)) {
            const double ps = w.psi[c];
            gr += -P.g * gFy;
            pr = P.g * gFy;
            if (!P.periodic_y && gj == 1) {
                gpsi += gFy * P.Gw_bottom * ps / 3.0;
                pg = gFy * ps * ps / 6.0;
            }
            if (!P.periodic_y && gj == P.ny - 2) gpsi += -gFy * P.Gw_top * ps / 3.0;
            gpsi += -P.G * (w.sx[c] * gFx + w.sy[c] * gFy);
            gsx = -P.G * ps * gFx + 2.0 * P.G * P.G * w.sx[c] * gQ;
            gsy = -P.G * ps * gFy + 2.0 * P.G * P.G * w.sy[c] * gQ;
        }
        w.grho[c] += gr;
        w.gpsi[c] = gpsi;
        w.gsx[c] = gsx;
        w.gsy[c] = gsy;
    }
    const double sr = block_sum<NTA>(pr, red);
    __syncthreads();
    const double sg = block_sum<NTA>(pg, red);
    if (threadIdx.x == 0) {
        w.part[2 * blockIdx.x] = sr;
        w.part[2 * blockIdx.x + 1] = sg;
    }
}

__global__ void a_reduce_force(AdjW w, int nb)
{
    __shared__ double red[NTA / 64];
    double sr = 0.0, sg = 0.0;
    for (int k = threadIdx.x; k < nb; k += NTA) {
        sr += w.part[2 * k];
        sg += w.part[2 * k + 1];
    }
    const double a = block_sum<NTA>(sr, red);
    __syncthreads();
    const double b = block_sum<NTA>(sg, red);
    if (threadIdx.x == 0) {
        w.scal[1] = a;
        w.scal[2] += b;
    }
}

// Interaction-force stencil transposed (gather of s over the neighbours),
// EOS transposed, rho = sum f, Zou-He completion transposed.
template <typename S>
__global__ __launch_bounds__(NTA) void a_final(DevParams P, AdjW w, const S *__restrict__ T, double *__restrict__ lf0,
                                               double *__restrict__ lT0)
{
    A_NODE
    if (!on) return;
    double gpsi = w.gpsi[c];
    for (int a = 1; a < 9; ++a) {
        size_t cp;
        if (!a_nbr(P, gi, gj, -kEX[a], -kEY[a], cp)) continue;
        if (a_wall(P, (int)(cp / P.nx))) continue;
        gpsi += kWpsi[a] * (kEX[a] * w.gsx[cp] + kEY[a] * w.gsy[cp]);
    }
    double gr = w.grho[c] + w.scal[1] / ((double)P.nx * (double)P.ny);
    if (gpsi != 0.0) {
        const double r = w.rho[c], Tv = P.T_ref + (double)T[c];
        double dpdr, dpdT;
        eos_derivs(P, r, Tv, dpdr, dpdT);
        const double gq = gpsi / (2.0 * w.psi[c]) * P.two_over_G;
        gr += gq * (dpdr - 1.0 / 3.0);
        lT0[c] += gq * dpdT;
    }
    double g[9];
    for (int a = 0; a < 9; ++a) g[a] = lf0[(size_t)a * N + c] + gr;
    if (!P.periodic_y && P.mode != MODE_THERMAL_ONLY) {
        if (gj == 0) zou_he_T(g, 1);
        else if (gj == P.ny - 1) zou_he_T(g, 0);
    }
    for (int a = 0; a < 9; ++a) lf0[(size_t)a * N + c] = g[a];
}

// The heat-flux sample of a state transposed, weight wq (= 1/N), added to
// the adjoint of that state.  One thread per bottom-wall node.
template <typename S>
__global__ void a_hf(DevParams P, const S *__restrict__ f, const S *__restrict__ T, double wq,
                     double *__restrict__ lf, double *__restrict__ lT)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.nx || P.periodic_y) return;
    const size_t N = (size_t)P.nx * P.ny;
    double fl[9];
    load_node(P, f, N, (size_t)i, 0, fl);
    double r0 = 0.0;
    for (int a = 0; a < 9; ++a) r0 += fl[a];
    const double t0 = (double)T[i], t1 = (double)T[P.nx + i], t2 = (double)T[2 * P.nx + i];
    const double k = -P.cv_chi / P.nx * wq;
    double g[9];
    for (int a = 0; a < 9; ++a) g[a] = k * (-3.0 * t0 + 4.0 * t1 - t2) / 2.0;
    zou_he_T(g, 1);
    for (int a = 0; a < 9; ++a) lf[(size_t)a * N + i] += g[a];
    lT[i] += k * r0 * (-1.5);
    lT[P.nx + i] += k * r0 * 2.0;
    lT[2 * P.nx + i] += k * r0 * (-0.5);
}

}  // namespace lbb
