/*
 * Discrete adjoint of the oracle's time step (TEST INFRASTRUCTURE ONLY; see
 * lbb_oracle.c).
 *
 * Objective: J = (1/N) sum_{n=1..N} q^n, the time-averaged bottom-wall heat
 * flux (Sec. 3.2) over N steps from the current state.  Parameters: the
 * bottom-wall temperatures T_b(x) (the Dirichlet row of the temperature,
 * Sec. 3.1) and the bottom fluid-solid strength G_w (Eq. (22)).
 *
 * The reverse sweep transposes each stage of the forward step of
 * lbb_oracle.c in reverse order, written out plainly over whole arrays:
 *   O13 heat flux        -> source terms on f and T of every sampled state
 *   O12 RK4 (Eqs. (19)-(20)) -> stage by stage, each K(T) of Eq. (18)
 *                           transposed (stencils scattered back, the
 *                           pressure-work term differentiated in T and rho)
 *   O11 Zou-He, O10 streaming -> the linear maps transposed
 *   O9  MRT collision    -> in moment space, including the rho-dependence of
 *                           the shear rate s_nu(rho)
 *   O8  velocity, O4-O7 forces (F_m stencil transposed, F_ads, buoyancy with
 *       the global rho_ave), O3 the EOS/pseudopotential, O1 the density.
 * Checkpoints every K steps; each segment is recomputed forward before its
 * reverse sweep.  Only the COUPLED mode with walls is differentiated.
 */
#include "lbb_oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WEQ[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double WPSI[9] = {0.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0,
                               1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0};
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};
static const double MNORM[9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};

static inline int wrap(int i, int n) { return (i % n + n) % n; }

/* ---------------------------------------------------------------------- */
/* Forward intermediates of one step, recomputed from the state (f, T)     */
/* ---------------------------------------------------------------------- */

typedef struct {
    int nx, ny;
    size_t n;
    double *rho, *psi, *sx, *sy, *Fx, *Fy, *Q, *jx, *jy, *vx, *vy, *vTx, *vTy;
    double rho_ave;
    double *Tk[4], *hk[4]; /* RK4 stage inputs and slopes */
    double *ws[7];
} fwd_t;

static int fwd_alloc(fwd_t *w, int nx, int ny)
{
    memset(w, 0, sizeof *w);
    w->nx = nx;
    w->ny = ny;
    w->n = (size_t)nx * ny;
    double **arr[] = {&w->rho, &w->psi, &w->sx, &w->sy, &w->Fx, &w->Fy, &w->Q, &w->jx, &w->jy,
                      &w->vx, &w->vy, &w->vTx, &w->vTy};
    int ok = 1;
    for (size_t k = 0; k < sizeof arr / sizeof arr[0]; ++k) ok = ok && (*arr[k] = calloc(w->n, sizeof(double)));
    for (int k = 0; k < 4; ++k) {
        ok = ok && (w->Tk[k] = calloc(w->n, sizeof(double)));
        ok = ok && (w->hk[k] = calloc(w->n, sizeof(double)));
    }
    for (int k = 0; k < 7; ++k) ok = ok && (w->ws[k] = calloc(w->n, sizeof(double)));
    return ok;
}

static void fwd_free(fwd_t *w)
{
    double *arr[] = {w->rho, w->psi, w->sx, w->sy, w->Fx, w->Fy, w->Q, w->jx, w->jy, w->vx, w->vy, w->vTx, w->vTy};
    for (size_t k = 0; k < sizeof arr / sizeof arr[0]; ++k) free(arr[k]);
    for (int k = 0; k < 4; ++k) {
        free(w->Tk[k]);
        free(w->hk[k]);
    }
    for (int k = 0; k < 7; ++k) free(w->ws[k]);
}

static int is_wall(const orc_params *p, int j) { return !p->periodic_y && (j == 0 || j == p->ny - 1); }

/* O1-O8 and the RK4 stages of one step from (f, T), as in the forward. */
static void fwd_intermediates(const orc_state *s, const double *f, const double *T, fwd_t *w)
{
    const orc_params *p = &s->p;
    const int nx = p->nx, ny = p->ny;
    const size_t n = w->n;
    double mass = 0.0;
    for (size_t c = 0; c < n; ++c) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int a = 0; a < 9; ++a) {
            r += f[(size_t)a * n + c];
            jx += EX[a] * f[(size_t)a * n + c];
            jy += EY[a] * f[(size_t)a * n + c];
        }
        w->rho[c] = r;
        w->jx[c] = jx;
        w->jy[c] = jy;
        mass += r;
    }
    w->rho_ave = mass / (double)n;
    for (size_t c = 0; c < n; ++c) {
        double pe = orc_p_eos(w->rho[c], T[c], p->a, p->b, p->R, s->Tc, s->kappa);
        w->psi[c] = sqrt(2.0 * (pe - w->rho[c] / 3.0) / p->G);
    }
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            w->sx[c] = w->sy[c] = w->Fx[c] = w->Fy[c] = w->Q[c] = 0.0;
            if (!is_wall(p, j)) {
                double sx = 0.0, sy = 0.0;
                for (int a = 1; a < 9; ++a) {
                    int ii = wrap(i + EX[a], nx), jj = p->periodic_y ? wrap(j + EY[a], ny) : j + EY[a];
                    sx += WPSI[a] * w->psi[(size_t)jj * nx + ii] * EX[a];
                    sy += WPSI[a] * w->psi[(size_t)jj * nx + ii] * EY[a];
                }
                w->sx[c] = sx;
                w->sy[c] = sy;
                w->Fx[c] = -p->G * w->psi[c] * sx;
                w->Fy[c] = -p->G * w->psi[c] * sy;
                w->Q[c] = p->G * p->G * (sx * sx + sy * sy);
                if (!p->periodic_y && j == 1) w->Fy[c] += p->Gw_bottom * w->psi[c] * w->psi[c] / 6.0;
                if (!p->periodic_y && j == ny - 2) w->Fy[c] -= p->Gw_top * w->psi[c] * w->psi[c] / 6.0;
                w->Fy[c] += -(w->rho[c] - w->rho_ave) * p->g;
            }
            w->vx[c] = (w->jx[c] + 0.5 * w->Fx[c]) / w->rho[c];
            w->vy[c] = (w->jy[c] + 0.5 * w->Fy[c]) / w->rho[c];
            w->vTx[c] = is_wall(p, j) ? 0.0 : w->vx[c];
            w->vTy[c] = is_wall(p, j) ? 0.0 : w->vy[c];
        }
    }
    /* RK4 stages: T1 = T, T2 = T + h1/2, T3 = T + h2/2, T4 = T + h3 */
    const double cst[4] = {0.0, 0.5, 0.5, 1.0};
    for (int k = 0; k < 4; ++k) {
        for (size_t c = 0; c < n; ++c) w->Tk[k][c] = T[c] + cst[k] * (k ? w->hk[k - 1][c] : 0.0);
        orc_thermal_rhs(p, w->rho, w->vTx, w->vTy, w->Tk[k], w->hk[k]);
    }
}

/* ---------------------------------------------------------------------- */
/* Transposes                                                              */
/* ---------------------------------------------------------------------- */

/* Scatter the adjoint of the isotropic stencils of a field phi at the
 * interior nodes: dx = 3 sum W e_x phi(n), dy = 3 sum W e_y phi(n),
 * lap = 6 sum W (phi(n) - phi(c)). */
static void stencil_T(const orc_params *p, const double *gdx, const double *gdy, const double *glap,
                      double *gphi)
{
    const int nx = p->nx, ny = p->ny;
    for (int j = 0; j < ny; ++j) {
        if (is_wall(p, j)) continue;
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            double gx = gdx ? gdx[c] : 0.0, gy = gdy ? gdy[c] : 0.0, gl = glap ? glap[c] : 0.0;
            for (int a = 1; a < 9; ++a) {
                int ii = wrap(i + EX[a], nx), jj = p->periodic_y ? wrap(j + EY[a], ny) : j + EY[a];
                size_t cn = (size_t)jj * nx + ii;
                gphi[cn] += 3.0 * WEQ[a] * EX[a] * gx + 3.0 * WEQ[a] * EY[a] * gy + 6.0 * WEQ[a] * gl;
                gphi[c] -= 6.0 * WEQ[a] * gl;
            }
        }
    }
}

/* Adjoint of h = K(T) at fixed rho, v (Eq. (18)): given gh, add to gT,
 * grho and gv (the velocity seen by the temperature equation). */
static void thermal_rhs_T(const orc_state *s, const fwd_t *w, const double *T, const double *gh, double *gT,
                          double *grho, double *gvx, double *gvy)
{
    const orc_params *p = &s->p;
    const int nx = p->nx, ny = p->ny;
    const size_t n = w->n;
    const double chi = p->cv_chi / p->cv;
    double *Tx = w->ws[0], *Ty = w->ws[1], *rx = w->ws[3], *ry = w->ws[4], *ux = w->ws[5], *vy_ = w->ws[6];
    orc_grad_iso(nx, ny, p->periodic_y, T, Tx, Ty, NULL);
    orc_grad_iso(nx, ny, p->periodic_y, w->rho, rx, ry, NULL);
    orc_grad_iso(nx, ny, p->periodic_y, w->vTx, ux, NULL, NULL);
    orc_grad_iso(nx, ny, p->periodic_y, w->vTy, NULL, vy_, NULL);
    double *gTx = calloc(n, sizeof(double)), *gTy = calloc(n, sizeof(double)), *gL = calloc(n, sizeof(double));
    double *grx = calloc(n, sizeof(double)), *gry = calloc(n, sizeof(double)), *gdiv = calloc(n, sizeof(double));
    const double a = p->a, b = p->b, R = p->R, Tc = s->Tc, kap = s->kappa;
    for (int j = 0; j < ny; ++j) {
        if (is_wall(p, j)) continue;
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            const double g = gh[c];
            if (g == 0.0) continue;
            const double r = w->rho[c], Tv = T[c];
            const double divv = ux[c] + vy_[c];
            /* K = -(v.DT) + chi (lap T + Drho.DT / rho) - T P(rho, T) divv / (rho c_v) */
            gTx[c] += g * (-w->vTx[c] + chi * rx[c] / r);
            gTy[c] += g * (-w->vTy[c] + chi * ry[c] / r);
            gL[c] += g * chi;
            gvx[c] += -g * Tx[c];
            gvy[c] += -g * Ty[c];
            grx[c] += g * chi * Tx[c] / r;
            gry[c] += g * chi * Ty[c] / r;
            /* pressure work: P = dp/dT = rho R/D1 - a rho^2 phi'(T)/D2 */
            const double D1 = 1.0 - b * r, D2 = 1.0 + 2.0 * b * r - b * b * r * r;
            const double dphi = orc_dphi_dT(Tv, Tc, kap);
            const double u = sqrt(Tv / Tc);
            const double d2phi = kap * (1.0 + kap) / (2.0 * Tc * Tc * u * u * u);
            const double P = r * R / D1 - a * r * r * dphi / D2;
            const double dPdT = -a * r * r * d2phi / D2;
            gT[c] += g * (-divv / (r * p->cv)) * (P + Tv * dPdT);
            gdiv[c] += -g * Tv * P / (r * p->cv);
            /* rho at the node: the conduction weight 1/rho and P/rho */
            const double dPrho_drho = R * b / (D1 * D1) - a * dphi * (1.0 + b * b * r * r) / (D2 * D2);
            grho[c] += g * (-chi * (rx[c] * Tx[c] + ry[c] * Ty[c]) / (r * r) - Tv * divv / p->cv * dPrho_drho);
        }
    }
    stencil_T(p, gTx, gTy, gL, gT);
    stencil_T(p, grx, gry, NULL, grho);
    stencil_T(p, gdiv, NULL, NULL, gvx);
    stencil_T(p, NULL, gdiv, NULL, gvy);
    free(gTx); free(gTy); free(gL); free(grx); free(gry); free(gdiv);
}

/* One step transposed.  In: lf1, lT1 (adjoints of the state after the step).
 * Out: lf0, lT0 (adjoints of the state before it); *gGw accumulates dJ/dG_w.
 * f, T: the state before the step. */
static void step_vjp(const orc_state *s, const double *f, const double *T, const double *lf1, const double *lT1,
                     double *lf0, double *lT0, double *gGw, fwd_t *w)
{
    const orc_params *p = &s->p;
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    fwd_intermediates(s, f, T, w);
    double *grho = calloc(n, sizeof(double)), *gvx = calloc(n, sizeof(double)), *gvy = calloc(n, sizeof(double));
    double *gvTx = calloc(n, sizeof(double)), *gvTy = calloc(n, sizeof(double));
    double *gFx = calloc(n, sizeof(double)), *gFy = calloc(n, sizeof(double)), *gQ = calloc(n, sizeof(double));
    double *gpsi = calloc(n, sizeof(double)), *gfs = calloc(9 * n, sizeof(double));
    double *gh[4], *gTk = calloc(n, sizeof(double));
    for (int k = 0; k < 4; ++k) gh[k] = calloc(n, sizeof(double));

    /* ---- O12 transposed: T1 = T + (h1 + 2 h2 + 2 h3 + h4)/6 on interior rows */
    const double wst[4] = {1.0, 2.0, 2.0, 1.0};
    for (size_t c = 0; c < n; ++c) lT0[c] = lT1[c];
    for (int j = 0; j < ny; ++j) {
        if (is_wall(p, j)) continue;
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            for (int k = 0; k < 4; ++k) gh[k][c] = wst[k] * lT1[c] / 6.0;
        }
    }
    const double cst[4] = {0.0, 0.5, 0.5, 1.0};
    for (int k = 3; k >= 0; --k) {
        memset(gTk, 0, n * sizeof(double));
        thermal_rhs_T(s, w, w->Tk[k], gh[k], gTk, grho, gvTx, gvTy);
        /* T_k = T + c_k h_{k-1} on interior rows (T on wall rows) */
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                size_t c = (size_t)j * nx + i;
                lT0[c] += gTk[c];
                if (k > 0 && !is_wall(p, j)) gh[k - 1][c] += cst[k] * gTk[c];
            }
        }
    }
    /* the temperature equation sees v on interior rows, 0 on wall rows */
    for (int j = 0; j < ny; ++j) {
        if (is_wall(p, j)) continue;
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            gvx[c] += gvTx[c];
            gvy[c] += gvTy[c];
        }
    }

    /* ---- O11 (Zou-He) and O10 (streaming) transposed into the adjoint of f* */
    double *lt = malloc(9 * n * sizeof(double));
    memcpy(lt, lf1, 9 * n * sizeof(double));
    if (!p->periodic_y) {
        for (int i = 0; i < nx; ++i) {
            double *L0[9];
            size_t c = (size_t)i;
            for (int a = 0; a < 9; ++a) L0[a] = &lt[(size_t)a * n + c];
            /* bottom: f2 = f4, f5 = f7 - (f1 - f3)/2, f6 = f8 + (f1 - f3)/2 */
            *L0[4] += *L0[2];
            *L0[7] += *L0[5];
            *L0[8] += *L0[6];
            *L0[1] += -0.5 * *L0[5] + 0.5 * *L0[6];
            *L0[3] += 0.5 * *L0[5] - 0.5 * *L0[6];
            *L0[2] = *L0[5] = *L0[6] = 0.0;
            c = (size_t)(ny - 1) * nx + i;
            for (int a = 0; a < 9; ++a) L0[a] = &lt[(size_t)a * n + c];
            /* top: f4 = f2, f7 = f5 + (f1 - f3)/2, f8 = f6 - (f1 - f3)/2 */
            *L0[2] += *L0[4];
            *L0[5] += *L0[7];
            *L0[6] += *L0[8];
            *L0[1] += 0.5 * *L0[7] - 0.5 * *L0[8];
            *L0[3] += -0.5 * *L0[7] + 0.5 * *L0[8];
            *L0[4] = *L0[7] = *L0[8] = 0.0;
        }
    }
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            for (int a = 0; a < 9; ++a) {
                int it = wrap(i + EX[a], nx), jt = j + EY[a];
                if (p->periodic_y) jt = wrap(jt, ny);
                if (jt < 0 || jt > ny - 1) continue; /* left through a wall */
                gfs[(size_t)a * n + c] = lt[(size_t)a * n + (size_t)jt * nx + it];
            }
        }
    }
    free(lt);

    /* ---- O9 transposed (moment space), then O8 */
    const double tauL = 3.0 * p->nu_L + 0.5, tauV = 3.0 * p->nu_V + 0.5;
    const double slope = (tauL - tauV) / (p->rho_L - p->rho_V);
    const double sig_e = p->sigma / (1.0 / p->s_e - 0.5), sig_z = p->sigma / (1.0 / p->s_zeta - 0.5);
    for (size_t k = 0; k < 9 * n; ++k) lf0[k] = 0.0;
    for (size_t c = 0; c < n; ++c) {
        double fl[9], m[9], meq[9], S[9], gms[9], gm[9], gmeq[9], gS[9];
        for (int a = 0; a < 9; ++a) fl[a] = f[(size_t)a * n + c];
        const double r = w->rho[c], vx = w->vx[c], vy = w->vy[c], Fx = w->Fx[c], Fy = w->Fy[c], Q = w->Q[c];
        for (int k = 0; k < 9; ++k) {
            m[k] = 0.0;
            for (int a = 0; a < 9; ++a) m[k] += MM[k][a] * fl[a];
        }
        const double v2 = vx * vx + vy * vy;
        meq[0] = r;
        meq[1] = r * (-2.0 + 3.0 * v2);
        meq[2] = r * (1.0 - 3.0 * v2);
        meq[3] = r * vx;
        meq[4] = -r * vx;
        meq[5] = r * vy;
        meq[6] = -r * vy;
        meq[7] = r * (vx * vx - vy * vy);
        meq[8] = r * vx * vy;
        orc_forcing_moments(p, vx, vy, Fx, Fy, Q, S);
        const double tau = tauV + (r - p->rho_V) * slope, s_nu = 1.0 / tau;
        const double L[9] = {p->s_rho, p->s_e, p->s_zeta, p->s_j, p->s_q, p->s_j, p->s_q, s_nu, s_nu};
        /* f* = M^T diag(1/n) m*  =>  gm* = diag(1/n) M gf* */
        for (int k = 0; k < 9; ++k) {
            gms[k] = 0.0;
            for (int a = 0; a < 9; ++a) gms[k] += MM[k][a] * gfs[(size_t)a * n + c];
            gms[k] /= MNORM[k];
        }
        /* m* = m - L (m - meq) + (1 - L/2) S */
        for (int k = 0; k < 9; ++k) {
            gm[k] = (1.0 - L[k]) * gms[k];
            gmeq[k] = L[k] * gms[k];
            gS[k] = (1.0 - 0.5 * L[k]) * gms[k];
        }
        double gsnu = 0.0;
        for (int k = 7; k < 9; ++k) gsnu += gms[k] * (-(m[k] - meq[k]) - 0.5 * S[k]);
        /* m = M f */
        for (int a = 0; a < 9; ++a) {
            double acc = 0.0;
            for (int k = 0; k < 9; ++k) acc += MM[k][a] * gm[k];
            lf0[(size_t)a * n + c] += acc;
        }
        /* meq(rho, v) of Eq. (5) */
        double gr = 0.0;
        for (int k = 0; k < 9; ++k) gr += gmeq[k] * meq[k] / r;
        double gvx_ = r * (gmeq[1] * 6.0 * vx - gmeq[2] * 6.0 * vx + gmeq[3] - gmeq[4] + gmeq[7] * 2.0 * vx + gmeq[8] * vy);
        double gvy_ = r * (gmeq[1] * 6.0 * vy - gmeq[2] * 6.0 * vy + gmeq[5] - gmeq[6] - gmeq[7] * 2.0 * vy + gmeq[8] * vx);
        /* S(v, F, Q) of Eq. (8) */
        const double a6 = gS[1] - gS[2];
        double gFx_ = 6.0 * a6 * vx, gFy_ = 6.0 * a6 * vy;
        gvx_ += 6.0 * a6 * Fx;
        gvy_ += 6.0 * a6 * Fy;
        double gQ_ = sig_e * gS[1] - sig_z * gS[2];
        gFx_ += gS[3] - gS[4];
        gFy_ += gS[5] - gS[6];
        gvx_ += 2.0 * Fx * gS[7] + Fy * gS[8];
        gvy_ += -2.0 * Fy * gS[7] + Fx * gS[8];
        gFx_ += 2.0 * vx * gS[7] + vy * gS[8];
        gFy_ += -2.0 * vy * gS[7] + vx * gS[8];
        /* s_nu = 1/tau(rho) */
        gr += gsnu * (-slope / (tau * tau));
        /* O8: v = (j + F/2)/rho (v also collects what the temperature equation saw) */
        gvx_ += gvx[c];
        gvy_ += gvy[c];
        const double gjx = gvx_ / r, gjy = gvy_ / r;
        gFx_ += 0.5 * gvx_ / r;
        gFy_ += 0.5 * gvy_ / r;
        gr += -(gvx_ * vx + gvy_ * vy) / r;
        for (int a = 0; a < 9; ++a) lf0[(size_t)a * n + c] += EX[a] * gjx + EY[a] * gjy;
        grho[c] += gr;
        gFx[c] += gFx_;
        gFy[c] += gFy_;
        gQ[c] += gQ_;
    }

    /* ---- O4-O7 transposed */
    double grho_ave = 0.0;
    for (int j = 0; j < ny; ++j) {
        if (is_wall(p, j)) continue; /* no force on the wall rows */
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            const double ps = w->psi[c];
            /* buoyancy F_y += -(rho - rho_ave) g */
            grho[c] += -p->g * gFy[c];
            grho_ave += p->g * gFy[c];
            /* fluid-solid force on the rows next to the walls */
            if (!p->periodic_y && j == 1) {
                gpsi[c] += gFy[c] * p->Gw_bottom * ps / 3.0;
                *gGw += gFy[c] * ps * ps / 6.0;
            }
            if (!p->periodic_y && j == ny - 2) gpsi[c] += -gFy[c] * p->Gw_top * ps / 3.0;
            /* F_m = -G psi s, Q = G^2 |s|^2 */
            gpsi[c] += -p->G * (w->sx[c] * gFx[c] + w->sy[c] * gFy[c]);
            const double gsx = -p->G * ps * gFx[c] + 2.0 * p->G * p->G * w->sx[c] * gQ[c];
            const double gsy = -p->G * ps * gFy[c] + 2.0 * p->G * p->G * w->sy[c] * gQ[c];
            for (int a = 1; a < 9; ++a) {
                int ii = wrap(i + EX[a], nx), jj = p->periodic_y ? wrap(j + EY[a], ny) : j + EY[a];
                gpsi[(size_t)jj * nx + ii] += WPSI[a] * (EX[a] * gsx + EY[a] * gsy);
            }
        }
    }
    for (size_t c = 0; c < n; ++c) grho[c] += grho_ave / (double)n;

    /* ---- O3 transposed: psi = sqrt(2 (p(rho, T) - rho/3)/G) */
    for (size_t c = 0; c < n; ++c) {
        if (gpsi[c] == 0.0) continue;
        const double gr_ = gpsi[c] / (2.0 * w->psi[c]) * 2.0 / p->G;
        grho[c] += gr_ * (orc_dp_drho(w->rho[c], T[c], p->a, p->b, p->R, s->Tc, s->kappa) - 1.0 / 3.0);
        lT0[c] += gr_ * orc_dp_dT(w->rho[c], T[c], p->a, p->b, p->R, s->Tc, s->kappa);
    }

    /* ---- O1 transposed: rho = sum_a f_a */
    for (size_t c = 0; c < n; ++c)
        for (int a = 0; a < 9; ++a) lf0[(size_t)a * n + c] += grho[c];

    free(grho); free(gvx); free(gvy); free(gvTx); free(gvTy); free(gFx); free(gFy); free(gQ); free(gpsi);
    free(gfs); free(gTk);
    for (int k = 0; k < 4; ++k) free(gh[k]);
}

/* O13 transposed: dq/df and dq/dT of the sampled state, scaled by wgt. */
static void heat_flux_T(const orc_params *p, const double *f, const double *T, double wgt, double *lf, double *lT)
{
    const int nx = p->nx;
    const size_t n = (size_t)nx * p->ny;
    for (int i = 0; i < nx; ++i) {
        double r0 = 0.0;
        for (int a = 0; a < 9; ++a) r0 += f[(size_t)a * n + i];
        const double d = (-3.0 * T[i] + 4.0 * T[(size_t)nx + i] - T[(size_t)2 * nx + i]) / 2.0;
        const double k = -p->cv_chi / nx * wgt;
        for (int a = 0; a < 9; ++a) lf[(size_t)a * n + i] += k * d;
        lT[i] += k * r0 * (-3.0 / 2.0);
        lT[(size_t)nx + i] += k * r0 * (4.0 / 2.0);
        lT[(size_t)2 * nx + i] += k * r0 * (-1.0 / 2.0);
    }
}

/* Public: one step transposed at the current state of s (for dot-product
 * tests).  lf1 [9n], lT1 [n] in; lf0 [9n], lT0 [n] out; *gGw accumulates. */
int orc_step_vjp(const orc_state *s, const double *lf1, const double *lT1, double *lf0, double *lT0, double *gGw)
{
    if (s->p.thermal_mode != ORC_COUPLED || s->p.ghost_layer) return ORC_EINVAL;
    fwd_t w;
    if (!fwd_alloc(&w, s->p.nx, s->p.ny)) return ORC_ENOMEM;
    step_vjp(s, s->f, s->T, lf1, lT1, lf0, lT0, gGw, &w);
    fwd_free(&w);
    return ORC_OK;
}

/* Public: J = (1/N) sum_{n=1..N} q^n over N steps from the current state and
 * its gradient with respect to T_b (all nx bottom cells) and G_w (bottom).
 * K: checkpoint interval (K <= 0: K = N).  The state of s is left unchanged
 * (the forward runs on a copy). */
int orc_adjoint(const orc_state *s, int64_t N, int64_t K, double *J, double *dJ_dTb, double *dJ_dGw)
{
    const orc_params *p = &s->p;
    if (p->thermal_mode != ORC_COUPLED || p->periodic_y || p->ghost_layer || N < 1) return ORC_EINVAL;
    if (K <= 0 || K > N) K = N;
    const int nx = p->nx;
    const size_t n = (size_t)nx * p->ny;
    const int64_t nck = (N + K - 1) / K;
    orc_state *run = NULL;
    {
        /* a private copy of the state to run the forward on */
        double *rho0 = malloc(n * sizeof(double));
        for (size_t c = 0; c < n; ++c) rho0[c] = 1.0;
        int rc = orc_create(p, rho0, NULL, NULL, NULL, s->Tb, &run);
        free(rho0);
        if (rc != ORC_OK) return rc;
        double *buf = malloc((size_t)orc_state_size(s) * sizeof(double));
        orc_save(s, buf);
        orc_load(run, buf);
        free(buf);
    }
    double *ck = malloc((size_t)nck * 10 * n * sizeof(double));   /* checkpoints (f, T) */
    double *seg = malloc((size_t)K * 10 * n * sizeof(double));    /* states of one segment */
    double *lf = calloc(9 * n, sizeof(double)), *lT = calloc(n, sizeof(double));
    double *lf0 = calloc(9 * n, sizeof(double)), *lT0 = calloc(n, sizeof(double));
    fwd_t w;
    if (!ck || !seg || !lf || !lT || !lf0 || !lT0 || !fwd_alloc(&w, nx, p->ny)) {
        orc_destroy(run);
        free(ck); free(seg); free(lf); free(lT); free(lf0); free(lT0);
        return ORC_ENOMEM;
    }
    /* forward: J and the checkpoints */
    double qsum = 0.0;
    for (int64_t t = 0; t < N; ++t) {
        if (t % K == 0) {
            memcpy(ck + (size_t)(t / K) * 10 * n, run->f, 9 * n * sizeof(double));
            memcpy(ck + (size_t)(t / K) * 10 * n + 9 * n, run->T, n * sizeof(double));
        }
        int rc = orc_step(run, 1);
        if (rc != ORC_OK) {
            orc_destroy(run);
            fwd_free(&w);
            free(ck); free(seg); free(lf); free(lT); free(lf0); free(lT0);
            return rc;
        }
        qsum += run->q_now;
    }
    *J = qsum / (double)N;
    /* the final state's heat-flux source */
    heat_flux_T(p, run->f, run->T, 1.0 / (double)N, lf, lT);
    double gGw = 0.0;
    for (int64_t sgi = nck - 1; sgi >= 0; --sgi) {
        const int64_t t0 = sgi * K, t1 = (t0 + K < N) ? t0 + K : N;
        /* recompute the segment's states t0 .. t1-1 */
        memcpy(run->f, ck + (size_t)sgi * 10 * n, 9 * n * sizeof(double));
        memcpy(run->T, ck + (size_t)sgi * 10 * n + 9 * n, n * sizeof(double));
        for (int64_t t = t0; t < t1; ++t) {
            memcpy(seg + (size_t)(t - t0) * 10 * n, run->f, 9 * n * sizeof(double));
            memcpy(seg + (size_t)(t - t0) * 10 * n + 9 * n, run->T, n * sizeof(double));
            if (t + 1 < t1) orc_step(run, 1);
        }
        for (int64_t t = t1 - 1; t >= t0; --t) {
            const double *fs = seg + (size_t)(t - t0) * 10 * n, *Ts = fs + 9 * n;
            step_vjp(run, fs, Ts, lf, lT, lf0, lT0, &gGw, &w);
            memcpy(lf, lf0, 9 * n * sizeof(double));
            memcpy(lT, lT0, n * sizeof(double));
            /* the heat-flux sample of state t (t >= 1) */
            if (t >= 1) heat_flux_T(p, fs, Ts, 1.0 / (double)N, lf, lT);
        }
    }
    /* T_b is the bottom row of the initial temperature */
    for (int i = 0; i < nx; ++i) dJ_dTb[i] = lT[i];
    *dJ_dGw = gGw;
    orc_destroy(run);
    fwd_free(&w);
    free(ck); free(seg); free(lf); free(lT); free(lf0); free(lT0);
    return ORC_OK;
}
