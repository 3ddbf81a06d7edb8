/*
 * Three-dimensional extension of the FP64 CPU oracle: the hybrid thermal
 * pseudopotential LB boiling model of Li, Kang, Francois, He and Luo
 * (arXiv:1501.03857) on the D3Q19 lattice, the extension the paper names as
 * its future work (Sec. 4).
 *
 * TEST INFRASTRUCTURE ONLY, like lbb_oracle.c: the GPU library's 3-D path is
 * checked against it; the product never loads it and shares nothing with it.
 *
 * The time step is the paper's (Sec. 2) with every two-dimensional piece
 * carried to three dimensions; the readings are:
 *  - D3Q19 velocities ordered rest, +x, -x, +y, -y, +z, -z, then the twelve
 *    edges (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1),
 *    (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1); lattice
 *    weights 1/3, 1/18, 1/36; c_s^2 = 1/3.
 *  - MRT in the standard orthogonal D3Q19 moment basis (rho, e, epsilon,
 *    j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww, p_xy, p_yz,
 *    p_xz, m_x, m_y, m_z), each row a polynomial in e_a (below).  Equilibrium
 *    moments m_eq = M f_eq and the forcing moments M F' of the Guo term,
 *    computed from their velocity-space definitions.  Rates
 *    diag(s_rho, s_e, s_zeta, s_j, s_q, s_j, s_q, s_j, s_q, s_nu, s_zeta,
 *    s_nu, s_zeta, s_nu, s_nu, s_nu, s_q, s_q, s_q): the fourth-order pi
 *    moments relax with the rate of the fourth-order epsilon, the
 *    third-order m moments with that of q.
 *  - Interaction force Eq. (7) with w_a = 3 W_a (1/6 on the axes, 1/12 on
 *    the edges): sum_a w_a e_a e_a = I, so the bulk pressure is again
 *    rho/3 + G psi^2/2 = p_EOS, and the fourth-order moments of w are
 *    isotropic with the same constant 1/3 as in two dimensions.
 *  - The sigma part of the improved forcing (Eq. (8)) adds the same
 *    isotropic increment s sigma Q / 6 to every diagonal component of the
 *    post-collision second moment as the two-dimensional term does:
 *    S_e += (19/2) sigma Q/(tau_e - 1/2), S_epsilon -= (19/5) sigma Q/
 *    (tau_epsilon - 1/2).  With equal rates this is an equal increment of
 *    every moving population, mass- and momentum-free.
 *  - Walls at y = 0 and y = ny-1 (gravity along -y), periodic x and z.  Wet
 *    Zou-He nodes with zero velocity, the transverse momentum carried by the
 *    populations parallel to the wall redistributed onto the unknowns, so
 *    the wall nodes carry no momentum.  No force on the wall rows; the
 *    fluid-solid force (Eq. (22), omega_a = w_a/3) on the rows next to them
 *    gives (0, +G_w psi^2/6, 0) at the bottom, as in two dimensions.
 *  - Temperature: Eq. (18) with the isotropic D3Q19 stencils
 *    d_i phi = 3 sum_a W_a e_ai phi(x + e_a),
 *    lap phi = 6 sum_a W_a (phi(x + e_a) - phi(x)), RK4 as in two
 *    dimensions; heat flux q_w(x, z) at the bottom wall, q = its mean.
 */
#include "lbb_oracle.h"
#include "lbb_oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#define ORC3_PARALLEL _Pragma("omp parallel for schedule(static)")
#else
#define ORC3_PARALLEL
#endif

static const int E3[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double W3(int a) { return a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

/* row k of the moment basis evaluated at velocity e_a */
static double basis(int k, int a)
{
    const double x = E3[a][0], y = E3[a][1], z = E3[a][2];
    const double e2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * e2 - 30.0;
    case 2: return (21.0 * e2 * e2 - 53.0 * e2 + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * e2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * e2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * e2 - 9.0) * z;
    case 9: return 3.0 * x * x - e2;
    case 10: return (3.0 * e2 - 5.0) * (3.0 * x * x - e2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * e2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
    }
}

static double M3[19][19], M3NORM[19];
static int m3_ready;

static void m3_init(void)
{
    if (m3_ready) return;
#ifdef _OPENMP
#pragma omp critical(orc3_basis)
#endif
    {
        if (!m3_ready) {
            for (int k = 0; k < 19; ++k) {
                double n = 0.0;
                for (int a = 0; a < 19; ++a) {
                    M3[k][a] = basis(k, a);
                    n += M3[k][a] * M3[k][a];
                }
                M3NORM[k] = n;
            }
            m3_ready = 1;
        }
    }
}

void orc3_lattice(int32_t e[57], double W[19], double M[361])
{
    m3_init();
    for (int a = 0; a < 19; ++a) {
        for (int d = 0; d < 3; ++d) e[3 * a + d] = E3[a][d];
        W[a] = W3(a);
    }
    for (int k = 0; k < 19; ++k)
        for (int a = 0; a < 19; ++a) M[19 * k + a] = M3[k][a];
}

/* second-order equilibrium, f_eq = W rho [1 + 3 e.v + 9/2 (e.v)^2 - 3/2 v^2] */
void orc3_feq(double rho, const double v[3], double feq[19])
{
    const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    for (int a = 0; a < 19; ++a) {
        const double ev = E3[a][0] * v[0] + E3[a][1] * v[1] + E3[a][2] * v[2];
        feq[a] = W3(a) * rho * (1.0 + 3.0 * ev + 4.5 * ev * ev - 1.5 * v2);
    }
}

static double tau3_nu(const orc_params *p, double rho)
{
    const double tL = 3.0 * p->nu_L + 0.5, tV = 3.0 * p->nu_V + 0.5;
    return tV + (rho - p->rho_V) * (tL - tV) / (p->rho_L - p->rho_V);
}

/* MRT collision at one node: m = M f; m_eq = M f_eq(rho, v);
 * S = M F' with F'_a = W_a [3 (e_a - v).F + 9 (e_a.v)(e_a.F)] plus the sigma
 * part of the improved forcing on e and epsilon;
 * m* = m - L (m - m_eq) + (I - L/2) S; f* = M^{-1} m*. */
void orc3_collide_site(const orc_params *p, const double f[19], double rho, const double v[3],
                       const double F[3], double Q, double fpost[19])
{
    m3_init();
    double feq[19], Fp[19], m[19], meq[19], S[19], ms[19];
    orc3_feq(rho, v, feq);
    for (int a = 0; a < 19; ++a) {
        const double eF = E3[a][0] * F[0] + E3[a][1] * F[1] + E3[a][2] * F[2];
        const double ev = E3[a][0] * v[0] + E3[a][1] * v[1] + E3[a][2] * v[2];
        const double vF = v[0] * F[0] + v[1] * F[1] + v[2] * F[2];
        Fp[a] = W3(a) * (3.0 * (eF - vF) + 9.0 * ev * eF);
    }
    for (int k = 0; k < 19; ++k) {
        m[k] = meq[k] = S[k] = 0.0;
        for (int a = 0; a < 19; ++a) {
            m[k] += M3[k][a] * f[a];
            meq[k] += M3[k][a] * feq[a];
            S[k] += M3[k][a] * Fp[a];
        }
    }
    const double tau_e = 1.0 / p->s_e, tau_eps = 1.0 / p->s_zeta;
    S[1] += 9.5 * p->sigma * Q / (tau_e - 0.5);
    S[2] -= 3.8 * p->sigma * Q / (tau_eps - 0.5);
    const double sn = 1.0 / tau3_nu(p, rho);
    const double L[19] = {p->s_rho, p->s_e, p->s_zeta, p->s_j, p->s_q, p->s_j, p->s_q, p->s_j, p->s_q, sn,
                          p->s_zeta, sn, p->s_zeta, sn, sn, sn, p->s_q, p->s_q, p->s_q};
    for (int k = 0; k < 19; ++k) ms[k] = m[k] - L[k] * (m[k] - meq[k]) + (1.0 - 0.5 * L[k]) * S[k];
    for (int a = 0; a < 19; ++a) {
        fpost[a] = 0.0;
        for (int k = 0; k < 19; ++k) fpost[a] += M3[k][a] * ms[k] / M3NORM[k];
    }
}

/* ---------------------------------------------------------------------- */

struct orc3_state {
    orc_params p;
    int nz;
    double Tc, kappa, Ts;
    int64_t t;
    double *f, *fpost; /* [19][nz][ny][nx] */
    double *T;         /* [nz][ny][nx] */
    double *Tb;        /* [nz][nx] bottom-wall temperature */
    double *rho, *psi, *F[3], *Q, *v[3], *vT[3];
    double *Tst, *h, *acc, *ws[11];
    double q_now, q_sum;
    int64_t n_samples;
    int store_bits;
};

static inline int wrap3(int i, int n) { return (i % n + n) % n; }

static size_t idx3(const orc3_state *s, int x, int y, int z)
{
    return ((size_t)z * s->p.ny + (size_t)y) * s->p.nx + (size_t)x;
}

/* neighbour of (x, y, z) along e_a: periodic in x and z (and y when
 * periodic_y); -1 beyond a wall */
static long nbr3(const orc3_state *s, int x, int y, int z, int a, int sign)
{
    const int xx = wrap3(x + sign * E3[a][0], s->p.nx), zz = wrap3(z + sign * E3[a][2], s->nz);
    int yy = y + sign * E3[a][1];
    if (s->p.periodic_y) yy = wrap3(yy, s->p.ny);
    else if (yy < 0 || yy >= s->p.ny) return -1;
    return (long)idx3(s, xx, yy, zz);
}

static int wall3(const orc3_state *s, int y) { return !s->p.periodic_y && (y == 0 || y == s->p.ny - 1); }

/* isotropic stencils on the D3Q19 neighbourhood where every neighbour exists
 * (interior rows, or all rows when periodic_y); 0 elsewhere */
static void grad3(const orc3_state *s, const double *phi, double *dx, double *dy, double *dz, double *lap)
{
    const int nx = s->p.nx, ny = s->p.ny, nz = s->nz;
    ORC3_PARALLEL
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t c = idx3(s, x, y, z);
                double g[3] = {0.0, 0.0, 0.0}, l = 0.0;
                if (!wall3(s, y)) {
                    for (int a = 1; a < 19; ++a) {
                        const double w = W3(a), val = phi[nbr3(s, x, y, z, a, 1)];
                        for (int d = 0; d < 3; ++d) g[d] += w * E3[a][d] * val;
                        l += w * (val - phi[c]);
                    }
                }
                if (dx) dx[c] = 3.0 * g[0];
                if (dy) dy[c] = 3.0 * g[1];
                if (dz) dz[c] = 3.0 * g[2];
                if (lap) lap[c] = 6.0 * l;
            }
}

void orc3_grad_iso(int32_t nx, int32_t ny, int32_t nz, int32_t periodic_y, const double *phi, double *dx,
                   double *dy, double *dz, double *lap)
{
    orc3_state s;
    memset(&s, 0, sizeof s);
    s.p.nx = nx;
    s.p.ny = ny;
    s.p.periodic_y = periodic_y;
    s.nz = nz;
    grad3(&s, phi, dx, dy, dz, lap);
}

void orc3_destroy(orc3_state *s)
{
    if (!s) return;
    free(s->f); free(s->fpost); free(s->T); free(s->Tb); free(s->rho); free(s->psi); free(s->Q);
    for (int d = 0; d < 3; ++d) { free(s->F[d]); free(s->v[d]); free(s->vT[d]); }
    free(s->Tst); free(s->h); free(s->acc);
    for (int k = 0; k < 11; ++k) free(s->ws[k]);
    free(s);
}

static void heat_flux3(orc3_state *s, double *q_local);

int orc3_create(const orc_params *p, int32_t nz, const double *rho0, const double *ux0, const double *uy0,
                const double *uz0, const double *T0, const double *T_bottom, orc3_state **out)
{
    *out = NULL;
    if (!p || !rho0 || nz < 3 || p->nx < 3 || (p->periodic_y ? p->ny < 3 : p->ny < 4) || p->ghost_layer ||
        !(p->G < 0) || !(p->rho_L != p->rho_V) || p->thermal_mode < ORC_COUPLED ||
        p->thermal_mode > ORC_THERMAL_ONLY)
        return ORC_EINVAL;
    m3_init();
    const size_t n = (size_t)p->nx * p->ny * nz;
    orc3_state *s = calloc(1, sizeof *s);
    if (!s) return ORC_ENOMEM;
    s->p = *p;
    s->nz = nz;
    s->Tc = orc_Tc(p->a, p->b, p->R);
    s->kappa = orc_kappa(p->omega);
    s->Ts = p->Ts_over_Tc * s->Tc;
    int ok = 1;
#define ALLOC3(ptr, cnt) ok = ok && ((ptr) = malloc((cnt) * sizeof(double))) != NULL
    ALLOC3(s->f, 19 * n);
    ALLOC3(s->fpost, 19 * n);
    ALLOC3(s->T, n);
    ALLOC3(s->Tb, (size_t)p->nx * nz);
    ALLOC3(s->rho, n);
    ALLOC3(s->psi, n);
    ALLOC3(s->Q, n);
    for (int d = 0; d < 3; ++d) {
        ALLOC3(s->F[d], n);
        ALLOC3(s->v[d], n);
        ALLOC3(s->vT[d], n);
    }
    ALLOC3(s->Tst, n);
    ALLOC3(s->h, n);
    ALLOC3(s->acc, n);
    for (int k = 0; k < 11; ++k) ALLOC3(s->ws[k], n);
#undef ALLOC3
    if (!ok) {
        orc3_destroy(s);
        return ORC_ENOMEM;
    }
    for (size_t c = 0; c < (size_t)p->nx * nz; ++c) s->Tb[c] = T_bottom ? T_bottom[c] : s->Ts;
    for (size_t c = 0; c < n; ++c) {
        if (!(rho0[c] > 0) || !isfinite(rho0[c]) || p->b * rho0[c] >= 1.0) {
            orc3_destroy(s);
            return ORC_EINVAL;
        }
        const double v[3] = {ux0 ? ux0[c] : 0.0, uy0 ? uy0[c] : 0.0, uz0 ? uz0[c] : 0.0};
        double feq[19];
        orc3_feq(rho0[c], v, feq);
        for (int a = 0; a < 19; ++a) s->f[(size_t)a * n + c] = feq[a];
        s->T[c] = T0 ? T0[c] : s->Ts;
    }
    if (!p->periodic_y)
        for (int z = 0; z < nz; ++z)
            for (int x = 0; x < p->nx; ++x) {
                s->T[idx3(s, x, 0, z)] = s->Tb[(size_t)z * p->nx + x];
                s->T[idx3(s, x, p->ny - 1, z)] = s->Ts;
            }
    for (size_t c = 0; c < n; ++c)
        if (!(s->T[c] > 0) || !isfinite(s->T[c])) {
            orc3_destroy(s);
            return ORC_EINVAL;
        }
    heat_flux3(s, NULL);
    *out = s;
    return ORC_OK;
}

int64_t orc3_time(const orc3_state *s) { return s->t; }

int orc3_set_storage_rounding(orc3_state *s, int bits)
{
    if (bits < 0 || bits > 52) return ORC_EINVAL;
    s->store_bits = bits;
    return ORC_OK;
}

static double round3(int bits, double x)
{
    if (bits == 0) return x;
    if (bits == 24) return (double)(float)x;
    const double c = ldexp(1.0, 53 - bits) + 1.0;
    const double y = c * x;
    return y - (y - x);
}

/* K(T) of Eq. (18) on the interior rows with rho and v_T frozen */
static void thermal_rhs3(orc3_state *s, const double *T, double *K)
{
    const orc_params *p = &s->p;
    const size_t n = (size_t)p->nx * p->ny * s->nz;
    const double chi = p->cv_chi / p->cv;
    double **w = s->ws;
    grad3(s, T, w[0], w[1], w[2], w[3]);
    grad3(s, s->rho, w[4], w[5], w[6], NULL);
    grad3(s, s->vT[0], w[7], NULL, NULL, NULL);
    grad3(s, s->vT[1], NULL, w[8], NULL, NULL);
    grad3(s, s->vT[2], NULL, NULL, w[9], NULL);
    ORC3_PARALLEL
    for (size_t c = 0; c < n; ++c) {
        const int y = (int)((c / (size_t)p->nx) % (size_t)p->ny);
        if (wall3(s, y)) {
            K[c] = 0.0;
            continue;
        }
        const double adv = s->vT[0][c] * w[0][c] + s->vT[1][c] * w[1][c] + s->vT[2][c] * w[2][c];
        const double cond = chi * (w[3][c] + (w[4][c] * w[0][c] + w[5][c] * w[1][c] + w[6][c] * w[2][c]) / s->rho[c]);
        const double divv = w[7][c] + w[8][c] + w[9][c];
        const double dpdT = orc_dp_dT(s->rho[c], T[c], p->a, p->b, p->R, s->Tc, s->kappa);
        K[c] = -adv + cond - T[c] / (s->rho[c] * p->cv) * dpdT * divv;
    }
}

static int one_step3(orc3_state *s)
{
    const orc_params *p = &s->p;
    const int nx = p->nx, ny = p->ny, nz = s->nz;
    const size_t n = (size_t)nx * ny * nz;
    int bad = 0;
    /* O1 density */
    for (size_t c = 0; c < n; ++c) {
        double r = 0.0;
        for (int a = 0; a < 19; ++a) r += s->f[(size_t)a * n + c];
        s->rho[c] = r;
        if (!(r > 0) || !isfinite(r)) bad = 1;
    }
    if (bad) return ORC_ENONFINITE;
    if (p->thermal_mode == ORC_THERMAL_ONLY) {
        for (size_t c = 0; c < n; ++c) {
            const int y = (int)((c / (size_t)nx) % (size_t)ny);
            for (int d = 0; d < 3; ++d) {
                double j = 0.0;
                for (int a = 0; a < 19; ++a) j += E3[a][d] * s->f[(size_t)a * n + c];
                s->vT[d][c] = wall3(s, y) ? 0.0 : j / s->rho[c];
            }
        }
    } else {
        /* O2 domain-mean density */
        double mass = 0.0;
        for (size_t c = 0; c < n; ++c) mass += s->rho[c];
        const double rho_ave = mass / (double)n;
        /* O3 pseudopotential */
        for (size_t c = 0; c < n; ++c) {
            const double pe = orc_p_eos(s->rho[c], s->T[c], p->a, p->b, p->R, s->Tc, s->kappa);
            const double r = 2.0 * (pe - s->rho[c] / 3.0) / p->G;
            if (!(r >= 0) || !isfinite(r)) bad = 1;
            s->psi[c] = round3(s->store_bits == 24 ? 0 : s->store_bits, sqrt(r));
        }
        if (bad) return ORC_ENONFINITE;
        /* O4-O8 forces and velocity */
        ORC3_PARALLEL
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t c = idx3(s, x, y, z);
                    double F[3] = {0.0, 0.0, 0.0}, Q = 0.0;
                    if (!wall3(s, y)) {
                        double sm[3] = {0.0, 0.0, 0.0};
                        for (int a = 1; a < 19; ++a) {
                            const double val = s->psi[nbr3(s, x, y, z, a, 1)];
                            for (int d = 0; d < 3; ++d) sm[d] += 3.0 * W3(a) * val * E3[a][d];
                        }
                        for (int d = 0; d < 3; ++d) F[d] = -p->G * s->psi[c] * sm[d];
                        Q = p->G * p->G * (sm[0] * sm[0] + sm[1] * sm[1] + sm[2] * sm[2]);
                        /* O5 fluid-solid force: the wall rows are the solid */
                        if (!p->periodic_y) {
                            double fs[3] = {0.0, 0.0, 0.0};
                            for (int a = 1; a < 19; ++a) {
                                const int yy = y + E3[a][1];
                                double Gws = 0.0;
                                if (yy == 0) Gws = p->Gw_bottom;
                                if (yy == ny - 1) Gws = p->Gw_top;
                                for (int d = 0; d < 3; ++d) fs[d] += W3(a) * Gws * s->psi[c] * E3[a][d];
                            }
                            for (int d = 0; d < 3; ++d) F[d] -= s->psi[c] * fs[d];
                        }
                        /* O6 buoyancy */
                        F[1] -= (s->rho[c] - rho_ave) * p->g;
                    }
                    for (int d = 0; d < 3; ++d) {
                        double j = 0.0;
                        for (int a = 0; a < 19; ++a) j += E3[a][d] * s->f[(size_t)a * n + c];
                        s->F[d][c] = F[d];
                        s->v[d][c] = (j + 0.5 * F[d]) / s->rho[c];
                        s->vT[d][c] = wall3(s, y) ? 0.0 : s->v[d][c];
                    }
                    s->Q[c] = Q;
                }
        /* O9 collision */
        ORC3_PARALLEL
        for (size_t c = 0; c < n; ++c) {
            double fl[19], fp[19];
            const double v[3] = {s->v[0][c], s->v[1][c], s->v[2][c]};
            const double F[3] = {s->F[0][c], s->F[1][c], s->F[2][c]};
            for (int a = 0; a < 19; ++a) fl[a] = s->f[(size_t)a * n + c];
            orc3_collide_site(p, fl, s->rho[c], v, F, s->Q[c], fp);
            for (int a = 0; a < 19; ++a) s->fpost[(size_t)a * n + c] = round3(s->store_bits, fp[a]);
        }
    }
    /* O12 temperature: RK4 with rho and v_T frozen, Dirichlet rows fixed */
    if (p->thermal_mode != ORC_ISOTHERMAL) {
        const double cst[4] = {0.0, 0.5, 0.5, 1.0}, wst[4] = {1.0, 2.0, 2.0, 1.0};
        for (size_t c = 0; c < n; ++c) s->acc[c] = 0.0;
        for (int k = 0; k < 4; ++k) {
            for (size_t c = 0; c < n; ++c) s->Tst[c] = s->T[c] + cst[k] * (k ? s->h[c] : 0.0);
            thermal_rhs3(s, s->Tst, s->h);
            for (size_t c = 0; c < n; ++c) s->acc[c] += wst[k] * s->h[c];
        }
        for (size_t c = 0; c < n; ++c) {
            const int y = (int)((c / (size_t)nx) % (size_t)ny);
            if (wall3(s, y)) continue;
            s->T[c] = s->T[c] + s->acc[c] / 6.0;
            if (s->store_bits != 24) s->T[c] = round3(s->store_bits, s->T[c]);
            if (!(s->T[c] > 0) || !isfinite(s->T[c])) bad = 1;
        }
        if (bad) return ORC_ENONFINITE;
    }
    /* O10 streaming and O11 Zou-He walls */
    if (p->thermal_mode != ORC_THERMAL_ONLY) {
        ORC3_PARALLEL
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t c = idx3(s, x, y, z);
                    for (int a = 0; a < 19; ++a) {
                        const long src = nbr3(s, x, y, z, a, -1);
                        if (src >= 0) s->f[(size_t)a * n + c] = s->fpost[(size_t)a * n + (size_t)src];
                    }
                }
        if (!p->periodic_y) {
            for (int z = 0; z < nz; ++z)
                for (int x = 0; x < nx; ++x) {
                    for (int side = 0; side < 2; ++side) {
                        const size_t c = idx3(s, x, side ? ny - 1 : 0, z);
                        double *f = s->f;
#define FA(a) f[(size_t)(a) * n + c]
                        /* transverse momentum of the populations parallel to the wall */
                        const double Nx = 0.5 * (FA(1) - FA(2) + FA(11) - FA(12) + FA(13) - FA(14));
                        const double Nz = 0.5 * (FA(5) - FA(6) + FA(11) - FA(12) - FA(13) + FA(14));
                        if (!side) { /* bottom: unknowns have e_y = +1 */
                            FA(3) = FA(4);
                            FA(7) = FA(8) - Nx;
                            FA(10) = FA(9) + Nx;
                            FA(15) = FA(16) - Nz;
                            FA(17) = FA(18) + Nz;
                        } else { /* top: unknowns have e_y = -1 */
                            FA(4) = FA(3);
                            FA(8) = FA(7) + Nx;
                            FA(9) = FA(10) - Nx;
                            FA(16) = FA(15) + Nz;
                            FA(18) = FA(17) - Nz;
                        }
#undef FA
                    }
                }
        }
    }
    s->t += 1;
    /* O13 heat flux of the new state */
    heat_flux3(s, NULL);
    s->q_sum += s->q_now;
    s->n_samples += 1;
    return ORC_OK;
}

int orc3_step(orc3_state *s, int64_t n)
{
    if (n < 0) return ORC_EINVAL;
    for (int64_t k = 0; k < n; ++k) {
        const int rc = one_step3(s);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}

/* q_w(x, z) = -c_v chi rho(x,0,z) (-3 T_0 + 4 T_1 - T_2)/2; q = mean */
static void heat_flux3(orc3_state *s, double *q_local)
{
    const orc_params *p = &s->p;
    const size_t n = (size_t)p->nx * p->ny * s->nz;
    if (p->periodic_y) {
        s->q_now = 0.0;
        return;
    }
    double sum = 0.0;
    for (int z = 0; z < s->nz; ++z)
        for (int x = 0; x < p->nx; ++x) {
            const size_t c0 = idx3(s, x, 0, z);
            double r = 0.0;
            for (int a = 0; a < 19; ++a) r += s->f[(size_t)a * n + c0];
            const double qw = -p->cv_chi * r *
                              (-3.0 * s->T[c0] + 4.0 * s->T[idx3(s, x, 1, z)] - s->T[idx3(s, x, 2, z)]) / 2.0;
            if (q_local) q_local[(size_t)z * p->nx + x] = qw;
            sum += qw;
        }
    s->q_now = sum / ((double)p->nx * s->nz);
}

void orc3_heat_flux(const orc3_state *cs, double *q_now, double *q_sum, int64_t *n_samples, double *q_local)
{
    orc3_state *s = (orc3_state *)cs;
    double keep = s->q_now;
    heat_flux3(s, q_local);
    s->q_now = keep;
    if (q_now) *q_now = s->q_now;
    if (q_sum) *q_sum = s->q_sum;
    if (n_samples) *n_samples = s->n_samples;
}

void orc3_reset_average(orc3_state *s)
{
    s->q_sum = 0.0;
    s->n_samples = 0;
}

/* rho = sum f; v from Eq. (6) with the force of the current state; T; f */
void orc3_fields(const orc3_state *cs, double *rho, double *ux, double *uy, double *uz, double *T, double *f)
{
    orc3_state *s = (orc3_state *)cs;
    const orc_params *p = &s->p;
    const size_t n = (size_t)p->nx * p->ny * s->nz;
    double *out_v[3] = {ux, uy, uz};
    /* forces of the current state, as the next step would form them */
    double mass = 0.0;
    for (size_t c = 0; c < n; ++c) {
        double r = 0.0;
        for (int a = 0; a < 19; ++a) r += s->f[(size_t)a * n + c];
        s->rho[c] = r;
        mass += r;
    }
    const double rho_ave = mass / (double)n;
    const int forces = p->thermal_mode != ORC_THERMAL_ONLY;
    if (forces)
        for (size_t c = 0; c < n; ++c) {
            const double pe = orc_p_eos(s->rho[c], s->T[c], p->a, p->b, p->R, s->Tc, s->kappa);
            const double r = 2.0 * (pe - s->rho[c] / 3.0) / p->G;
            s->psi[c] = sqrt(r);
        }
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const size_t c = idx3(s, x, y, z);
                double F[3] = {0.0, 0.0, 0.0};
                if (forces && !wall3(s, y)) {
                    double sm[3] = {0.0, 0.0, 0.0};
                    for (int a = 1; a < 19; ++a) {
                        const double val = s->psi[nbr3(s, x, y, z, a, 1)];
                        for (int d = 0; d < 3; ++d) sm[d] += 3.0 * W3(a) * val * E3[a][d];
                    }
                    for (int d = 0; d < 3; ++d) F[d] = -p->G * s->psi[c] * sm[d];
                    if (!p->periodic_y) {
                        double fs[3] = {0.0, 0.0, 0.0};
                        for (int a = 1; a < 19; ++a) {
                            const int yy = y + E3[a][1];
                            double Gws = 0.0;
                            if (yy == 0) Gws = p->Gw_bottom;
                            if (yy == p->ny - 1) Gws = p->Gw_top;
                            for (int d = 0; d < 3; ++d) fs[d] += W3(a) * Gws * s->psi[c] * E3[a][d];
                        }
                        for (int d = 0; d < 3; ++d) F[d] -= s->psi[c] * fs[d];
                    }
                    F[1] -= (s->rho[c] - rho_ave) * p->g;
                }
                if (rho) rho[c] = s->rho[c];
                for (int d = 0; d < 3; ++d) {
                    if (!out_v[d]) continue;
                    double j = 0.0;
                    for (int a = 0; a < 19; ++a) j += E3[a][d] * s->f[(size_t)a * n + c];
                    out_v[d][c] = (j + 0.5 * F[d]) / s->rho[c];
                }
                if (T) T[c] = s->T[c];
            }
    if (f) memcpy(f, s->f, 19 * n * sizeof(double));
}

void orc3_set_heater(orc3_state *s, const double *T_bottom)
{
    if (s->p.periodic_y) return;
    for (int z = 0; z < s->nz; ++z)
        for (int x = 0; x < s->p.nx; ++x) {
            s->Tb[(size_t)z * s->p.nx + x] = T_bottom[(size_t)z * s->p.nx + x];
            s->T[idx3(s, x, 0, z)] = s->Tb[(size_t)z * s->p.nx + x];
        }
}
