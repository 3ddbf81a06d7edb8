/*
 * Private layout of the oracle state, shared by the forward (lbb_oracle.c)
 * and its adjoint (lbb_oracle_adjoint.c).  TEST INFRASTRUCTURE ONLY.
 */
#ifndef LBB_ORACLE_INTERNAL_H
#define LBB_ORACLE_INTERNAL_H

#include "lbb_oracle.h"

struct orc_state {
    orc_params p;
    double Tc, kappa, Ts;
    int64_t t;
    double *f, *fpost;           /* [9][ny][nx] */
    double *T;                   /* [ny][nx]    */
    double *Tb;                  /* [nx] bottom-wall temperature */
    /* work arrays of one step */
    double *rho, *psi, *Fx, *Fy, *Q, *vx, *vy, *vTx, *vTy;
    double *Tst, *h, *acc;
    double *ws[7];               /* stencil scratch of the RK4 stages */
    double q_now, q_sum;
    int64_t n_samples;
    int store_bits;              /* 0, or the significant bits the post-collision
                                    populations are rounded to each step */
};

#endif
