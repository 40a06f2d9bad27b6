/*
 * ifdlbm_oracle.c -- TEST INFRASTRUCTURE ONLY (see ifdlbm_oracle.h).
 *
 * Plain serial FP64 IFDLBM for the lid-driven isosceles-trapezoid cavity,
 * written from the paper, arXiv:2306.07603.  Every routine follows one
 * equation or one Step of the calculational process in Section 4, in the
 * paper's order and notation; there is no blocking, fusion or reordering.
 * Build with -O2 -ffp-contract=off.
 *
 * Readings taken where the paper is silent, ambiguous or garbled (each one is
 * pinned by a test where a pin exists):
 *  R1  Eq. (2.8): the second-order term is divided by 2 c_s^4 (printed as
 *      2 c_s^2); only this satisfies the moment design (A1) and inverts
 *      Eq. (2.11).
 *  R2  Eqs. (2.3)-(2.4): the collision operator is -(f - f_eq)/lambda, the
 *      BGK term of Eq. (2.0); the conversions (2.15)-(2.18) follow from it.
 *  R3  Eq. (2.7), c < 0 branch: the third point is Pi(chi + 2 dchi), the
 *      mirror of the c >= 0 branch.
 *  R4  The sign test of Eq. (2.7) uses the contravariant velocity component
 *      of the direction being differenced, at that node (Section 4 notes it
 *      varies with position); c = 0 takes the c >= 0 branch.
 *  R5  c_s^2 = c^2 / 3 with c = 1 (the D2Q9 weights of Eq. (2.9) give
 *      sum omega_k c_k c_k = I/3).
 *  R6  Upwind points that would leave the grid (i = 1 or i = nx-2 in the
 *      outward direction) fall back to the first-order one-sided difference.
 *  R7  Boundary nodes use the non-equilibrium extrapolation named in
 *      Section 4: X_b = f_eq(P_nb, u_wall) + (X_nb - f_eq(P_nb, u_nb)),
 *      nb = the node one index inward (diagonal at corners).  It is applied
 *      to the stage variable of each half of the step: f-bar at t + dt/2
 *      (Step 4) and f-hat at t + dt (Step 6).
 *  R8  The lid condition of Eq. (1.5) holds on the closed top edge, so the
 *      two top corners move with the lid; bottom corners are at rest.
 *  R9  Eq. (1.4) at zero shear: mu = K max(gamma^2, gamma_min^2)^((n-1)/2),
 *      gamma^2 = 2 D:D.  Initial lambda_0 = U L / (Re c_s^2).
 *  R10 Eq. (2.15.1): K = U^(2-n) L^n / Re with L = 1 (cavity height) and
 *      U = |u_lid|.
 *  R11 CFL = 0.5 of Section 5 is the Courant number of the transformed
 *      equations (3.6)-(3.7): dt = cfl / max(|c_k,xi|/dxi, |c_k,eta|/deta),
 *      where max |c_k,xi| = 1 + cot(theta) (diagonal populations at the
 *      bottom corners, Eqs. 3.2, 3.8.2) and |c_k,eta| <= 1; on the square
 *      this is the paper's dt = cfl * dx / c.  (The literal Cartesian rule
 *      dt = cfl * min(dxi, deta) / c is kept as an option; on trapezoids it
 *      puts the corner Courant number at 1 + cot(theta)/2 and is unstable
 *      where the fluid is nearly collisionless.)  dxi = 1/(nx-1),
 *      deta = 1/(ny-1); periodic directions hold N distinct nodes and use
 *      spacing 1/N.
 *  R12 Step (2) uses the lambda stored with f-hat (the previous step's, as
 *      Section 3 prescribes) both to recover f by Eq. (2.18) and in
 *      Eq. (2.12); the new lambda is used by Steps (3)-(5).
 *  R13 The half-step macroscopic quantities come from f-bar (Eqs. 2.10-2.11
 *      allow it); they give f_eq(t + dt/2) for Eq. (2.17).
 *  R14 Eq. (2.19) is evaluated over all nodes with the velocities and
 *      pressures computed from f-hat before and after the step; 0/0 counts 0.
 *  R15 Eq. (5.1): area integral with trapezoid weights in (xi, eta) times J.
 *  R16 Eq. (2.19) for P is also given with the spatial mean of P removed
 *      before and after the step.  The level of P is a gauge of the
 *      incompressible model (u depends on grad P only); the extrapolation
 *      walls leak the pressure moment at a constant rate at steady state, so
 *      the raw E(P) falls only as 1/n while the gauge-fixed E(P) converges.
 *  R20 (option) The lag of Step (2) can be removed: with lambda_mode
 *      IMPLICIT, lambda is the fixed point of Step (2) at the node (the
 *      strain rate taken with the lambda being solved for), Section 3 notes
 *      the lag keeps the scheme explicit; the default is the paper's lag.
 */
#include "ifdlbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_COMPLEX_STEP
/* Complex-step build: every operation is the analytic extension of the real one; ordered comparisons, and
   with them every branch (upwind side, shear-rate floor, time-step rule), take the real part, so the
   derivative is that of the branch the real computation takes.  |x| continues as x sign(Re x), and cot at
   90 degrees, exactly 0 in the real build, as -i tanh(Im(theta) pi / 180). */
#define RE(x) creal(x)
#define ORC_POW cpow
#define ORC_TAN ctan
#define ORC_SQRT csqrt
#define ORC_ABS(x) (creal(x) < 0.0 ? -(x) : (x))
#define ORC_FINITE(x) (isfinite(creal(x)) && isfinite(cimag(x)))
#define ORC_COT_AT_90(t) (-I * tanh(cimag(t) * (M_PI / 180.0)))
/* The upwind side of Eq. (2.7) at c = 0 (theta = 90 degrees, populations 2 and 4): the real computation has
   c exactly 0 and takes the c >= 0 side (reading R4); in complex arithmetic the real part of c also carries
   products of two imaginary parts, O(h^2) with h <= 1e-15, whose sign would pick a side node by node. */
#define ORC_UPWIND_NONNEG(c) (creal(c) >= -1e-25)
#else
#define RE(x) (x)
#define ORC_POW pow
#define ORC_TAN tan
#define ORC_SQRT sqrt
#define ORC_ABS(x) fabs(x)
#define ORC_FINITE(x) isfinite(x)
#define ORC_COT_AT_90(t) 0.0
#define ORC_UPWIND_NONNEG(c) ((c) >= 0.0)
#endif

/* ---------------------------------------------------------------- lattice */

/* Eq. (2.9): D2Q9 velocities (c = 1) and weights. */
static const double CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const double CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double OMEGA[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double OMEGABAR[9] = {-5.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* R5 */
static const double CS2 = 1.0 / 3.0;

void orc_lattice(orc_real cx[9], orc_real cy[9], orc_real w[9], orc_real wbar[9], orc_real* cs2)
{
    for (int k = 0; k < 9; ++k) {
        cx[k] = CX[k];
        cy[k] = CY[k];
        w[k] = OMEGA[k];
        wbar[k] = OMEGABAR[k];
    }
    *cs2 = CS2;
}

/* Eq. (2.8), reading R1. */
void orc_equilibrium(orc_real P, orc_real ux, orc_real uy, orc_real rho0, orc_real feq[9])
{
    orc_real uu = ux * ux + uy * uy;
    for (int k = 0; k < 9; ++k) {
        orc_real cu = CX[k] * ux + CY[k] * uy;
        /* u u : (c_k c_k - c_s^2 I) = (c_k . u)^2 - c_s^2 |u|^2 */
        orc_real uu_cc = cu * cu - CS2 * uu;
        feq[k] = OMEGABAR[k] * P / CS2 + OMEGA[k] * rho0
               + OMEGA[k] * (cu / CS2 + uu_cc / (2.0 * CS2 * CS2));
    }
}

/* Eqs. (2.10) and (2.11). */
void orc_moments(const orc_real f[9], orc_real rho0, orc_real* P, orc_real* ux, orc_real* uy)
{
    orc_real sx = 0.0, sy = 0.0, s = 0.0;
    for (int k = 0; k < 9; ++k) {
        sx += CX[k] * f[k];
        sy += CY[k] * f[k];
    }
    for (int k = 1; k < 9; ++k) s += f[k];
    *ux = sx;
    *uy = sy;
    *P = CS2 / OMEGABAR[0] * (-s + (1.0 - OMEGA[0]) * rho0 + OMEGA[0] / (2.0 * CS2) * (sx * sx + sy * sy));
}

/* ---------------------------------------------------------- parameters */

static orc_real cot_deg(orc_real theta_deg)
{
    if (RE(theta_deg) == 90.0) return ORC_COT_AT_90(theta_deg);   /* the unit square, exactly */
    return 1.0 / ORC_TAN(theta_deg * (M_PI / 180.0));
}

int orc_derive(const orc_params* p, orc_derived* d)
{
    if (p->nx < 5 || p->ny < 5) return -1;
    if (!(RE(p->theta_deg) > 0.0 && RE(p->theta_deg) <= 90.0)) return -1;
    if (!(RE(p->n) > 0.0) || !(RE(p->re) > 0.0) || !(RE(p->cfl) > 0.0)) return -1;
    if (!(RE(ORC_ABS(p->u_lid)) > 0.0)) return -1;   /* Re of Eq. (2.15.1) needs U > 0 */
    if (!(RE(p->mix) >= 0.0 && RE(p->mix) <= 1.0) || !(RE(p->gamma_min) > 0.0)) return -1;
    if (p->bc_mode != ORC_CAVITY && RE(p->theta_deg) != 90.0) return -1;
    if (p->bc_mode < ORC_CAVITY || p->bc_mode > ORC_PERIODIC) return -1;
    if (p->dt_rule != ORC_DT_CONTRAVARIANT && p->dt_rule != ORC_DT_CARTESIAN) return -1;
    if (p->lambda_mode != ORC_LAMBDA_LAGGED && p->lambda_mode != ORC_LAMBDA_IMPLICIT) return -1;
    /* R11 */
    d->dxi = (p->bc_mode == ORC_CAVITY) ? 1.0 / (p->nx - 1) : 1.0 / p->nx;
    d->deta = (p->bc_mode == ORC_PERIODIC) ? 1.0 / p->ny : 1.0 / (p->ny - 1);
    d->cot = cot_deg(p->theta_deg);
    if (p->dt_rule == ORC_DT_CARTESIAN) {
        d->dt = p->cfl * (RE(d->dxi) < RE(d->deta) ? d->dxi : d->deta) / 1.0;
    } else {
        orc_real sxi = (1.0 + d->cot) / d->dxi, seta = 1.0 / d->deta;
        /* a tie (theta = 90 on a square grid) takes the xi speed: equal values, and the derivative with
           respect to theta is the one from inside the domain (0, 90] */
        d->dt = p->cfl / (RE(sxi) >= RE(seta) ? sxi : seta);
    }
    /* R10: Re = U^(2-n) L^n / K with L = 1 */
    orc_real U = ORC_ABS(p->u_lid);
    d->K = ORC_POW(U, 2.0 - p->n) / p->re;
    /* R9: lambda_0 = U L / (Re c_s^2) */
    d->lam0 = U / (p->re * CS2);
    return 0;
}

/* ---------------------------------------------------------- geometry */

/* Eq. (3.8.1) */
void orc_node_xy(const orc_params* p, int i, int j, orc_real* x, orc_real* y)
{
    orc_derived d;
    orc_derive(p, &d);
    orc_real xi = i * d.dxi, eta = j * d.deta;
    orc_real C = d.cot;
    *x = 2.0 * C * xi * eta + xi - C * eta + C;
    *y = eta;
}

/* Eqs. (3.2), (3.3), (3.4) with the derivatives of Eq. (3.8.2). */
static void contravariant(const orc_derived* d, int i, int j, orc_real cxi[9], orc_real ceta[9], orc_real* J)
{
    orc_real xi = i * d->dxi, eta = j * d->deta;
    orc_real C = d->cot;
    orc_real x_xi = 2.0 * C * eta + 1.0;
    orc_real x_eta = 2.0 * C * xi - C;
    orc_real y_xi = 0.0, y_eta = 1.0;
    orc_real jac = x_xi * y_eta - x_eta * y_xi;
    orc_real xi_x = y_eta / jac, xi_y = -x_eta / jac;
    orc_real eta_x = -y_xi / jac, eta_y = x_xi / jac;
    for (int k = 0; k < 9; ++k) {
        cxi[k] = CX[k] * xi_x + CY[k] * xi_y;
        ceta[k] = CX[k] * eta_x + CY[k] * eta_y;
    }
    if (J) *J = jac;
}

void orc_contravariant(const orc_params* p, int i, int j, orc_real cxi[9], orc_real ceta[9], orc_real* J)
{
    orc_derived d;
    orc_derive(p, &d);
    contravariant(&d, i, j, cxi, ceta, J);
}

/* ---------------------------------------------------------- transport */

/* Value of a field plane at (i, j), wrapping periodic directions. */
static orc_real at(const orc_params* p, const orc_real* plane, int i, int j)
{
    if (p->bc_mode != ORC_CAVITY) i = (i % p->nx + p->nx) % p->nx;
    if (p->bc_mode == ORC_PERIODIC) j = (j % p->ny + p->ny) % p->ny;
    return plane[j * p->nx + i];
}

/* Eq. (2.5) along one grid direction: eps * central (2.6) + (1 - eps) *
 * second-order upwind (2.7), readings R3, R4 and R6.  (di, dj) is the unit
 * index step of the direction, h its spacing, c the contravariant velocity
 * that selects the upwind side, and npts the node count along it. */
static orc_real mixed_derivative(const orc_params* p, const orc_real* plane, int i, int j,
                               int di, int dj, orc_real h, orc_real c, int pos, int npts, int periodic)
{
    orc_real m1 = at(p, plane, i - di, j - dj);
    orc_real c0 = at(p, plane, i, j);
    orc_real p1 = at(p, plane, i + di, j + dj);
    orc_real central = (p1 - m1) / (2.0 * h);
    orc_real upwind;
    if (ORC_UPWIND_NONNEG(c)) {
        if (periodic || pos >= 2)
            upwind = (3.0 * c0 - 4.0 * m1 + at(p, plane, i - 2 * di, j - 2 * dj)) / (2.0 * h);
        else
            upwind = (c0 - m1) / h;
    } else {
        if (periodic || pos <= npts - 3)
            upwind = -(3.0 * c0 - 4.0 * p1 + at(p, plane, i + 2 * di, j + 2 * dj)) / (2.0 * h);
        else
            upwind = -(c0 - p1) / h;
    }
    return p->mix * central + (1.0 - p->mix) * upwind;
}

/* Eq. (3.4): c_k . grad Phi_k = c_k,xi dPhi/dxi + c_k,eta dPhi/deta. */
static orc_real stream_term(const orc_params* p, const orc_derived* dd, const orc_real* Phi, int k, int i, int j)
{
    orc_derived d = *dd;
    size_t nn = (size_t)p->nx * p->ny;
    const orc_real* plane = Phi + (size_t)k * nn;
    orc_real cxi[9], ceta[9];
    contravariant(&d, i, j, cxi, ceta, NULL);
    int per_xi = p->bc_mode != ORC_CAVITY;
    int per_eta = p->bc_mode == ORC_PERIODIC;
    orc_real term = 0.0;
    if (cxi[k] != 0.0)
        term += cxi[k] * mixed_derivative(p, plane, i, j, 1, 0, d.dxi, cxi[k], i, p->nx, per_xi);
    if (ceta[k] != 0.0)
        term += ceta[k] * mixed_derivative(p, plane, i, j, 0, 1, d.deta, ceta[k], j, p->ny, per_eta);
    return term;
}

orc_real orc_stream_term(const orc_params* p, const orc_real* Phi, int k, int i, int j)
{
    orc_derived d;
    orc_derive(p, &d);
    return stream_term(p, &d, Phi, k, i, j);
}

/* ---------------------------------------------------------- boundary */

static int is_boundary(const orc_params* p, int i, int j)
{
    int wall_i = (p->bc_mode == ORC_CAVITY) && (i == 0 || i == p->nx - 1);
    int wall_j = (p->bc_mode != ORC_PERIODIC) && (j == 0 || j == p->ny - 1);
    return wall_i || wall_j;
}

/* R7: the inward neighbour of a boundary node. */
static void inward(const orc_params* p, int i, int j, int* ni, int* nj)
{
    *ni = i;
    *nj = j;
    if (p->bc_mode == ORC_CAVITY) {
        if (i == 0) *ni = 1;
        if (i == p->nx - 1) *ni = p->nx - 2;
    }
    if (p->bc_mode != ORC_PERIODIC) {
        if (j == 0) *nj = 1;
        if (j == p->ny - 1) *nj = p->ny - 2;
    }
}

/* Eq. (1.5) with reading R8: the top row (corners included) moves with the lid. */
static void wall_velocity(const orc_params* p, int i, int j, orc_real* ux, orc_real* uy)
{
    (void)i;
    *ux = (j == p->ny - 1) ? p->u_lid : 0.0;
    *uy = 0.0;
}

/* R7: fill every boundary node of the nine-plane field X from its inward
 * neighbour: X_b = f_eq(P_nb, u_wall) + (X_nb - f_eq(P_nb, u_nb)), where
 * (P_nb, u_nb) are the moments of X at nb. */
static void nonequilibrium_extrapolation(const orc_params* p, orc_real* X)
{
    size_t nn = (size_t)p->nx * p->ny;
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            if (!is_boundary(p, i, j)) continue;
            int ni, nj;
            inward(p, i, j, &ni, &nj);
            size_t nb = (size_t)nj * p->nx + ni, b = (size_t)j * p->nx + i;
            orc_real fnb[9], feq_nb[9], feq_w[9], P, ux, uy, wx, wy;
            for (int k = 0; k < 9; ++k) fnb[k] = X[k * nn + nb];
            orc_moments(fnb, p->rho0, &P, &ux, &uy);
            orc_equilibrium(P, ux, uy, p->rho0, feq_nb);
            wall_velocity(p, i, j, &wx, &wy);
            orc_equilibrium(P, wx, wy, p->rho0, feq_w);
            for (int k = 0; k < 9; ++k) X[k * nn + b] = feq_w[k] + (fnb[k] - feq_nb[k]);
        }
}

/* ---------------------------------------------------------- per node */

/* Step (7), Eq. (2.18): f from f-hat. */
void orc_f_from_fhat_node(const orc_real fh[9], const orc_real feq[9], orc_real lam, orc_real dt, orc_real f[9])
{
    for (int k = 0; k < 9; ++k) f[k] = 2.0 * lam / (2.0 * lam + dt) * fh[k] + dt / (2.0 * lam + dt) * feq[k];
}

/* Step (4), Eq. (2.17): f from f-bar. */
void orc_f_from_fbar(const orc_real fb[9], const orc_real feq[9], orc_real lam, orc_real dt, orc_real f[9])
{
    for (int k = 0; k < 9; ++k) f[k] = 4.0 * lam / (4.0 * lam + dt) * fb[k] + dt / (4.0 * lam + dt) * feq[k];
}

/* Step (3), Eq. (2.15), and Step (4), Eq. (2.16). */
void orc_collide(const orc_real fh[9], const orc_real feq[9], orc_real lam, orc_real dt, orc_real fhat_plus[9], orc_real fbar_plus[9])
{
    for (int k = 0; k < 9; ++k) {
        fhat_plus[k] = (2.0 * lam - dt) / (2.0 * lam + dt) * fh[k] + 2.0 * dt / (2.0 * lam + dt) * feq[k];
        fbar_plus[k] = (4.0 * lam - dt) / (4.0 * lam + 2.0 * dt) * fh[k] + 3.0 * dt / (4.0 * lam + 2.0 * dt) * feq[k];
    }
}

/* Step (2): lambda from f^(1) = f - f_eq, Eqs. (2.12)-(2.14) with Eq. (1.4),
 * readings R9 and R12.  f is recovered from f-hat with the stored lambda by
 * Eq. (2.18). */
orc_real orc_relaxation_time(const orc_real fh[9], const orc_real feq[9], orc_real lam_old, orc_real dt,
                           orc_real K, orc_real n, orc_real gamma_min)
{
    orc_real f[9];
    orc_f_from_fhat_node(fh, feq, lam_old, dt, f);
    orc_real sxx = 0.0, sxy = 0.0, syy = 0.0;   /* sum_k c c f^ne, Eq. (2.13) */
    for (int k = 0; k < 9; ++k) {
        orc_real fne = f[k] - feq[k];
        sxx += CX[k] * CX[k] * fne;
        sxy += CX[k] * CY[k] * fne;
        syy += CY[k] * CY[k] * fne;
    }
    /* Eq. (2.12): grad u + grad u^T = -(1/(lambda c_s^2)) sum c c f^ne */
    orc_real gxx = -sxx / (lam_old * CS2), gxy = -sxy / (lam_old * CS2), gyy = -syy / (lam_old * CS2);
    /* Eq. (1.3.1): D = (grad u + grad u^T)/2; Eq. (1.4): mu = K (2 D:D)^((n-1)/2) */
    orc_real Dxx = 0.5 * gxx, Dxy = 0.5 * gxy, Dyy = 0.5 * gyy;
    orc_real gamma2 = 2.0 * (Dxx * Dxx + 2.0 * Dxy * Dxy + Dyy * Dyy);
    orc_real floor2 = gamma_min * gamma_min;
    orc_real mu = K * ORC_POW(RE(gamma2) > RE(floor2) ? gamma2 : floor2, 0.5 * (n - 1.0));
    /* Eq. (2.14) */
    return mu / CS2;
}

/* Implicit Step (2): lambda = mu(gamma(lambda)) / c_s^2.  With f recovered
 * from f-hat at the same lambda (Eq. 2.18), f - f_eq = 2 lambda (f-hat - f_eq)
 * / (2 lambda + dt), so Eq. (2.12) gives D = -Pi / (c_s^2 (2 lambda + dt)),
 * Pi = sum_k c_k c_k (f-hat_k - f_eq,k), and gamma^2 = 2 D:D = 2 Q / (c_s^4
 * (2 lambda + dt)^2), Q = Pi:Pi = Pxx^2 + 2 Pxy^2 + Pyy^2.  The map lambda ->
 * mu(gamma(lambda)) / c_s^2 is non-increasing for n >= 1 and, for n < 1,
 * increasing, concave in (2 lambda + dt) up to the floor and bounded by
 * K gamma_min^(n-1) / c_s^2; lambda minus it is negative at 0 and crosses zero
 * once.  Bisection on [0, upper] to the resolution of a orc_real. */
static orc_real implicit_map(orc_real lam, orc_real Q, orc_real dt, orc_real K, orc_real n, orc_real gamma_min)
{
    orc_real s = 2.0 * lam + dt;
    orc_real gamma2 = 2.0 * Q / (CS2 * CS2 * s * s);
    orc_real floor2 = gamma_min * gamma_min;
    return K * ORC_POW(RE(gamma2) > RE(floor2) ? gamma2 : floor2, 0.5 * (n - 1.0)) / CS2;
}

orc_real orc_relaxation_time_implicit(const orc_real fh[9], const orc_real feq[9], orc_real dt, orc_real K, orc_real n,
                                    orc_real gamma_min)
{
    orc_real pxx = 0.0, pxy = 0.0, pyy = 0.0;
    for (int k = 0; k < 9; ++k) {
        orc_real d = fh[k] - feq[k];
        pxx += CX[k] * CX[k] * d;
        pxy += CX[k] * CY[k] * d;
        pyy += CY[k] * CY[k] * d;
    }
    orc_real Q = pxx * pxx + 2.0 * pxy * pxy + pyy * pyy;
    if (RE(n) == 1.0) return K / CS2;
    orc_real lo = 0.0, hi;
    if (RE(n) > 1.0)
        hi = implicit_map(0.0, Q, dt, K, n, gamma_min);   /* the map only falls from here */
    else
        hi = K * ORC_POW(gamma_min * gamma_min, 0.5 * (n - 1.0)) / CS2;   /* the floor caps the map */
    for (int it = 0; it < 200; ++it) {
        orc_real mid = 0.5 * (lo + hi);
        if (RE(mid) <= RE(lo) || RE(mid) >= RE(hi)) break;
        if (RE(mid - implicit_map(mid, Q, dt, K, n, gamma_min)) < 0.0)
            lo = mid;
        else
            hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ---------------------------------------------------------- Step (1) */

int orc_init(const orc_params* p, orc_real* F, orc_real* Lam)
{
    orc_derived d;
    if (orc_derive(p, &d)) return -1;
    size_t nn = (size_t)p->nx * p->ny;
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            orc_real ux = 0.0, uy = 0.0, feq[9];
            if (p->bc_mode != ORC_PERIODIC) wall_velocity(p, i, j, &ux, &uy);
            orc_equilibrium(0.0, ux, uy, p->rho0, feq);
            size_t id = (size_t)j * p->nx + i;
            for (int k = 0; k < 9; ++k) F[k * nn + id] = feq[k];
            Lam[id] = d.lam0;
        }
    return 0;
}

/* ---------------------------------------------------------- Steps (2)-(8) */

typedef struct {
    orc_real *fhat_plus, *fbar_plus, *fbar, *fhalf, *lam, *u_old, *v_old, *P_old;
} workspace;

static void velocities(const orc_params* p, const orc_real* F, orc_real* u, orc_real* v, orc_real* P)
{
    size_t nn = (size_t)p->nx * p->ny;
    for (size_t id = 0; id < nn; ++id) {
        orc_real f[9];
        for (int k = 0; k < 9; ++k) f[k] = F[k * nn + id];
        orc_moments(f, p->rho0, &P[id], &u[id], &v[id]);
    }
}

static int one_step(const orc_params* p, const orc_derived* d, orc_real* F, orc_real* Lam,
                    workspace* w, orc_real* res_u, orc_real* res_p)
{
    const size_t nn = (size_t)p->nx * p->ny;
    const orc_real dt = d->dt;

    velocities(p, F, w->u_old, w->v_old, w->P_old);

    /* Steps (2)-(3) and the first half of Step (4), at every node. */
    for (size_t id = 0; id < nn; ++id) {
        orc_real fh[9], feq[9], fhp[9], fbp[9], P, ux, uy;
        for (int k = 0; k < 9; ++k) fh[k] = F[k * nn + id];
        orc_moments(fh, p->rho0, &P, &ux, &uy);
        orc_equilibrium(P, ux, uy, p->rho0, feq);
        orc_real lam = p->lambda_mode == ORC_LAMBDA_IMPLICIT
                         ? orc_relaxation_time_implicit(fh, feq, dt, d->K, p->n, p->gamma_min)
                         : orc_relaxation_time(fh, feq, Lam[id], dt, d->K, p->n, p->gamma_min);
        w->lam[id] = lam;
        orc_collide(fh, feq, lam, dt, fhp, fbp);
        for (int k = 0; k < 9; ++k) {
            w->fhat_plus[k * nn + id] = fhp[k];
            w->fbar_plus[k * nn + id] = fbp[k];
        }
    }

    /* Step (4): half-step evolution, Eq. (3.7), at interior nodes. */
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            if (is_boundary(p, i, j)) continue;
            size_t id = (size_t)j * p->nx + i;
            for (int k = 0; k < 9; ++k)
                w->fbar[k * nn + id] = w->fbar_plus[k * nn + id] - 0.5 * dt * stream_term(p, d, w->fbar_plus, k, i, j);
        }
    /* boundary populations of f-bar (R7) */
    nonequilibrium_extrapolation(p, w->fbar);
    /* f(t + dt/2) by Eq. (2.17), with f_eq(t + dt/2) from the moments of f-bar (R13) */
    for (size_t id = 0; id < nn; ++id) {
        orc_real fb[9], feq[9], f[9], P, ux, uy;
        for (int k = 0; k < 9; ++k) fb[k] = w->fbar[k * nn + id];
        orc_moments(fb, p->rho0, &P, &ux, &uy);
        orc_equilibrium(P, ux, uy, p->rho0, feq);
        orc_f_from_fbar(fb, feq, w->lam[id], dt, f);
        for (int k = 0; k < 9; ++k) w->fhalf[k * nn + id] = f[k];
    }

    /* Step (5): full-step evolution, Eq. (3.6), at interior nodes. */
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            if (is_boundary(p, i, j)) continue;
            size_t id = (size_t)j * p->nx + i;
            for (int k = 0; k < 9; ++k)
                F[k * nn + id] = w->fhat_plus[k * nn + id] - dt * stream_term(p, d, w->fhalf, k, i, j);
        }
    /* Step (6): macroscopic quantities and the boundary populations (R7). */
    nonequilibrium_extrapolation(p, F);
    for (size_t id = 0; id < nn; ++id) Lam[id] = w->lam[id];

    /* Step (8): global relative errors, Eq. (2.19), R14. */
    orc_real du2 = 0.0, u2 = 0.0, dp2 = 0.0, p2 = 0.0;
    int finite = 1;
    for (size_t id = 0; id < nn; ++id) {
        orc_real f[9], P, ux, uy;
        for (int k = 0; k < 9; ++k) f[k] = F[k * nn + id];
        orc_moments(f, p->rho0, &P, &ux, &uy);
        if (!ORC_FINITE(P) || !ORC_FINITE(ux) || !ORC_FINITE(uy)) finite = 0;
        du2 += (ux - w->u_old[id]) * (ux - w->u_old[id]) + (uy - w->v_old[id]) * (uy - w->v_old[id]);
        u2 += ux * ux + uy * uy;
        dp2 += (P - w->P_old[id]) * (P - w->P_old[id]);
        p2 += P * P;
    }
    if (res_u) *res_u = (du2 == 0.0) ? 0.0 : ORC_SQRT(du2) / ORC_SQRT(u2);
    if (res_p) *res_p = (dp2 == 0.0) ? 0.0 : ORC_SQRT(dp2) / ORC_SQRT(p2);
    return finite ? 0 : -2;
}

int orc_run(const orc_params* p, orc_real* F, orc_real* Lam, long nsteps, orc_real* res_u, orc_real* res_p)
{
    orc_derived d;
    if (orc_derive(p, &d)) return -1;
    size_t nn = (size_t)p->nx * p->ny;
    workspace w;
    w.fhat_plus = malloc(9 * nn * sizeof(orc_real));
    w.fbar_plus = malloc(9 * nn * sizeof(orc_real));
    w.fbar = calloc(9 * nn, sizeof(orc_real));
    w.fhalf = malloc(9 * nn * sizeof(orc_real));
    w.lam = malloc(nn * sizeof(orc_real));
    w.u_old = malloc(nn * sizeof(orc_real));
    w.v_old = malloc(nn * sizeof(orc_real));
    w.P_old = malloc(nn * sizeof(orc_real));
    int rc = 0;
    if (res_u) *res_u = 0.0;
    if (res_p) *res_p = 0.0;
    for (long s = 0; s < nsteps && rc == 0; ++s) rc = one_step(p, &d, F, Lam, &w, res_u, res_p);
    free(w.fhat_plus);
    free(w.fbar_plus);
    free(w.fbar);
    free(w.fhalf);
    free(w.lam);
    free(w.u_old);
    free(w.v_old);
    free(w.P_old);
    return rc;
}

/* ---------------------------------------------------------- outputs */

void orc_residuals(const orc_params* p, const orc_real* F_old, const orc_real* F_new,
                   orc_real* e_u, orc_real* e_p, orc_real* e_p_gauge)
{
    size_t nn = (size_t)p->nx * p->ny;
    orc_real *u0 = malloc(nn * sizeof(orc_real)), *v0 = malloc(nn * sizeof(orc_real)), *P0 = malloc(nn * sizeof(orc_real));
    orc_real *u1 = malloc(nn * sizeof(orc_real)), *v1 = malloc(nn * sizeof(orc_real)), *P1 = malloc(nn * sizeof(orc_real));
    velocities(p, F_old, u0, v0, P0);
    velocities(p, F_new, u1, v1, P1);
    orc_real m0 = 0.0, m1 = 0.0;
    for (size_t id = 0; id < nn; ++id) {
        m0 += P0[id];
        m1 += P1[id];
    }
    m0 /= (orc_real)nn;
    m1 /= (orc_real)nn;
    orc_real du2 = 0.0, u2 = 0.0, dp2 = 0.0, p2 = 0.0, dg2 = 0.0, g2 = 0.0;
    for (size_t id = 0; id < nn; ++id) {
        du2 += (u1[id] - u0[id]) * (u1[id] - u0[id]) + (v1[id] - v0[id]) * (v1[id] - v0[id]);
        u2 += u1[id] * u1[id] + v1[id] * v1[id];
        dp2 += (P1[id] - P0[id]) * (P1[id] - P0[id]);
        p2 += P1[id] * P1[id];
        orc_real dg = (P1[id] - m1) - (P0[id] - m0);
        dg2 += dg * dg;
        g2 += (P1[id] - m1) * (P1[id] - m1);
    }
    *e_u = du2 == 0.0 ? 0.0 : ORC_SQRT(du2) / ORC_SQRT(u2);
    *e_p = dp2 == 0.0 ? 0.0 : ORC_SQRT(dp2) / ORC_SQRT(p2);
    *e_p_gauge = dg2 == 0.0 ? 0.0 : ORC_SQRT(dg2) / ORC_SQRT(g2);
    free(u0); free(v0); free(P0); free(u1); free(v1); free(P1);
}

void orc_fields(const orc_params* p, const orc_real* F, orc_real* u, orc_real* v, orc_real* P)
{
    velocities(p, F, u, v, P);
}

void orc_f_from_fhat(const orc_params* p, const orc_real* F, const orc_real* Lam, orc_real* f)
{
    orc_derived d;
    orc_derive(p, &d);
    size_t nn = (size_t)p->nx * p->ny;
    for (size_t id = 0; id < nn; ++id) {
        orc_real fh[9], feq[9], fo[9], P, ux, uy;
        for (int k = 0; k < 9; ++k) fh[k] = F[k * nn + id];
        orc_moments(fh, p->rho0, &P, &ux, &uy);
        orc_equilibrium(P, ux, uy, p->rho0, feq);
        orc_f_from_fhat_node(fh, feq, Lam[id], d.dt, fo);
        for (int k = 0; k < 9; ++k) f[k * nn + id] = fo[k];
    }
}

orc_real orc_kinetic_energy(const orc_params* p, const orc_real* F)
{
    orc_derived d;
    orc_derive(p, &d);
    size_t nn = (size_t)p->nx * p->ny;
    orc_real e = 0.0;
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            size_t id = (size_t)j * p->nx + i;
            orc_real f[9], P, ux, uy, cxi[9], ceta[9], J;
            for (int k = 0; k < 9; ++k) f[k] = F[k * nn + id];
            orc_moments(f, p->rho0, &P, &ux, &uy);
            contravariant(&d, i, j, cxi, ceta, &J);
            orc_real wi = (p->bc_mode == ORC_CAVITY && (i == 0 || i == p->nx - 1)) ? 0.5 : 1.0;
            orc_real wj = (p->bc_mode != ORC_PERIODIC && (j == 0 || j == p->ny - 1)) ? 0.5 : 1.0;
            e += 0.5 * wi * wj * J * d.dxi * d.deta * (ux * ux + uy * uy);
        }
    return e;
}

void orc_kinetic_energy_into(const orc_params* p, const orc_real* F, orc_real* out)
{
    *out = orc_kinetic_energy(p, F);
}
