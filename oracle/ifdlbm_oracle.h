/*
 * ifdlbm_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, FP64 CPU implementation of the incompressible
 * finite-difference lattice Boltzmann method (IFDLBM) of Chen, Chai, Zhao and
 * Shi, "Numerical Simulation of Power-Law Fluid Flow in a Trapezoidal Cavity
 * using the Incompressible Finite-Difference Lattice Boltzmann Method"
 * (arXiv:2306.07603), for the lid-driven isosceles-trapezoid cavity.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no source with the GPU library.
 *
 * Equation numbers are the paper's equation labels: (1.1)-(1.5) Section 2,
 * (2.0)-(2.15.1) Section 3, (3.1)-(3.8.2) and the conversions (2.15)-(2.19)
 * of the calculational process (Steps (1)-(8)) in Section 4, (A1)-(A12) the
 * Chapman-Enskog appendix.
 *
 * State of a grid of nx * ny nodes: the nine planes F[k * nx*ny + j*nx + i]
 * of the distribution f-hat (Eq. 2.3) and the plane Lam[j*nx + i] of the
 * relaxation time lambda that produced it (Eq. 2.14).  Node (i, j) sits at
 * xi = i*dxi, eta = j*deta in the computational square.
 */
#ifndef IFDLBM_ORACLE_H
#define IFDLBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* The oracle's arithmetic type: double, or with ORC_COMPLEX_STEP a complex double, for the complex-step
   derivative of its outputs with respect to a parameter (J(x + i h) = J(x) + i h J'(x) + O(h^2)). */
#ifdef ORC_COMPLEX_STEP
#include <complex.h>
typedef double _Complex orc_real;
#else
typedef double orc_real;
#endif

/* bc_mode values.  ORC_CAVITY is the paper's problem (Eq. 1.5).  The two
 * periodic modes are test-only geometries (theta must be 90 degrees) used to
 * pin the oracle against closed forms and exact conservation. */
enum { ORC_CAVITY = 0, ORC_COUETTE = 1, ORC_PERIODIC = 2 };

typedef struct {
    int    nx, ny;      /* nodes along xi and eta, boundary nodes included   */
    orc_real re;          /* generalised Reynolds number, Eq. (2.15.1), L = 1  */
    orc_real n;           /* power-law index, Eq. (1.4)                        */
    orc_real theta_deg;   /* top angle of the isosceles trapezoid, (0, 90]     */
    orc_real u_lid;       /* lid speed u0, Eq. (1.5); may be negative in tests */
    orc_real cfl;         /* dt = cfl * min(dxi, deta) / c, c = 1              */
    orc_real mix;         /* weight of the central scheme in Eq. (2.5)         */
    orc_real rho0;        /* constant density rho_0 of Eq. (2.8)               */
    orc_real gamma_min;   /* floor of the shear rate in Eq. (1.4)              */
    int    bc_mode;     /* ORC_CAVITY, ORC_COUETTE or ORC_PERIODIC           */
    int    dt_rule;     /* ORC_DT_CONTRAVARIANT or ORC_DT_CARTESIAN          */
    int    lambda_mode; /* ORC_LAMBDA_LAGGED or ORC_LAMBDA_IMPLICIT          */
} orc_params;

/* lambda_mode values.  LAGGED: Step (2) evaluates the strain rate with the
 * lambda stored with f-hat (the previous step's), the paper's explicit
 * scheme.  IMPLICIT: lambda solves lambda = mu(gamma(lambda)) / c_s^2 at the
 * node, with the strain rate of Eqs. (2.12) and (2.18) taken at that same
 * lambda (solved by bisection to machine precision). */
enum { ORC_LAMBDA_LAGGED = 0, ORC_LAMBDA_IMPLICIT = 1 };

/* dt_rule values (reading R11).  CONTRAVARIANT: dt = cfl / max(|c_xi|/dxi,
 * |c_eta|/deta) over the grid, the Courant number of the transformed
 * equations (3.6)-(3.7); max |c_xi| = 1 + cot(theta) at the bottom corners.
 * CARTESIAN: dt = cfl * min(dxi, deta) / c.  Both equal cfl * dxi on the
 * square. */
enum { ORC_DT_CONTRAVARIANT = 0, ORC_DT_CARTESIAN = 1 };

/* Derived constants of one run. */
typedef struct {
    orc_real dxi, deta;   /* grid spacings of the computational square          */
    orc_real dt;          /* time step                                          */
    orc_real K;           /* consistency coefficient from Eq. (2.15.1)          */
    orc_real cot;         /* 1/tan(theta), exactly 0 at 90 degrees              */
    orc_real lam0;        /* initial relaxation time U L / (Re c_s^2)           */
} orc_derived;

/* Returns 0, or -1 when the parameters are outside the method's domain. */
int  orc_derive(const orc_params* p, orc_derived* d);

/* D2Q9 constants of Eq. (2.9): c_k (as orc_reals), omega_k, omegabar_k. */
void orc_lattice(orc_real cx[9], orc_real cy[9], orc_real w[9], orc_real wbar[9], orc_real* cs2);

/* Eq. (2.8): incompressible equilibrium at (P, u). */
void orc_equilibrium(orc_real P, orc_real ux, orc_real uy, orc_real rho0, orc_real feq[9]);

/* Eqs. (2.10)-(2.11): velocity and pressure from any of f, f-bar, f-hat. */
void orc_moments(const orc_real f[9], orc_real rho0, orc_real* P, orc_real* ux, orc_real* uy);

/* Per-node conversions of the calculational process (Section 4):
 * Eq. (2.18) f from f-hat, Eq. (2.17) f from f-bar, Eqs. (2.15)-(2.16) the
 * post-collision f-hat+ and f-bar+, and Step (2), lambda from the
 * non-equilibrium part by Eqs. (2.12)-(2.14) and (1.4) given the lambda that
 * produced f-hat. */
void   orc_f_from_fhat_node(const orc_real fh[9], const orc_real feq[9], orc_real lam, orc_real dt, orc_real f[9]);
void   orc_f_from_fbar(const orc_real fb[9], const orc_real feq[9], orc_real lam, orc_real dt, orc_real f[9]);
void   orc_collide(const orc_real fh[9], const orc_real feq[9], orc_real lam, orc_real dt,
                   orc_real fhat_plus[9], orc_real fbar_plus[9]);
orc_real orc_relaxation_time(const orc_real fh[9], const orc_real feq[9], orc_real lam_old, orc_real dt,
                           orc_real K, orc_real n, orc_real gamma_min);
/* The implicit reading: the lambda for which orc_relaxation_time returns the
 * lambda it was given (a fixed point), found by bisection. */
orc_real orc_relaxation_time_implicit(const orc_real fh[9], const orc_real feq[9], orc_real dt, orc_real K, orc_real n,
                                    orc_real gamma_min);

/* Eq. (3.8.1): physical position of node (i, j). */
void orc_node_xy(const orc_params* p, int i, int j, orc_real* x, orc_real* y);

/* Eqs. (3.2)-(3.8.2): contravariant velocities (c_k,xi , c_k,eta) at (i, j),
 * and the Jacobian J of Eq. (3.3). */
void orc_contravariant(const orc_params* p, int i, int j, orc_real cxi[9], orc_real ceta[9], orc_real* J);

/* Mixed-difference transport term c_k,xi dPhi_k/dxi + c_k,eta dPhi_k/deta of
 * Eqs. (2.5)-(2.7) and (3.4) at interior node (i, j), for population k of
 * the nine-plane field Phi. */
orc_real orc_stream_term(const orc_params* p, const orc_real* Phi, int k, int i, int j);

/* Step (1): rest state plus moving lid; F = f-hat = f_eq, Lam = lambda_0. */
int  orc_init(const orc_params* p, orc_real* F, orc_real* Lam);

/* Steps (2)-(8), nsteps times, in place.  res_u / res_p (may be NULL) receive
 * the global relative errors of Eq. (2.19) of the last step.  Returns 0, or
 * -1 on bad parameters, or -2 if the state became non-finite. */
int  orc_run(const orc_params* p, orc_real* F, orc_real* Lam, long nsteps, orc_real* res_u, orc_real* res_p);

/* Eq. (2.19) between two states: E(u), E(P), and E(P) of the pressure with
 * its spatial mean removed (reading R16). */
void orc_residuals(const orc_params* p, const orc_real* F_old, const orc_real* F_new,
                   orc_real* e_u, orc_real* e_p, orc_real* e_p_gauge);

/* Macroscopic fields u, v, P (each nx*ny, [j][i]) of the state. */
void orc_fields(const orc_params* p, const orc_real* F, orc_real* u, orc_real* v, orc_real* P);

/* Step (7), Eq. (2.18): the distribution f from f-hat and the stored lambda. */
void orc_f_from_fhat(const orc_params* p, const orc_real* F, const orc_real* Lam, orc_real* f);

/* Eq. (5.1): kinetic energy 1/2 sum |u|^2 dA over the physical cavity,
 * trapezoid-rule weights in (xi, eta) times the Jacobian J. */
orc_real orc_kinetic_energy(const orc_params* p, const orc_real* F);
/* The same into *out (for callers, such as ctypes, that cannot take a complex return value). */
void orc_kinetic_energy_into(const orc_params* p, const orc_real* F, orc_real* out);

#ifdef __cplusplus
}
#endif
#endif
