/*
 * goc_oracle.c -- plain FP64 CPU oracle of the GOC-LBM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * HIP library: every formula below is restated from the paper
 * (Yahia & Premnath, "Lattice Boltzmann Methods for Navier-Stokes Equations
 * in General Orthogonal Coordinates ...").
 *
 * Scope: the central-moment MRT GOC-LBM for the Navier-Stokes equations
 * (Appendix E of the paper, with the shear stress of Appendix A and the
 * initial / boundary conditions of Appendix C), its two simpler collision
 * variants on the same grid and streaming -- the raw-moment MRT model (the
 * appendix summarising the raw-moment algorithm) and the single-relaxation-
 * time model in velocity space (the appendix on collisions in velocity
 * space) -- and the D2Q5 vector distribution GOC-LBM for the magnetic
 * induction equation (Appendix G).
 * The metric is a general 2-D orthogonal one (h1, h2 and all four theta_ij
 * per node); straight clustered grids are the special case theta12 =
 * theta21 = 0.
 *
 * Every step is written as plain loops over nodes in the paper's order:
 *   pass 1   hydrodynamic fields rho, U (App. E step 7, lagged force) and,
 *            with MHD, B plus the local dB, J3 and Lorentz force (App. G)
 *   pass 2   finite-difference gradients, stresses, effective force,
 *            central-moment collision (App. E steps 1-5), D2Q5 collision
 *   pass 3   pull streaming with boundary conditions (App. E step 6,
 *            App. C momentum-augmented bounce-back, App. G anti-bounce-back)
 *
 * Readings of the paper where it is silent or inconsistent are marked
 * "reading:" and are listed in the design document of the repository.
 *
 * Conventions:
 *   node (i, j) sits at xi1 = i + 1/2, xi2 = j + 1/2; walls lie on the
 *   cell faces xi = 0 and xi = n (half-way bounce-back).
 *   populations f[a][j][i]   -> f[(a*ny + j)*nx + i], a = 0..8
 *   D2Q5 populations g[c][a] -> plane p = c*5 + a (c = 0: B1, c = 1: B2)
 *   lattice velocities (Sec. 3, D2Q9): e = (0,0) (1,0) (0,1) (-1,0) (0,-1)
 *                                          (1,1) (-1,1) (-1,-1) (1,-1)
 *   bare raw-moment order m = (k00,k10,k01,k20,k02,k11,k21,k12,k22)
 *   (Sec. 4, bare moments of the transformation matrix P).
 *
 * parity: the node collision is pinned by tests against the explicit matrix
 * form P^-1 F^-1 [...] of App. E, the binomial definitions of the central
 * moments, the symbolic Chapman-Enskog constraints of Sec. 4-5, the h = 1
 * reduction to a textbook central-moment LBM, mass conservation and the
 * Poiseuille / Couette / Hartmann closed forms.  The raw-moment collision is
 * pinned against its matrix form P^-1 [m + B^-1 L (...)], the SRT collision
 * against the raw-moment one with equal rates (the identity of the two
 * formulations through the linear map P), both against the h = 1 textbook
 * product-form BGK scheme and the Poiseuille closed form.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ 9
#define NM 5

static const int EX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[NQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

enum { K00 = 0, K10, K01, K20, K02, K11, K21, K12, K22 };

typedef struct {
    int32_t nx, ny;
    int32_t bc_x, bc_y;          /* 0 periodic, 1 wall                      */
    int32_t gi_terms;            /* 1: full correction coefficients (Sec. 4)
                                    0: App. B(ii) low-Mach straight-grid forms */
    int32_t q3_sign;             /* 0: binomial transform (reading), 1: printed q21, q12 */
    int32_t lid_corners;         /* 1: a moving y-wall owns the corner ghosts */
    int32_t rho_terms;           /* 0: density-gradient coefficients from the
                                    Chapman-Enskog deviation terms (reading),
                                    1: as printed                              */
    int32_t mhd;                 /* 1: couple the D2Q5 induction equation      */
    double u_wall_lo, u_wall_hi; /* tangential velocity of the xi2 = 0 / ny walls */
    double cs2;                  /* c_s^2 = q^2/3 (Sec. 3.2.1)                   */
    double omega[9];             /* omega_0..omega_8                           */
    double nu, zeta;             /* shear and bulk kinematic viscosity          */
    double rho0;
    double Fext[2];              /* external body force, GOC components          */
    double csm2, tau_m, eta, mu_m, B0;   /* App. G                              */
    /* metric per node, [ny][nx] */
    const double *h1, *h2, *th11, *th12, *th21, *th22;
    /* metric on the wall faces: h2 on xi2 = 0 / ny (per column), h1 on
       xi1 = 0 / nx (per row) and h1 under / above the wall faces (per column)
       and h2 beside the x-wall faces (per row) */
    const double *h2_face_lo, *h2_face_hi, *h1_face_ylo, *h1_face_yhi;  /* [nx] */
    const double *h1_face_lo, *h1_face_hi, *h2_face_xlo, *h2_face_xhi;  /* [ny] */
    int32_t collision;           /* 0 central-moment MRT, 1 raw-moment MRT,
                                    2 SRT with tau = 1/omega_4              */
    double v_wall_lo, v_wall_hi; /* tangential (xi2) velocity of the xi1 = 0 / nx walls */
} OracleCfg;

/* ------------------------------------------------------------------ */
/* Moment maps of App. E (steps 1, 2, 4, 5)                            */
/* ------------------------------------------------------------------ */

/* Step 1: raw moments m = P f. */
static void raw_moments(const double f[NQ], double m[NQ])
{
    m[K00] = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    m[K10] = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
    m[K01] = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
    m[K20] = f[1] + f[3] + f[5] + f[6] + f[7] + f[8];
    m[K02] = f[2] + f[4] + f[5] + f[6] + f[7] + f[8];
    m[K11] = f[5] - f[6] + f[7] - f[8];
    m[K21] = f[5] + f[6] - f[7] - f[8];
    m[K12] = f[5] - f[6] - f[7] + f[8];
    m[K22] = f[5] + f[6] + f[7] + f[8];
}

/* Step 2: central moments k = F(U) m (binomial expansion). */
static void central_from_raw(const double m[NQ], double U1, double U2, double k[NQ])
{
    k[K00] = m[K00];
    k[K10] = m[K10] - U1 * m[K00];
    k[K01] = m[K01] - U2 * m[K00];
    k[K20] = m[K20] - 2.0 * U1 * m[K10] + U1 * U1 * m[K00];
    k[K02] = m[K02] - 2.0 * U2 * m[K01] + U2 * U2 * m[K00];
    k[K11] = m[K11] - U2 * m[K10] - U1 * m[K01] + U1 * U2 * m[K00];
    k[K21] = m[K21] - 2.0 * U1 * m[K11] + U1 * U1 * m[K01] - U2 * m[K20]
           + 2.0 * U1 * U2 * m[K10] - U1 * U1 * U2 * m[K00];
    k[K12] = m[K12] - 2.0 * U2 * m[K11] + U2 * U2 * m[K10] - U1 * m[K02]
           + 2.0 * U1 * U2 * m[K01] - U1 * U2 * U2 * m[K00];
    k[K22] = m[K22] - 2.0 * U1 * m[K12] + U1 * U1 * m[K02] - 2.0 * U2 * m[K21]
           + 4.0 * U1 * U2 * m[K11] - 2.0 * U1 * U1 * U2 * m[K01]
           + U2 * U2 * m[K20] - 2.0 * U1 * U2 * U2 * m[K10]
           + U1 * U1 * U2 * U2 * m[K00];
}

/* Step 4: raw moments back from central ones, m = F(-U) k.  The paper's
   listing swaps the primes on the left and right; the map implemented is the
   inverse frame transformation F^-1 = F(-U) stated with the frame matrix. */
static void raw_from_central(const double k[NQ], double U1, double U2, double m[NQ])
{
    m[K00] = k[K00];
    m[K10] = k[K10] + U1 * k[K00];
    m[K01] = k[K01] + U2 * k[K00];
    m[K20] = k[K20] + 2.0 * U1 * k[K10] + U1 * U1 * k[K00];
    m[K02] = k[K02] + 2.0 * U2 * k[K01] + U2 * U2 * k[K00];
    m[K11] = k[K11] + U2 * k[K10] + U1 * k[K01] + U1 * U2 * k[K00];
    m[K21] = k[K21] + 2.0 * U1 * k[K11] + U1 * U1 * k[K01] + U2 * k[K20]
           + 2.0 * U1 * U2 * k[K10] + U1 * U1 * U2 * k[K00];
    m[K12] = k[K12] + 2.0 * U2 * k[K11] + U2 * U2 * k[K10] + U1 * k[K02]
           + 2.0 * U1 * U2 * k[K01] + U1 * U2 * U2 * k[K00];
    m[K22] = k[K22] + 2.0 * U1 * k[K12] + U1 * U1 * k[K02] + 2.0 * U2 * k[K21]
           + 4.0 * U1 * U2 * k[K11] + 2.0 * U1 * U1 * U2 * k[K01]
           + U2 * U2 * k[K20] + 2.0 * U1 * U2 * U2 * k[K10]
           + U1 * U1 * U2 * U2 * k[K00];
}

/* Step 5 (and App. C initial conditions): f = P^-1 m. */
static void pops_from_raw(const double m[NQ], double f[NQ])
{
    f[0] = m[K00] - m[K20] - m[K02] + m[K22];
    f[1] = 0.5 * (m[K10] + m[K20] - m[K12] - m[K22]);
    f[2] = 0.5 * (m[K01] + m[K02] - m[K21] - m[K22]);
    f[3] = 0.5 * (-m[K10] + m[K20] + m[K12] - m[K22]);
    f[4] = 0.5 * (-m[K01] + m[K02] + m[K21] - m[K22]);
    f[5] = 0.25 * (m[K11] + m[K21] + m[K12] + m[K22]);
    f[6] = 0.25 * (-m[K11] + m[K21] - m[K12] + m[K22]);
    f[7] = 0.25 * (m[K11] - m[K21] - m[K12] + m[K22]);
    f[8] = 0.25 * (-m[K11] - m[K21] + m[K12] + m[K22]);
}

/* ------------------------------------------------------------------ */
/* Viscous stresses, effective body force and the local shear stress    */
/* ------------------------------------------------------------------ */

typedef struct {
    double h1, h2, th11, th12, th21, th22;
} Metric;

typedef struct {
    double rho, U1, U2;                 /* hydrodynamic fields, App. E step 7 */
    double d1U1, d2U2, d1rho, d2rho;    /* second-order finite differences    */
    double Fx1, Fx2;                    /* external force (body + Lorentz)    */
} NodeFlow;

typedef struct {
    double tc11, tc22, t11, t22, Ft1, Ft2, t12, F1, F2;
} ForceTerms;

/* Sec. 2: normal viscous stresses tau11, tau22 with their curvature parts
   tau^c (bulk viscosity zeta, shear viscosity nu). */
static void normal_stresses(const OracleCfg *c, const Metric *g, const NodeFlow *n, ForceTerms *t)
{
    const double rho = n->rho, U1 = n->U1, U2 = n->U2;
    const double nu = c->nu, zeta = c->zeta;
    t->tc11 = rho * (zeta + nu) * U2 * g->th12 + rho * (zeta - nu) * U1 * g->th21;
    t->tc22 = rho * (zeta + nu) * U1 * g->th21 + rho * (zeta - nu) * U2 * g->th12;
    t->t11 = rho * (zeta + nu) * n->d1U1 / g->h1 + rho * (zeta - nu) * n->d2U2 / g->h2 + t->tc11;
    t->t22 = rho * (zeta + nu) * n->d2U2 / g->h2 + rho * (zeta - nu) * n->d1U1 / g->h1 + t->tc22;
}

/* App. A: reduced effective force F~ (tau12 set to zero) from the normal
   stresses, the local implicit solution for tau12 from the non-equilibrium
   raw moment k'11 (relaxed at rate w5), and the full effective force
   F = F~ + 2 h theta tau12.  The same for every collision model. */
static void effective_force(const OracleCfg *c, const Metric *g, const NodeFlow *n, double k11raw,
                            double w5, ForceTerms *t)
{
    const double rho = n->rho, U1 = n->U1, U2 = n->U2;
    const double P = rho * c->cs2;
    t->Ft1 = g->h2 * (n->Fx1 + (g->th21 - g->th11) * P
                      + g->th11 * (t->t11 - rho * U1 * U1)
                      + 2.0 * g->th12 * (0.0 - rho * U1 * U2)
                      - g->th21 * (t->t22 - rho * U2 * U2));
    t->Ft2 = g->h1 * (n->Fx2 + (g->th12 - g->th22) * P
                      + g->th22 * (t->t22 - rho * U2 * U2)
                      + 2.0 * g->th21 * (0.0 - rho * U1 * U2)
                      - g->th12 * (t->t11 - rho * U1 * U1));
    const double a = 1.0 - 0.5 * w5;
    const double num = k11raw + 0.5 * (t->Ft1 * U2 / g->h2 + t->Ft2 * U1 / g->h1) - rho * U1 * U2;
    t->t12 = -a * num / (1.0 + a * (g->th12 * U2 + g->th21 * U1));
    t->F1 = t->Ft1 + 2.0 * g->h2 * g->th12 * t->t12;
    t->F2 = t->Ft2 + 2.0 * g->h1 * g->th21 * t->t12;
}

/* Stresses and effective force of the MRT models. */
static void force_terms(const OracleCfg *c, const Metric *g, const NodeFlow *n,
                        double k11raw, ForceTerms *t)
{
    normal_stresses(c, g, n, t);
    effective_force(c, g, n, k11raw, c->omega[5], t);
}

/* Sec. 4: equilibrium corrections n3^eq(1) (combined k2s) and n4^eq(1)
   (combined k2d), Delta t = 1.  gi_terms = 1 uses the full coefficient sets
   D3k, C3, D4k, C4; gi_terms = 0 uses App. B(ii) (straight grids, no cubic
   Galilean-invariance terms). */
static void eq_corrections(const OracleCfg *c, const Metric *g, const NodeFlow *n,
                           const ForceTerms *t, double *n3, double *n4)
{
    const double rho = n->rho, U1 = n->U1, U2 = n->U2;
    const double nu = c->nu, zeta = c->zeta, cs2 = c->cs2;
    const double h1 = g->h1, h2 = g->h2;
    double D31, D32, D33, D34, C3, D41, D42, D43, D44, C4;
    if (c->gi_terms) {
        D31 = rho * (2.0 * zeta - (zeta + nu) * h2 / (h1 * h1) - (zeta - nu) / h2
                     - zeta * (2.0 - h2 / cs2 + (3.0 * U1 * U1 / cs2 + 1.0) * h2 / (h1 * h1)));
        D32 = rho * (2.0 * zeta - (zeta + nu) * h1 / (h2 * h2) - (zeta - nu) / h1
                     - zeta * (2.0 - h1 / cs2 + (3.0 * U2 * U2 / cs2 + 1.0) * h1 / (h2 * h2)));
        if (c->rho_terms) {
            D33 = -zeta * ((3.0 - U1 * U1 / cs2) * h2 / (h1 * h1) - h2 / cs2 - (U2 * U2 / cs2) / h2) * U1;
            D34 = -zeta * ((3.0 - U2 * U2 / cs2) * h1 / (h2 * h2) - h1 / cs2 - (U1 * U1 / cs2) / h1) * U2;
        } else {
            /* reading: the U d(rho) parts of the deviation terms E3, E4 that
               follow from the Sec. 3 equilibria through the O(eps) moment
               system are U1 [(3 cs2 + U1^2) h2/h1^2 - h2] (and the xi2
               analogue); the printed ones carry -U1^2 and an extra
               -U2^2/h2.  The coefficients below are built from the former,
               as the construction of the corrections prescribes. */
            D33 = -zeta * ((3.0 + U1 * U1 / cs2) * h2 / (h1 * h1) - h2 / cs2) * U1;
            D34 = -zeta * ((3.0 + U2 * U2 / cs2) * h1 / (h2 * h2) - h1 / cs2) * U2;
        }
        C3 = -(h2 / h1 * t->tc11 + h1 / h2 * t->tc22)
             - rho * zeta * (-2.0 * U1 * (U1 * U1 / cs2 + 1.0) * h2 / h1 * g->th11
                             - 2.0 * U2 * (U2 * U2 / cs2 + 1.0) * h1 / h2 * g->th22
                             + U1 * ((3.0 + U1 * U1 / cs2) * h2 / h1 + 2.0 * h1 / h2 - h1 * h2 / cs2) * g->th21
                             + U2 * ((3.0 + U2 * U2 / cs2) * h1 / h2 + 2.0 * h2 / h1 - h1 * h2 / cs2) * g->th12);
        D41 = rho * (2.0 * nu - (zeta + nu) * h2 / (h1 * h1) + (zeta - nu) / h2
                     - nu * (2.0 - h2 / cs2 + (3.0 * U1 * U1 / cs2 + 1.0) * h2 / (h1 * h1)));
        D42 = rho * (-2.0 * nu + (zeta + nu) * h1 / (h2 * h2) - (zeta - nu) / h1
                     - nu * (-2.0 + h1 / cs2 - (3.0 * U2 * U2 / cs2 + 1.0) * h1 / (h2 * h2)));
        if (c->rho_terms) {
            D43 = -nu * ((3.0 - U1 * U1 / cs2) * h2 / (h1 * h1) - h2 / cs2 + (U2 * U2 / cs2) / h2) * U1;
            D44 = -nu * (-(3.0 - U2 * U2 / cs2) * h1 / (h2 * h2) + h1 / cs2 - (U1 * U1 / cs2) / h1) * U2;
        } else {
            D43 = -nu * ((3.0 + U1 * U1 / cs2) * h2 / (h1 * h1) - h2 / cs2) * U1;
            D44 = -nu * (-(3.0 + U2 * U2 / cs2) * h1 / (h2 * h2) + h1 / cs2) * U2;
        }
        /* reading: the theta21 bracket of C4 carries h2/h1 (as in the deviation
           term E4 it is derived from), not the printed h1/h2. */
        C4 = -(h2 / h1 * t->tc11 - h1 / h2 * t->tc22)
             - rho * nu * (-2.0 * U1 * (U1 * U1 / cs2 + 1.0) * h2 / h1 * g->th11
                           + 2.0 * U2 * (U2 * U2 / cs2 + 1.0) * h1 / h2 * g->th22
                           + U1 * ((3.0 + U1 * U1 / cs2) * h2 / h1 - 2.0 * h1 / h2 - h1 * h2 / cs2) * g->th21
                           + U2 * (-(3.0 + U2 * U2 / cs2) * h1 / h2 + 2.0 * h2 / h1 + h1 * h2 / cs2) * g->th12);
    } else {
        D31 = rho * (zeta * h2 / cs2 - (zeta - nu) / h2 - (2.0 * zeta + nu) * h2 / (h1 * h1));
        D32 = rho * (zeta * h1 / cs2 - (zeta - nu) / h1 - (2.0 * zeta + nu) * h1 / (h2 * h2));
        D33 = 0.0;
        D34 = 0.0;
        C3 = -rho * zeta * (-2.0 * U1 * h2 / h1 * g->th11 - 2.0 * U2 * h1 / h2 * g->th22);
        D41 = rho * (nu * h2 / cs2 + (zeta - nu) / h2 - (2.0 * nu + zeta) * h2 / (h1 * h1));
        D42 = rho * (-nu * h1 / cs2 - (zeta - nu) / h1 + (2.0 * nu + zeta) * h1 / (h2 * h2));
        D43 = 0.0;
        D44 = 0.0;
        C4 = -rho * nu * (-2.0 * U1 * h2 / h1 * g->th11 + 2.0 * U2 * h1 / h2 * g->th22);
    }
    *n3 = D31 * n->d1U1 + D32 * n->d2U2 + D33 * n->d1rho + D34 * n->d2rho + C3;
    *n4 = D41 * n->d1U1 + D42 * n->d2U2 + D43 * n->d1rho + D44 * n->d2rho + C4;
}

/* App. E: central-moment equilibria (base forms, combined k2s / k2d). */
static void central_equilibria(const OracleCfg *c, const Metric *g, double rho, double U1,
                               double U2, double eq[NQ])
{
    const double h1 = g->h1, h2 = g->h2, cs2 = c->cs2;
    const double q20 = h2 / h1 * (h1 - 1.0) * (h1 - 1.0);
    const double q02 = h1 / h2 * (h2 - 1.0) * (h2 - 1.0);
    const double q11 = (h1 - 1.0) * (h2 - 1.0);
    double q21, q12;
    if (c->q3_sign) {
        q21 = (h1 - 1.0) * (h1 - 1.0) * (h2 - 1.0) / h1;
        q12 = (h1 - 1.0) * (h2 - 1.0) * (h2 - 1.0) / h2;
    } else {
        /* reading: the binomial transform of the raw equilibria, which the
           paper states as the construction rule, gives the opposite sign of
           the printed coefficients. */
        q21 = (1.0 - h1) * (1.0 - h1) * (1.0 - h2) / h1;
        q12 = (1.0 - h1) * (1.0 - h2) * (1.0 - h2) / h2;
    }
    eq[K00] = h1 * h2 * rho;
    eq[K10] = (1.0 - h1) * h2 * rho * U1;
    eq[K01] = (1.0 - h2) * h1 * rho * U2;
    eq[K20] = q20 * rho * U1 * U1 + q02 * rho * U2 * U2 + (h2 / h1 + h1 / h2) * rho * cs2; /* k2s */
    eq[K02] = q20 * rho * U1 * U1 - q02 * rho * U2 * U2 + (h2 / h1 - h1 / h2) * rho * cs2; /* k2d */
    eq[K11] = q11 * rho * U1 * U2;
    eq[K21] = q21 * rho * U1 * U1 * U2 + (1.0 - h2) * rho * cs2 * U2 / h1;
    eq[K12] = q12 * rho * U1 * U2 * U2 + (1.0 - h1) * rho * cs2 * U1 / h2;
    eq[K22] = cs2 * cs2 * rho;
}

/* App. E: source central moments (combined k2s / k2d slots). */
static void central_sources(const Metric *g, double U1, double U2, double F1, double F2,
                            double s[NQ])
{
    const double h1 = g->h1, h2 = g->h2;
    s[K00] = 0.0;
    s[K10] = F1;
    s[K01] = F2;
    s[K20] = 2.0 * (1.0 / h1 - 1.0) * F1 * U1 + 2.0 * (1.0 / h2 - 1.0) * F2 * U2; /* s2s */
    s[K02] = 2.0 * (1.0 / h1 - 1.0) * F1 * U1 - 2.0 * (1.0 / h2 - 1.0) * F2 * U2; /* s2d */
    s[K11] = (1.0 / h2 - 1.0) * F1 * U2 + (1.0 / h1 - 1.0) * F2 * U1;
    s[K21] = 0.0;
    s[K12] = 0.0;
    s[K22] = 0.0;
}

/* App. E steps 1-5 at one node: pre-collision populations f (post-stream)
   -> post-collision populations ft and the effective force F used for the
   sources. */
static void cm_collide(const OracleCfg *c, const Metric *g, const double f[NQ],
                       const NodeFlow *n, double ft[NQ], double Fout[2])
{
    double m[NQ], k[NQ], eq[NQ], s[NQ], kt[NQ], mt[NQ];
    ForceTerms t;
    double n3, n4;
    raw_moments(f, m);
    force_terms(c, g, n, m[K11], &t);
    central_from_raw(m, n->U1, n->U2, k);
    central_equilibria(c, g, n->rho, n->U1, n->U2, eq);
    eq_corrections(c, g, n, &t, &n3, &n4);
    eq[K20] += n3;   /* k2s^eq */
    eq[K02] += n4;   /* k2d^eq */
    central_sources(g, n->U1, n->U2, t.F1, t.F2, s);
    /* combined second-order diagonal moments (operator B) */
    const double k2s = k[K20] + k[K02];
    const double k2d = k[K20] - k[K02];
    const double *w = c->omega;
    /* reading: the conserved k00 relaxes to k00^eq = h1 h2 rho = k00; it is
       kept as k00 exactly so that mass is conserved to rounding. */
    kt[K00] = k[K00];
    kt[K10] = k[K10] + w[1] * (eq[K10] - k[K10]) + (1.0 - 0.5 * w[1]) * s[K10];
    kt[K01] = k[K01] + w[2] * (eq[K01] - k[K01]) + (1.0 - 0.5 * w[2]) * s[K01];
    const double kt2s = k2s + w[3] * (eq[K20] - k2s) + (1.0 - 0.5 * w[3]) * s[K20];
    const double kt2d = k2d + w[4] * (eq[K02] - k2d) + (1.0 - 0.5 * w[4]) * s[K02];
    kt[K11] = k[K11] + w[5] * (eq[K11] - k[K11]) + (1.0 - 0.5 * w[5]) * s[K11];
    kt[K21] = k[K21] + w[6] * (eq[K21] - k[K21]) + (1.0 - 0.5 * w[6]) * s[K21];
    kt[K12] = k[K12] + w[7] * (eq[K12] - k[K12]) + (1.0 - 0.5 * w[7]) * s[K12];
    kt[K22] = k[K22] + w[8] * (eq[K22] - k[K22]) + (1.0 - 0.5 * w[8]) * s[K22];
    /* split back to the bare second-order moments (operator B^-1) */
    kt[K20] = 0.5 * (kt2s + kt2d);
    kt[K02] = 0.5 * (kt2s - kt2d);
    raw_from_central(kt, n->U1, n->U2, mt);
    pops_from_raw(mt, ft);
    Fout[0] = t.F1;
    Fout[1] = t.F2;
}

/* ------------------------------------------------------------------ */
/* Raw-moment MRT GOC-LBM (appendix summarising the raw-moment model)    */
/* ------------------------------------------------------------------ */

/* Sec. 3, base raw-moment equilibria in the combined basis n^eq = B m^eq:
   slot K20 holds n3 = k20 + k02, slot K02 holds n4 = k20 - k02. */
static void raw_equilibria(const OracleCfg *c, const Metric *g, double rho, double U1, double U2,
                           double eq[NQ])
{
    const double h1 = g->h1, h2 = g->h2, cs2 = c->cs2;
    const double P = rho * cs2;
    eq[K00] = h1 * h2 * rho;
    eq[K10] = h2 * rho * U1;
    eq[K01] = h1 * rho * U2;
    eq[K20] = h2 / h1 * rho * U1 * U1 + h1 / h2 * rho * U2 * U2 + (h2 / h1 + h1 / h2) * P;
    eq[K02] = h2 / h1 * rho * U1 * U1 - h1 / h2 * rho * U2 * U2 + (h2 / h1 - h1 / h2) * P;
    eq[K11] = rho * U1 * U2;
    eq[K21] = rho * (cs2 + U1 * U1) * U2 / h1;
    eq[K12] = rho * (cs2 + U2 * U2) * U1 / h2;
    eq[K22] = rho * cs2 * cs2 + rho * cs2 * (U1 * U1 + U2 * U2) + rho * U1 * U1 * U2 * U2;
}

/* Sec. 3, raw source moments in the combined basis Psi = B sigma. */
static void raw_sources(const Metric *g, double U1, double U2, double F1, double F2, double s[NQ])
{
    const double h1 = g->h1, h2 = g->h2;
    s[K00] = 0.0;
    s[K10] = F1;
    s[K01] = F2;
    s[K20] = 2.0 * (F1 * U1 / h1 + F2 * U2 / h2);   /* sigma2s */
    s[K02] = 2.0 * (F1 * U1 / h1 - F2 * U2 / h2);   /* sigma2d */
    s[K11] = F1 * U2 / h2 + F2 * U1 / h1;
    s[K21] = 0.0;
    s[K12] = 0.0;
    s[K22] = 0.0;
}

/* Raw-moment collision at one node: step 1 (m = P f), step 2 (stresses,
   local tau12, effective force, sources, base equilibria plus the Sec. 4
   corrections on the combined diagonal moments, relaxation of the nine
   combined moments, split back to k20, k02) and step 3 (f~ = P^-1 m~). */
static void raw_collide(const OracleCfg *c, const Metric *g, const double f[NQ],
                        const NodeFlow *n, double ft[NQ], double Fout[2])
{
    double m[NQ], eq[NQ], s[NQ], mt[NQ];
    ForceTerms t;
    double n3, n4;
    raw_moments(f, m);
    force_terms(c, g, n, m[K11], &t);
    raw_sources(g, n->U1, n->U2, t.F1, t.F2, s);
    raw_equilibria(c, g, n->rho, n->U1, n->U2, eq);
    eq_corrections(c, g, n, &t, &n3, &n4);
    eq[K20] += n3;   /* k2s^eq */
    eq[K02] += n4;   /* k2d^eq */
    const double k2s = m[K20] + m[K02];
    const double k2d = m[K20] - m[K02];
    const double *w = c->omega;
    /* reading: as in the central-moment model, the conserved k'00 relaxes
       to h1 h2 rho = k'00 and is kept exactly. */
    mt[K00] = m[K00];
    mt[K10] = m[K10] + w[1] * (eq[K10] - m[K10]) + (1.0 - 0.5 * w[1]) * s[K10];
    mt[K01] = m[K01] + w[2] * (eq[K01] - m[K01]) + (1.0 - 0.5 * w[2]) * s[K01];
    const double mt2s = k2s + w[3] * (eq[K20] - k2s) + (1.0 - 0.5 * w[3]) * s[K20];
    const double mt2d = k2d + w[4] * (eq[K02] - k2d) + (1.0 - 0.5 * w[4]) * s[K02];
    mt[K11] = m[K11] + w[5] * (eq[K11] - m[K11]) + (1.0 - 0.5 * w[5]) * s[K11];
    mt[K21] = m[K21] + w[6] * (eq[K21] - m[K21]) + (1.0 - 0.5 * w[6]) * s[K21];
    mt[K12] = m[K12] + w[7] * (eq[K12] - m[K12]) + (1.0 - 0.5 * w[7]) * s[K12];
    mt[K22] = m[K22] + w[8] * (eq[K22] - m[K22]) + (1.0 - 0.5 * w[8]) * s[K22];
    mt[K20] = 0.5 * (mt2s + mt2d);
    mt[K02] = 0.5 * (mt2s - mt2d);
    pops_from_raw(mt, ft);
    Fout[0] = t.F1;
    Fout[1] = t.F2;
}

/* ------------------------------------------------------------------ */
/* SRT GOC-LBM in velocity space (appendix on velocity-space collisions) */
/* ------------------------------------------------------------------ */

/* SRT collision at one node with the single relaxation time tau =
   1/omega_4; bulk and shear viscosity coincide, nu = zeta = c_s^2 (tau - 1/2).
   The normal stresses take their reduced forms tau11 = 2 rho nu d1U1/h1 +
   tau^c11 with tau^c11 = 2 rho nu U2 theta12 (and symmetrically); the shear
   stress and the effective force are those of every model (App. A, relaxed
   at 1/tau).  The bare second-order equilibria carry the corrections through
   the coefficients G_j, H_j; f^eq = P^-1 m^eq and S = P^-1 sigma, then
   f~ = f + (f^eq - f)/tau + (1 - 1/(2 tau)) S. */
static void srt_collide(const OracleCfg *c, const Metric *g, const double f[NQ],
                        const NodeFlow *n, double ft[NQ], double Fout[2])
{
    const double tau = 1.0 / c->omega[4];
    const double cs2 = c->cs2, nu = cs2 * (tau - 0.5);
    const double rho = n->rho, U1 = n->U1, U2 = n->U2;
    const double h1 = g->h1, h2 = g->h2;
    double m[NQ];
    raw_moments(f, m);            /* k'11 for the local shear stress */
    ForceTerms t;
    t.tc11 = 2.0 * rho * nu * U2 * g->th12;
    t.tc22 = 2.0 * rho * nu * U1 * g->th21;
    t.t11 = 2.0 * rho * nu / h1 * n->d1U1 + t.tc11;
    t.t22 = 2.0 * rho * nu / h2 * n->d2U2 + t.tc22;
    effective_force(c, g, n, m[K11], 1.0 / tau, &t);
    const double u1s = U1 * U1 / cs2, u2s = U2 * U2 / cs2;
    double G1, G3, G5, H2, H4, H5;
    if (c->gi_terms) {
        G1 = rho * nu * (h2 / cs2 - 3.0 * (1.0 + u1s) * h2 / (h1 * h1));
        /* reading: the H2 bracket carries h1/h2^2 (as D3,2 it is half of),
           not the printed h1/h1^2. */
        H2 = rho * nu * (h1 / cs2 - 3.0 * (1.0 + u2s) * h1 / (h2 * h2));
        /* reading: G3, H4 keep the cubic U^2/c_s^2 part of the Chapman-Enskog
           density coefficients D3,3 and D4,3 at zeta = nu, from which the
           coefficients are stated to reduce (the printed G3, H4 drop it while
           G1, H2 keep the analogous term). */
        G3 = -nu * ((3.0 + u1s) * h2 / (h1 * h1) - h2 / cs2) * U1;
        H4 = -nu * ((3.0 + u2s) * h1 / (h2 * h2) - h1 / cs2) * U2;
        G5 = -h2 / h1 * t.tc11
             - rho * nu * (-2.0 * U1 * (u1s + 1.0) * h2 / h1 * g->th11
                           + U1 * ((3.0 + u1s) * h2 / h1 - h1 * h2 / cs2) * g->th21
                           + 2.0 * U2 * h2 / h1 * g->th12);
        H5 = -h1 / h2 * t.tc22
             - rho * nu * (-2.0 * U2 * (u2s + 1.0) * h1 / h2 * g->th22
                           + U2 * ((3.0 + u2s) * h1 / h2 - h1 * h2 / cs2) * g->th12
                           + 2.0 * U1 * h1 / h2 * g->th21);
    } else {
        /* App. B(ii) low-Mach straight-grid limit of the same coefficients:
           no cubic velocity terms, theta12 = theta21 = 0. */
        G1 = rho * nu * (h2 / cs2 - 3.0 * h2 / (h1 * h1));
        H2 = rho * nu * (h1 / cs2 - 3.0 * h1 / (h2 * h2));
        G3 = 0.0;
        H4 = 0.0;
        G5 = 2.0 * rho * nu * U1 * h2 / h1 * g->th11;
        H5 = 2.0 * rho * nu * U2 * h1 / h2 * g->th22;
    }
    double meq[NQ], sig[NQ], feq[NQ], S[NQ];
    meq[K00] = rho * h1 * h2;
    meq[K10] = rho * U1 * h2;
    meq[K01] = rho * U2 * h1;
    meq[K20] = h2 / h1 * rho * (U1 * U1 + cs2) + G1 * n->d1U1 + G3 * n->d1rho + G5;
    meq[K02] = h1 / h2 * rho * (U2 * U2 + cs2) + H2 * n->d2U2 + H4 * n->d2rho + H5;
    meq[K11] = rho * U1 * U2;
    meq[K21] = rho * U2 / h1 * (cs2 + U1 * U1);
    meq[K12] = rho * U1 / h2 * (cs2 + U2 * U2);
    meq[K22] = rho * cs2 * cs2 + rho * cs2 * (U1 * U1 + U2 * U2) + rho * U1 * U1 * U2 * U2;
    sig[K00] = 0.0;
    sig[K10] = t.F1;
    sig[K01] = t.F2;
    sig[K20] = 2.0 * t.F1 * U1 / h1;
    sig[K02] = 2.0 * t.F2 * U2 / h2;
    /* reading: sigma'11 without the printed extra factor 2 on F1 U2/h2, as in
       the raw-moment sources of Sec. 3 it restates. */
    sig[K11] = t.F1 * U2 / h2 + t.F2 * U1 / h1;
    sig[K21] = 0.0;
    sig[K12] = 0.0;
    sig[K22] = 0.0;
    pops_from_raw(meq, feq);
    pops_from_raw(sig, S);
    for (int a = 0; a < NQ; ++a)
        ft[a] = f[a] + (feq[a] - f[a]) / tau + (1.0 - 0.5 / tau) * S[a];
    Fout[0] = t.F1;
    Fout[1] = t.F2;
}

/* Collision of the selected model. */
static void collide_node(const OracleCfg *c, const Metric *g, const double f[NQ],
                         const NodeFlow *n, double ft[NQ], double Fout[2])
{
    if (c->collision == 1) raw_collide(c, g, f, n, ft, Fout);
    else if (c->collision == 2) srt_collide(c, g, f, n, ft, Fout);
    else cm_collide(c, g, f, n, ft, Fout);
}

/* ------------------------------------------------------------------ */
/* D2Q5 vector-distribution GOC-LBM for the induction equation (App. G) */
/* ------------------------------------------------------------------ */

static void mie_weights(double csm2, double W[NM])
{
    /* reading: the zeroth-order weight constraint sums to one (the printed
       sum of zero contradicts the solution W0 + 4 W1 = 1 given with it). */
    W[0] = 1.0 - 2.0 * csm2;
    W[1] = W[2] = W[3] = W[4] = 0.5 * csm2;
}

/* Antisymmetric flux tensor A_ij = U_j B_i - B_j U_i. */
static double Aij(int i, int j, const double U[2], const double B[2])
{
    return U[j] * B[i] - B[j] * U[i];
}

/* Base equilibria g^eq(0)_ai = W_a [h1 h2 B_i + e_a1 h2 A_i1 / csm2 + e_a2 h1 A_i2 / csm2]. */
static void mie_geq0(const OracleCfg *c, const Metric *g, const double U[2], const double B[2],
                     double geq[2][NM])
{
    double W[NM];
    mie_weights(c->csm2, W);
    for (int i = 0; i < 2; ++i)
        for (int a = 0; a < NM; ++a)
            geq[i][a] = W[a] * (g->h1 * g->h2 * B[i] + EX[a] * g->h2 * Aij(i, 0, U, B) / c->csm2
                                + EY[a] * g->h1 * Aij(i, 1, U, B) / c->csm2);
}

/* Source Y_i = h1 h2 (A_i1 theta_i1 + A_i2 theta_i2) of the GOC induction equation. */
static void mie_source(const Metric *g, const double U[2], const double B[2], double Y[2])
{
    const double th[2][2] = {{g->th11, g->th12}, {g->th21, g->th22}};
    for (int i = 0; i < 2; ++i)
        Y[i] = g->h1 * g->h2 * (Aij(i, 0, U, B) * th[i][0] + Aij(i, 1, U, B) * th[i][1]);
}

/* Magnetic field from the transformed populations:
   h1 h2 B_i = sum_a gbar_ai - Y_i / 2, with Y linear in B (2x2 solve). */
static void mie_field(const Metric *g, const double S[2], const double U[2], double B[2])
{
    const double h = g->h1 * g->h2;
    /* h B1 = S1 - h/2 (U2 B1 - B2 U1) th12 ; h B2 = S2 - h/2 (U1 B2 - B1 U2) th21 */
    const double a11 = h * (1.0 + 0.5 * U[1] * g->th12), a12 = -0.5 * h * U[0] * g->th12;
    const double a21 = -0.5 * h * U[1] * g->th21, a22 = h * (1.0 + 0.5 * U[0] * g->th21);
    const double det = a11 * a22 - a12 * a21;
    B[0] = (S[0] * a22 - a12 * S[1]) / det;
    B[1] = (a11 * S[1] - a21 * S[0]) / det;
}

typedef struct {
    double B[2];
    double dB[2][2];  /* dB[p][i] = d B_i / d xi_p */
    double J3;
    double FL[2];
} MieLocal;

/* App. G: local field derivatives from the non-equilibrium first moments,
   current density J3 and Lorentz force. */
static void mie_local(const OracleCfg *c, const Metric *g, const double gb[2][NM],
                      const double U[2], MieLocal *L)
{
    double S[2];
    for (int i = 0; i < 2; ++i) {
        S[i] = 0.0;
        for (int a = 0; a < NM; ++a) S[i] += gb[i][a];
    }
    mie_field(g, S, U, L->B);
    double geq[2][NM];
    mie_geq0(c, g, U, L->B, geq);
    const double csm2 = c->csm2, tm = c->tau_m;
    for (int i = 0; i < 2; ++i) {
        double Lam1 = 0.0, Lam2 = 0.0;
        for (int a = 0; a < NM; ++a) {
            Lam1 += EX[a] * (gb[i][a] - geq[i][a]);
            Lam2 += EY[a] * (gb[i][a] - geq[i][a]);
        }
        L->dB[0][i] = -(Lam1 + 0.5 * csm2 * g->h1 * g->h1 * g->h2 * (g->th11 + g->th21) * L->B[i])
                      / (csm2 * (0.5 * g->h1 * g->h2 + (tm - 0.5) * g->h2 / g->h1));
        L->dB[1][i] = -(Lam2 + 0.5 * csm2 * g->h1 * g->h2 * g->h2 * (g->th22 + g->th12) * L->B[i])
                      / (csm2 * (0.5 * g->h1 * g->h2 + (tm - 0.5) * g->h1 / g->h2));
    }
    L->J3 = (1.0 / c->mu_m) / (g->h1 * g->h2)
            * (g->h2 * L->dB[0][1] - g->h1 * L->dB[1][0]
               + g->h1 * g->h2 * (L->B[1] * g->th21 - L->B[0] * g->th12));
    L->FL[0] = -L->J3 * L->B[1];
    L->FL[1] = L->J3 * L->B[0];
}

/* App. G step 3: SRT collision of the transformed populations with the
   corrected equilibria and the source S^m_ai = -W_a Y_i. */
static void mie_collide(const OracleCfg *c, const Metric *g, const double gb[2][NM],
                        const double U[2], const MieLocal *L, double gt[2][NM])
{
    double W[NM], geq[2][NM], Y[2];
    mie_weights(c->csm2, W);
    mie_geq0(c, g, U, L->B, geq);
    mie_source(g, U, L->B, Y);
    const double eta = c->eta, tm = c->tau_m, csm2 = c->csm2;
    const double h1 = g->h1, h2 = g->h2;
    for (int i = 0; i < 2; ++i) {
        const double Lc1 = eta * (h1 * h2 - h2 / h1) * L->dB[0][i]
                         + eta * h1 * h1 * h2 * (g->th11 + g->th21) * L->B[i];
        const double Lc2 = eta * (h1 * h2 - h1 / h2) * L->dB[1][i]
                         + eta * h1 * h2 * h2 * (g->th22 + g->th12) * L->B[i];
        for (int a = 0; a < NM; ++a) {
            const double gcorr = W[a] * (EX[a] * Lc1 / csm2 + EY[a] * Lc2 / csm2);
            const double geff = geq[i][a] + gcorr;
            const double Sm = -W[a] * Y[i];
            gt[i][a] = gb[i][a] - (gb[i][a] - geff) / tm + (1.0 - 0.5 / tm) * Sm;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Grid driver                                                          */
/* ------------------------------------------------------------------ */

static inline size_t nid(const OracleCfg *c, int i, int j) { return (size_t)j * c->nx + i; }

static void metric_at(const OracleCfg *c, size_t n, Metric *g)
{
    g->h1 = c->h1[n];
    g->h2 = c->h2[n];
    g->th11 = c->th11[n];
    g->th12 = c->th12[n];
    g->th21 = c->th21[n];
    g->th22 = c->th22[n];
}

/* Hydrodynamic fields (App. E step 7): rho = k00/(h1 h2),
   U1 = (k10 + F1/2)/(rho h2), U2 = (k01 + F2/2)/(rho h1).
   reading: F is the effective force of the node's previous collision. */
static void macro_node(const OracleCfg *c, const double *f, const double *Fp, size_t N, size_t n,
                       double *rho, double *U1, double *U2)
{
    double fl[NQ], m[NQ];
    for (int a = 0; a < NQ; ++a) fl[a] = f[a * N + n];
    raw_moments(fl, m);
    const double r = m[K00] / (c->h1[n] * c->h2[n]);
    *rho = r;
    *U1 = (m[K10] + 0.5 * Fp[n]) / (r * c->h2[n]);
    *U2 = (m[K01] + 0.5 * Fp[N + n]) / (r * c->h1[n]);
}

/* Second-order finite difference of a node field along one axis:
   central in the interior and across periodic boundaries; reading: one-sided
   second order (-3 p0 + 4 p1 - p2)/2 on nodes next to a wall. */
static double fd(const double *phi, int idx, int n, int stride, int periodic)
{
    if (periodic) {
        const int ip = (idx + 1) % n, im = (idx - 1 + n) % n;
        return 0.5 * (phi[ip * stride] - phi[im * stride]);
    }
    if (idx == 0) return 0.5 * (-3.0 * phi[0] + 4.0 * phi[stride] - phi[2 * stride]);
    if (idx == n - 1)
        return 0.5 * (3.0 * phi[(n - 1) * stride] - 4.0 * phi[(n - 2) * stride] + phi[(n - 3) * stride]);
    return 0.5 * (phi[(idx + 1) * stride] - phi[(idx - 1) * stride]);
}

typedef struct {
    double *rho, *U1, *U2;     /* [N] */
    double *B1, *B2, *FL1, *FL2; /* [N], MHD */
    double *dB;                /* [4][N], MHD: dB1/dxi1, dB2/dxi1, dB1/dxi2, dB2/dxi2 */
    double *ft;                /* [9][N] post-collision */
    double *gt;                /* [10][N] post-collision (MHD) */
    double *Fn;                /* [2][N] new effective force */
} Work;

static int work_alloc(const OracleCfg *c, Work *w)
{
    const size_t N = (size_t)c->nx * c->ny;
    memset(w, 0, sizeof(*w));
    w->rho = malloc(3 * N * sizeof(double));
    w->ft = malloc(NQ * N * sizeof(double));
    w->Fn = malloc(2 * N * sizeof(double));
    if (!w->rho || !w->ft || !w->Fn) return -1;
    w->U1 = w->rho + N;
    w->U2 = w->rho + 2 * N;
    if (c->mhd) {
        w->B1 = malloc(8 * N * sizeof(double));
        w->gt = malloc(2 * NM * N * sizeof(double));
        if (!w->B1 || !w->gt) return -1;
        w->B2 = w->B1 + N;
        w->FL1 = w->B1 + 2 * N;
        w->FL2 = w->B1 + 3 * N;
        w->dB = w->B1 + 4 * N;
    }
    return 0;
}

static void work_free(Work *w)
{
    free(w->rho);
    free(w->ft);
    free(w->Fn);
    free(w->B1);
    free(w->gt);
}

/* pass 1: hydrodynamic fields, and with MHD the local magnetic quantities. */
static void pass1(const OracleCfg *c, const double *f, const double *Fp, const double *g, Work *w)
{
    const size_t N = (size_t)c->nx * c->ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
            const size_t n = nid(c, i, j);
            macro_node(c, f, Fp, N, n, &w->rho[n], &w->U1[n], &w->U2[n]);
            if (c->mhd) {
                Metric gm;
                metric_at(c, n, &gm);
                double gb[2][NM];
                for (int ci = 0; ci < 2; ++ci)
                    for (int a = 0; a < NM; ++a) gb[ci][a] = g[(ci * NM + a) * N + n];
                const double U[2] = {w->U1[n], w->U2[n]};
                MieLocal L;
                mie_local(c, &gm, gb, U, &L);
                w->B1[n] = L.B[0];
                w->B2[n] = L.B[1];
                w->FL1[n] = L.FL[0];
                w->FL2[n] = L.FL[1];
                w->dB[0 * N + n] = L.dB[0][0];
                w->dB[1 * N + n] = L.dB[0][1];
                w->dB[2 * N + n] = L.dB[1][0];
                w->dB[3 * N + n] = L.dB[1][1];
            }
        }
}

/* pass 2 at one node: gradients, collision of f (and g). */
static void collide_at(const OracleCfg *c, const double *f, const double *g, Work *w, int i, int j)
{
    const size_t N = (size_t)c->nx * c->ny;
    const size_t n = nid(c, i, j);
    Metric gm;
    metric_at(c, n, &gm);
    NodeFlow nf;
    nf.rho = w->rho[n];
    nf.U1 = w->U1[n];
    nf.U2 = w->U2[n];
    const int px = (c->bc_x == 0), py = (c->bc_y == 0);
    nf.d1U1 = fd(w->U1 + (size_t)j * c->nx, i, c->nx, 1, px);
    nf.d1rho = fd(w->rho + (size_t)j * c->nx, i, c->nx, 1, px);
    nf.d2U2 = fd(w->U2 + i, j, c->ny, c->nx, py);
    nf.d2rho = fd(w->rho + i, j, c->ny, c->nx, py);
    nf.Fx1 = c->Fext[0];
    nf.Fx2 = c->Fext[1];
    if (c->mhd) {
        nf.Fx1 += w->FL1[n];
        nf.Fx2 += w->FL2[n];
    }
    double fl[NQ], ft[NQ], F[2];
    for (int a = 0; a < NQ; ++a) fl[a] = f[a * N + n];
    collide_node(c, &gm, fl, &nf, ft, F);
    for (int a = 0; a < NQ; ++a) w->ft[a * N + n] = ft[a];
    w->Fn[n] = F[0];
    w->Fn[N + n] = F[1];
    if (c->mhd) {
        double gb[2][NM], gt[2][NM];
        for (int ci = 0; ci < 2; ++ci)
            for (int a = 0; a < NM; ++a) gb[ci][a] = g[(ci * NM + a) * N + n];
        MieLocal L;
        L.B[0] = w->B1[n];
        L.B[1] = w->B2[n];
        L.dB[0][0] = w->dB[0 * N + n];
        L.dB[0][1] = w->dB[1 * N + n];
        L.dB[1][0] = w->dB[2 * N + n];
        L.dB[1][1] = w->dB[3 * N + n];
        const double U[2] = {nf.U1, nf.U2};
        mie_collide(c, &gm, gb, U, &L, gt);
        for (int ci = 0; ci < 2; ++ci)
            for (int a = 0; a < NM; ++a) w->gt[(ci * NM + a) * N + n] = gt[ci][a];
    }
}

/* pass 3 at one node: pull streaming with boundary conditions.
   Interior and periodic: f_a(x) = ft_a(x - e_a).
   Wall (half-way bounce-back): f_a(x) = ft_opp(a)(x) plus, for a moving
   y-wall, the App. C momentum correction e_a1 rho_w cs2 U_w / (2 h2_wall),
   which gives f7 = ft5 - rho_w cs2 U_w/(2 h2_wall) and f8 = ft6 + ... at the
   top wall; for a moving x-wall (tangential velocity V_w along xi2) the same
   construction, f^eq of App. C at (rho_w, 0, V_w), gives
   e_a2 rho_w cs2 V_w / (2 h1_wall).  reading: rho_w is the density of the
   wall-adjacent node at the collision time level; with lid_corners the
   moving walls also own the corner ghost nodes, where the terms of both
   walls add (the wall equilibria at (rho_w, U_w, V_w) to first order in the
   speeds), which keeps each wall's pair of terms and so the mass; without
   it the corner ghosts take none.
   D2Q5 walls use the App. G anti-bounce-back g_a,i(x) = -gt_opp(a),i(x)
   + 2 W h_wall B_i,wall with B_wall = (0, B0). */
static void stream_at(const OracleCfg *c, const Work *w, double *fo, double *go, int i, int j)
{
    const size_t N = (size_t)c->nx * c->ny;
    const size_t n = nid(c, i, j);
    for (int a = 0; a < NQ; ++a) {
        int si = i - EX[a], sj = j - EY[a];
        int outx = 0, outy = 0;
        if (si < 0 || si >= c->nx) {
            if (c->bc_x == 0) si = (si + c->nx) % c->nx;
            else outx = (si < 0) ? -1 : 1;
        }
        if (sj < 0 || sj >= c->ny) {
            if (c->bc_y == 0) sj = (sj + c->ny) % c->ny;
            else outy = (sj < 0) ? -1 : 1;
        }
        if (!outx && !outy) {
            fo[a * N + n] = w->ft[a * N + nid(c, si, sj)];
            continue;
        }
        double v = w->ft[OPP[a] * N + n];
        if (outy && (!outx || c->lid_corners)) {
            const double uw = (outy < 0) ? c->u_wall_lo : c->u_wall_hi;
            const double hw = (outy < 0) ? c->h2_face_lo[i] : c->h2_face_hi[i];
            v += EX[a] * w->rho[n] * c->cs2 * uw / (2.0 * hw);
        }
        if (outx && (!outy || c->lid_corners)) {
            const double vw = (outx < 0) ? c->v_wall_lo : c->v_wall_hi;
            const double hw = (outx < 0) ? c->h1_face_lo[j] : c->h1_face_hi[j];
            v += EY[a] * w->rho[n] * c->cs2 * vw / (2.0 * hw);
        }
        fo[a * N + n] = v;
    }
    if (!c->mhd) return;
    double W[NM];
    mie_weights(c->csm2, W);
    const double Bw[2] = {0.0, c->B0};
    for (int a = 0; a < NM; ++a) {
        int si = i - EX[a], sj = j - EY[a];
        double hw = 0.0;
        int out = 0;
        if (si < 0 || si >= c->nx) {
            if (c->bc_x == 0) si = (si + c->nx) % c->nx;
            else {
                out = 1;
                hw = ((si < 0) ? c->h1_face_lo[j] : c->h1_face_hi[j])
                     * ((si < 0) ? c->h2_face_xlo[j] : c->h2_face_xhi[j]);
            }
        }
        if (sj < 0 || sj >= c->ny) {
            if (c->bc_y == 0) sj = (sj + c->ny) % c->ny;
            else {
                out = 1;
                hw = ((sj < 0) ? c->h1_face_ylo[i] : c->h1_face_yhi[i])
                     * ((sj < 0) ? c->h2_face_lo[i] : c->h2_face_hi[i]);
            }
        }
        for (int ci = 0; ci < 2; ++ci) {
            if (!out)
                go[(ci * NM + a) * N + n] = w->gt[(ci * NM + a) * N + nid(c, si, sj)];
            else
                go[(ci * NM + a) * N + n] = -w->gt[(ci * NM + OPP[a]) * N + n] + 2.0 * W[a] * hw * Bw[ci];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Exported entry points (called through ctypes by the tests)           */
/* ------------------------------------------------------------------ */

/* Advance the state (f, Fprev, g) by nsteps time steps in place. */
int oracle_step(const OracleCfg *c, double *f, double *Fp, double *g, int nsteps)
{
    const size_t N = (size_t)c->nx * c->ny;
    Work w;
    if (work_alloc(c, &w)) {
        work_free(&w);
        return -1;
    }
    for (int s = 0; s < nsteps; ++s) {
        pass1(c, f, Fp, g, &w);
#pragma omp parallel for schedule(static)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) collide_at(c, f, g, &w, i, j);
#pragma omp parallel for schedule(static)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) stream_at(c, &w, f, g, i, j);
        memcpy(Fp, w.Fn, 2 * N * sizeof(double));
    }
    work_free(&w);
    return 0;
}

/* One time step evaluated only at the sampled nodes (ix[s], iy[s]).  The
   hydrodynamic pass runs over the whole grid, the collision only on the
   nodes the samples pull from.  Outputs: f_out[9][ns], F_out[2][ns] (the
   sampled nodes' new effective force) and g_out[10][ns]. */
int oracle_step_sample(const OracleCfg *c, const double *f, const double *Fp, const double *g,
                       const int32_t *ix, const int32_t *iy, int ns, double *f_out,
                       double *F_out, double *g_out)
{
    const size_t N = (size_t)c->nx * c->ny;
    Work w;
    if (work_alloc(c, &w)) {
        work_free(&w);
        return -1;
    }
    pass1(c, f, Fp, g, &w);
    for (int s = 0; s < ns; ++s)
        for (int a = 0; a < NQ; ++a) {
            int si = ix[s] - EX[a], sj = iy[s] - EY[a], wall = 0;
            if (si < 0 || si >= c->nx) {
                if (c->bc_x == 0) si = (si + c->nx) % c->nx;
                else wall = 1;
            }
            if (sj < 0 || sj >= c->ny) {
                if (c->bc_y == 0) sj = (sj + c->ny) % c->ny;
                else wall = 1;
            }
            if (wall) { /* bounce-back reads the node's own post-collision state */
                si = ix[s];
                sj = iy[s];
            }
            collide_at(c, f, g, &w, si, sj);
        }
    double *fo = malloc(NQ * N * sizeof(double));
    double *go = c->mhd ? malloc(2 * NM * N * sizeof(double)) : NULL;
    for (int s = 0; s < ns; ++s) {
        stream_at(c, &w, fo, go, ix[s], iy[s]);
        const size_t n = nid(c, ix[s], iy[s]);
        for (int a = 0; a < NQ; ++a) f_out[a * ns + s] = fo[a * N + n];
        F_out[s] = w.Fn[n];
        F_out[ns + s] = w.Fn[N + n];
        if (c->mhd)
            for (int p = 0; p < 2 * NM; ++p) g_out[p * ns + s] = go[p * N + n];
    }
    free(fo);
    free(go);
    work_free(&w);
    return 0;
}

/* Hydrodynamic and magnetic fields of a state (the quantities of pass 1). */
int oracle_fields(const OracleCfg *c, const double *f, const double *Fp, const double *g,
                  double *rho, double *U1, double *U2, double *B1, double *B2)
{
    const size_t N = (size_t)c->nx * c->ny;
    Work w;
    if (work_alloc(c, &w)) {
        work_free(&w);
        return -1;
    }
    pass1(c, f, Fp, g, &w);
    memcpy(rho, w.rho, N * sizeof(double));
    memcpy(U1, w.U1, N * sizeof(double));
    memcpy(U2, w.U2, N * sizeof(double));
    if (c->mhd && B1 && B2) {
        memcpy(B1, w.B1, N * sizeof(double));
        memcpy(B2, w.B2, N * sizeof(double));
    }
    work_free(&w);
    return 0;
}

/* Initial state (App. C): f = P^-1 m^eq,eff(rho_i, U_i) with the raw-moment
   equilibria of Sec. 3 and the corrections of Sec. 4 (gradients of the
   initial fields by the same finite differences); g = g^eq(0)(B_i, U_i)
   (App. G) with B_i the given field, or (0, B0) when B1_i / B2_i are NULL;
   reading: the lagged force before the first step is zero, so the first
   hydrodynamic fields equal the initial ones. */
int oracle_init(const OracleCfg *c, const double *rho_i, const double *U1_i, const double *U2_i,
                const double *B1_i, const double *B2_i, double *f, double *Fp, double *g)
{
    const size_t N = (size_t)c->nx * c->ny;
    const int px = (c->bc_x == 0), py = (c->bc_y == 0);
    for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
            const size_t n = nid(c, i, j);
            Metric gm;
            metric_at(c, n, &gm);
            NodeFlow nf;
            nf.rho = rho_i[n];
            nf.U1 = U1_i[n];
            nf.U2 = U2_i[n];
            nf.d1U1 = fd(U1_i + (size_t)j * c->nx, i, c->nx, 1, px);
            nf.d1rho = fd(rho_i + (size_t)j * c->nx, i, c->nx, 1, px);
            nf.d2U2 = fd(U2_i + i, j, c->ny, c->nx, py);
            nf.d2rho = fd(rho_i + i, j, c->ny, c->nx, py);
            nf.Fx1 = c->Fext[0];
            nf.Fx2 = c->Fext[1];
            const double h1 = gm.h1, h2 = gm.h2, r = nf.rho, u1 = nf.U1, u2 = nf.U2;
            const double P = r * c->cs2;
            ForceTerms t;
            /* tau^c only (no tau12 is needed by the corrections) */
            force_terms(c, &gm, &nf, r * u1 * u2, &t);
            double n3, n4;
            eq_corrections(c, &gm, &nf, &t, &n3, &n4);
            /* raw equilibria, Sec. 3 */
            const double k2s = h2 / h1 * r * u1 * u1 + h1 / h2 * r * u2 * u2 + (h2 / h1 + h1 / h2) * P + n3;
            const double k2d = h2 / h1 * r * u1 * u1 - h1 / h2 * r * u2 * u2 + (h2 / h1 - h1 / h2) * P + n4;
            double m[NQ], fl[NQ];
            m[K00] = h1 * h2 * r;
            m[K10] = h2 * r * u1;
            m[K01] = h1 * r * u2;
            m[K20] = 0.5 * (k2s + k2d);
            m[K02] = 0.5 * (k2s - k2d);
            m[K11] = r * u1 * u2;
            m[K21] = r * (c->cs2 + u1 * u1) * u2 / h1;
            m[K12] = r * (c->cs2 + u2 * u2) * u1 / h2;
            m[K22] = r * c->cs2 * c->cs2 + r * c->cs2 * (u1 * u1 + u2 * u2) + r * u1 * u1 * u2 * u2;
            pops_from_raw(m, fl);
            for (int a = 0; a < NQ; ++a) f[a * N + n] = fl[a];
            Fp[n] = 0.0;
            Fp[N + n] = 0.0;
            if (c->mhd) {
                const double U[2] = {u1, u2};
                const double B[2] = {B1_i ? B1_i[n] : 0.0, B2_i ? B2_i[n] : c->B0};
                double geq[2][NM];
                mie_geq0(c, &gm, U, B, geq);
                for (int ci = 0; ci < 2; ++ci)
                    for (int a = 0; a < NM; ++a) g[(ci * NM + a) * N + n] = geq[ci][a];
            }
        }
    return 0;
}

/* ---- single-node entry points used by the unit pins ---------------- */

/* Collision of one node from explicit inputs:
   in[0..8] f, in[9..14] h1 h2 th11 th12 th21 th22, in[15..17] rho U1 U2,
   in[18..21] d1U1 d2U2 d1rho d2rho, in[22..23] external force.
   out[0..8] ft, out[9..10] F of the selected collision model; out[11]
   tau12, out[12] n3eq1, out[13] n4eq1, out[14..15] F~ of the MRT models'
   stresses. */
int oracle_collide_node(const OracleCfg *c, const double *in, double *out)
{
    Metric g = {in[9], in[10], in[11], in[12], in[13], in[14]};
    NodeFlow n = {in[15], in[16], in[17], in[18], in[19], in[20], in[21], in[22], in[23]};
    double ft[NQ], F[2], m[NQ];
    collide_node(c, &g, in, &n, ft, F);
    for (int a = 0; a < NQ; ++a) out[a] = ft[a];
    out[9] = F[0];
    out[10] = F[1];
    raw_moments(in, m);
    ForceTerms t;
    force_terms(c, &g, &n, m[K11], &t);
    out[11] = t.t12;
    double n3, n4;
    eq_corrections(c, &g, &n, &t, &n3, &n4);
    out[12] = n3;
    out[13] = n4;
    out[14] = t.Ft1;
    out[15] = t.Ft2;
    return 0;
}

/* Moment maps exposed for the matrix-form pins: which = 0 P, 1 F(U),
   2 F(-U) (inverse), 3 P^-1; vector of 9 in, 9 out. */
int oracle_moment_map(int which, const double *v, double U1, double U2, double *out)
{
    switch (which) {
    case 0: raw_moments(v, out); return 0;
    case 1: central_from_raw(v, U1, U2, out); return 0;
    case 2: raw_from_central(v, U1, U2, out); return 0;
    case 3: pops_from_raw(v, out); return 0;
    default: return -1;
    }
}

/* Central equilibria (combined k2s in slot 3, k2d in slot 4) and central
   sources for the binomial pins. */
int oracle_central_eq(const OracleCfg *c, double h1, double h2, double rho, double U1, double U2,
                      double F1, double F2, double *eq, double *src)
{
    Metric g = {h1, h2, 0, 0, 0, 0};
    central_equilibria(c, &g, rho, U1, U2, eq);
    central_sources(&g, U1, U2, F1, F2, src);
    return 0;
}

/* D2Q5 single-node entry: in gb[10] (plane c*5+a), U[2], metric[6];
   out: B[2], dB[4] (dB1/dxi1, dB2/dxi1, dB1/dxi2, dB2/dxi2), J3, FL[2], gt[10]. */
int oracle_mie_node(const OracleCfg *c, const double *gbin, const double *Uin, const double *met,
                    double *out)
{
    Metric g = {met[0], met[1], met[2], met[3], met[4], met[5]};
    double gb[2][NM], gt[2][NM];
    for (int ci = 0; ci < 2; ++ci)
        for (int a = 0; a < NM; ++a) gb[ci][a] = gbin[ci * NM + a];
    MieLocal L;
    mie_local(c, &g, gb, Uin, &L);
    mie_collide(c, &g, gb, Uin, &L, gt);
    out[0] = L.B[0];
    out[1] = L.B[1];
    out[2] = L.dB[0][0];
    out[3] = L.dB[0][1];
    out[4] = L.dB[1][0];
    out[5] = L.dB[1][1];
    out[6] = L.J3;
    out[7] = L.FL[0];
    out[8] = L.FL[1];
    for (int ci = 0; ci < 2; ++ci)
        for (int a = 0; a < NM; ++a) out[9 + ci * NM + a] = gt[ci][a];
    return 0;
}

/* Number of threads the OpenMP loops use (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads of the OpenMP loops (for timing the oracle on
   one core and on all of them); returns the number now in use. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return oracle_threads();
}
