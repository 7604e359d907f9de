/*
 * goc_lbm.h -- C-ABI of the MI355X GOC-LBM library (libgoclbm.so).
 *
 * The library advances the central-moment multiple-relaxation-time lattice
 * Boltzmann method in general orthogonal coordinates (Yahia & Premnath,
 * App. E, with the local shear stress of App. A and the boundary and initial
 * conditions of App. C), optionally coupled to the D2Q5 vector-distribution
 * scheme for the magnetic induction equation (App. G), on the uniform
 * computational lattice of a straight clustered grid (metric factors
 * h1(xi1), h2(xi2); theta12 = theta21 = 0, the case of App. B(i)).  Two
 * simpler collision models run on the same data path: the raw-moment MRT
 * model (the appendix summarising the raw-moment algorithm) and the
 * single-relaxation-time model in velocity space (the appendix on
 * velocity-space collisions); goc_params.collision selects one.
 *
 * Conventions shared by every entry point:
 *   - nodes (i, j), 0 <= i < nx, 0 <= j < ny, sit at xi = (i + 1/2, j + 1/2);
 *     walls lie on the cell faces xi = 0 and xi = n (half-way bounce-back);
 *   - node arrays are row-major [ny][nx] FP64, index j*nx + i;
 *   - D2Q9 directions e_a = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
 *     (-1,-1) (1,-1); D2Q5 uses the first five;
 *   - "device" pointers are HIP device allocations valid on the handle's
 *     device (e.g. a torch tensor's data_ptr()); "host" pointers are plain
 *     CPU memory.  Calls are ordered on the stream given at creation.
 *   - Every function returns GOC_OK (0) or a negative goc_status; it never
 *     aborts or prints.  goc_lbm_last_error() gives a thread-local message.
 *   - One handle must not be used by two threads at once.
 */
#ifndef GOC_LBM_H
#define GOC_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GOC_OK = 0,
    GOC_EINVAL = -1,     /* bad argument                                  */
    GOC_ENOMEM = -2,     /* device or host allocation failed              */
    GOC_EDEVICE = -3,    /* a HIP call failed                             */
    GOC_EUNSTABLE = -4,  /* the watchdog found a non-finite value         */
    GOC_ESTATE = -5      /* state blob of another version, size or grid   */
} goc_status;

typedef enum { GOC_BC_PERIODIC = 0, GOC_BC_WALL = 1 } goc_bc;

typedef enum {
    GOC_F64 = 0,      /* populations FP64, arithmetic FP64                       */
    GOC_F32 = 1,      /* populations FP32, arithmetic FP32                       */
    GOC_F16DEV = 2,   /* populations FP16 as scaled deviations from the rest state,
                         less a per-row reference (below), arithmetic FP32       */
    GOC_BF16DEV = 3   /* as GOC_F16DEV with bfloat16                              */
} goc_storage;
/* The 16-bit forms (GOC_F16DEV, GOC_BF16DEV) store each slot as the deviation
   of its population from the rest state (rho0, U = 0; App. C), minus a
   reference: the mean over the reader's row of the deviations pulled along
   the reader's direction (one table of 19 FP32 values per row and run: nine
   D2Q9 and ten D2Q5 directions), times a fixed scale per direction class,
   rounded stochastically.  Where the flow varies little along a row the
   stored residual is far smaller than the deviation, which carries the
   velocity, the lagged force and the magnetic field.  Every initialisation
   (goc_lbm_init*, goc_lbm_set_populations) forms the table from the state it
   writes; goc_lbm_step refreshes it from the current state after the first
   step and then every 100 steps (the step then decodes with the old table
   and encodes with the new one); checkpoints carry it.  The 16-bit forms
   step with the tiled kernel only (goc_lbm_set_launch). */

typedef enum {
    GOC_COLL_CENTRAL = 0,  /* central-moment MRT (App. E)                          */
    GOC_COLL_RAW = 1,      /* raw-moment MRT: the nine combined raw moments relax
                              to the Sec. 3 equilibria with the Sec. 4 corrections */
    GOC_COLL_SRT = 2       /* single relaxation time tau = 1/omega[4] in velocity
                              space, f^eq = P^-1 m^eq and S = P^-1 sigma; every
                              rate is 1/tau, so zeta = nu.  Computed as the
                              raw-moment body with equal rates (P is linear). */
} goc_collision;

typedef enum {
    GOC_STRETCH_ARRAY = 0,    /* metric factors given as arrays                   */
    GOC_STRETCH_UNIFORM = 1,  /* h = 1                                            */
    GOC_STRETCH_TANH = 2,     /* Sec. 6.1 two-wall hyperbolic tangent, parameter beta */
    GOC_STRETCH_ROBERTS = 3,  /* Sec. 6.2 Roberts transformation, parameter gamma,
                                 clustered at both walls (alpha = 1/2)           */
    /* General 2-D metrics (kind_x only; kind_y is then ignored): */
    GOC_STRETCH_ANNULUS = 4,  /* the conformal annular sector of the curvilinear
                                 section, Z = a exp(pi W / N_theta) shifted and
                                 scaled: xi1 in [0, nx] spans the radii a = param_x
                                 .. Ro = param_y, xi2 in [0, ny] the angle
                                 2 pi / n_theta; h1, h2 and theta11 = theta21 in
                                 closed form, theta12 = theta22 = 0              */
    GOC_STRETCH_ARRAY2D = 5   /* node arrays h1_2d, h2_2d [ny*nx]               */
} goc_stretch;

typedef enum {
    GOC_FLOW_CHANNEL = 0,   /* body-force channel, Sec. 7.1: Re = U (H/2)/nu, tau given */
    GOC_FLOW_CAVITY = 1,    /* lid-driven cavity, Sec. 7.3: Re = U_lid L / nu,
                               U_lid = u_lid, or Ma c_s when u_lid <= 0, then
                               lowered so that tau <= tau_max when tau_max > 1/2  */
    GOC_FLOW_HARTMANN = 2,  /* MHD channel, Sec. 7.4: Re = U_c H / nu, H half-width,
                               U_c = Ma c_s lowered so that tau <= tau_max when
                               tau_max > 1/2; eta = nu / Pm                          */
    GOC_FLOW_FREE = 3       /* no derived forcing: tau and F_ext given                */
} goc_flow;

/* Lattice and boundaries.  u_wall_lo / u_wall_hi are the tangential (xi1)
   velocities of the walls at xi2 = 0 and xi2 = ny (momentum-augmented
   bounce-back of App. C); they are used only when bc_y is GOC_BC_WALL.
   v_wall_lo / v_wall_hi are the tangential (xi2) velocities of the walls at
   xi1 = 0 and xi1 = nx (the same construction: e_a2 rho_w c_s^2 V_w /
   (2 h1_wall)), used only when bc_x is GOC_BC_WALL.  With lid_corners the
   corner ghosts take the terms of both walls. */
typedef struct {
    int32_t nx, ny;           /* >= 3 each                                   */
    int32_t bc_x, bc_y;       /* goc_bc                                      */
    double u_wall_lo, u_wall_hi;
    double v_wall_lo, v_wall_hi;
} goc_grid;

/* Metric factors of a straight orthogonal grid.  For GOC_STRETCH_ARRAY the
   caller passes h1[nx] and h2[ny] (host, FP64, > 0, borrowed for the call)
   at the node centres, optionally their derivatives dh1[nx], dh2[ny]
   (NULL: second-order finite differences, one-sided at the ends), and the
   values on the wall faces h1_face[2] (xi1 = 0, nx) and h2_face[2]
   (xi2 = 0, ny); a face value <= 0 means "the adjacent node's value".
   For the analytic kinds only the kind and its parameter are read.
   General 2-D metrics (kind_x GOC_STRETCH_ANNULUS or GOC_STRETCH_ARRAY2D):
   for the annulus param_x, param_y and n_theta (> 0, param_y > param_x > 0);
   for arrays h1_2d, h2_2d [ny*nx] (host, FP64, > 0) and either all four
   derivative arrays d1h1, d2h1, d1h2, d2h2 [ny*nx] or none (second-order
   differences: central, wrapped along a periodic axis, one-sided at the
   ends of a walled one); their face values are the adjacent nodes'.  A run
   on a 2-D metric takes the curvilinear step (one launch per run and step,
   the metric read per node); it cannot be MHD (the paper's GOC induction
   equation diffuses each component of B as a scalar, which is the vector
   Laplacian only on straight grids), and the runs of a batch share the
   metric kind (2-D or straight). */
typedef struct {
    int32_t kind_x, kind_y;   /* goc_stretch                                 */
    double param_x, param_y;  /* beta (tanh) or gamma (Roberts); annulus radii */
    const double *h1, *h2;
    const double *dh1, *dh2;
    double h1_face[2], h2_face[2];
    double n_theta;           /* annulus: sectors in a full circle           */
    const double *h1_2d, *h2_2d;
    const double *d1h1, *d2h1, *d1h2, *d2h2;
} goc_metric;

/* Lattice parameters of a run (all in lattice units).  The physical
   parameters of the paper's flows (Reynolds number Re, Hartmann number Ha,
   magnetic Prandtl number Pm, Mach number Ma) are not fields here: they
   enter through goc_lbm_derive, which turns a goc_physics description into
   these fields (omega[4] = omega[5] from the viscosity that Re fixes;
   F_ext from Re, or from Re and Ha for the Hartmann flow; tau_m from
   eta = nu / Pm; B0 from Ha), and the caller passes the result to
   goc_lbm_create.  c_s^2 = q^2/3 with
   q the minimum metric factor (Sec. 3.2.1) is derived by the library from
   the metric, as is the MHD sound speed c_sm = c_s (App. G).  nu and zeta
   follow from omega[4] (= omega[5] for the default reading) and omega[3]:
   nu = c_s^2 (1/omega5 - 1/2), zeta = c_s^2 (1/omega3 - 1/2) (Sec. 4). */
typedef struct {
    double omega[9];          /* relaxation rates, each in (0, 2)            */
    double rho0;              /* reference (initial) density                 */
    double F_ext[2];          /* external body-force density, GOC components */
    int32_t gi_terms;         /* 1: full correction coefficients (Sec. 4);
                                 0: App. B(ii) low-Mach forms                */
    int32_t q3_sign;          /* 0: binomial-transform sign of q21, q12; 1: as printed */
    int32_t rho_terms;        /* 0: density-gradient coefficients from the
                                 Chapman-Enskog analysis; 1: as printed      */
    int32_t lid_corners;      /* 1: a moving y-wall owns the corner ghosts   */
    int32_t mhd;              /* 1: couple the D2Q5 induction equation       */
    double tau_m;             /* magnetic relaxation time (> 1/2)            */
    double mu_m;              /* magnetic permeability                       */
    double B0;                /* applied field: wall and initial B2          */
    int32_t collision;        /* goc_collision.  GOC_COLL_SRT reads omega[4]
                                 only (the other entries are ignored) and
                                 needs rho_terms = 0: its coefficients G_j,
                                 H_j reduce from the Chapman-Enskog reading.
                                 The runs of a batch share one model.        */
} goc_params;

/* Physical description used by goc_lbm_derive. */
typedef struct {
    int32_t flow;             /* goc_flow                                    */
    double Re, Ha, Pm, Ma;
    double tau;               /* channel / free flows: shear relaxation time */
    double tau_max;           /* Hartmann, cavity with u_lid <= 0: cap on the
                                 shear relaxation time (<= 1/2: no cap)      */
    double u_lid;             /* cavity: lid (xi2 = ny wall) speed           */
    double rho0, mu_m;
    double F_ext[2];          /* free flows: body force                      */
} goc_physics;

typedef struct goc_lbm goc_lbm_t;

/* Derive lattice parameters from physical ones (Sec. 3.2.1, Sec. 4,
   App. G, Sec. 7), for the given grid and metric: the bridge from the
   paper's dimensionless numbers (Re, Ha, Pm, Ma in *phys) to goc_params,
   which goc_lbm_create takes.  c_s^2 from the metric;
   channel: nu = c_s^2 (tau - 1/2), U = Re nu/(H/2), F = 2 nu U rho0/(H/2)^2
   with H = ny; cavity: nu = U_lid nx / Re (U_lid reduced if tau would
   exceed tau_max and u_lid <= 0) and grid->u_wall_hi = U_lid;
   Hartmann: U_c = Ma c_s (reduced if tau would exceed tau_max),
   nu = U_c (ny/2)/Re, eta = nu/Pm, B0 from Ha, F from the analytic
   centre-line speed; omega4 = omega5 from nu, the other rates 1.  Writes
   *out and may update grid->u_wall_*.  Host only. */
int goc_lbm_derive(goc_grid *grid, const goc_metric *metric, const goc_physics *phys,
                   goc_params *out);

/* Create a run on the current HIP device.  Copies the metric (FP64
   precompute on the device: theta = dh/h^2, q = min h), allocates the
   state (two slot buffers, holding with MHD the D2Q5 slots too, and the
   lagged force) and initialises it at rest (rho0, U = 0, B = (0, B0)).
   stream: a hipStream_t (NULL = the default stream).  *out receives the
   handle, owned by the caller until goc_lbm_destroy.  Size limits: nx, ny
   >= 3, nx*ny <= 2^31, and the slot pool of one run (9 planes, or 20 with
   the D2Q5 slots, which share its rows; each plane padded to an odd number
   of 64-node pieces, over ny + 2 rows, plus 256 storage elements) at most
   4 GiB, i.e. about 27M nodes in FP64 with MHD (59M without), 53M in FP32
   (119M), 107M in the 16-bit forms (238M) for wide grids; GOC_EINVAL
   beyond. */
int goc_lbm_create(goc_lbm_t **out, const goc_grid *grid, const goc_metric *metric,
                   const goc_params *params, int32_t storage, void *stream);

/* Initial state of App. C from node fields rho[ny*nx], u1, u2 (FP64,
   device if on_device else host): f = P^-1 m^eq,eff(rho, U), g = g^eq(0)
   with B = (0, B0); lagged force zero; step counter zero.  All three NULL
   re-initialises at rest. */
int goc_lbm_init(goc_lbm_t *h, const double *rho, const double *u1, const double *u2,
                 int32_t on_device);

/* As goc_lbm_init, with the magnetic field too: b1[ny*nx], b2 (FP64, same
   memory space as rho) give B, so that g = g^eq(0)(B, U) of App. G.  b1 and
   b2 must be given together, with rho, u1, u2, on an MHD run; both NULL is
   goc_lbm_init.  GOC_EINVAL otherwise. */
int goc_lbm_init_mhd(goc_lbm_t *h, const double *rho, const double *u1, const double *u2,
                     const double *b1, const double *b2, int32_t on_device);

/* Initial state of one run of a batch from its node fields (as
   goc_lbm_init_mhd; b1, b2 may be NULL): rho, u1, u2 [ny*nx] of that run.
   The other runs and the handle's step count are unchanged.  GOC_EINVAL for
   a run outside [0, num_runs) or missing fields. */
int goc_lbm_init_run(goc_lbm_t *h, int32_t run, const double *rho, const double *u1, const double *u2,
                     const double *b1, const double *b2, int32_t on_device);

/* Advance n >= 0 time steps (App. E steps 1-7 and App. G steps 1-6 per
   step, one fused kernel launch each; with a non-NULL stream, blocks of 100
   steps replay a captured HIP graph).  16-bit storage: the reference table
   is refreshed on the steps given above the storage enum, and graph blocks
   start on them.  Asynchronous on the stream unless the watchdog check is
   due at its return (goc_lbm_set_watchdog). */
int goc_lbm_step(goc_lbm_t *h, int64_t n);

/* Hydrodynamic and magnetic fields of the current state (App. E step 7,
   App. G): rho[ny*nx], u[2*ny*nx] (U1 then U2; the Cartesian components
   on a straight grid) and B[2*ny*nx] (B1 then B2, MHD runs only; NULL
   allowed).  FP64; device pointers if on_device else host.  Synchronises
   the stream when on_device is 0. */
int goc_lbm_moments(goc_lbm_t *h, double *rho, double *u, double *B, int32_t on_device);

/* Global sums in FP64 over the nodes of run 0 (host out[8]): [0] mass
   sum f (App. E step 7: the populations sum to h1 h2 rho), [1] sum h2 rho U1,
   [2] sum h1 rho U2 (the momentum of App. E step 7 without the lagged
   force's half), [3] mean over columns of the flow rate sum_j h2 rho U1
   (the physical integral of rho u across the channel), [4] sum h1 h2 B1,
   [5] sum h1 h2 B2 (the fluxes of the field of App. G; 0 without MHD),
   [6] max |U|, [7] number of non-finite populations.  Work-group partials
   summed in a fixed order: deterministic.  Synchronises the stream. */
int goc_lbm_diagnostics(goc_lbm_t *h, double out[8]);
/* The same for run `run` of a batch (GOC_EINVAL outside [0, num_runs)). */
int goc_lbm_diagnostics_run(goc_lbm_t *h, int32_t run, double out[8]);
/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, hosts that forbid hipMalloc): the eight
   outputs of goc_lbm_diagnostics_run, computed by the same kernels, written
   to the device buffer out_dev (8 doubles, on the handle's device), queued
   on the handle's stream with no synchronisation and no allocation.  The
   partial sums live in a static device array of the library (4096 x 7
   doubles, 229 KB on every device it runs on, held until the process ends;
   every grid fits it, since the first pass strides over the nodes).  Calls
   that overlap on one GPU (other streams, other threads) race on that array.
   GOC_EINVAL for a run outside [0, num_runs), a NULL out_dev, or a current
   device other than the handle's. */
int goc_lbm_diagnostics_noalloc(goc_lbm_t *h, int32_t run, double *out_dev);

/* The watchdog: when a goc_lbm_step call returns having completed at
   least `every` steps since the last check (or since initialisation,
   set_state or this call), every run's populations are checked for
   non-finite values (the diagnostics pass, App. E step 7 sums), and a hit
   makes that goc_lbm_step return GOC_EUNSTABLE.  Default 1000; 0 turns it
   off.  The check synchronises the stream. */
int goc_lbm_set_watchdog(goc_lbm_t *h, int64_t every);

/* Form and launch plan of the step.  Two kernels compute the same step
   (App. E, every node once per step):
   - the march: one work-group (a wave of 64 lanes) owns 64 columns of a
     run and a segment of rows (whole groups of 4 rows, the last segment of
     a run taking the remainder) and marches up it; every run gets segments
     in proportion to its nodes so that the launch holds about waves_per_cu
     work-groups per compute unit (default 16; fewer where a run has too
     few row groups).  Fewer, longer segments re-read fewer halo rows; more
     segments fill the chip and balance uneven batches.  It can step every
     handle on straight metrics;
   - the tiled step: one thread per node, 64 x 4, 8 or 16 nodes per
     work-group (by default 8, 4 in FP64; goc_lbm_set_tile) or, on straight
     metrics, 128 x 4 (goc_lbm_set_tile_shape), the moments
     of the tile and its ring in LDS, non-temporal or plain stores, one launch
     over the tiles of every run of the handle.  It steps straight runs,
     with or without MHD, alone or batched (the default for a single run:
     it is the faster form on most sizes; batches start on the march), and
     every run on a 2-D metric or in 16-bit storage (its only form).  The two
     forms agree to rounding.
   goc_lbm_set_launch: waves_per_cu = 0 selects the tiled step;
   waves_per_cu in [0.5, 1024] the march with that plan (GOC_EINVAL
   outside, on a 2-D metric and in 16-bit storage).  Synchronous.
   goc_lbm_launch_info writes out[0] = waves_per_cu (0 for the tiled step),
   out[1] = work-groups per step, out[2] = mean rows per segment (rows per
   tile), out[3] = strips (column tiles), over all runs, out[4] = 1 when the
   tiled step stores non-temporally, else 0, out[5] = columns per tile
   (64 for the march's strips). */
int goc_lbm_set_launch(goc_lbm_t *h, double waves_per_cu);
int goc_lbm_launch_info(const goc_lbm_t *h, double out[6]);
/* Select the tiled step with tiles of `rows` rows (4, 8 or 16, FP64 4 or
   8; 64 columns each, one thread per node) and non-temporal stores
   (nontemporal = 1) or plain ones (0); GOC_EINVAL otherwise.  Taller tiles
   re-read fewer ring rows, shorter ones spread a grid over more
   work-groups; non-temporal stores suit a state larger than the caches
   (the default where one copy of the state exceeds 128 MiB), plain ones a
   state the next step finds in the Infinity Cache.  Synchronous; captured
   step graphs are dropped. */
int goc_lbm_set_tile(goc_lbm_t *h, int32_t rows, int32_t nontemporal);
/* As goc_lbm_set_tile with the tile width too: cols = 64 with the heights
   above, or cols = 128 with rows = 4 (two waves per row of the tile, whose
   longer row pieces suit wide grids larger than the caches; straight
   metrics only); GOC_EINVAL otherwise. */
int goc_lbm_set_tile_shape(goc_lbm_t *h, int32_t cols, int32_t rows, int32_t nontemporal);

/* Autotuner of the step form and launch plan: times trial_steps step
   launches (1..10000, plus one warm-up) for the tiled step at each tile
   shape (64 x 4, 8, 16; FP64 64 x 4, 8; 128 x 4 on straight metrics), with
   non-temporal and with plain stores, and, for straight FP64 / FP32
   handles, the march
   at each waves_per_cu in {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128,
   192, 256, 384, 512}, on the handle's stream; the candidates within 5 %
   of the fastest are timed again with three times the steps (at most
   10000), and the fastest of that second timing is kept (a run on a 2-D
   metric or in 16-bit storage has the tiled step only: its heights are
   timed).  The trials step the state as a run does (each launch reads what
   the previous one wrote) from a device copy of it, which is put back
   afterwards, so the state does not change; the copy is freed before the
   call returns (GOC_ENOMEM when it does not fit).  out[0] = chosen
   waves_per_cu (0: the
   tiled step; its height, stores and width are launch_info's out[2],
   out[4], out[5]),
   out[1] = its
   microseconds per step (second timing), out[2] = microseconds per step of
   the form in use before in the first timing (-1 if it was not a
   candidate), out[3] = number of candidates.  Synchronous. */
int goc_lbm_tune(goc_lbm_t *h, int32_t trial_steps, double out[4]);

/* Post-stream populations in FP64 (the quantities App. E step 1 reads):
   f[9][ny][nx], F[2][ny][nx] (the lagged effective force) and, for MHD,
   g[10][ny][nx] (plane c*5 + a for component c of B).  set takes the same
   layout and encodes it in the storage precision.  Device pointers if
   on_device else host. */
int goc_lbm_get_populations(goc_lbm_t *h, double *f, double *F, double *g, int32_t on_device);
int goc_lbm_set_populations(goc_lbm_t *h, const double *f, const double *F, const double *g,
                            int32_t on_device);

/* Checkpoint in storage precision (host buffer).  get: with buf NULL writes
   the required size to *bytes; otherwise *bytes must be >= that size.
   The blob holds a header (format version 3, storage, run count, step
   counter, the byte sizes of its regions, the step of the last
   initialisation), each run's (nx, ny, mhd), then the raw device state: the
   16-bit reference table, the slots (with MHD, the D2Q5 slots in their
   rows) and the lagged force.  Blobs of another format version are
   refused.
   set: checks the header, the region sizes and every run's shape against
   the handle before copying anything and returns GOC_ESTATE on any
   mismatch (the handle is then unchanged).  Restoring a blob and stepping
   reproduces an uninterrupted run bit for bit. */
int goc_lbm_get_state(goc_lbm_t *h, void *buf, size_t *bytes);
int goc_lbm_set_state(goc_lbm_t *h, const void *buf, size_t bytes);

/* Derived quantities (host out[16]): [0] c_s^2, [1] nu, [2] zeta, [3] q,
   [4] c_sm^2, [5] eta, [6] tau_m, [7] B0, [8] F_ext1, [9] F_ext2,
   [10] h2 on the xi2 = 0 face, [11] on the xi2 = ny face, [12] step count,
   [13] storage bytes per node per step (algorithmic), [14] nx, [15] ny. */
int goc_lbm_derived(const goc_lbm_t *h, double out[16]);
/* The same for run `run` of a batch (GOC_EINVAL outside [0, num_runs)). */
int goc_lbm_derived_run(const goc_lbm_t *h, int32_t run, double out[16]);

/* Metric arrays as used by the kernels (FP64 host): h1, theta11 [nx],
   h2, theta22 [ny]; any pointer may be NULL.  GOC_EINVAL for a run on a
   2-D metric (use goc_lbm_metric_2d). */
int goc_lbm_metric(const goc_lbm_t *h, double *h1, double *th11, double *h2, double *th22);
/* Node metric of run `run` (FP64 host arrays [ny*nx], any may be NULL):
   h1, h2 and the curvature elements theta11 = d1h1/h1^2, theta12 =
   d2h1/(h1 h2), theta21 = d1h2/(h1 h2), theta22 = d2h2/h2^2 (Sec. 2.1), for
   straight and 2-D metrics alike. */
int goc_lbm_metric_2d(const goc_lbm_t *h, int32_t run, double *h1, double *h2, double *th11, double *th12,
                      double *th21, double *th22);

void goc_lbm_destroy(goc_lbm_t *h);
const char *goc_lbm_last_error(void);

/* ---- batched form --------------------------------------------------------
 * nruns independent runs (each its own grid, metric and parameters, same
 * storage) advanced by one kernel launch per step over a shared work list;
 * blocks of steps are captured in a HIP graph.  The arrays grid[], metric[]
 * and params[] have nruns entries. */
int goc_lbm_create_batch(goc_lbm_t **out, int32_t nruns, const goc_grid *grid,
                         const goc_metric *metric, const goc_params *params, int32_t storage,
                         void *stream);
/* Fields of one run of a batch, as goc_lbm_moments. */
int goc_lbm_moments_run(goc_lbm_t *h, int32_t run, double *rho, double *u, double *B,
                        int32_t on_device);
/* Populations of one run of a batch, as goc_lbm_get_populations. */
int goc_lbm_get_populations_run(goc_lbm_t *h, int32_t run, double *f, double *F, double *g,
                                int32_t on_device);
int32_t goc_lbm_num_runs(const goc_lbm_t *h);

#ifdef __cplusplus
}
#endif
#endif /* GOC_LBM_H */
