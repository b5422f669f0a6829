/*
 * roeam_oracle.h -- FP64 CPU oracle for the Roe-AM finite-volume Euler solver
 * on structured 2-D grids (Li, Ren, Gu: "An Improved Roe Scheme for All
 * Mach-Number Flows Simultaneously Curing Known Problems", arXiv 1711.09272).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU path is checked against.  It shares no code, header, table or
 * constant with the HIP library.  Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark may load it.
 *
 * Layout: conserved state q is [4 + ns][ny][nx] row-major FP64, rows (rho,
 * rho*u, rho*v, rho*E) followed by the ns transported scalars rho*k_m of
 * Eq. (85) (ns = orc_grid.nscalars, 0 .. ORC_MAX_SCALARS).  Node coordinates
 * are [ny+1][nx+1].
 *
 * Parity unpinned (documented readings, checked only oracle == GPU): the
 * modified-entropy-fix / rotated-Riemann term of Eq. (86) (readings D6-D8),
 * the expansion-shock weight of Eq. (92) (reading D2), MUSCL-minmod
 * details, the slip-wall ghost rule and the time-step rule.
 */
#ifndef ROEAM_ORACLE_H
#define ROEAM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary kinds (the paper names none; the test configurations do).
 * ORC_BC_MOVING (uniform grids): a side split at a + b t along it (cell-centre
 * coordinate, x for south/north, y for west/east, t = orc_grid.t_bc): below the
 * split its split_lo kind, either the side's Dirichlet state bc_state or a slip
 * wall; above it its split_hi kind, either a Dirichlet state bc_state_hi or a
 * slip wall.  The double-Mach reflection (Sec. 7.4) needs it (a wall that starts
 * at x = 1/6 and a top boundary that follows the exact incident shock), and so
 * does the supersonic corner (Sec. 7.3: the step's face below the corner, the
 * inflow channel above it). */
enum { ORC_BC_PERIODIC = 0, ORC_BC_TRANSMISSIVE = 1, ORC_BC_SLIPWALL = 2, ORC_BC_DIRICHLET = 3, ORC_BC_MOVING = 4 };
/* Sides. */
enum { ORC_WEST = 0, ORC_EAST = 1, ORC_SOUTH = 2, ORC_NORTH = 3 };
/* Numerical flux families. */
enum { ORC_SCHEME_ROEAM = 0, ORC_SCHEME_ROE = 1, ORC_SCHEME_ROE_HARTEN = 2 };

/* Variant bits: alternative readings of ambiguous passages and the paper's
 * ablations of Sec. 7.  All zero = the Roe-AM scheme of Eqs. (85)-(109) with
 * the default readings. */
#define ORC_V_XI_UNGATED    (1u << 0) /* xi as printed in Eq. (86) instead of the Eq. (68) gate   */
#define ORC_V_EXPFIX_F8     (1u << 1) /* f^8(Mbar) weight of Eq. (73) instead of f(Mbar), Eq. (92)  */
#define ORC_V_CLAMP_UPRIME  (1u << 2) /* clamp |U|' at zero                                        */
#define ORC_V_NO_EQ92       (1u << 3) /* |U|' = |U| (ablation of Fig. 3b / Fig. 8d)                */
#define ORC_V_XI_ROE        (1u << 4) /* xi = |U| of Eq. (13) (Fig. 6d)                             */
#define ORC_V_DUP_ROE       (1u << 5) /* dU_p of Eq. (17) (Fig. 6d, 6e, 11c)                        */
#define ORC_V_XI_EQ46       (1u << 6) /* xi = |U_R+U_L|/2 of Eq. (46): no velocity positivity (6f)  */
#define ORC_V_DUP_ZERO      (1u << 7) /* dU_p = 0 (Fig. 11b)                                        */

typedef struct {
    double gamma;     /* ratio of specific heats, Eq. (54)                       */
    double cfl;       /* Courant number of the time-step rule                     */
    double mach_ref;  /* global reference Mach number of Eq. (101)               */
    double u_ref;     /* reference speed of Eq. (108)                             */
    double eps1;      /* switch of Eq. (111), 0 or 1                              */
    double eps2;      /* entropy-fix constant of Eq. (112)                        */
    double eps_lambda;/* Harten constant of Eq. (115) (Roe + entropy fix only)   */
    int s1_mode;      /* 0: detector of Eqs. (95)-(97); 1: s1 = 1 (Eq. 110)       */
    int order;        /* 1: piecewise constant; 2: MUSCL-minmod                   */
    int time_scheme;  /* 0: forward Euler; 1: SSP-RK3 (Shu-Osher); 2: four-stage RK */
    int scheme;       /* ORC_SCHEME_*                                             */
    unsigned variant; /* ORC_V_* bits                                             */
} orc_params;

/* Transported scalars (the rho k rows of Eq. 85) a 2-D grid may carry. */
#define ORC_MAX_SCALARS 2

typedef struct {
    int nx, ny;
    int metric;            /* 0: uniform dx, dy; 1: node coordinates            */
    double dx, dy;
    const double *xn, *yn; /* metric 1: [ny+1][nx+1]                            */
    int bc[4];             /* west, east, south, north                          */
    double bc_state[4][4]; /* Dirichlet conserved state per side                */
    int nscalars;          /* transported scalars, 0 .. ORC_MAX_SCALARS          */
    double bc_scalar[4][ORC_MAX_SCALARS]; /* Dirichlet rho k_m per side          */
    double split_a[4], split_b[4]; /* ORC_BC_MOVING: split at a + b t          */
    int split_hi[4];               /* ORC_BC_MOVING: kind above the split       */
    double bc_state_hi[4][4];      /* ORC_BC_MOVING: Dirichlet state above it   */
    double t_bc;           /* time of moving boundaries for orc_residual; orc_run
                              uses the time of each stage's input state          */
    int split_lo[4];       /* ORC_BC_MOVING: kind below the split               */
} orc_grid;

/* Every intermediate of one face evaluation, for property tests. */
typedef struct {
    double UL, UR, U, dU, dp;          /* normal velocities and jumps            */
    double rho, u, v, H, c;            /* Roe averages                           */
    double M, Mbar, theta, ct, Ut;     /* Eqs. (93), (94), (101), (99), (100)    */
    double absUp;                      /* |U|' of Eq. (92)                       */
    double s1, fef, frr;               /* Eqs. (95), (102), (103)                */
    double xi, dpp, dpu, dUp, dUuR, dUuL; /* Eqs. (86)-(91)                      */
} orc_face_diag;

typedef struct {
    double t, dt_last, max_rate;
    long steps;
    int nonphys;
    long neg_uprime_faces;  /* faces where |U|' < 0 was seen (reading D4)       */
} orc_run_stats;

/* Eq. (98). */
double orc_f(double phi);
/* Eq. (97): detector ratio of two neighbouring cells. */
double orc_detector_P(double pA, double rhoA, double pB, double rhoB);
/* One face: W = (rho, u, v, p) on each side, unit normal (nx, ny), switch s1.
 * Writes the numerical flux per unit face length; diag may be NULL. */
void orc_face_flux(const orc_params *prm, const double WL[4], const double WR[4],
                   double nx, double ny, double s1, double F[4], orc_face_diag *diag);
/* One face with ns transported scalars: W = (rho, u, v, p, k_1 .. k_ns) on
 * each side, F = 4 + ns rows.  The scalar rows are those of Eq. (85): central
 * U rho k, minus half of xi Delta(rho k) + dU_p rho^ k^ + dU_uR (rho k)_R +
 * dU_uL (rho k)_L (classical Roe: xi Delta(rho k) + (dU_u + dU_p) rho^ k^),
 * with k^ the sqrt(rho)-weighted Roe average. */
void orc_face_flux_sc(const orc_params *prm, const double *WL, const double *WR, double nx, double ny,
                      double s1, int ns, double *F);
/* Physical face flux of Eq. (4) for one state. */
void orc_physical_flux(double gamma, const double W[4], double nx, double ny, double F[4]);

/* R = dQ/dt.  q, r: [4 + nscalars][ny][nx].  scale (nullable): per-cell sum over the
 * four faces of |F_k| |S| / Omega, used by the cancellation-aware error norm.
 * Returns 0, or -4 if a cell has rho <= 0, p <= 0 or a non-finite value. */
int orc_residual(const orc_params *prm, const orc_grid *g, const double *q, double *r, double *scale);
/* Diagnostic of Sec. 7.2 (Fig. 7): the rotated Mach number f_rr / c of
 * Eqs. (103)-(109) on every i-face [ny][nx+1] and j-face [ny+1][nx] (either
 * pointer nullable), from the same face states as orc_residual. */
int orc_rotated_mach(const orc_params *prm, const orc_grid *g, const double *q, double *frr_x, double *frr_y);
/* Largest explicit rate lambda over cells (time-step rule). */
int orc_max_rate(const orc_params *prm, const orc_grid *g, const double *q, double *max_rate);
/* Advance q in place: nsteps steps or until t reaches t_end (t_end <= 0: no
 * clip).  Returns 0 or -4 (non-physical state: q undefined). */
int orc_run(const orc_params *prm, const orc_grid *g, double *q, long nsteps, double t_end,
            orc_run_stats *stats);
/* Cell areas [ny][nx] (shoelace); face vectors for tests. */
void orc_cell_areas(const orc_grid *g, double *omega);

/* ------------------------------------------------------------------------ */
/* 3-D, uniform Cartesian grids (roeam_oracle3d.c)                          */
/* ------------------------------------------------------------------------ */
/* Sides in 3-D: west, east (x), south, north (y), bottom, top (z). */
enum { ORC_BOTTOM = 4, ORC_TOP = 5 };

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    int bc[6];             /* west, east, south, north, bottom, top            */
    double bc_state[6][5]; /* Dirichlet conserved state per side              */
    int nscalars;          /* transported scalars, 0 .. ORC_MAX_SCALARS          */
    double bc_scalar[6][ORC_MAX_SCALARS]; /* Dirichlet rho k_m per side          */
} orc3_grid;

/* Layout: q is [5 + ns][nz][ny][nx], rows (rho, rho u, rho v, rho w, rho E)
 * and the ns transported scalars rho k_m. */
void orc3_physical_flux(double gamma, const double W[5], const double n[3], double F[5]);
/* Eqs. (85)-(109) (or the classical schemes) in 3-D, per unit face area;
 * W = (rho, u, v, w, p), n a unit normal. */
void orc3_face_flux(const orc_params *prm, const double WL[5], const double WR[5], const double n[3], double s1,
                    double F[5]);
/* The same with ns transported scalars: W = (rho, u, v, w, p, k_1 ..), F = 5 + ns rows
 * (the rho k rows of Eq. 85 as printed, in three dimensions). */
void orc3_face_flux_sc(const orc_params *prm, const double *WL, const double *WR, const double n[3], double s1,
                       int ns, double *F);
int orc3_residual(const orc_params *prm, const orc3_grid *g, const double *q, double *r, double *scale);
int orc3_max_rate(const orc_params *prm, const orc3_grid *g, const double *q, double *max_rate);
int orc3_run(const orc_params *prm, const orc3_grid *g, double *q, long nsteps, double t_end, orc_run_stats *stats);

/* Threads used by the row loops (OpenMP); the results are bitwise the same
 * for any count. */
void orc_set_threads(int n);
int orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
