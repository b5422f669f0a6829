/*
 * roeam_oracle.c -- plain FP64 CPU oracle of the Roe-AM finite-volume solver
 * (arXiv 1711.09272), 2-D structured grids.
 *
 * TEST INFRASTRUCTURE ONLY: slow and obviously correct on purpose.  It is
 * compiled with -O2 -ffp-contract=off, uses libm sqrt and true division, and
 * fixed loop and summation orders.  It shares nothing with the HIP library.
 *
 * 2-D specialisation of the paper's 3-D equations: w = 0, n_z = 0, four
 * conserved rows (rho, rho u, rho v, rho E).  Face quantities without a
 * subscript are Roe averages (Sec. 2.2, remark after Eq. 6; Sec. 4.2 says the
 * Roe average is the one in use).
 */
#include "roeam_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ENONPHYS (-4)
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* sign with sign(0) = 0 (reading D5). */
static double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }
static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

/* Eq. (98): f(phi) = min(phi sqrt(4 + (1 - phi^2)^2) / (1 + phi^2), 1). */
double orc_f(double phi)
{
    double one_minus = 1.0 - phi * phi;
    double val = phi * sqrt(4.0 + one_minus * one_minus) / (1.0 + phi * phi);
    return dmin(val, 1.0);
}

/* f^8 is the eighth power of f (reading D3), by repeated squaring. */
static double pow8(double x)
{
    double x2 = x * x;
    double x4 = x2 * x2;
    return x4 * x4;
}

/* Eq. (97): P = min(pA/pB, pB/pA, rhoA/rhoB, rhoB/rhoA). */
double orc_detector_P(double pA, double rhoA, double pB, double rhoB)
{
    double a = dmin(pA / pB, pB / pA);
    double b = dmin(rhoA / rhoB, rhoB / rhoA);
    return dmin(a, b);
}

/* Ideal gas (Eq. 54 and the definitions of E and H after Eq. 1):
 * rho E = p/(gamma-1) + rho |V|^2 / 2,  H = (rho E + p) / rho. */
static double total_enthalpy(double gamma, const double W[4])
{
    double rhoE = W[3] / (gamma - 1.0) + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2]);
    return (rhoE + W[3]) / W[0];
}

/* Eq. (4): Fbar = U (rho, rho u, rho v, rho H) + p (0, nx, ny, 0). */
void orc_physical_flux(double gamma, const double W[4], double nx, double ny, double F[4])
{
    double U = nx * W[1] + ny * W[2];
    double H = total_enthalpy(gamma, W);
    F[0] = U * W[0];
    F[1] = U * (W[0] * W[1]) + W[3] * nx;
    F[2] = U * (W[0] * W[2]) + W[3] * ny;
    F[3] = U * (W[0] * H);
}

/* Rotated-Riemann speed f_rr of Eqs. (103)-(109), 2-D.
 * n1 from the reconstructed velocity jump (Eq. 108, reading D6); n2 is the
 * unit vector along (n1 x n) x n1 (reading D7); U1, U2 use the Roe-averaged
 * velocity (reading D8). */
static double rotated_speed(double nx, double ny, double du, double dv, double u, double v,
                            double u_ref)
{
    double dV = sqrt(du * du + dv * dv);
    double n1x, n1y;
    if (dV < 1e-5 * u_ref || dV == 0.0) {
        n1x = nx;
        n1y = ny;
    } else {
        n1x = du / dV;
        n1y = dv / dV;
    }
    double alpha1 = n1x * nx + n1y * ny;  /* Eq. (106) */
    double U1 = n1x * u + n1y * v;        /* Eq. (104) */
    /* (n1 x n) x n1 = s (-n1y, n1x) with s the z-component of n1 x n. */
    double s = n1x * ny - n1y * nx;
    double a2U2 = 0.0;
    if (s != 0.0) {
        double n2x = -sgn(s) * n1y, n2y = sgn(s) * n1x;
        double alpha2 = n2x * nx + n2y * ny; /* Eq. (107) */
        double U2 = n2x * u + n2y * v;       /* Eq. (105) */
        a2U2 = alpha2 * U2;
    }
    return fabs(alpha1 * U1) + fabs(a2U2);  /* Eq. (103) */
}

void orc_face_flux(const orc_params *prm, const double WL[4], const double WR[4],
                   double nx, double ny, double s1, double F[4], orc_face_diag *diag)
{
    const double g = prm->gamma;
    const double rL = WL[0], uL = WL[1], vL = WL[2], pL = WL[3];
    const double rR = WR[0], uR = WR[1], vR = WR[2], pR = WR[3];

    /* Side quantities, Eq. (4). */
    double UL = nx * uL + ny * vL;
    double UR = nx * uR + ny * vR;
    double HL = total_enthalpy(g, WL);
    double HR = total_enthalpy(g, WR);
    double PsiL[4] = {rL, rL * uL, rL * vL, rL * HL};
    double PsiR[4] = {rR, rR * uR, rR * vR, rR * HR};
    double FbL[4], FbR[4];
    orc_physical_flux(g, WL, nx, ny, FbL);
    orc_physical_flux(g, WR, nx, ny, FbR);

    /* Roe averages (Sec. 4.2): sqrt(rho) weights. */
    double rr = sqrt(rR / rL);
    double rho = rr * rL;
    double u = (uL + rr * uR) / (1.0 + rr);
    double v = (vL + rr * vR) / (1.0 + rr);
    double H = (HL + rr * HR) / (1.0 + rr);
    double c = sqrt((g - 1.0) * (H - 0.5 * (u * u + v * v)));
    double U = nx * u + ny * v;
    double PsiHat[4] = {rho, rho * u, rho * v, rho * H};

    double dU = UR - UL;
    double dp = pR - pL;
    double pvec[4] = {0.0, nx, ny, 0.0};
    double diss[4];

    orc_face_diag d;
    memset(&d, 0, sizeof d);
    d.UL = UL; d.UR = UR; d.U = U; d.dU = dU; d.dp = dp;
    d.rho = rho; d.u = u; d.v = v; d.H = H; d.c = c;

    if (prm->scheme == ORC_SCHEME_ROE || prm->scheme == ORC_SCHEME_ROE_HARTEN) {
        /* Classical Roe in the scale form, Eq. (7) with Eqs. (8)-(12) and the
         * eigenvalues of Eq. (6); Harten's fix of Eqs. (114)-(115) optional. */
        double l1 = fabs(U), l4 = fabs(U - c), l5 = fabs(U + c);
        if (prm->scheme == ORC_SCHEME_ROE_HARTEN) {
            double h = prm->eps_lambda * dmax(l1, dmax(l4, l5));
            if (l1 < h) l1 = 0.5 * (l1 * l1 / h + h);
            if (l4 < h) l4 = 0.5 * (l4 * l4 / h + h);
            if (l5 < h) l5 = 0.5 * (l5 * l5 / h + h);
        }
        double xi = l1;                                      /* Eq. (8)  */
        double dpu = (0.5 * (l5 + l4) - l1) * rho * dU;      /* Eq. (9)  */
        double dpp = 0.5 * (l5 - l4) * dp / c;               /* Eq. (10) */
        double dUu = 0.5 * (l5 - l4) * dU / c;               /* Eq. (11) */
        double dUp = (0.5 * (l5 + l4) - l1) * dp / (rho * c * c); /* Eq. (12) */
        /* Eq. (7): conserved jump with rho E, pressure vector (0, n, U). */
        double rEL = pL / (g - 1.0) + 0.5 * rL * (uL * uL + vL * vL);
        double rER = pR / (g - 1.0) + 0.5 * rR * (uR * uR + vR * vR);
        double dQ[4] = {rR - rL, rR * uR - rL * uL, rR * vR - rL * vL, rER - rEL};
        double pv7[4] = {0.0, nx, ny, U};
        for (int k = 0; k < 4; ++k)
            diss[k] = xi * dQ[k] + (dpu + dpp) * pv7[k] + (dUu + dUp) * PsiHat[k];
        d.xi = xi; d.dpu = dpu; d.dpp = dpp; d.dUp = dUp; d.dUuR = 0.5 * dUu; d.dUuL = 0.5 * dUu;
        d.absUp = fabs(U); d.s1 = s1; d.Mbar = fabs(U) / c;
    } else {
        const unsigned var = prm->variant;
        /* Mach numbers, Eqs. (93)-(94); f and f^8 of Eq. (98). */
        double cL = sqrt(g * pL / rL), cR = sqrt(g * pR / rR);
        double M = 0.5 * (sqrt(uL * uL + vL * vL) / cL + sqrt(uR * uR + vR * vR) / cR);
        double Mbar = fabs(U) / c;
        double fM = orc_f(M), f8M = pow8(fM);
        double fMbar = orc_f(Mbar), f8Mbar = pow8(fMbar);

        /* Preconditioning quantities, Eqs. (99)-(101). */
        double mr2 = prm->mach_ref * prm->mach_ref;
        double theta = dmin(dmax(mr2, M * M), 1.0);
        double ct = 0.5 * sqrt(4.0 * c * c * theta + (1.0 - theta) * (1.0 - theta) * U * U);
        double Ut = 0.5 * (1.0 + theta) * U;

        /* Expansion-shock fix, Eq. (92) (weight f, reading D2). */
        double absU = fabs(U);
        double absUp = absU;
        if (!(var & ORC_V_NO_EQ92)) {
            double w = (var & ORC_V_EXPFIX_F8) ? f8Mbar : fMbar;
            absUp = absU - w * (sgn(U + c) - sgn(U - c)) * dmax(0.0, dU) / 4.0;
        }
        if (var & ORC_V_CLAMP_UPRIME) absUp = dmax(absUp, 0.0);

        /* Basic upwind dissipation, Eq. (86) with the Eq. (68) gate (D1). */
        double gate = (var & ORC_V_XI_UNGATED) ? 1.0 : (1.0 - f8Mbar);
        double xi_pos = fabs(0.5 * (UR + UL)) + gate * (0.5 * dU);
        double fef = prm->eps2 * c;                                       /* Eq. (102) */
        double frr = rotated_speed(nx, ny, uR - uL, vR - vL, u, v, prm->u_ref);
        double xi_fix = prm->eps1 * (1.0 - f8Mbar) * f8M * dmin(fef, frr);
        double xi = dmax(xi_pos, xi_fix);
        if (var & ORC_V_XI_EQ46) xi = fabs(UR + UL) / 2.0;               /* Eq. (46) */
        if (var & ORC_V_XI_ROE) xi = absU;                               /* Eq. (13) */

        /* Eqs. (87)-(91). */
        double dpp = sgn(U) * dmin(absUp, c) * dp / c;
        double dpu = (1.0 - s1 + s1 * fM) * dmax(0.0, c - absUp) * rho * dU;
        double bracket = dmax(0.0, ct - absUp)
                       + (1.0 - theta) * (absUp - U / (2.0 * ct) * sgn(Ut) * dmin(fabs(Ut), ct));
        double dUp = s1 * (1.0 - f8M) * bracket * dp / (rho * theta * c * c);
        if (var & ORC_V_DUP_ROE) dUp = dmax(0.0, c - absU) * dp / (rho * c * c); /* Eq. (17) */
        if (var & ORC_V_DUP_ZERO) dUp = 0.0;
        double dUuR = 0.5 * sgn(U) * dmin(absUp, c) * dU / c;
        double dUuL = 0.5 * sgn(U) * dmin(absUp, c) * dU / c;

        /* Eq. (85), 2-D, energy row with Delta(rho H) and 0 in the pressure
         * vector (Eq. 49 and the remark after it). */
        double dPsi[4];
        for (int k = 0; k < 4; ++k) dPsi[k] = PsiR[k] - PsiL[k];
        for (int k = 0; k < 4; ++k)
            diss[k] = xi * dPsi[k] + (dpp + dpu) * pvec[k] + dUp * PsiHat[k]
                    + dUuR * PsiR[k] + dUuL * PsiL[k];

        d.M = M; d.Mbar = Mbar; d.theta = theta; d.ct = ct; d.Ut = Ut; d.absUp = absUp;
        d.s1 = s1; d.fef = fef; d.frr = frr;
        d.xi = xi; d.dpp = dpp; d.dpu = dpu; d.dUp = dUp; d.dUuR = dUuR; d.dUuL = dUuL;
    }

    /* Eq. (2)-(3): central term minus half the dissipation braces. */
    for (int k = 0; k < 4; ++k) F[k] = 0.5 * (FbL[k] + FbR[k]) - 0.5 * diss[k];
    if (diag) *diag = d;
}

/* Eq. (85) with the transported-scalar rows (rho k, ...): the same xi,
 * dU_p, dU_u of the face; rho^ k^ with the Roe average of k (sqrt(rho)
 * weights, like u, v and H); no pressure term. */
void orc_face_flux_sc(const orc_params *prm, const double *WL, const double *WR, double nx, double ny,
                      double s1, int ns, double *F)
{
    orc_face_diag d;
    orc_face_flux(prm, WL, WR, nx, ny, s1, F, &d);
    const double rL = WL[0], rR = WR[0];
    const double rr = sqrt(rR / rL);
    const int classical = prm->scheme == ORC_SCHEME_ROE || prm->scheme == ORC_SCHEME_ROE_HARTEN;
    for (int m = 0; m < ns; ++m) {
        double kL = WL[4 + m], kR = WR[4 + m];
        double PsiL = rL * kL, PsiR = rR * kR;
        double khat = (kL + rr * kR) / (1.0 + rr);
        double diss;
        if (classical)
            diss = d.xi * (PsiR - PsiL) + (d.dUuR + d.dUuL + d.dUp) * (d.rho * khat); /* Eq. (7) */
        else
            diss = d.xi * (PsiR - PsiL) + d.dUp * (d.rho * khat) + d.dUuR * PsiR + d.dUuL * PsiL;
        F[4 + m] = 0.5 * (d.UL * PsiL + d.UR * PsiR) - 0.5 * diss;
    }
}

/* ------------------------------------------------------------------------ */
/* Grid, ghosts and the residual                                             */
/* ------------------------------------------------------------------------ */

/* Largest number of components of a cell: (rho, u, v, p) and the scalars k_m. */
#define ORC_MAXC (4 + ORC_MAX_SCALARS)

typedef struct {
    int nx, ny, NX, NY;   /* NX = nx + 4, NY = ny + 4 (two ghost layers) */
    int nc;               /* components: 4 + scalars */
    double *W;            /* primitives [nc][NY][NX]: rho, u, v, p, k_1 .. */
} prim_field;

#define PIDX(pf, k, i, j) ((size_t)(k) * (pf)->NX * (pf)->NY + (size_t)((j) + 2) * (pf)->NX + (size_t)((i) + 2))

/* (rho, rho u, rho v, rho E, rho k_1 ..) -> (rho, u, v, p, k_1 ..); nc components. */
static void conserved_to_prim(double gamma, const double *Q, double *W, int nc)
{
    double rho = Q[0];
    double u = Q[1] / rho, v = Q[2] / rho;
    double p = (gamma - 1.0) * (Q[3] - 0.5 * rho * (u * u + v * v));
    W[0] = rho; W[1] = u; W[2] = v; W[3] = p;
    for (int k = 4; k < nc; ++k) W[k] = Q[k] / rho;
}

static int physical(const double W[4])
{
    for (int k = 0; k < 4; ++k)
        if (!isfinite(W[k])) return 0;
    return W[0] > 0.0 && W[3] > 0.0;
}

/* Face vector of the i-face between cells (i-1, j) and (i, j), and of the
 * j-face between (i, j-1) and (i, j); the vector points from the lower to the
 * higher index and its length is the face length. */
static void xface_vector(const orc_grid *g, int i, int j, double S[2])
{
    if (g->metric == 0) { S[0] = g->dy; S[1] = 0.0; return; }
    int NXn = g->nx + 1;
    double ddx = g->xn[(size_t)(j + 1) * NXn + i] - g->xn[(size_t)j * NXn + i];
    double ddy = g->yn[(size_t)(j + 1) * NXn + i] - g->yn[(size_t)j * NXn + i];
    S[0] = ddy; S[1] = -ddx;
}
static void yface_vector(const orc_grid *g, int i, int j, double S[2])
{
    if (g->metric == 0) { S[0] = 0.0; S[1] = g->dx; return; }
    int NXn = g->nx + 1;
    double ddx = g->xn[(size_t)j * NXn + i + 1] - g->xn[(size_t)j * NXn + i];
    double ddy = g->yn[(size_t)j * NXn + i + 1] - g->yn[(size_t)j * NXn + i];
    S[0] = -ddy; S[1] = ddx;
}
static void unit_normal(const orc_grid *g, const double S[2], double n[2], double *len)
{
    if (g->metric == 0) {
        /* axis-aligned: exact unit vectors */
        if (S[1] == 0.0) { n[0] = 1.0; n[1] = 0.0; *len = S[0]; }
        else { n[0] = 0.0; n[1] = 1.0; *len = S[1]; }
        return;
    }
    *len = sqrt(S[0] * S[0] + S[1] * S[1]);
    n[0] = S[0] / *len;
    n[1] = S[1] / *len;
}

/* Cell area: shoelace formula over the four corner nodes. */
static double cell_area(const orc_grid *g, int i, int j)
{
    if (g->metric == 0) return g->dx * g->dy;
    int NXn = g->nx + 1;
    const double *x = g->xn, *y = g->yn;
    double x00 = x[(size_t)j * NXn + i], y00 = y[(size_t)j * NXn + i];
    double x10 = x[(size_t)j * NXn + i + 1], y10 = y[(size_t)j * NXn + i + 1];
    double x11 = x[(size_t)(j + 1) * NXn + i + 1], y11 = y[(size_t)(j + 1) * NXn + i + 1];
    double x01 = x[(size_t)(j + 1) * NXn + i], y01 = y[(size_t)(j + 1) * NXn + i];
    return 0.5 * ((x11 - x00) * (y01 - y10) - (x01 - x10) * (y11 - y00));
}

void orc_cell_areas(const orc_grid *g, double *omega)
{
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) omega[(size_t)j * g->nx + i] = cell_area(g, i, j);
}

/* Slip wall: mirror the velocity about the wall-face unit normal. */
static void reflect(double W[4], const double n[2])
{
    double vn = W[1] * n[0] + W[2] * n[1];
    W[1] = W[1] - 2.0 * vn * n[0];
    W[2] = W[2] - 2.0 * vn * n[1];
}

static void get_prim(const prim_field *pf, int i, int j, double *W)
{
    for (int k = 0; k < pf->nc; ++k) W[k] = pf->W[PIDX(pf, k, i, j)];
}
static void set_prim(prim_field *pf, int i, int j, const double *W)
{
    for (int k = 0; k < pf->nc; ++k) pf->W[PIDX(pf, k, i, j)] = W[k];
}

/* Dirichlet state of a side (or, hi != 0, its state above a moving split),
 * primitive, scalars included. */
static void dirichlet_prim_of(const orc_params *prm, const orc_grid *g, int side, int hi, int nc, double *W)
{
    double Q[ORC_MAXC];
    for (int k = 0; k < 4; ++k) Q[k] = hi ? g->bc_state_hi[side][k] : g->bc_state[side][k];
    for (int k = 4; k < nc; ++k) Q[k] = g->bc_scalar[side][k - 4];
    conserved_to_prim(prm->gamma, Q, W, nc);
}
static void dirichlet_prim(const orc_params *prm, const orc_grid *g, int side, int nc, double *W)
{
    dirichlet_prim_of(prm, g, side, 0, nc, W);
}

/* A moving-split side at coordinate xc (cell centre) along it: below the
 * split point a + b t_bc the lo kind, above it the hi kind; a Dirichlet kind
 * fills W (the side's state below, bc_state_hi above) and returns -1, a slip
 * wall is returned. */
static int moving_side(const orc_params *prm, const orc_grid *g, int side, double xc, int nc, double *W)
{
    const int lo = xc < g->split_a[side] + g->split_b[side] * g->t_bc;
    if ((lo ? g->split_lo[side] : g->split_hi[side]) == ORC_BC_DIRICHLET) {
        dirichlet_prim_of(prm, g, side, !lo, nc, W);
        return -1;
    }
    return ORC_BC_SLIPWALL;
}

/* Ghost cells, two layers.  Boundary conditions are not in the paper; the
 * test configurations name them.  x-ghosts are filled for interior rows
 * first, then y-ghosts for every column including the x-ghost columns, which
 * defines the corners. */
static void fill_ghosts(const orc_params *prm, const orc_grid *g, prim_field *pf)
{
    const int nx = g->nx, ny = g->ny, nc = pf->nc;
    double W[ORC_MAXC], n[2], S[2], len;
    for (int j = 0; j < ny; ++j) {
        for (int gi = 1; gi <= 2; ++gi) {
            /* west ghost i = -gi */
            int kind = g->bc[ORC_WEST];
            if (kind == ORC_BC_MOVING) kind = moving_side(prm, g, ORC_WEST, (j + 0.5) * g->dy, nc, W);
            switch (kind) {
            case -1: break;
            case ORC_BC_PERIODIC: get_prim(pf, nx - gi, j, W); break;
            case ORC_BC_TRANSMISSIVE: get_prim(pf, 0, j, W); break;
            case ORC_BC_SLIPWALL:
                get_prim(pf, gi - 1, j, W);
                xface_vector(g, 0, j, S); unit_normal(g, S, n, &len); reflect(W, n); break;
            default: dirichlet_prim(prm, g, ORC_WEST, nc, W); break;
            }
            set_prim(pf, -gi, j, W);
            /* east ghost i = nx - 1 + gi */
            kind = g->bc[ORC_EAST];
            if (kind == ORC_BC_MOVING) kind = moving_side(prm, g, ORC_EAST, (j + 0.5) * g->dy, nc, W);
            switch (kind) {
            case -1: break;
            case ORC_BC_PERIODIC: get_prim(pf, gi - 1, j, W); break;
            case ORC_BC_TRANSMISSIVE: get_prim(pf, nx - 1, j, W); break;
            case ORC_BC_SLIPWALL:
                get_prim(pf, nx - gi, j, W);
                xface_vector(g, nx, j, S); unit_normal(g, S, n, &len); reflect(W, n); break;
            default: dirichlet_prim(prm, g, ORC_EAST, nc, W); break;
            }
            set_prim(pf, nx - 1 + gi, j, W);
        }
    }
    for (int i = -2; i < nx + 2; ++i) {
        int ic = i < 0 ? 0 : (i > nx - 1 ? nx - 1 : i); /* wall normal of the nearest column */
        for (int gj = 1; gj <= 2; ++gj) {
            int kind = g->bc[ORC_SOUTH];
            if (kind == ORC_BC_MOVING) kind = moving_side(prm, g, ORC_SOUTH, (i + 0.5) * g->dx, nc, W);
            switch (kind) {
            case -1: break;
            case ORC_BC_PERIODIC: get_prim(pf, i, ny - gj, W); break;
            case ORC_BC_TRANSMISSIVE: get_prim(pf, i, 0, W); break;
            case ORC_BC_SLIPWALL:
                get_prim(pf, i, gj - 1, W);
                yface_vector(g, ic, 0, S); unit_normal(g, S, n, &len); reflect(W, n); break;
            default: dirichlet_prim(prm, g, ORC_SOUTH, nc, W); break;
            }
            set_prim(pf, i, -gj, W);
            kind = g->bc[ORC_NORTH];
            if (kind == ORC_BC_MOVING) kind = moving_side(prm, g, ORC_NORTH, (i + 0.5) * g->dx, nc, W);
            switch (kind) {
            case -1: break;
            case ORC_BC_PERIODIC: get_prim(pf, i, gj - 1, W); break;
            case ORC_BC_TRANSMISSIVE: get_prim(pf, i, ny - 1, W); break;
            case ORC_BC_SLIPWALL:
                get_prim(pf, i, ny - gj, W);
                yface_vector(g, ic, ny, S); unit_normal(g, S, n, &len); reflect(W, n); break;
            default: dirichlet_prim(prm, g, ORC_NORTH, nc, W); break;
            }
            set_prim(pf, i, ny - 1 + gj, W);
        }
    }
}

/* minmod limiter: 0 if the slopes disagree in sign, else the smaller one. */
static double minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return sgn(a) * dmin(fabs(a), fabs(b));
}

/* Face states from four cells m2, m1 | p0, p1 along the face normal.
 * First order (Sec. 7.1): the two adjacent cells.  MUSCL-minmod on the
 * primitive variables (not in the paper; named by the test configurations). */
static void reconstruct(int order, int nc, const double *m2, const double *m1, const double *p0,
                        const double *p1, double *WL, double *WR)
{
    for (int k = 0; k < nc; ++k) {
        if (order == 1) {
            WL[k] = m1[k];
            WR[k] = p0[k];
        } else {
            WL[k] = m1[k] + 0.5 * minmod(m1[k] - m2[k], p0[k] - m1[k]);
            WR[k] = p0[k] - 0.5 * minmod(p0[k] - m1[k], p1[k] - p0[k]);
        }
    }
}

static double P_between(const prim_field *pf, int ia, int ja, int ib, int jb)
{
    double A[ORC_MAXC], B[ORC_MAXC];
    get_prim(pf, ia, ja, A);
    get_prim(pf, ib, jb, B);
    return orc_detector_P(A[3], A[0], B[3], B[0]);
}

/* Eqs. (95)-(96) in 2-D: the face and the four transverse faces of its two
 * cells; P from cell-centre values (reading D11). */
static double s1_xface(const orc_params *prm, const prim_field *pf, int i, int j)
{
    if (prm->s1_mode == 1) return 1.0; /* Eq. (110) */
    double a = P_between(pf, i - 1, j, i, j);
    a = dmin(a, P_between(pf, i - 1, j - 1, i - 1, j));
    a = dmin(a, P_between(pf, i - 1, j, i - 1, j + 1));
    a = dmin(a, P_between(pf, i, j - 1, i, j));
    a = dmin(a, P_between(pf, i, j, i, j + 1));
    return pow8(orc_f(a));
}
static double s1_yface(const orc_params *prm, const prim_field *pf, int i, int j)
{
    if (prm->s1_mode == 1) return 1.0;
    double a = P_between(pf, i, j - 1, i, j);
    a = dmin(a, P_between(pf, i - 1, j - 1, i, j - 1));
    a = dmin(a, P_between(pf, i, j - 1, i + 1, j - 1));
    a = dmin(a, P_between(pf, i - 1, j, i, j));
    a = dmin(a, P_between(pf, i, j, i + 1, j));
    return pow8(orc_f(a));
}

static int load_prims(const orc_params *prm, const orc_grid *g, const double *q, prim_field *pf)
{
    const int nx = g->nx, ny = g->ny, nc = pf->nc;
    const size_t plane = (size_t)nx * ny;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            double Q[ORC_MAXC], W[ORC_MAXC];
            for (int k = 0; k < nc; ++k) Q[k] = q[k * plane + c];
            conserved_to_prim(prm->gamma, Q, W, nc);
            if (!physical(W)) bad = 1;
            set_prim(pf, i, j, W);
        }
    if (bad) return ORC_ENONPHYS;
    fill_ghosts(prm, g, pf);
    return 0;
}

static int check_args(const orc_params *prm, const orc_grid *g)
{
    if (!prm || !g) return ORC_EINVAL;
    if (g->nx < 2 || g->ny < 2) return ORC_EINVAL;
    if (!(prm->gamma > 1.0)) return ORC_EINVAL;
    if (prm->scheme == ORC_SCHEME_ROEAM && !(prm->mach_ref > 0.0)) return ORC_EINVAL;
    if (g->metric == 1 && (!g->xn || !g->yn)) return ORC_EINVAL;
    if (prm->order != 1 && prm->order != 2) return ORC_EINVAL;
    if (g->nscalars < 0 || g->nscalars > ORC_MAX_SCALARS) return ORC_EINVAL;
    for (int s = 0; s < 4; ++s) {
        if (g->bc[s] < ORC_BC_PERIODIC || g->bc[s] > ORC_BC_MOVING) return ORC_EINVAL;
        if (g->bc[s] != ORC_BC_MOVING) continue;
        if (g->metric != 0 || g->bc[s ^ 1] == ORC_BC_PERIODIC) return ORC_EINVAL;
        if (g->split_hi[s] != ORC_BC_DIRICHLET && g->split_hi[s] != ORC_BC_SLIPWALL) return ORC_EINVAL;
        if (g->split_lo[s] != ORC_BC_DIRICHLET && g->split_lo[s] != ORC_BC_SLIPWALL) return ORC_EINVAL;
    }
    return 0;
}

/* frr_x, frr_y (nullable): f_rr / c of every i-face [ny][nx+1] and j-face
 * [ny+1][nx] (the rotated Mach number of Eqs. 103-109; 0 where eps1 = 0). */
static int residual_impl_diag(const orc_params *prm, const orc_grid *g, const double *q, double *r,
                              double *scale, long *neg_uprime, double *frr_x, double *frr_y);

static int residual_impl(const orc_params *prm, const orc_grid *g, const double *q, double *r,
                         double *scale, long *neg_uprime)
{
    return residual_impl_diag(prm, g, q, r, scale, neg_uprime, NULL, NULL);
}

static int residual_impl_diag(const orc_params *prm, const orc_grid *g, const double *q, double *r,
                              double *scale, long *neg_uprime, double *frr_x, double *frr_y)
{
    int rc = check_args(prm, g);
    if (rc) return rc;
    const int nx = g->nx, ny = g->ny, nc = 4 + g->nscalars;
    prim_field pf = {nx, ny, nx + 4, ny + 4, nc, NULL};
    pf.W = (double *)malloc(sizeof(double) * nc * (size_t)pf.NX * pf.NY);
    double *Fx = (double *)malloc(sizeof(double) * nc * (size_t)ny * (nx + 1));
    double *Fy = (double *)malloc(sizeof(double) * nc * (size_t)(ny + 1) * nx);
    if (!pf.W || !Fx || !Fy) { free(pf.W); free(Fx); free(Fy); return ORC_ENOMEM; }
    rc = load_prims(prm, g, q, &pf);
    if (rc) { free(pf.W); free(Fx); free(Fy); return rc; }

    /* Rows of faces are independent; with OpenMP they are shared out among
     * threads (each face is computed by one thread with the same arithmetic,
     * so the result does not depend on the thread count). */
    long negc = 0;
    /* i-faces: between (i-1, j) and (i, j), i = 0..nx */
#pragma omp parallel for schedule(static) reduction(+ : negc)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            double m2[ORC_MAXC], m1[ORC_MAXC], p0[ORC_MAXC], p1[ORC_MAXC], WL[ORC_MAXC], WR[ORC_MAXC];
            double F[ORC_MAXC], S[2], n[2], len;
            orc_face_diag d;
            get_prim(&pf, i - 2, j, m2); get_prim(&pf, i - 1, j, m1);
            get_prim(&pf, i, j, p0); get_prim(&pf, i + 1, j, p1);
            reconstruct(prm->order, nc, m2, m1, p0, p1, WL, WR);
            xface_vector(g, i, j, S);
            unit_normal(g, S, n, &len);
            double s1 = s1_xface(prm, &pf, i, j);
            orc_face_flux(prm, WL, WR, n[0], n[1], s1, F, &d);
            if (nc > 4) orc_face_flux_sc(prm, WL, WR, n[0], n[1], s1, nc - 4, F);
            if (d.absUp < 0.0) ++negc;
            if (frr_x) frr_x[(size_t)j * (nx + 1) + i] = d.frr / d.c;
            for (int k = 0; k < nc; ++k) Fx[((size_t)j * (nx + 1) + i) * nc + k] = F[k] * len;
        }
    /* j-faces: between (i, j-1) and (i, j), j = 0..ny */
#pragma omp parallel for schedule(static) reduction(+ : negc)
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double m2[ORC_MAXC], m1[ORC_MAXC], p0[ORC_MAXC], p1[ORC_MAXC], WL[ORC_MAXC], WR[ORC_MAXC];
            double F[ORC_MAXC], S[2], n[2], len;
            orc_face_diag d;
            get_prim(&pf, i, j - 2, m2); get_prim(&pf, i, j - 1, m1);
            get_prim(&pf, i, j, p0); get_prim(&pf, i, j + 1, p1);
            reconstruct(prm->order, nc, m2, m1, p0, p1, WL, WR);
            yface_vector(g, i, j, S);
            unit_normal(g, S, n, &len);
            double s1 = s1_yface(prm, &pf, i, j);
            orc_face_flux(prm, WL, WR, n[0], n[1], s1, F, &d);
            if (nc > 4) orc_face_flux_sc(prm, WL, WR, n[0], n[1], s1, nc - 4, F);
            if (d.absUp < 0.0) ++negc;
            if (frr_y) frr_y[(size_t)j * nx + i] = d.frr / d.c;
            for (int k = 0; k < nc; ++k) Fy[((size_t)j * nx + i) * nc + k] = F[k] * len;
        }
    if (neg_uprime) *neg_uprime += negc;
    /* Conservative sum: R = -(1/Omega) [(F_e - F_w) + (G_n - G_s)]. */
    const size_t plane = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double omega = cell_area(g, i, j);
            for (int k = 0; k < nc; ++k) {
                double fw = Fx[((size_t)j * (nx + 1) + i) * nc + k];
                double fe = Fx[((size_t)j * (nx + 1) + i + 1) * nc + k];
                double gs = Fy[((size_t)j * nx + i) * nc + k];
                double gn = Fy[((size_t)(j + 1) * nx + i) * nc + k];
                r[k * plane + (size_t)j * nx + i] = -((fe - fw) + (gn - gs)) / omega;
                if (scale)
                    scale[k * plane + (size_t)j * nx + i] =
                        (fabs(fe) + fabs(fw) + fabs(gn) + fabs(gs)) / omega;
            }
        }
    free(pf.W); free(Fx); free(Fy);
    return 0;
}

int orc_residual(const orc_params *prm, const orc_grid *g, const double *q, double *r, double *scale)
{
    return residual_impl(prm, g, q, r, scale, NULL);
}

int orc_rotated_mach(const orc_params *prm, const orc_grid *g, const double *q, double *frr_x, double *frr_y)
{
    const size_t n = (4 + (size_t)g->nscalars) * g->nx * g->ny;
    double *r = (double *)malloc(sizeof(double) * n);
    if (!r) return ORC_ENOMEM;
    int rc = residual_impl_diag(prm, g, q, r, NULL, NULL, frr_x, frr_y);
    free(r);
    return rc;
}

/* Explicit rate of one cell (time-step rule; the paper prints none):
 * lambda = (|V.Sbar_i| + c_eff |Sbar_i| + |V.Sbar_j| + c_eff |Sbar_j|) / Omega,
 * Sbar = mean of the two opposite face vectors, c_eff = c / sqrt(theta_cell)
 * with theta_cell = min(max(M_ref^2, M^2), 1) as in Eq. (101).  The extra
 * factor bounds the pressure-diffusion speed of the preconditioned dU_p term
 * of Eq. (89) at low Mach. */
static double cell_rate(const orc_params *prm, const orc_grid *g, const double W[4], int i, int j)
{
    double c = sqrt(prm->gamma * W[3] / W[0]);
    double M = sqrt(W[1] * W[1] + W[2] * W[2]) / c;
    double mr2 = prm->mach_ref * prm->mach_ref;
    double theta = dmin(dmax(mr2, M * M), 1.0);
    double ceff = c / sqrt(theta);
    double Sw[2], Se[2], Ss[2], Sn[2];
    xface_vector(g, i, j, Sw); xface_vector(g, i + 1, j, Se);
    yface_vector(g, i, j, Ss); yface_vector(g, i, j + 1, Sn);
    double Si[2] = {0.5 * (Sw[0] + Se[0]), 0.5 * (Sw[1] + Se[1])};
    double Sj[2] = {0.5 * (Ss[0] + Sn[0]), 0.5 * (Ss[1] + Sn[1])};
    double li, lj;
    if (g->metric == 0) { li = g->dy; lj = g->dx; }
    else { li = sqrt(Si[0] * Si[0] + Si[1] * Si[1]); lj = sqrt(Sj[0] * Sj[0] + Sj[1] * Sj[1]); }
    double sum = fabs(W[1] * Si[0] + W[2] * Si[1]) + ceff * li
               + fabs(W[1] * Sj[0] + W[2] * Sj[1]) + ceff * lj;
    return sum / cell_area(g, i, j);
}

int orc_max_rate(const orc_params *prm, const orc_grid *g, const double *q, double *max_rate)
{
    int rc = check_args(prm, g);
    if (rc) return rc;
    const int nx = g->nx, ny = g->ny;
    const size_t plane = (size_t)nx * ny;
    double mx = 0.0;
    int bad = 0;
    /* the maximum does not depend on the order it is taken in */
#pragma omp parallel for schedule(static) reduction(max : mx) reduction(| : bad)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            double Q[4] = {q[c], q[plane + c], q[2 * plane + c], q[3 * plane + c]};
            double W[4];
            conserved_to_prim(prm->gamma, Q, W, 4);
            if (!physical(W)) { bad = 1; continue; }
            mx = dmax(mx, cell_rate(prm, g, W, i, j));
        }
    if (bad) return ORC_ENONPHYS;
    *max_rate = mx;
    return 0;
}

int orc_run(const orc_params *prm, const orc_grid *g, double *q, long nsteps, double t_end,
            orc_run_stats *stats)
{
    int rc = check_args(prm, g);
    if (rc) return rc;
    if (!(prm->cfl > 0.0) || prm->time_scheme < 0 || prm->time_scheme > 2) return ORC_EINVAL;
    const size_t n = (4 + (size_t)g->nscalars) * g->nx * g->ny;
    double *r = (double *)malloc(sizeof(double) * n);
    double *q1 = (double *)malloc(sizeof(double) * n);
    double *q2 = (double *)malloc(sizeof(double) * n);
    if (!r || !q1 || !q2) { free(r); free(q1); free(q2); return ORC_ENOMEM; }
    double t = stats ? stats->t : 0.0;
    /* moving boundaries are evaluated at the time of each stage's input state */
    orc_grid gs = *g;
    long steps = 0, neg = 0;
    double dt = 0.0, rate = 0.0;
    rc = 0;
    for (long s = 0; s < nsteps; ++s) {
        if (t_end > 0.0 && t >= t_end) break;
        rc = orc_max_rate(prm, g, q, &rate);
        if (rc) break;
        dt = prm->cfl / rate;
        int last = 0;
        if (t_end > 0.0 && t + dt >= t_end) { dt = t_end - t; last = 1; }
        if (prm->time_scheme == 0) {
            /* forward Euler: Q^{n+1} = Q^n + dt R(Q^n) */
            gs.t_bc = t;
            rc = residual_impl(prm, &gs, q, r, NULL, &neg);
            if (rc) break;
#pragma omp parallel for schedule(static)
            for (size_t m = 0; m < n; ++m) q[m] = q[m] + dt * r[m];
        } else if (prm->time_scheme == 2) {
            /* Four-stage Runge-Kutta (the paper's time scheme, Sec. 7.1; reading:
             * the low-storage form of Jameson, Schmidt and Turkel):
             * Q^(k) = Q^n + alpha_k dt R(Q^(k-1)), alpha = 1/4, 1/3, 1/2, 1. */
            const double alpha[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};
            const double *in = q;
            for (int k = 0; k < 4 && !rc; ++k) {
                gs.t_bc = t + (k == 0 ? 0.0 : alpha[k - 1] * dt);
                rc = residual_impl(prm, &gs, in, r, NULL, &neg);
                if (rc) break;
                double *out = (k == 3) ? q : (k == 1 ? q2 : q1);
#pragma omp parallel for schedule(static)
                for (size_t m = 0; m < n; ++m) out[m] = q[m] + alpha[k] * dt * r[m];
                in = out;
            }
            if (rc) break;
        } else {
            /* SSP-RK3 (Shu-Osher form); stage inputs at t, t + dt, t + dt/2 */
            gs.t_bc = t;
            rc = residual_impl(prm, &gs, q, r, NULL, &neg);
            if (rc) break;
#pragma omp parallel for schedule(static)
            for (size_t m = 0; m < n; ++m) q1[m] = q[m] + dt * r[m];
            gs.t_bc = t + dt;
            rc = residual_impl(prm, &gs, q1, r, NULL, &neg);
            if (rc) break;
#pragma omp parallel for schedule(static)
            for (size_t m = 0; m < n; ++m) q2[m] = 0.75 * q[m] + 0.25 * (q1[m] + dt * r[m]);
            gs.t_bc = t + 0.5 * dt;
            rc = residual_impl(prm, &gs, q2, r, NULL, &neg);
            if (rc) break;
#pragma omp parallel for schedule(static)
            for (size_t m = 0; m < n; ++m)
                q[m] = (1.0 / 3.0) * q[m] + (2.0 / 3.0) * (q2[m] + dt * r[m]);
        }
        t = last ? t_end : t + dt;
        ++steps;
    }
    if (!rc) {
        /* the final state must be physical too */
        double dummy;
        rc = orc_max_rate(prm, g, q, &dummy);
    }
    if (stats) {
        stats->t = t; stats->dt_last = dt; stats->max_rate = rate; stats->steps = steps;
        stats->nonphys = (rc == ORC_ENONPHYS); stats->neg_uprime_faces = neg;
    }
    free(r); free(q1); free(q2);
    return rc;
}

/* Threads of the row loops (OpenMP); results do not depend on them. */
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int orc_max_threads(void) { return omp_get_max_threads(); }
