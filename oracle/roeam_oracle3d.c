/*
 * roeam_oracle3d.c -- plain FP64 CPU oracle of the Roe-AM scheme on uniform
 * Cartesian 3-D grids: the paper's equations in their own dimension (five
 * conserved rows, the velocity component w, the nine-face detector of
 * Eq. (96) and the 3-D cross products of Eq. (109)).
 *
 * TEST INFRASTRUCTURE ONLY, like roeam_oracle.c: slow and plain on purpose,
 * -O2 -ffp-contract=off, libm sqrt and true division, fixed loop and sum
 * orders, rows of cells shared out by OpenMP without changing any value's
 * arithmetic.  It shares nothing with the HIP library.
 *
 * Layout: q is [5 + ns][nz][ny][nx], rows (rho, rho u, rho v, rho w, rho E)
 * and ns transported scalars rho k_m.
 */
#include "roeam_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ENONPHYS (-4)
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

static double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }
static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }
static double pow8(double x)
{
    double x2 = x * x;
    double x4 = x2 * x2;
    return x4 * x4;
}
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* rho E = p/(gamma-1) + rho |V|^2 / 2,  H = (rho E + p) / rho. */
static double rhoE3(double gamma, const double W[5])
{
    return W[4] / (gamma - 1.0) + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
}
static double enthalpy3(double gamma, const double W[5]) { return (rhoE3(gamma, W) + W[4]) / W[0]; }

/* Eq. (4) in 3-D: U (rho, rho u, rho v, rho w, rho H) + p (0, n, 0). */
void orc3_physical_flux(double gamma, const double W[5], const double n[3], double F[5])
{
    double U = n[0] * W[1] + n[1] * W[2] + n[2] * W[3];
    double H = enthalpy3(gamma, W);
    F[0] = U * W[0];
    F[1] = U * (W[0] * W[1]) + W[4] * n[0];
    F[2] = U * (W[0] * W[2]) + W[4] * n[1];
    F[3] = U * (W[0] * W[3]) + W[4] * n[2];
    F[4] = U * (W[0] * H);
}

/* Eqs. (103)-(109): n1 from the velocity jump (Eq. 108), n2 the unit vector
 * along (n1 x n) x n1 (reading D7), U1, U2 with the Roe-averaged velocity. */
static double rotated_speed3(const double n[3], const double dV[3], const double V[3], double u_ref)
{
    double m = sqrt(dot3(dV, dV));
    double n1[3];
    if (m < 1e-5 * u_ref || m == 0.0) {
        n1[0] = n[0]; n1[1] = n[1]; n1[2] = n[2];
    } else {
        n1[0] = dV[0] / m; n1[1] = dV[1] / m; n1[2] = dV[2] / m;
    }
    double alpha1 = dot3(n1, n); /* Eq. (106) */
    double U1 = dot3(n1, V);     /* Eq. (104) */
    double c1[3], c2[3];
    cross3(n1, n, c1);
    cross3(c1, n1, c2);          /* Eq. (109) before normalisation */
    double l2 = sqrt(dot3(c2, c2));
    double a2U2 = 0.0;
    if (l2 > 0.0) {
        double n2[3] = {c2[0] / l2, c2[1] / l2, c2[2] / l2};
        a2U2 = dot3(n2, n) * dot3(n2, V); /* Eqs. (107), (105) */
    }
    return fabs(alpha1 * U1) + fabs(a2U2); /* Eq. (103) */
}

/* Eq. (85) in 3-D with ns transported scalars after the five flow rows: each
 * scalar row has Psi = rho k, Psi^ = rho^ k^ (k^ the sqrt(rho)-weighted Roe
 * average), no pressure term, and the face's xi, dU_p, dU_u (classical Roe:
 * xi Delta(rho k) + (dU_u + dU_p) rho^ k^). */
void orc3_face_flux_sc(const orc_params *prm, const double *WL, const double *WR, const double n[3], double s1,
                       int ns, double *F)
{
    const double g = prm->gamma;
    const double rL = WL[0], rR = WR[0], pL = WL[4], pR = WR[4];
    const double VL[3] = {WL[1], WL[2], WL[3]}, VR[3] = {WR[1], WR[2], WR[3]};
    double UL = dot3(n, VL), UR = dot3(n, VR);
    double HL = enthalpy3(g, WL), HR = enthalpy3(g, WR);
    const int nc = 5 + ns;
    double PsiL[5 + ORC_MAX_SCALARS] = {rL, rL * VL[0], rL * VL[1], rL * VL[2], rL * HL};
    double PsiR[5 + ORC_MAX_SCALARS] = {rR, rR * VR[0], rR * VR[1], rR * VR[2], rR * HR};
    double FbL[5 + ORC_MAX_SCALARS], FbR[5 + ORC_MAX_SCALARS];
    orc3_physical_flux(g, WL, n, FbL);
    orc3_physical_flux(g, WR, n, FbR);
    for (int m = 0; m < ns; ++m) {
        PsiL[5 + m] = rL * WL[5 + m];
        PsiR[5 + m] = rR * WR[5 + m];
        FbL[5 + m] = dot3(n, VL) * PsiL[5 + m];
        FbR[5 + m] = dot3(n, VR) * PsiR[5 + m];
    }

    /* Roe averages (sqrt(rho) weights) */
    double rr = sqrt(rR / rL);
    double rho = rr * rL;
    double V[3];
    for (int d = 0; d < 3; ++d) V[d] = (VL[d] + rr * VR[d]) / (1.0 + rr);
    double H = (HL + rr * HR) / (1.0 + rr);
    double c = sqrt((g - 1.0) * (H - 0.5 * dot3(V, V)));
    double U = dot3(n, V);
    double PsiHat[5 + ORC_MAX_SCALARS] = {rho, rho * V[0], rho * V[1], rho * V[2], rho * H};
    for (int m = 0; m < ns; ++m) PsiHat[5 + m] = rho * ((WL[5 + m] + rr * WR[5 + m]) / (1.0 + rr));
    double dU = UR - UL, dp = pR - pL;
    double pvec[5 + ORC_MAX_SCALARS] = {0.0, n[0], n[1], n[2], 0.0};
    double diss[5 + ORC_MAX_SCALARS];

    if (prm->scheme == ORC_SCHEME_ROE || prm->scheme == ORC_SCHEME_ROE_HARTEN) {
        /* classical Roe, Eq. (7) with Eqs. (8)-(12); Harten's fix, Eqs. (114)-(115) */
        double l1 = fabs(U), l4 = fabs(U - c), l5 = fabs(U + c);
        if (prm->scheme == ORC_SCHEME_ROE_HARTEN) {
            double h = prm->eps_lambda * dmax(l1, dmax(l4, l5));
            if (l1 < h) l1 = 0.5 * (l1 * l1 / h + h);
            if (l4 < h) l4 = 0.5 * (l4 * l4 / h + h);
            if (l5 < h) l5 = 0.5 * (l5 * l5 / h + h);
        }
        double xi = l1;
        double dpu = (0.5 * (l5 + l4) - l1) * rho * dU;
        double dpp = 0.5 * (l5 - l4) * dp / c;
        double dUu = 0.5 * (l5 - l4) * dU / c;
        double dUp = (0.5 * (l5 + l4) - l1) * dp / (rho * c * c);
        double dQ[5 + ORC_MAX_SCALARS] = {rR - rL, PsiR[1] - PsiL[1], PsiR[2] - PsiL[2], PsiR[3] - PsiL[3],
                                          rhoE3(g, WR) - rhoE3(g, WL)};
        double pv7[5 + ORC_MAX_SCALARS] = {0.0, n[0], n[1], n[2], U};
        for (int m = 0; m < ns; ++m) dQ[5 + m] = PsiR[5 + m] - PsiL[5 + m];
        for (int k = 0; k < nc; ++k) diss[k] = xi * dQ[k] + (dpu + dpp) * pv7[k] + (dUu + dUp) * PsiHat[k];
    } else {
        const unsigned var = prm->variant;
        double cL = sqrt(g * pL / rL), cR = sqrt(g * pR / rR);
        double M = 0.5 * (sqrt(dot3(VL, VL)) / cL + sqrt(dot3(VR, VR)) / cR); /* Eq. (93) */
        double Mbar = fabs(U) / c;                                            /* Eq. (94) */
        double fM = orc_f(M), f8M = pow8(fM);
        double fMbar = orc_f(Mbar), f8Mbar = pow8(fMbar);
        double mr2 = prm->mach_ref * prm->mach_ref;
        double theta = dmin(dmax(mr2, M * M), 1.0);                                            /* Eq. (101) */
        double ct = 0.5 * sqrt(4.0 * c * c * theta + (1.0 - theta) * (1.0 - theta) * U * U);   /* Eq. (99)  */
        double Ut = 0.5 * (1.0 + theta) * U;                                                   /* Eq. (100) */
        double absU = fabs(U), absUp = absU;
        if (!(var & ORC_V_NO_EQ92)) {
            double w = (var & ORC_V_EXPFIX_F8) ? f8Mbar : fMbar;
            absUp = absU - w * (sgn(U + c) - sgn(U - c)) * dmax(0.0, dU) / 4.0; /* Eq. (92) */
        }
        if (var & ORC_V_CLAMP_UPRIME) absUp = dmax(absUp, 0.0);
        double gate = (var & ORC_V_XI_UNGATED) ? 1.0 : (1.0 - f8Mbar);
        double xi_pos = fabs(0.5 * (UR + UL)) + gate * (0.5 * dU);
        double dV[3] = {VR[0] - VL[0], VR[1] - VL[1], VR[2] - VL[2]};
        double fef = prm->eps2 * c;                                     /* Eq. (102) */
        double frr = rotated_speed3(n, dV, V, prm->u_ref);
        double xi = dmax(xi_pos, prm->eps1 * (1.0 - f8Mbar) * f8M * dmin(fef, frr)); /* Eq. (86) */
        if (var & ORC_V_XI_EQ46) xi = fabs(UR + UL) / 2.0;
        if (var & ORC_V_XI_ROE) xi = absU;
        double dpp = sgn(U) * dmin(absUp, c) * dp / c;                                   /* Eq. (87) */
        double dpu = (1.0 - s1 + s1 * fM) * dmax(0.0, c - absUp) * rho * dU;              /* Eq. (88) */
        double bracket = dmax(0.0, ct - absUp) + (1.0 - theta) * (absUp - U / (2.0 * ct) * sgn(Ut) * dmin(fabs(Ut), ct));
        double dUp = s1 * (1.0 - f8M) * bracket * dp / (rho * theta * c * c);            /* Eq. (89) */
        if (var & ORC_V_DUP_ROE) dUp = dmax(0.0, c - absU) * dp / (rho * c * c);
        if (var & ORC_V_DUP_ZERO) dUp = 0.0;
        double dUu = 0.5 * sgn(U) * dmin(absUp, c) * dU / c;                             /* Eqs. (90)-(91) */
        for (int k = 0; k < nc; ++k)
            diss[k] = xi * (PsiR[k] - PsiL[k]) + (dpp + dpu) * pvec[k] + dUp * PsiHat[k] + dUu * PsiR[k]
                    + dUu * PsiL[k];
    }
    for (int k = 0; k < nc; ++k) F[k] = 0.5 * (FbL[k] + FbR[k]) - 0.5 * diss[k]; /* Eq. (85) */
}

void orc3_face_flux(const orc_params *prm, const double WL[5], const double WR[5], const double n[3], double s1,
                    double F[5])
{
    orc3_face_flux_sc(prm, WL, WR, n, s1, 0, F);
}

/* ------------------------------------------------------------------------ */
/* grid, ghosts, residual                                                   */
/* ------------------------------------------------------------------------ */

#define ORC3_MAXC (5 + ORC_MAX_SCALARS)

typedef struct {
    int nx, ny, nz, NX, NY, NZ; /* N* = n* + 4 (two ghost layers) */
    int nc;                     /* components: 5 + scalars */
    double *W;                  /* primitives [nc][NZ][NY][NX]: rho, u, v, w, p, k_1 .. */
} prim3;

static size_t P3(const prim3 *f, int k, int i, int j, int l)
{
    return (((size_t)k * f->NZ + (size_t)(l + 2)) * f->NY + (size_t)(j + 2)) * f->NX + (size_t)(i + 2);
}
static void get3(const prim3 *f, int i, int j, int l, double *W)
{
    for (int k = 0; k < f->nc; ++k) W[k] = f->W[P3(f, k, i, j, l)];
}
static void set3(prim3 *f, int i, int j, int l, const double *W)
{
    for (int k = 0; k < f->nc; ++k) f->W[P3(f, k, i, j, l)] = W[k];
}
/* nc components: the five flow primitives and k_m = (rho k_m) / rho */
static void prim_of3(double gamma, const double *Q, double *W, int nc)
{
    double rho = Q[0];
    double u = Q[1] / rho, v = Q[2] / rho, w = Q[3] / rho;
    W[0] = rho; W[1] = u; W[2] = v; W[3] = w;
    W[4] = (gamma - 1.0) * (Q[4] - 0.5 * rho * (u * u + v * v + w * w));
    for (int k = 5; k < nc; ++k) W[k] = Q[k] / rho;
}
static int physical3(const double W[5])
{
    for (int k = 0; k < 5; ++k)
        if (!isfinite(W[k])) return 0;
    return W[0] > 0.0 && W[4] > 0.0;
}

/* The ghost of side s for a ghost cell at distance gd (1 or 2) from the
 * boundary, given the line of cells along the side's axis: a[] is the index
 * of interior cell m (0 .. n-1) along that axis. */
static void ghost3(const orc_params *prm, const orc3_grid *g, const prim3 *f, int side, int gd, int i, int j, int l,
                   double *W)
{
    const int axis = side / 2, hi = side & 1;
    const int n = axis == 0 ? g->nx : (axis == 1 ? g->ny : g->nz);
    int m;
    switch (g->bc[side]) {
    case ORC_BC_PERIODIC: m = hi ? gd - 1 : n - gd; break;
    case ORC_BC_TRANSMISSIVE: m = hi ? n - 1 : 0; break;
    case ORC_BC_SLIPWALL: m = hi ? n - gd : gd - 1; break;
    default: {
        double Q[ORC3_MAXC];
        for (int k = 0; k < 5; ++k) Q[k] = g->bc_state[side][k];
        for (int k = 5; k < f->nc; ++k) Q[k] = g->bc_scalar[side][k - 5];
        prim_of3(prm->gamma, Q, W, f->nc);
        return;
    }
    }
    int ii = i, jj = j, ll = l;
    if (axis == 0) ii = m;
    else if (axis == 1) jj = m;
    else ll = m;
    get3(f, ii, jj, ll, W);
    if (g->bc[side] == ORC_BC_SLIPWALL) W[1 + axis] = -W[1 + axis]; /* mirror the wall-normal velocity */
}

/* x-ghosts for interior (j, l), then y-ghosts for every i (incl. x-ghosts)
 * and interior l, then z-ghosts for every (i, j): edges and corners follow. */
static void fill_ghosts3(const orc_params *prm, const orc3_grid *g, prim3 *f)
{
    double W[ORC3_MAXC];
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int gd = 1; gd <= 2; ++gd) {
                ghost3(prm, g, f, 0, gd, -gd, j, l, W); set3(f, -gd, j, l, W);
                ghost3(prm, g, f, 1, gd, nx - 1 + gd, j, l, W); set3(f, nx - 1 + gd, j, l, W);
            }
    for (int l = 0; l < nz; ++l)
        for (int i = -2; i < nx + 2; ++i)
            for (int gd = 1; gd <= 2; ++gd) {
                ghost3(prm, g, f, 2, gd, i, -gd, l, W); set3(f, i, -gd, l, W);
                ghost3(prm, g, f, 3, gd, i, ny - 1 + gd, l, W); set3(f, i, ny - 1 + gd, l, W);
            }
    for (int j = -2; j < ny + 2; ++j)
        for (int i = -2; i < nx + 2; ++i)
            for (int gd = 1; gd <= 2; ++gd) {
                ghost3(prm, g, f, 4, gd, i, j, -gd, W); set3(f, i, j, -gd, W);
                ghost3(prm, g, f, 5, gd, i, j, nz - 1 + gd, W); set3(f, i, j, nz - 1 + gd, W);
            }
}

static int load_prims3(const orc_params *prm, const orc3_grid *g, const double *q, prim3 *f)
{
    const size_t vol = (size_t)g->nx * g->ny * g->nz;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int l = 0; l < g->nz; ++l)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = ((size_t)l * g->ny + j) * g->nx + i;
                double Q[ORC3_MAXC], W[ORC3_MAXC];
                for (int k = 0; k < f->nc; ++k) Q[k] = q[k * vol + c];
                prim_of3(prm->gamma, Q, W, f->nc);
                if (!physical3(W)) bad = 1;
                set3(f, i, j, l, W);
            }
    if (bad) return ORC_ENONPHYS;
    fill_ghosts3(prm, g, f);
    return 0;
}

static double minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return sgn(a) * dmin(fabs(a), fabs(b));
}

static double P3between(const prim3 *f, int ia, int ja, int la, int ib, int jb, int lb)
{
    double A[ORC3_MAXC], B[ORC3_MAXC];
    get3(f, ia, ja, la, A);
    get3(f, ib, jb, lb, B);
    return orc_detector_P(A[4], A[0], B[4], B[0]);
}

/* Eq. (96): the face between cells a = c - e_axis and b = c, and the faces of
 * both cells in the two transverse directions (nine ratios). */
static double s1_face3(const orc_params *prm, const prim3 *f, int axis, int i, int j, int l)
{
    if (prm->s1_mode == 1) return 1.0; /* Eq. (110) */
    int e[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    const int *ea = e[axis];
    int ai = i - ea[0], aj = j - ea[1], al = l - ea[2];
    double a = P3between(f, ai, aj, al, i, j, l);
    for (int t = 0; t < 3; ++t) {
        if (t == axis) continue;
        const int *et = e[t];
        /* faces of cell a and of cell b on both sides in direction t */
        a = dmin(a, P3between(f, ai - et[0], aj - et[1], al - et[2], ai, aj, al));
        a = dmin(a, P3between(f, ai, aj, al, ai + et[0], aj + et[1], al + et[2]));
        a = dmin(a, P3between(f, i - et[0], j - et[1], l - et[2], i, j, l));
        a = dmin(a, P3between(f, i, j, l, i + et[0], j + et[1], l + et[2]));
    }
    return pow8(orc_f(a));
}

static int check3(const orc_params *prm, const orc3_grid *g)
{
    if (!prm || !g) return ORC_EINVAL;
    if (g->nx < 2 || g->ny < 2 || g->nz < 2) return ORC_EINVAL;
    if (!(g->dx > 0.0) || !(g->dy > 0.0) || !(g->dz > 0.0)) return ORC_EINVAL;
    if (!(prm->gamma > 1.0)) return ORC_EINVAL;
    if (prm->scheme == ORC_SCHEME_ROEAM && !(prm->mach_ref > 0.0)) return ORC_EINVAL;
    if (prm->order != 1 && prm->order != 2) return ORC_EINVAL;
    if (g->nscalars < 0 || g->nscalars > ORC_MAX_SCALARS) return ORC_EINVAL;
    return 0;
}

/* Faces normal to `axis`: face (i, j, l) lies between cell (i, j, l) - e_axis
 * and (i, j, l).  Flux per unit area into F[(face index) * nc + k]. */
static void face_fluxes3(const orc_params *prm, const orc3_grid *g, const prim3 *f, int axis, double *F)
{
    const int fx = g->nx + (axis == 0), fy = g->ny + (axis == 1), fz = g->nz + (axis == 2);
    const int e[3] = {axis == 0, axis == 1, axis == 2};
    const double n[3] = {(double)e[0], (double)e[1], (double)e[2]};
    const int nc = f->nc;
#pragma omp parallel for schedule(static)
    for (int l = 0; l < fz; ++l)
        for (int j = 0; j < fy; ++j)
            for (int i = 0; i < fx; ++i) {
                double m2[ORC3_MAXC], m1[ORC3_MAXC], p0[ORC3_MAXC], p1[ORC3_MAXC], WL[ORC3_MAXC], WR[ORC3_MAXC];
                get3(f, i - 2 * e[0], j - 2 * e[1], l - 2 * e[2], m2);
                get3(f, i - e[0], j - e[1], l - e[2], m1);
                get3(f, i, j, l, p0);
                get3(f, i + e[0], j + e[1], l + e[2], p1);
                for (int k = 0; k < nc; ++k) {
                    if (prm->order == 1) {
                        WL[k] = m1[k];
                        WR[k] = p0[k];
                    } else {
                        WL[k] = m1[k] + 0.5 * minmod(m1[k] - m2[k], p0[k] - m1[k]);
                        WR[k] = p0[k] - 0.5 * minmod(p0[k] - m1[k], p1[k] - p0[k]);
                    }
                }
                double Fc[ORC3_MAXC];
                orc3_face_flux_sc(prm, WL, WR, n, s1_face3(prm, f, axis, i, j, l), nc - 5, Fc);
                size_t idx = ((size_t)l * fy + j) * fx + i;
                for (int k = 0; k < nc; ++k) F[idx * nc + k] = Fc[k];
            }
}

static int residual3_impl(const orc_params *prm, const orc3_grid *g, const double *q, double *r, double *scale)
{
    int rc = check3(prm, g);
    if (rc) return rc;
    const int nx = g->nx, ny = g->ny, nz = g->nz, nc = 5 + g->nscalars;
    prim3 f = {nx, ny, nz, nx + 4, ny + 4, nz + 4, nc, NULL};
    f.W = (double *)malloc(sizeof(double) * nc * (size_t)f.NX * f.NY * f.NZ);
    double *Fx = (double *)malloc(sizeof(double) * nc * (size_t)(nx + 1) * ny * nz);
    double *Fy = (double *)malloc(sizeof(double) * nc * (size_t)nx * (ny + 1) * nz);
    double *Fz = (double *)malloc(sizeof(double) * nc * (size_t)nx * ny * (nz + 1));
    if (!f.W || !Fx || !Fy || !Fz) { free(f.W); free(Fx); free(Fy); free(Fz); return ORC_ENOMEM; }
    rc = load_prims3(prm, g, q, &f);
    if (rc) { free(f.W); free(Fx); free(Fy); free(Fz); return rc; }
    face_fluxes3(prm, g, &f, 0, Fx);
    face_fluxes3(prm, g, &f, 1, Fy);
    face_fluxes3(prm, g, &f, 2, Fz);
    /* R = -(1/Omega) [((F_e - F_w) A_x + (G_n - G_s) A_y) + (H_t - H_b) A_z] */
    const double Ax = g->dy * g->dz, Ay = g->dx * g->dz, Az = g->dx * g->dy, vol = g->dx * g->dy * g->dz;
    const size_t plane = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = ((size_t)l * ny + j) * nx + i;
                for (int k = 0; k < nc; ++k) {
                    double fw = Fx[(((size_t)l * ny + j) * (nx + 1) + i) * nc + k] * Ax;
                    double fe = Fx[(((size_t)l * ny + j) * (nx + 1) + i + 1) * nc + k] * Ax;
                    double gs = Fy[(((size_t)l * (ny + 1) + j) * nx + i) * nc + k] * Ay;
                    double gn = Fy[(((size_t)l * (ny + 1) + j + 1) * nx + i) * nc + k] * Ay;
                    double hb = Fz[(((size_t)l * ny + j) * nx + i) * nc + k] * Az;
                    double ht = Fz[(((size_t)(l + 1) * ny + j) * nx + i) * nc + k] * Az;
                    r[k * plane + c] = -(((fe - fw) + (gn - gs)) + (ht - hb)) / vol;
                    if (scale)
                        scale[k * plane + c] =
                            (fabs(fe) + fabs(fw) + fabs(gn) + fabs(gs) + fabs(ht) + fabs(hb)) / vol;
                }
            }
    free(f.W); free(Fx); free(Fy); free(Fz);
    return 0;
}

int orc3_residual(const orc_params *prm, const orc3_grid *g, const double *q, double *r, double *scale)
{
    return residual3_impl(prm, g, q, r, scale);
}

/* Explicit rate of a cell: (|u| + c_e)/dx + (|v| + c_e)/dy + (|w| + c_e)/dz in the
 * face-area form of the 2-D rule, c_e = c / sqrt(theta_cell). */
int orc3_max_rate(const orc_params *prm, const orc3_grid *g, const double *q, double *max_rate)
{
    int rc = check3(prm, g);
    if (rc) return rc;
    const size_t vol = (size_t)g->nx * g->ny * g->nz;
    const double Ax = g->dy * g->dz, Ay = g->dx * g->dz, Az = g->dx * g->dy, V = g->dx * g->dy * g->dz;
    const double mr2 = prm->mach_ref * prm->mach_ref;
    double mx = 0.0;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : mx) reduction(| : bad)
    for (int l = 0; l < g->nz; ++l)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = ((size_t)l * g->ny + j) * g->nx + i;
                double Q[5], W[5];
                for (int k = 0; k < 5; ++k) Q[k] = q[k * vol + c];
                prim_of3(prm->gamma, Q, W, 5);
                if (!physical3(W)) { bad = 1; continue; }
                double cs = sqrt(prm->gamma * W[4] / W[0]);
                double M = sqrt(W[1] * W[1] + W[2] * W[2] + W[3] * W[3]) / cs;
                double theta = dmin(dmax(mr2, M * M), 1.0);
                double ce = cs / sqrt(theta);
                double sum = (fabs(W[1]) * Ax + ce * Ax) + (fabs(W[2]) * Ay + ce * Ay) + (fabs(W[3]) * Az + ce * Az);
                mx = dmax(mx, sum / V);
            }
    if (bad) return ORC_ENONPHYS;
    *max_rate = mx;
    return 0;
}

int orc3_run(const orc_params *prm, const orc3_grid *g, double *q, long nsteps, double t_end, orc_run_stats *stats)
{
    int rc = check3(prm, g);
    if (rc) return rc;
    if (!(prm->cfl > 0.0) || prm->time_scheme < 0 || prm->time_scheme > 2) return ORC_EINVAL;
    const size_t n = (5 + (size_t)g->nscalars) * g->nx * g->ny * g->nz;
    double *r = (double *)malloc(sizeof(double) * n);
    double *q1 = (double *)malloc(sizeof(double) * n);
    double *q2 = (double *)malloc(sizeof(double) * n);
    if (!r || !q1 || !q2) { free(r); free(q1); free(q2); return ORC_ENOMEM; }
    double t = stats ? stats->t : 0.0, dt = 0.0, rate = 0.0;
    long steps = 0;
    for (long s = 0; s < nsteps; ++s) {
        if (t_end > 0.0 && t >= t_end) break;
        rc = orc3_max_rate(prm, g, q, &rate);
        if (rc) break;
        dt = prm->cfl / rate;
        int last = 0;
        if (t_end > 0.0 && t + dt >= t_end) { dt = t_end - t; last = 1; }
        if (prm->time_scheme == 0) {
            if ((rc = residual3_impl(prm, g, q, r, NULL))) break;
#pragma omp parallel for schedule(static)
            for (size_t m = 0; m < n; ++m) q[m] = q[m] + dt * r[m];
        } else if (prm->time_scheme == 2) {
            const double alpha[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};
            const double *in = q;
            for (int k = 0; k < 4 && !rc; ++k) {
                if ((rc = residual3_impl(prm, g, in, r, NULL))) break;
                double *out = (k == 3) ? q : (k == 1 ? q2 : q1);
#pragma omp parallel for schedule(static)
                for (size_t m = 0; m < n; ++m) out[m] = q[m] + alpha[k] * dt * r[m];
                in = out;
            }
            if (rc) break;
        } else {
            if ((rc = residual3_impl(prm, g, q, r, NULL))) break;
#pragma omp parallel for schedule(static)
            for (size_t m = 0; m < n; ++m) q1[m] = q[m] + dt * r[m];
            if ((rc = residual3_impl(prm, g, q1, r, NULL))) break;
#pragma omp parallel for schedule(static)
            for (size_t m = 0; m < n; ++m) q2[m] = 0.75 * q[m] + 0.25 * (q1[m] + dt * r[m]);
            if ((rc = residual3_impl(prm, g, q2, r, NULL))) break;
#pragma omp parallel for schedule(static)
            for (size_t m = 0; m < n; ++m) q[m] = (1.0 / 3.0) * q[m] + (2.0 / 3.0) * (q2[m] + dt * r[m]);
        }
        t = last ? t_end : t + dt;
        ++steps;
    }
    if (!rc) {
        double dummy;
        rc = orc3_max_rate(prm, g, q, &dummy);
    }
    if (stats) {
        stats->t = t; stats->dt_last = dt; stats->max_rate = rate; stats->steps = steps;
        stats->nonphys = (rc == ORC_ENONPHYS); stats->neg_uprime_faces = 0;
    }
    free(r); free(q1); free(q2);
    return rc;
}
