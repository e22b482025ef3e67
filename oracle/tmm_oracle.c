/*
 * Reference CPU implementation of the transport-matrix time step.
 *
 * TEST INFRASTRUCTURE ONLY: a plain float64 restatement of the method of
 * Piwonski & Slawig, "The Idea and Concept of Metos3D" (arXiv 1410.0204),
 * written for readability, not speed.  It is loaded by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the GPU library,
 * and shares no code with it.
 *
 * What it computes (paper sections in brackets):
 *   step      y_{j+1} = Ai(t_j) (Ae(t_j) y_j + dt * q(y_j, u))        [3]
 *   matrices  A(t_j) = (1-w) A_k0 + w A_k1, monthly anchors          [3, 7]
 *   year map  phi(y_0) = y_nstep, residual ||y - phi(y)||_2           [4, 7]
 *   BGC       PO4-DOP model: production, light, DOP, Martin export    [2.2.1]
 *             PO4-DOP-PHY model: explicit phytoplankton               [2.2.2]
 *             evaluated per water column through the interface of     [5]
 *   tangent   phi'(y) v, exactly (forward mode) and by finite         [6.1]
 *             differences
 *   reverse   gradient of a least-squares misfit with respect to the
 *             parameters u and to y_0, by storing the whole trajectory
 *             (the paper names algorithmic differentiation as the route
 *             to exact derivatives, sections 1.2, 6.1 and 9)
 *
 * Readings where the paper is silent (each also listed with the design notes):
 *   - dt multiplies q, and the rates are per day: dt_d = 360/nstep days.
 *   - Monthly matrices sit at mid-month; step j lies at t_j = j/nstep; the
 *     year is periodic, so December is interpolated towards January.
 *   - Remineralisation adds nutrient: layer k of the aphotic zone receives
 *     the flux divergence (F(d_{k-1}) - F(d_k))/h_k with F(z) = Phi*(z/l')^-b;
 *     the bottom wet layer receives all flux that reaches it; a column no
 *     deeper than the euphotic zone remineralises its export in its bottom
 *     layer.
 *   - The production integral over [0, l'] is the layer sum sum_k h_k f_k;
 *     light is taken at layer centres, the Martin curve at layer bottoms.
 *   - sigma_PAR = 0.4, sigma_ice = 0; I_SWR is the daily-mean top-of-
 *     atmosphere insolation with solar constant 1361 W/m^2.
 *   - Michaelis-Menten uses max(N, 0), with derivative 0 for N <= 0.
 *   - The one-tracer N model is the PO4-DOP model without the DOP tracer
 *     (sigma_2 = 0, all production exported).
 *   - PO4-DOP-PHY: production f_1 = mu_1 PHY N+/(N+ + K_1) I/(I + K_I) with
 *     PHY entering linearly (not clipped); the exported part is
 *     (1 - sigma_2) sigma_3 f_1, remineralised as in PO4-DOP; the losses
 *     lambda_3 PHY + kappa_3 PHY^2 act in the euphotic zone only.
 *   - With nbgc > 1 internal BGC steps per ocean step (section 7), the source
 *     is the increment of nbgc explicit Euler sub-steps of length dt/nbgc at
 *     the step's forcing; nbgc = 1 is dt*q(y).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* The CPU-baseline timing build (-fopenmp) runs the row loops of the
 * products and the column loop of the sources of a step in parallel.  Every
 * output element is still computed by one thread in the order written here,
 * so that build gives the plain build's results bit for bit; without
 * -fopenmp the macro is empty. */
#ifdef _OPENMP
#include <omp.h>
#define ROWS_IN_PARALLEL _Pragma("omp parallel for schedule(static)")
#else
#define ROWS_IN_PARALLEL
#endif

#define PI 3.14159265358979323846
#define SIGMA_PAR 0.4
#define SIGMA_ICE 0.0
#define SOLAR_CONSTANT 1361.0
#define DAYS_PER_YEAR 360.0
#define MAX_LAYERS 256
#define MAX_TRACERS 3
#define MAX_PARAMS 11

int oracle_ntracer(int model)
{
    if (model == ORACLE_MODEL_N) return 1;
    if (model == ORACLE_MODEL_NDOP) return 2;
    if (model == ORACLE_MODEL_NDOPPHY) return 3;
    return -1;
}

/* Threads the step's loops use (1 without OpenMP); n < 1 leaves it alone. */
int oracle_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

int oracle_nparam(int model)
{
    if (model == ORACLE_MODEL_N) return 5;
    if (model == ORACLE_MODEL_NDOP) return 7;
    if (model == ORACLE_MODEL_NDOPPHY) return 11;
    return -1;
}

static int floor_div(int a, int b)
{
    int q = a / b;
    if (a % b != 0 && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

/* Section 3: twelve monthly matrices, linearly interpolated in time.  The
 * matrix of month k represents the middle of that month, so step j sits
 * tau = j - spm/2 steps after the middle of January. */
void oracle_phase(int j, int nstep, int nmat, int *k0, int *k1, double *w)
{
    int spm = nstep / nmat;
    int jj = ((j % nstep) + nstep) % nstep;
    int tau = jj - spm / 2;
    int kk = floor_div(tau, spm);
    int r = tau - kk * spm;
    *k0 = ((kk % nmat) + nmat) % nmat;
    *k1 = (*k0 + 1) % nmat;
    *w = (double)r / (double)spm;
}

/* Section 2.2.1: short-wave radiation as a function of latitude and season.
 * Daily mean over the sunlit part of the day at the top of the atmosphere;
 * solar declination from a cosine of the 360-day year with the December
 * solstice ten days before t = 0. */
double oracle_insolation(double lat_deg, double t)
{
    double decl = -23.44 * PI / 180.0 * cos(2.0 * PI * (t + 10.0 / DAYS_PER_YEAR));
    double phi = lat_deg * PI / 180.0;
    double x = -tan(phi) * tan(decl);
    double h0;
    if (x >= 1.0) h0 = 0.0;          /* polar night */
    else if (x <= -1.0) h0 = PI;     /* polar day */
    else h0 = acos(x);
    double q = SOLAR_CONSTANT / PI * (h0 * sin(phi) * sin(decl) + cos(phi) * cos(decl) * sin(h0));
    return q > 0.0 ? q : 0.0;
}

void oracle_spmm_interp(int n, const int *rowptr, const int *colidx,
                        const double *v0, const double *v1, double w,
                        int W, const double *x, double *y)
{
    ROWS_IN_PARALLEL
    for (int i = 0; i < n; ++i) {
        for (int c = 0; c < W; ++c) {
            double acc = 0.0;
            for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                double a = (1.0 - w) * v0[e] + w * v1[e];
                acc += a * x[(size_t)colidx[e] * W + c];
            }
            y[(size_t)i * W + c] = acc;
        }
    }
}

/* y = ((1-w) A_k0 + w A_k1)^T x */
static void spmm_interp_transposed(int n, const int *rowptr, const int *colidx,
                                   const double *v0, const double *v1, double w,
                                   int W, const double *x, double *y)
{
    memset(y, 0, sizeof(double) * (size_t)n * W);
    for (int i = 0; i < n; ++i) {
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            double a = (1.0 - w) * v0[e] + w * v1[e];
            for (int c = 0; c < W; ++c)
                y[(size_t)colidx[e] * W + c] += a * x[(size_t)i * W + c];
        }
    }
}

/* ---------------------------------------------------------------------------
 * Biogeochemical model of one water column (sections 2.2.1 and 5).
 * ------------------------------------------------------------------------ */

typedef struct {
    int ntracer;            /* 1 (N), 2 (PO4, DOP) or 3 (PO4, DOP, PHY) */
    int nl;                 /* wet layers in this column */
    int neu;                /* euphotic layers */
    const double *h;        /* layer heights of the grid, at least max(nl, neu) */
    double insol;           /* I_SWR, W/m^2 */
    double alpha, kw, k1, ki, lam, sig, b;     /* alpha is mu_1 in PO4-DOP-PHY */
    double lam3, kap3, lam3p, sig3;            /* PO4-DOP-PHY only */
} column_ctx;

static void column_params(column_ctx *c, int model, const double *u)
{
    c->alpha = u[0];
    c->kw = u[1];
    c->k1 = u[2];
    c->ki = u[3];
    c->lam3 = c->kap3 = c->lam3p = c->sig3 = 0.0;
    if (model == ORACLE_MODEL_NDOPPHY) {
        c->lam = u[4];
        c->sig = u[5];
        c->lam3 = u[6];
        c->kap3 = u[7];
        c->lam3p = u[8];
        c->sig3 = u[9];
        c->b = u[10];
    } else if (model == ORACLE_MODEL_NDOP) {
        c->lam = u[4];
        c->sig = u[5];
        c->b = u[6];
    } else {
        c->lam = 0.0;
        c->sig = 0.0;
        c->b = u[4];
    }
}

/* Parameter slots of the gradient for each model. */
static void param_slots(int model, int *ia, int *ikw, int *ik1, int *iki, int *ilam, int *isig, int *ib)
{
    *ia = 0; *ikw = 1; *ik1 = 2; *iki = 3;
    if (model == ORACLE_MODEL_NDOP) { *ilam = 4; *isig = 5; *ib = 6; }
    else if (model == ORACLE_MODEL_NDOPPHY) { *ilam = 4; *isig = 5; *ib = 10; }
    else { *ilam = -1; *isig = -1; *ib = 4; }
}

/* Bottom depth d_k of layer k. */
static double layer_bottom(const double *h, int k)
{
    double d = 0.0;
    for (int i = 0; i <= k; ++i) d += h[i];
    return d;
}

/* Production f_1 = alpha N/(N+K_1) I/(I+K_I) at layer k and its partial
 * derivatives with respect to N and the parameters. */
typedef struct { double f, dfdN, dalpha, dkw, dk1, dki; } production_t;

static production_t production(const column_ctx *c, int k, double N)
{
    production_t p;
    double z = layer_bottom(c->h, k) - 0.5 * c->h[k];
    double I = c->insol * SIGMA_PAR * (1.0 - SIGMA_ICE) * exp(-z * c->kw);
    double Np = N > 0.0 ? N : 0.0;
    double limN = Np / (Np + c->k1);
    double limI = I / (I + c->ki);
    p.f = c->alpha * limN * limI;
    p.dfdN = N > 0.0 ? c->alpha * c->k1 / ((N + c->k1) * (N + c->k1)) * limI : 0.0;
    p.dalpha = limN * limI;
    p.dkw = c->alpha * limN * c->ki / ((I + c->ki) * (I + c->ki)) * (-z * I);
    p.dk1 = -c->alpha * Np / ((Np + c->k1) * (Np + c->k1)) * limI;
    p.dki = -c->alpha * limN * I / ((I + c->ki) * (I + c->ki));
    return p;
}

/* Fraction rho_k of the export Phi remineralised per metre in layer k, and
 * (when drho_db is not NULL) d rho_k / d b.  sum_k h_k rho_k = 1. */
static void remineralisation(const column_ctx *c, double *rho, double *drho_db)
{
    int nl = c->nl, neu = c->neu;
    for (int k = 0; k < nl; ++k) {
        rho[k] = 0.0;
        if (drho_db) drho_db[k] = 0.0;
    }
    if (nl <= neu) {
        rho[nl - 1] = 1.0 / c->h[nl - 1];
        return;
    }
    /* Martin curve m(z) = (z/l')^-b at the bottom of layers neu-1 .. nl-2;
     * the bottom of layer neu-1 is l' itself, where m = 1. */
    double lp = layer_bottom(c->h, neu - 1);
    double m[MAX_LAYERS], dm[MAX_LAYERS];
    for (int k = neu - 1; k < nl - 1; ++k) {
        double z = layer_bottom(c->h, k);
        m[k] = pow(z / lp, -c->b);
        dm[k] = drho_db ? -log(z / lp) * m[k] : 0.0;
    }
    for (int k = neu; k < nl; ++k) {
        double mbot = k < nl - 1 ? m[k] : 0.0;      /* sea floor: nothing passes */
        double dmbot = k < nl - 1 ? dm[k] : 0.0;
        rho[k] = (m[k - 1] - mbot) / c->h[k];
        if (drho_db) drho_db[k] = (dm[k - 1] - dmbot) / c->h[k];
    }
}

/* Section 2.2.2, PO4-DOP-PHY, one column; y and q are [3][nl] (PO4, DOP, PHY).
 * In the euphotic zone (k < neu):
 *   q_1 = -f_1 + lambda'_2 DOP + (1 - sigma_2) Phi rho_k
 *   q_2 = sigma_2 f_3 + lambda_3 PHY + kappa_3 PHY^2 - lambda'_2 DOP + lambda'_3 PHY
 *   q_3 = (1 - sigma_3) f_1 - lambda_3 PHY - kappa_3 PHY^2 - lambda'_3 PHY
 * below it f_1 = 0 and the lambda_3, kappa_3 terms vanish; f_3 = sigma_3 f_1 and
 * the export is Phi = sum_k h_k f_3,k over the euphotic layers. */
static void column_q_phy(const column_ctx *c, const double *y, double *q)
{
    int nl = c->nl, neu = c->neu;
    const double *N = y, *D = y + nl, *P = y + 2 * nl;
    double rho[MAX_LAYERS], f[MAX_LAYERS];
    remineralisation(c, rho, NULL);
    double Phi = 0.0;
    for (int k = 0; k < nl; ++k) {
        f[k] = 0.0;
        if (k < neu) {
            f[k] = production(c, k, N[k]).f * P[k];
            Phi += c->h[k] * (c->sig3 * f[k]);
        }
    }
    for (int k = 0; k < nl; ++k) {
        double loss = k < neu ? c->lam3 * P[k] + c->kap3 * P[k] * P[k] : 0.0;
        q[k] = -f[k] + c->lam * D[k] + (1.0 - c->sig) * Phi * rho[k];
        q[nl + k] = c->sig * (c->sig3 * f[k]) + loss - c->lam * D[k] + c->lam3p * P[k];
        q[2 * nl + k] = (1.0 - c->sig3) * f[k] - loss - c->lam3p * P[k];
    }
}

static void column_q_phy_tangent(const column_ctx *c, const double *y, const double *yd, double *qd)
{
    int nl = c->nl, neu = c->neu;
    const double *N = y, *P = y + 2 * nl;
    const double *Nd = yd, *Dd = yd + nl, *Pd = yd + 2 * nl;
    double rho[MAX_LAYERS], fd[MAX_LAYERS];
    remineralisation(c, rho, NULL);
    double Phid = 0.0;
    for (int k = 0; k < nl; ++k) {
        fd[k] = 0.0;
        if (k < neu) {
            production_t pr = production(c, k, N[k]);
            fd[k] = pr.dfdN * Nd[k] * P[k] + pr.f * Pd[k];
            Phid += c->h[k] * (c->sig3 * fd[k]);
        }
    }
    for (int k = 0; k < nl; ++k) {
        double lossd = k < neu ? (c->lam3 + 2.0 * c->kap3 * P[k]) * Pd[k] : 0.0;
        qd[k] = -fd[k] + c->lam * Dd[k] + (1.0 - c->sig) * Phid * rho[k];
        qd[nl + k] = c->sig * (c->sig3 * fd[k]) + lossd - c->lam * Dd[k] + c->lam3p * Pd[k];
        qd[2 * nl + k] = (1.0 - c->sig3) * fd[k] - lossd - c->lam3p * Pd[k];
    }
}

/* ybar = (dq/dy)^T mu, ubar += (dq/du)^T mu in the parameter order of the
 * table of section 2.2.2. */
static void column_q_phy_adjoint(const column_ctx *c, const double *y, const double *mu, double *ybar,
                                 double *ubar)
{
    int nl = c->nl, neu = c->neu;
    const double *N = y, *D = y + nl, *P = y + 2 * nl;
    const double *m1 = mu, *m2 = mu + nl, *m3 = mu + 2 * nl;
    double rho[MAX_LAYERS], drho[MAX_LAYERS];
    remineralisation(c, rho, drho);
    double Phi = 0.0, Phibar = 0.0;
    for (int k = 0; k < nl; ++k) {
        if (k < neu) Phi += c->h[k] * (c->sig3 * (production(c, k, N[k]).f * P[k]));
        Phibar += (1.0 - c->sig) * rho[k] * m1[k];
    }
    for (int k = 0; k < nl; ++k) {
        double *bN = ybar + k, *bD = ybar + nl + k, *bP = ybar + 2 * nl + k;
        *bN = 0.0;
        *bP = 0.0;
        if (k < neu) {
            production_t pr = production(c, k, N[k]);
            double f = pr.f * P[k];
            /* f_1 enters q_1 (-1), q_2 (sigma_2 sigma_3), q_3 (1 - sigma_3) and Phi (h_k sigma_3) */
            double fbar = -m1[k] + c->sig * c->sig3 * m2[k] + (1.0 - c->sig3) * m3[k] + c->sig3 * c->h[k] * Phibar;
            double dloss = c->lam3 + 2.0 * c->kap3 * P[k];
            *bN = fbar * pr.dfdN * P[k];
            *bP += fbar * pr.f + dloss * (m2[k] - m3[k]);
            ubar[0] += fbar * pr.dalpha * P[k];
            ubar[1] += fbar * pr.dkw * P[k];
            ubar[2] += fbar * pr.dk1 * P[k];
            ubar[3] += fbar * pr.dki * P[k];
            ubar[5] += c->sig3 * f * m2[k];
            ubar[6] += P[k] * (m2[k] - m3[k]);
            ubar[7] += P[k] * P[k] * (m2[k] - m3[k]);
            ubar[9] += f * (c->sig * m2[k] - m3[k] + c->h[k] * Phibar);
        }
        *bD = c->lam * (m1[k] - m2[k]);
        *bP += c->lam3p * (m2[k] - m3[k]);
        ubar[4] += D[k] * (m1[k] - m2[k]);
        ubar[5] += -Phi * rho[k] * m1[k];
        ubar[8] += P[k] * (m2[k] - m3[k]);
        ubar[10] += (1.0 - c->sig) * Phi * drho[k] * m1[k];
    }
}

/* q for one column: y and q are [ntracer][nl] (tracer-major, as in the
 * Fortran form of the interface). */
static void column_q(const column_ctx *c, const double *y, double *q)
{
    if (c->ntracer == 3) {
        column_q_phy(c, y, q);
        return;
    }
    int nl = c->nl, neu = c->neu, ntr = c->ntracer;
    double rho[MAX_LAYERS], f[MAX_LAYERS];
    remineralisation(c, rho, NULL);
    double Phi = 0.0;
    for (int k = 0; k < nl; ++k) {
        f[k] = 0.0;
        if (k < neu) {
            f[k] = production(c, k, y[k]).f;
            Phi += c->h[k] * f[k];
        }
    }
    for (int k = 0; k < nl; ++k) {
        double dop = ntr > 1 ? y[nl + k] : 0.0;
        q[k] = -f[k] + c->lam * dop + (1.0 - c->sig) * Phi * rho[k];
        if (ntr > 1) q[nl + k] = c->sig * f[k] - c->lam * dop;
    }
}

/* Tangent: qdot = (dq/dy) ydot. */
static void column_q_tangent(const column_ctx *c, const double *y, const double *ydot, double *qdot)
{
    if (c->ntracer == 3) {
        column_q_phy_tangent(c, y, ydot, qdot);
        return;
    }
    int nl = c->nl, neu = c->neu, ntr = c->ntracer;
    double rho[MAX_LAYERS], fdot[MAX_LAYERS];
    remineralisation(c, rho, NULL);
    double Phidot = 0.0;
    for (int k = 0; k < nl; ++k) {
        fdot[k] = 0.0;
        if (k < neu) {
            fdot[k] = production(c, k, y[k]).dfdN * ydot[k];
            Phidot += c->h[k] * fdot[k];
        }
    }
    for (int k = 0; k < nl; ++k) {
        double dopdot = ntr > 1 ? ydot[nl + k] : 0.0;
        qdot[k] = -fdot[k] + c->lam * dopdot + (1.0 - c->sig) * Phidot * rho[k];
        if (ntr > 1) qdot[nl + k] = c->sig * fdot[k] - c->lam * dopdot;
    }
}

/* Adjoint: ybar = (dq/dy)^T mu, ubar += (dq/du)^T mu. */
static void column_q_adjoint(const column_ctx *c, int model, const double *y, const double *mu,
                             double *ybar, double *ubar)
{
    if (c->ntracer == 3) {
        column_q_phy_adjoint(c, y, mu, ybar, ubar);
        return;
    }
    int nl = c->nl, neu = c->neu, ntr = c->ntracer;
    int ia, ikw, ik1, iki, ilam, isig, ib;
    param_slots(model, &ia, &ikw, &ik1, &iki, &ilam, &isig, &ib);
    double rho[MAX_LAYERS], drho[MAX_LAYERS];
    remineralisation(c, rho, drho);

    double Phi = 0.0, Phibar = 0.0;
    for (int k = 0; k < nl; ++k) {
        if (k < neu) Phi += c->h[k] * production(c, k, y[k]).f;
        Phibar += (1.0 - c->sig) * rho[k] * mu[k];
    }
    for (int k = 0; k < nl; ++k) {
        double mu1 = mu[k];
        double mu2 = ntr > 1 ? mu[nl + k] : 0.0;
        double dop = ntr > 1 ? y[nl + k] : 0.0;
        ybar[k] = 0.0;
        if (k < neu) {
            production_t p = production(c, k, y[k]);
            double fbar = -mu1 + c->sig * mu2 + c->h[k] * Phibar;
            ybar[k] = fbar * p.dfdN;
            ubar[ia] += fbar * p.dalpha;
            ubar[ikw] += fbar * p.dkw;
            ubar[ik1] += fbar * p.dk1;
            ubar[iki] += fbar * p.dki;
            if (isig >= 0) ubar[isig] += p.f * mu2;
        }
        if (ntr > 1) {
            ybar[nl + k] = c->lam * (mu1 - mu2);
            ubar[ilam] += dop * (mu1 - mu2);
            ubar[isig] += -Phi * rho[k] * mu1;
        }
        ubar[ib] += (1.0 - c->sig) * Phi * drho[k] * mu1;
    }
}

/* Section 7: the biogeochemical models take eight internal time steps per
 * ocean step.  The source over one ocean step of length dt is the increment of
 * nsub explicit Euler sub-steps of length dt/nsub at fixed forcing:
 *   inc_0 = 0,  inc_{s+1} = inc_s + (dt/nsub) q(y + inc_s),  source = inc_nsub.
 * With nsub = 1 this is dt*q(y). */
#define MAX_SUBSTEPS 32

static void column_source(const column_ctx *c, const double *y, double dt, int nsub, double *inc)
{
    int len = c->ntracer * c->nl;
    double yt[MAX_TRACERS * MAX_LAYERS], q[MAX_TRACERS * MAX_LAYERS];
    double h = dt / nsub;
    for (int i = 0; i < len; ++i) inc[i] = 0.0;
    for (int s = 0; s < nsub; ++s) {
        for (int i = 0; i < len; ++i) yt[i] = y[i] + inc[i];
        column_q(c, yt, q);
        for (int i = 0; i < len; ++i) inc[i] += h * q[i];
    }
}

/* Tangent of column_source in direction ydot. */
static void column_source_tangent(const column_ctx *c, const double *y, const double *ydot, double dt, int nsub,
                                  double *incdot)
{
    int len = c->ntracer * c->nl;
    double inc[MAX_TRACERS * MAX_LAYERS], yt[MAX_TRACERS * MAX_LAYERS], ytd[MAX_TRACERS * MAX_LAYERS], q[MAX_TRACERS * MAX_LAYERS], qd[MAX_TRACERS * MAX_LAYERS];
    double h = dt / nsub;
    for (int i = 0; i < len; ++i) { inc[i] = 0.0; incdot[i] = 0.0; }
    for (int s = 0; s < nsub; ++s) {
        for (int i = 0; i < len; ++i) { yt[i] = y[i] + inc[i]; ytd[i] = ydot[i] + incdot[i]; }
        column_q(c, yt, q);
        column_q_tangent(c, yt, ytd, qd);
        for (int i = 0; i < len; ++i) { inc[i] += h * q[i]; incdot[i] += h * qd[i]; }
    }
}

/* Adjoint of column_source: given mu, the cotangent of the source,
 * ybar = (d source/dy)^T mu and ubar += (d source/du)^T mu. */
static void column_source_adjoint(const column_ctx *c, int model, const double *y, const double *mu, double dt,
                                  int nsub, double *ybar, double *ubar)
{
    int len = c->ntracer * c->nl;
    double ytraj[MAX_SUBSTEPS][MAX_TRACERS * MAX_LAYERS];
    double inc[MAX_TRACERS * MAX_LAYERS], q[MAX_TRACERS * MAX_LAYERS], ibar[MAX_TRACERS * MAX_LAYERS], yb[MAX_TRACERS * MAX_LAYERS];
    double h = dt / nsub;
    for (int i = 0; i < len; ++i) inc[i] = 0.0;
    for (int s = 0; s < nsub; ++s) {
        for (int i = 0; i < len; ++i) ytraj[s][i] = y[i] + inc[i];
        column_q(c, ytraj[s], q);
        for (int i = 0; i < len; ++i) inc[i] += h * q[i];
    }
    for (int i = 0; i < len; ++i) { ibar[i] = mu[i]; ybar[i] = 0.0; }
    for (int s = nsub - 1; s >= 0; --s) {
        double ucol[MAX_PARAMS] = {0};
        column_q_adjoint(c, model, ytraj[s], ibar, yb, ucol);
        for (int i = 0; i < len; ++i) {
            ybar[i] += h * yb[i];
            ibar[i] += h * yb[i];
        }
        for (int p = 0; p < MAX_PARAMS; ++p) ubar[p] += h * ucol[p];
    }
}

int oracle_bgc_source(int model, double insol, int nlayer, const double *h, const double *y, double *inc,
                      const double *u, int neuphotic, double dt, int nsub)
{
    int ntr = oracle_ntracer(model);
    if (ntr < 0 || nlayer < 1 || nlayer > MAX_LAYERS || neuphotic < 1 || nsub < 1 || nsub > MAX_SUBSTEPS)
        return -1;
    column_ctx c;
    c.ntracer = ntr; c.nl = nlayer; c.neu = neuphotic; c.h = h; c.insol = insol;
    column_params(&c, model, u);
    column_source(&c, y, dt, nsub, inc);
    return 0;
}

int oracle_bgc_column(int model, double insol, int nlayer, const double *h,
                      const double *y, double *q, const double *u, int neuphotic)
{
    int ntr = oracle_ntracer(model);
    if (ntr < 0 || nlayer < 1 || nlayer > MAX_LAYERS || neuphotic < 1) return -1;
    column_ctx c;
    c.ntracer = ntr; c.nl = nlayer; c.neu = neuphotic; c.h = h; c.insol = insol;
    column_params(&c, model, u);
    column_q(&c, y, q);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Step, year, tangent, reverse mode.
 * ------------------------------------------------------------------------ */

static int check_desc(const oracle_desc *g, int nbatch)
{
    if (!g || g->n < 1 || g->ncol < 1 || g->nlayer < 1 || g->nlayer > MAX_LAYERS) return -1;
    if (oracle_ntracer(g->model) < 0 || nbatch < 1) return -1;
    if (g->nmat < 1 || g->nstep < 1 || g->nstep % g->nmat != 0 || (g->nstep / g->nmat) % 2 != 0) return -1;
    if (g->neuphotic < 1 || g->neuphotic > g->nlayer) return -1;
    if (g->nbgc < 0 || g->nbgc > MAX_SUBSTEPS) return -1;
    if (g->col_start[0] != 0 || g->col_start[g->ncol] != g->n) return -1;
    for (int c = 0; c < g->ncol; ++c) {
        int nl = g->col_start[c + 1] - g->col_start[c];
        if (nl < 1 || nl > g->nlayer) return -1;
    }
    return 0;
}

static double step_days(const oracle_desc *g) { return DAYS_PER_YEAR / (double)g->nstep; }
static int substeps(const oracle_desc *g) { return g->nbgc > 1 ? g->nbgc : 1; }

/* Gathers member b of column c from the n x W state into [ntracer][nl]. */
static void gather_column(const oracle_desc *g, int W, int b, int c, const double *y, double *col)
{
    int ntr = oracle_ntracer(g->model);
    int s = g->col_start[c], nl = g->col_start[c + 1] - s;
    for (int tr = 0; tr < ntr; ++tr)
        for (int k = 0; k < nl; ++k)
            col[tr * nl + k] = y[(size_t)(s + k) * W + b * ntr + tr];
}

static void scatter_add_column(const oracle_desc *g, int W, int b, int c, const double *col,
                               double scale, double *y)
{
    int ntr = oracle_ntracer(g->model);
    int s = g->col_start[c], nl = g->col_start[c + 1] - s;
    for (int tr = 0; tr < ntr; ++tr)
        for (int k = 0; k < nl; ++k)
            y[(size_t)(s + k) * W + b * ntr + tr] += scale * col[tr * nl + k];
}

static void make_column(const oracle_desc *g, int c, double t, const double *u, int model, column_ctx *cc)
{
    cc->ntracer = oracle_ntracer(model);
    cc->nl = g->col_start[c + 1] - g->col_start[c];
    cc->neu = g->neuphotic;
    cc->h = g->dz;
    cc->insol = oracle_insolation(g->lat[c], t);
    column_params(cc, model, u);
}

/* z += dt_d * q(y) for every column and member. */
static void add_sources(const oracle_desc *g, int nbatch, const double *u, int j,
                        const double *y, double *z)
{
    int ntr = oracle_ntracer(g->model), np = oracle_nparam(g->model), W = nbatch * ntr;
    double t = (double)(((j % g->nstep) + g->nstep) % g->nstep) / (double)g->nstep;
    ROWS_IN_PARALLEL
    for (int c = 0; c < g->ncol; ++c) {
        double col[MAX_TRACERS * MAX_LAYERS], inc[MAX_TRACERS * MAX_LAYERS];
        for (int b = 0; b < nbatch; ++b) {
            column_ctx cc;
            make_column(g, c, t, u + (size_t)b * np, g->model, &cc);
            gather_column(g, W, b, c, y, col);
            column_source(&cc, col, step_days(g), substeps(g), inc);
            scatter_add_column(g, W, b, c, inc, 1.0, z);
        }
    }
}

int oracle_step(const oracle_desc *g, int nbatch, const double *u, int j,
                const double *y_in, double *y_out)
{
    if (check_desc(g, nbatch)) return -1;
    int W = nbatch * oracle_ntracer(g->model);
    int k0, k1;
    double w;
    oracle_phase(j, g->nstep, g->nmat, &k0, &k1, &w);
    double *z = malloc(sizeof(double) * (size_t)g->n * W);
    if (!z) return -2;
    oracle_spmm_interp(g->n, g->ae_rowptr, g->ae_colidx, g->ae_val + (size_t)k0 * g->ae_nnz,
                       g->ae_val + (size_t)k1 * g->ae_nnz, w, W, y_in, z);
    add_sources(g, nbatch, u, j, y_in, z);
    oracle_spmm_interp(g->n, g->ai_rowptr, g->ai_colidx, g->ai_val + (size_t)k0 * g->ai_nnz,
                       g->ai_val + (size_t)k1 * g->ai_nnz, w, W, z, y_out);
    free(z);
    return 0;
}

int oracle_year(const oracle_desc *g, int nbatch, const double *u, int nyears,
                const double *y0, double *y1, double *resid)
{
    if (check_desc(g, nbatch) || nyears < 0) return -1;
    int ntr = oracle_ntracer(g->model), W = nbatch * ntr;
    size_t len = (size_t)g->n * W;
    double *a = malloc(sizeof(double) * len), *b = malloc(sizeof(double) * len);
    if (!a || !b) { free(a); free(b); return -2; }
    memcpy(a, y0, sizeof(double) * len);
    for (int yr = 0; yr < nyears; ++yr) {
        double *start = malloc(sizeof(double) * len);
        if (!start) { free(a); free(b); return -2; }
        memcpy(start, a, sizeof(double) * len);
        for (int j = 0; j < g->nstep; ++j) {
            int rc = oracle_step(g, nbatch, u, j, a, b);
            if (rc) { free(a); free(b); free(start); return rc; }
            double *t = a; a = b; b = t;
        }
        if (resid) {
            for (int m = 0; m < nbatch; ++m) {
                double s = 0.0;
                for (size_t i = 0; i < (size_t)g->n; ++i)
                    for (int tr = 0; tr < ntr; ++tr) {
                        double d = start[i * W + m * ntr + tr] - a[i * W + m * ntr + tr];
                        s += d * d;
                    }
                resid[(size_t)yr * nbatch + m] = sqrt(s);
            }
        }
        free(start);
    }
    memcpy(y1, a, sizeof(double) * len);
    free(a);
    free(b);
    return 0;
}

int oracle_year_tangent(const oracle_desc *g, int nbatch, const double *u,
                        const double *y, const double *v, double *phi_y, double *jv)
{
    if (check_desc(g, nbatch)) return -1;
    int ntr = oracle_ntracer(g->model), np = oracle_nparam(g->model), W = nbatch * ntr;
    size_t len = (size_t)g->n * W;
    double *ya = malloc(sizeof(double) * len), *yb = malloc(sizeof(double) * len);
    double *va = malloc(sizeof(double) * len), *vb = malloc(sizeof(double) * len);
    double *z = malloc(sizeof(double) * len);
    if (!ya || !yb || !va || !vb || !z) { free(ya); free(yb); free(va); free(vb); free(z); return -2; }
    memcpy(ya, y, sizeof(double) * len);
    memcpy(va, v, sizeof(double) * len);
    double col[MAX_TRACERS * MAX_LAYERS], dcol[MAX_TRACERS * MAX_LAYERS], qd[MAX_TRACERS * MAX_LAYERS];
    for (int j = 0; j < g->nstep; ++j) {
        int k0, k1;
        double w;
        oracle_phase(j, g->nstep, g->nmat, &k0, &k1, &w);
        double t = (double)j / (double)g->nstep;
        /* tangent: zdot = Ae vdot + dt_d qdot(y; vdot); vdot' = Ai zdot */
        oracle_spmm_interp(g->n, g->ae_rowptr, g->ae_colidx, g->ae_val + (size_t)k0 * g->ae_nnz,
                           g->ae_val + (size_t)k1 * g->ae_nnz, w, W, va, z);
        for (int c = 0; c < g->ncol; ++c)
            for (int b = 0; b < nbatch; ++b) {
                column_ctx cc;
                make_column(g, c, t, u + (size_t)b * np, g->model, &cc);
                gather_column(g, W, b, c, ya, col);
                gather_column(g, W, b, c, va, dcol);
                column_source_tangent(&cc, col, dcol, step_days(g), substeps(g), qd);
                scatter_add_column(g, W, b, c, qd, 1.0, z);
            }
        oracle_spmm_interp(g->n, g->ai_rowptr, g->ai_colidx, g->ai_val + (size_t)k0 * g->ai_nnz,
                           g->ai_val + (size_t)k1 * g->ai_nnz, w, W, z, vb);
        /* primal step */
        oracle_step(g, nbatch, u, j, ya, yb);
        double *t1 = ya; ya = yb; yb = t1;
        double *t2 = va; va = vb; vb = t2;
    }
    if (phi_y) memcpy(phi_y, ya, sizeof(double) * len);
    memcpy(jv, va, sizeof(double) * len);
    free(ya); free(yb); free(va); free(vb); free(z);
    return 0;
}

int oracle_year_jvp_fd(const oracle_desc *g, int nbatch, const double *u,
                       const double *y, const double *v, double *phi_y, double *jv)
{
    if (check_desc(g, nbatch)) return -1;
    int ntr = oracle_ntracer(g->model), W = nbatch * ntr;
    size_t len = (size_t)g->n * W;
    double *yp = malloc(sizeof(double) * len), *fp = malloc(sizeof(double) * len);
    double *f0 = malloc(sizeof(double) * len);
    double *h = malloc(sizeof(double) * nbatch);
    if (!yp || !fp || !f0 || !h) { free(yp); free(fp); free(f0); free(h); return -2; }
    for (int b = 0; b < nbatch; ++b) {
        double ny = 0.0, nv = 0.0;
        for (size_t i = 0; i < (size_t)g->n; ++i)
            for (int tr = 0; tr < ntr; ++tr) {
                double a = y[i * W + b * ntr + tr], d = v[i * W + b * ntr + tr];
                ny += a * a;
                nv += d * d;
            }
        h[b] = nv > 0.0 ? 1e-8 * sqrt(ny) / sqrt(nv) : 0.0;
    }
    for (size_t i = 0; i < (size_t)g->n; ++i)
        for (int b = 0; b < nbatch; ++b)
            for (int tr = 0; tr < ntr; ++tr) {
                size_t e = i * W + b * ntr + tr;
                yp[e] = y[e] + h[b] * v[e];
            }
    int rc = oracle_year(g, nbatch, u, 1, y, f0, NULL);
    if (!rc) rc = oracle_year(g, nbatch, u, 1, yp, fp, NULL);
    if (!rc) {
        for (size_t i = 0; i < (size_t)g->n; ++i)
            for (int b = 0; b < nbatch; ++b)
                for (int tr = 0; tr < ntr; ++tr) {
                    size_t e = i * W + b * ntr + tr;
                    jv[e] = h[b] > 0.0 ? (fp[e] - f0[e]) / h[b] : 0.0;
                }
        if (phi_y) memcpy(phi_y, f0, sizeof(double) * len);
    }
    free(yp); free(fp); free(f0); free(h);
    return rc;
}

/* Cell volumes V_i = area_c h_k. */
static double *cell_volumes(const oracle_desc *g, double *vtot)
{
    double *V = malloc(sizeof(double) * g->n);
    if (!V) return NULL;
    double s = 0.0;
    for (int c = 0; c < g->ncol; ++c)
        for (int r = g->col_start[c]; r < g->col_start[c + 1]; ++r) {
            V[r] = g->area[c] * g->dz[r - g->col_start[c]];
            s += V[r];
        }
    *vtot = s;
    return V;
}

/* Snapshot index m of step s (s = (m+1)*nstep/nmat), or -1. */
static int snapshot_of(const oracle_desc *g, int s)
{
    int spm = g->nstep / g->nmat;
    if (s <= 0 || s % spm != 0) return -1;
    return s / spm - 1;
}

/* Forward with the whole trajectory kept, then the reverse sweep.  The
 * cotangent of y_nstep is wbar (nullable) plus the misfit source; the misfit
 * and its sources are skipped when obs is NULL. */
static int reverse_year(const oracle_desc *g, int nbatch, const double *u, const double *y0,
                        const double *obs, const double *wbar,
                        double *J, double *ubar, double *ybar0)
{
    if (check_desc(g, nbatch)) return -1;
    int ntr = oracle_ntracer(g->model), np = oracle_nparam(g->model), W = nbatch * ntr;
    int nstep = g->nstep;
    size_t len = (size_t)g->n * W;
    double vtot;
    double *V = cell_volumes(g, &vtot);
    double *traj = malloc(sizeof(double) * len * (size_t)(nstep + 1));
    double *lam = malloc(sizeof(double) * len), *mu = malloc(sizeof(double) * len);
    double *lam2 = malloc(sizeof(double) * len);
    double *ub = calloc((size_t)nbatch * np, sizeof(double));
    if (!V || !traj || !lam || !mu || !lam2 || !ub) {
        free(V); free(traj); free(lam); free(mu); free(lam2); free(ub);
        return -2;
    }
    memcpy(traj, y0, sizeof(double) * len);
    for (int j = 0; j < nstep; ++j)
        oracle_step(g, nbatch, u, j, traj + (size_t)j * len, traj + (size_t)(j + 1) * len);

    if (J) for (int b = 0; b < nbatch; ++b) J[b] = 0.0;
    if (J && obs) {
        for (int m = 0; m < g->nmat; ++m) {
            const double *ys = traj + (size_t)((m + 1) * (nstep / g->nmat)) * len;
            const double *o = obs + (size_t)m * len;
            for (size_t i = 0; i < (size_t)g->n; ++i)
                for (int b = 0; b < nbatch; ++b)
                    for (int tr = 0; tr < ntr; ++tr) {
                        size_t e = i * W + b * ntr + tr;
                        double d = ys[e] - o[e];
                        J[b] += V[i] * d * d / (2.0 * g->nmat * vtot);
                    }
        }
    }

    /* cotangent of the final state */
    for (size_t e = 0; e < len; ++e) lam[e] = wbar ? wbar[e] : 0.0;
    if (obs) {
        const double *ys = traj + (size_t)nstep * len;
        const double *o = obs + (size_t)(g->nmat - 1) * len;
        for (size_t i = 0; i < (size_t)g->n; ++i)
            for (int c = 0; c < W; ++c)
                lam[i * W + c] += V[i] * (ys[i * W + c] - o[i * W + c]) / (g->nmat * vtot);
    }

    double col[MAX_TRACERS * MAX_LAYERS], mcol[MAX_TRACERS * MAX_LAYERS], yb[MAX_TRACERS * MAX_LAYERS];
    for (int j = nstep - 1; j >= 0; --j) {
        int k0, k1;
        double w;
        oracle_phase(j, nstep, g->nmat, &k0, &k1, &w);
        double t = (double)j / (double)nstep;
        const double *yj = traj + (size_t)j * len;
        /* mu = Ai(t_j)^T lam_{j+1} is the cotangent of z_j */
        spmm_interp_transposed(g->n, g->ai_rowptr, g->ai_colidx, g->ai_val + (size_t)k0 * g->ai_nnz,
                               g->ai_val + (size_t)k1 * g->ai_nnz, w, W, lam, mu);
        /* lam_j = Ae(t_j)^T mu + dt_d (dq/dy)^T mu */
        spmm_interp_transposed(g->n, g->ae_rowptr, g->ae_colidx, g->ae_val + (size_t)k0 * g->ae_nnz,
                               g->ae_val + (size_t)k1 * g->ae_nnz, w, W, mu, lam2);
        for (int c = 0; c < g->ncol; ++c)
            for (int b = 0; b < nbatch; ++b) {
                column_ctx cc;
                double ucol[MAX_PARAMS] = {0};
                make_column(g, c, t, u + (size_t)b * np, g->model, &cc);
                gather_column(g, W, b, c, yj, col);
                gather_column(g, W, b, c, mu, mcol);
                column_source_adjoint(&cc, g->model, col, mcol, step_days(g), substeps(g), yb, ucol);
                scatter_add_column(g, W, b, c, yb, 1.0, lam2);
                for (int p = 0; p < np; ++p) ub[(size_t)b * np + p] += ucol[p];
            }
        int m = snapshot_of(g, j);
        if (obs && m >= 0) {
            const double *o = obs + (size_t)m * len;
            for (size_t i = 0; i < (size_t)g->n; ++i)
                for (int c = 0; c < W; ++c)
                    lam2[i * W + c] += V[i] * (yj[i * W + c] - o[i * W + c]) / (g->nmat * vtot);
        }
        double *tmp = lam; lam = lam2; lam2 = tmp;
    }
    if (ybar0) memcpy(ybar0, lam, sizeof(double) * len);
    if (ubar) memcpy(ubar, ub, sizeof(double) * (size_t)nbatch * np);
    free(V); free(traj); free(lam); free(mu); free(lam2); free(ub);
    return 0;
}

int oracle_year_misfit(const oracle_desc *g, int nbatch, const double *u,
                       const double *y0, const double *obs, double *J)
{
    if (check_desc(g, nbatch) || !obs || !J) return -1;
    int ntr = oracle_ntracer(g->model), W = nbatch * ntr;
    size_t len = (size_t)g->n * W;
    double vtot;
    double *V = cell_volumes(g, &vtot);
    double *a = malloc(sizeof(double) * len), *b = malloc(sizeof(double) * len);
    if (!V || !a || !b) { free(V); free(a); free(b); return -2; }
    memcpy(a, y0, sizeof(double) * len);
    for (int m = 0; m < nbatch; ++m) J[m] = 0.0;
    for (int j = 0; j < g->nstep; ++j) {
        oracle_step(g, nbatch, u, j, a, b);
        double *t = a; a = b; b = t;
        int m = snapshot_of(g, j + 1);
        if (m >= 0) {
            const double *o = obs + (size_t)m * len;
            for (size_t i = 0; i < (size_t)g->n; ++i)
                for (int mb = 0; mb < nbatch; ++mb)
                    for (int tr = 0; tr < ntr; ++tr) {
                        size_t e = i * W + mb * ntr + tr;
                        double d = a[e] - o[e];
                        J[mb] += V[i] * d * d / (2.0 * g->nmat * vtot);
                    }
        }
    }
    free(V); free(a); free(b);
    return 0;
}

int oracle_year_adjoint(const oracle_desc *g, int nbatch, const double *u,
                        const double *y0, const double *obs,
                        double *J, double *dJdu, double *dJdy0)
{
    if (!obs) return -1;
    return reverse_year(g, nbatch, u, y0, obs, NULL, J, dJdu, dJdy0);
}

int oracle_year_vjp(const oracle_desc *g, int nbatch, const double *u,
                    const double *y0, const double *wbar, double *ybar, double *ubar)
{
    if (!wbar) return -1;
    return reverse_year(g, nbatch, u, y0, NULL, wbar, NULL, ubar, ybar);
}
