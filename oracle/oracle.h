/*
 * Reference CPU implementation of the transport-matrix time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, float64 restatement of the
 * method of Piwonski & Slawig, "The Idea and Concept of Metos3D" (arXiv
 * 1410.0204), used to check the GPU library.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * source with the GPU library and the GPU library never calls it.
 *
 * State layout: row-major n x W with W = nbatch*ntracer, element
 * y[i*W + b*ntracer + tr] (row i, ensemble member b, tracer tr).  Rows of one
 * water column are contiguous, surface first (section 5.1).
 *
 * All functions return 0 on success and a negative value on invalid input.
 */
#ifndef TMM_ORACLE_H
#define TMM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_MODEL_N = 1, ORACLE_MODEL_NDOP = 2, ORACLE_MODEL_NDOPPHY = 3 };

typedef struct {
    int n, ncol, nlayer;
    const int *col_start;   /* [ncol+1] */
    const double *lat;      /* [ncol] degrees */
    const double *area;     /* [ncol] m^2 */
    const double *dz;       /* [nlayer] layer heights h_k, m */
    int nmat, nstep, model, neuphotic;
    int ae_nnz;
    const int *ae_rowptr, *ae_colidx;
    const double *ae_val;   /* [nmat][ae_nnz] */
    int ai_nnz;
    const int *ai_rowptr, *ai_colidx;
    const double *ai_val;   /* [nmat][ai_nnz] */
    int nbgc;               /* internal BGC steps per ocean step (section 7); 0 or 1 = one */
} oracle_desc;

int oracle_ntracer(int model);
int oracle_nparam(int model);

/* Month pair and weight of step j (section 3: linear interpolation between
 * monthly matrices; anchors at mid-month, periodic in the year). */
void oracle_phase(int j, int nstep, int nmat, int *k0, int *k1, double *w);

/* Daily-mean top-of-atmosphere short-wave radiation (W/m^2) at latitude
 * lat_deg (degrees) and time t (fraction of a 360-day year). */
double oracle_insolation(double lat_deg, double t);

/* y = ((1-w) A_k0 + w A_k1) x for a CSR pattern and W right-hand sides. */
void oracle_spmm_interp(int n, const int *rowptr, const int *colidx,
                        const double *v0, const double *v1, double w,
                        int W, const double *x, double *y);

/* Source-minus-sink term q (per day) of one water column, in the layout of
 * the biogeochemical interface (section 5.2): y and q are [ntracer][nlayer]. */
int oracle_bgc_column(int model, double insol, int nlayer, const double *h,
                      const double *y, double *q, const double *u, int neuphotic);

/* Source of one ocean step of length dt for one column with nsub internal
 * BGC steps (section 7): inc = y_nsub - y of explicit Euler at fixed forcing. */
int oracle_bgc_source(int model, double insol, int nlayer, const double *h, const double *y, double *inc,
                      const double *u, int neuphotic, double dt, int nsub);

/* Sets the thread count of the step's parallel loops when n >= 1 (timing
 * build with OpenMP only) and returns the count in use (1 without OpenMP). */
int oracle_threads(int n);

/* One step y_out = Ai(t_j) (Ae(t_j) y_in + dt*q(y_in)) (section 3). */
int oracle_step(const oracle_desc *g, int nbatch, const double *u, int j,
                const double *y_in, double *y_out);

/* nyears model years (nstep steps each).  resid (nullable) receives
 * ||y - phi(y)||_2 per year and member: [nyears][nbatch]. */
int oracle_year(const oracle_desc *g, int nbatch, const double *u, int nyears,
                const double *y0, double *y1, double *resid);

/* Forward tangent of one model year: phi_y = phi(y), jv = phi'(y) v. */
int oracle_year_tangent(const oracle_desc *g, int nbatch, const double *u,
                        const double *y, const double *v, double *phi_y, double *jv);

/* Finite-difference directional derivative (phi(y+h v) - phi(y))/h with
 * h = 1e-8*||y||_2/||v||_2 per member. */
int oracle_year_jvp_fd(const oracle_desc *g, int nbatch, const double *u,
                       const double *y, const double *v, double *phi_y, double *jv);

/* Misfit J_b = sum_m sum_i sum_tr V_i (y_{s_m} - obs_m)^2 / (2*nmat*V_tot) over
 * the nmat month-end snapshots s_m = (m+1)*nstep/nmat.  obs: [nmat][n][W]. */
int oracle_year_misfit(const oracle_desc *g, int nbatch, const double *u,
                       const double *y0, const double *obs, double *J);

/* Reverse mode of the misfit over one model year, storing the full
 * trajectory: J [nbatch], dJdu [nbatch][nparam], dJdy0 [n][W] (nullable). */
int oracle_year_adjoint(const oracle_desc *g, int nbatch, const double *u,
                        const double *y0, const double *obs,
                        double *J, double *dJdu, double *dJdy0);

/* Vector-Jacobian product of the year map: ybar = phi'(y)^T wbar and
 * ubar = (d phi / d u)^T wbar (nullable). */
int oracle_year_vjp(const oracle_desc *g, int nbatch, const double *u,
                    const double *y0, const double *wbar, double *ybar, double *ubar);

#ifdef __cplusplus
}
#endif
#endif
