/*
 * libtmm -- transport-matrix time stepping of marine biogeochemical tracers
 * on one AMD Instinct MI355X (gfx950), float64 throughout.
 *
 * The method is the one of Piwonski & Slawig, "The Idea and Concept of
 * Metos3D" (arXiv 1410.0204):
 *
 *   y_{j+1} = A_imp(t_j) (A_exp(t_j) y_j + dt * q(y_j, u)),   j = 0..nstep-1
 *
 * (section 3), where A_exp / A_imp are linear interpolations between twelve
 * monthly explicit (horizontal) and implicit (vertical) transport matrices
 * (sections 3 and 7), q is a biogeochemical model evaluated per water column
 * (sections 2.2 and 5), and nstep = 2880 steps make one model year.  The
 * year map y(T) = phi(y(0)) (section 4) is the unit of work of spin-up and of
 * matrix-free Newton-Krylov solvers (section 6).
 *
 * Conventions (following the C form of the paper's interface, section 5.2):
 * reals are double, counts are int, arrays are a pointer plus int sizes.
 *
 * State layout.  A state is a device array of n rows by W = nbatch*ntracer
 * columns, row-major: y[i*W + b*ntracer + tr] is tracer tr of ensemble member
 * b at grid point i.  Grid points of one water column are contiguous, surface
 * first (section 5.1).
 *
 * Ownership.  The caller owns every buffer.  The library never allocates
 * device memory: it works inside one caller-provided device workspace of
 * tmm_workspace_bytes() bytes, which must stay allocated until tmm_destroy().
 * Host arrays of the descriptor are read during tmm_create() only.
 *
 * Errors.  Every call returns TMM_OK (0) or a negative status; a call that
 * fails validation changes nothing.  Kernels run asynchronously on the stream
 * given at creation; calls that return host results (resid_host, J_host,
 * dJdu_host) synchronise that stream and report device errors there.
 * A handle is not thread-safe; use one handle per stream.
 */
#ifndef TMM_H
#define TMM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tmm_ctx *tmm_handle;

enum {
    TMM_OK = 0,
    TMM_EINVAL = -1,        /* invalid argument or descriptor */
    TMM_ENOMEM = -2,        /* workspace too small */
    TMM_EDEVICE = -3,       /* HIP runtime error, or a wait of the persistent kernels gave up */
    TMM_ESTATE = -4,        /* call not valid in the handle's state (e.g. no parameters set) */
    TMM_ENONFINITE = -5,    /* non-finite value found in a result (or in the state at the end of a
                               model year of tmm_year) */
    TMM_EUNSUPPORTED = -6,  /* valid request outside what this build supports */
    TMM_ETOOBIG = -7        /* request exceeds the fixed scratch of tmm_year_noalloc */
};

/* Biogeochemical models (section 2.2).  Parameter order is the order of the
 * paper's parameter table. */
enum {
    TMM_MODEL_N = 1,        /* 1 tracer (nutrient); u = alpha, K_H2O, K_N, K_I, b */
    TMM_MODEL_NDOP = 2,     /* PO4-DOP (section 2.2.1), 2 tracers;
                               u = alpha, K_H2O, K_1, K_I, lambda'_2, sigma_2, b */
    TMM_MODEL_NDOPPHY = 3   /* PO4-DOP-PHY (section 2.2.2), 3 tracers (PO4, DOP, PHY);
                               u = mu_1, K_H2O, K_1, K_I, lambda'_2, sigma_2, lambda_3, kappa_3,
                               lambda'_3, sigma_3, b */
};

/* Directional derivative of the year map (section 6.1). */
enum {
    TMM_JVP_FD = 0,         /* finite difference (phi(y+h v) - phi(y))/h, h = 1e-8 |y|/|v| per member */
    TMM_JVP_TANGENT = 1,    /* exact forward-mode tangent */
    TMM_JVP_FD_GIVEN_PHI = 2 /* as TMM_JVP_FD with phi_y = phi(y) supplied by the caller (input): one
                               year map per product, as inside a Krylov solve at a fixed Newton iterate */
};

typedef struct {
    int n;                  /* wet grid points */
    int ncol;               /* water columns */
    int nlayer;             /* maximum layers per column (<= 64) */
    const int *col_start;   /* [ncol+1] first row of each column; col_start[ncol] = n */
    const double *lat;      /* [ncol] latitude of each column, degrees */
    const double *area;     /* [ncol] horizontal area of each column, m^2 */
    const double *dz;       /* [nlayer] layer heights h_k, m, surface first */
    int nmat;               /* monthly matrices of each kind (12) */
    int nstep;              /* steps per model year (2880); nstep/nmat must be even */
    int model;              /* TMM_MODEL_* */
    int neuphotic;          /* euphotic layers (2 in the paper's experiments, section 7) */
    int nbgc;               /* internal BGC time steps per ocean step (section 7; 8 in the paper's
                               experiments): the source of a step is the increment of nbgc explicit
                               Euler steps of dt/nbgc at the step's forcing.  0 or 1 = one evaluation
                               dt*q(y).  At most 16; above 1 needs neuphotic <= 4 */
    int nbatch_max;         /* largest ensemble (member count) the handle must hold */
    int adjoint_nbatch_max; /* largest ensemble for tmm_year_adjoint (0 disables it) */
    int ckpt_every;         /* steps between adjoint checkpoints; divides nstep (ignored if no adjoint) */
    /* explicit (horizontal) matrices, CSR with one pattern for all months */
    int ae_nnz;
    const int *ae_rowptr;   /* [n+1] */
    const int *ae_colidx;   /* [ae_nnz] */
    const double *ae_val;   /* [nmat][ae_nnz] */
    /* implicit (vertical) matrices, CSR; every entry must couple two points
     * of the same water column (section 3: implicit operators act vertically) */
    int ai_nnz;
    const int *ai_rowptr;
    const int *ai_colidx;
    const double *ai_val;   /* [nmat][ai_nnz] */
    /* optional */
    const double *lon;      /* [ncol] longitude of each column, degrees, or NULL.  Only orders the
                               work of the member-parallel ensemble kernel (horizontal neighbours
                               close together, for cache reuse); results do not depend on it */
} tmm_desc;

/* Device workspace size for a descriptor.  Returns TMM_EINVAL for a bad
 * descriptor. */
int tmm_workspace_bytes(const tmm_desc *desc, size_t *bytes);

/* Validates the descriptor, converts the matrices to the device formats and
 * uploads them into the workspace (device pointer, at least
 * tmm_workspace_bytes() bytes, 256-byte aligned).  hip_stream is a
 * hipStream_t (NULL = default stream) used by every later call. */
int tmm_create(const tmm_desc *desc, void *dev_workspace, size_t bytes,
               void *hip_stream, tmm_handle *out);

/* Synchronises the stream and releases host-side state.  Safe on NULL. */
int tmm_destroy(tmm_handle h);

/* Sets nbatch parameter vectors (host array [nbatch][nparam], order of the
 * paper's parameter table, section 2.2.1) and rebuilds the per-member
 * tables (light attenuation, Martin-curve remineralisation).  Every
 * parameter must be finite, K_1, K_I > 0, 0 <= sigma_2 <= 1. */
int tmm_set_params(tmm_handle h, int nbatch, const double *u);

/* One time step j (section 3): y_out = Ai(t_j)(Ae(t_j) y_in + dt q(y_in)).
 * y_in, y_out: device, n x W, must not overlap. */
int tmm_step(tmm_handle h, int j, const double *y_in, double *y_out);

/* Model years (section 4).  Runs nyears years from y0 and writes the final
 * state to y1 (device, n x W; y1 may equal y0).  years_per_member (host,
 * [nbatch], nullable) gives per-member lengths <= nyears: member b stops after
 * years_per_member[b] years and y1 holds its state then.  resid_host
 * (nullable, [nyears][nbatch]) receives ||y - phi(y)||_2 of each member for
 * each year it ran (0 afterwards); passing it synchronises.  The state is
 * checked for NaN and infinity at the end of every year (unless
 * TMM_OPT_CHECK_FINITE is 0): if any year produced one, the call still runs
 * all its years, writes y1 and resid_host, and returns TMM_ENONFINITE. */
int tmm_year(tmm_handle h, int nyears, const int *years_per_member,
             const double *y0, double *y1, double *resid_host);

/* tmm_year for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * model years with the same kernels, but every buffer besides y0 and y1 --
 * the ping-pong state, a copy of the year's start state, the residual
 * partial sums, the non-finite flag -- lives in a fixed device array of the
 * library (32 MiB, one per device, held until the process ends) instead of
 * the workspace's state buffers, and the call makes no allocation of any
 * kind.  It always runs one launch per time step (the single-launch year
 * kernel needs the workspace's state ring) and has no per-member lengths.
 * Requests that do not fit, 2 n W + (tiles + 1) nbatch doubles > 32 MiB
 * (about 2 million state values: the global grid with up to 19 members),
 * return TMM_ETOOBIG before anything runs.  y1 may equal y0; resid_host and
 * the non-finite check as for tmm_year.  With resid_host NULL and
 * TMM_OPT_CHECK_FINITE 0 the call only enqueues kernels and does not
 * synchronise.  The fixed array is shared by every call on a device: calls
 * that overlap on one device (different streams or threads) race, and must
 * be serialised by the caller. */
int tmm_year_noalloc(tmm_handle h, int nyears, const double *y0, double *y1, double *resid_host);

/* Directional derivative of the year map (section 6.1): jv = phi'(y) v by
 * mode TMM_JVP_FD or TMM_JVP_TANGENT, where phi_y (nullable) receives phi(y);
 * with TMM_JVP_FD_GIVEN_PHI, phi_y must hold phi(y) and is read.
 * All device, n x W; jv must not overlap y, v or phi_y. */
int tmm_year_jvp(tmm_handle h, int mode, const double *y, const double *v,
                 double *phi_y, double *jv);

/* Gradient of the least-squares misfit
 *   J_b = sum_m sum_i sum_tr V_i (y_{s_m} - obs_m)^2 / (2 nmat V_tot),
 * s_m = (m+1) nstep/nmat, over one model year from y0, by a discrete adjoint
 * (the derivative route the paper names in sections 1.2, 6.1 and 9) with
 * checkpoints every ckpt_every steps and recomputation in between.  The
 * forward sweep keeps the states of the last checkpoint segment, so that
 * segment is not recomputed: ckpt_every = nstep stores the whole year
 * (nstep x n x W doubles of workspace) and recomputes nothing.
 * y0, obs ([nmat][n][W]) and dJdy0 (nullable, n x W) are device arrays;
 * J_host [nbatch] and dJdu_host [nbatch][nparam] are host arrays.
 * ckpt_every must equal the descriptor's value.  Synchronises. */
int tmm_year_adjoint(tmm_handle h, const double *y0, const double *obs, int ckpt_every,
                     double *J_host, double *dJdu_host, double *dJdy0);

/* Options (tmm_set_option). */
enum {
    TMM_OPT_PERSISTENT = 1,  /* 1 (default): single-member model years run as one persistent
                                cooperative launch when the grid fits; 0: one launch per step */
    TMM_OPT_DOMAIN_ROWS = 2, /* target rows per workgroup of the persistent kernel (<= 512);
                                0 = the default (256) */
    TMM_OPT_MEMBER_KERNEL_MIN = 3, /* forward steps of batches with at least this many members use the
                                     member-parallel kernel (one wavefront per water column, lane =
                                     member); -1 = the default: 2 where its packed forms run (two
                                     tracers, one BGC evaluation per step, at most 24 layers,
                                     TMM_OPT_MEMBER_PACK on), else 6, about where it overtakes the
                                     tile kernel on grids of 50k to 500k points; 0 = never */
    TMM_OPT_GRAPH = 4,           /* 1 (default): model years on the launch-per-step path are captured
                                    once per (members, buffers) into a hipGraph and replayed */
    TMM_OPT_SPIN_LIMIT = 5,      /* polls after which a wait of the persistent kernels gives up
                                    (the call then returns TMM_EDEVICE; the next call starts
                                    afresh); 0 = the default (2^22, seconds); small values are for
                                    tests of that failure path */
    TMM_OPT_CHECK_FINITE = 6,    /* 1 (default): tmm_year checks the state for non-finite values at
                                    the end of every model year (one read of the state per year);
                                    0: no check */
    TMM_OPT_MEMBER_WAVES = 7,    /* wavefronts (water columns) per workgroup of the member-parallel
                                    kernel for two-tracer models: 2, 4 or 8; 0 = the default (4) */
    TMM_OPT_MEMBER_BAND_ROWS = 8, /* latitude rows per band of the member-parallel kernel's column
                                    order (needs the descriptor's longitudes); 0 = the default (16),
                                    -1 = the natural column order */
    TMM_OPT_TILE_ROWS = 9,       /* largest tile (rows per workgroup) of the launch-per-step tile
                                    kernels: 32, 64, 128 or 256 (a tiling no deeper than the
                                    deepest column is used as the smallest); 0 = by state width
                                    (128 up to 4 state columns, else 256) */
    TMM_OPT_WAVE_LOCAL = 10,     /* 1 (default): the persistent forward kernels place each water
                                    column within one wavefront where the domains allow it (more,
                                    smaller domains if needed), so that a time step needs one
                                    workgroup barrier instead of three; 0: packed columns and
                                    three barriers per step.  Rebuilds the domains; the results
                                    are the same bit for bit */
    TMM_OPT_MEMBER_TILE = 11,    /* 0 (default): member-parallel steps of two-tracer models use one
                                    wavefront per water column that reads its stencil's state rows
                                    itself; 4 or 8: workgroups of that many neighbouring columns
                                    (from the band order, which must be on) load each state row
                                    their explicit rows read once per layer into LDS.  Needs one
                                    BGC evaluation per step, at most 5 explicit entries per row,
                                    at most 24 layers and the descriptor's longitudes
                                    (TMM_EUNSUPPORTED otherwise, or when a tile's layer reads
                                    more rows than a workgroup stages: 16 for 4 columns, 24 for
                                    8; the option is then left as it was).  The results are the
                                    same bit for bit */
    TMM_OPT_MEMBER_PACK = 12     /* 1 (default): member-parallel steps of two-tracer models with at
                                    most 32 (16) members place 2 (4) water columns in one wavefront,
                                    32 (16) lanes each, so that the step's time follows the member
                                    count; 0: one column per wavefront at every width.  Same
                                    results bit for bit */
};

/* Queries (tmm_query). */
enum {
    TMM_Q_PERSISTENT = 1,   /* 1 if the persistent year kernel is available on this handle */
    TMM_Q_DOMAINS = 2,      /* workgroups (column domains) of the persistent kernel */
    TMM_Q_WORKSPACE = 3,    /* workspace bytes in use */
    TMM_Q_COMPUTE_UNITS = 4, /* compute units of the device */
    TMM_Q_PERSISTENT_ADJOINT = 5, /* 1 if single-member adjoints use the persistent reverse kernel (its
                                    store of internal BGC steps must fit the workgroup's LDS) */
    TMM_Q_INSOLATION_LDS = 6, /* 1 if the persistent forward kernel (state only) holds the year's
                                insolation of each domain's latitude rows in LDS (no internal BGC steps,
                                at most 8 latitude rows per domain, and the table fits beside the halo
                                with every domain resident); 0 if it loads it every step.  The tangent
                                kernel decides the same on its own, larger LDS */
    TMM_Q_WAVE_LOCAL = 7     /* 1 if the persistent forward kernels run with wave-aligned water
                                columns (option TMM_OPT_WAVE_LOCAL) */
};

/* Sets an execution option; results are the same either way up to rounding
 * order.  TMM_EINVAL for an unknown option. */
int tmm_set_option(tmm_handle h, int option, int value);

/* Reads a property of the handle into *value.  TMM_EINVAL for an unknown query. */
int tmm_query(tmm_handle h, int what, long long *value);

/* Measures, on the handle's device and stream, the latency of the primitives
 * that the single-launch year kernels chain in every time step, so that a
 * step's time can be set against the floor they impose (no effect on any
 * result; uses a small reserved part of the workspace).  rounds (1 ..
 * 1000000) repetitions of each; out (host, [8]) receives
 *   out[0]  us per round trip of an agent-scope store and poll between two
 *           workgroups on the same XCD (two hand-overs of a value),
 *   out[1]  the same between workgroups on two different XCDs,
 *   out[2]  us per workgroup barrier of 256 threads,
 *   out[3]  us per dependent agent-scope load,
 *   out[4..7] the XCDs the two pairs of workgroups ran on.
 * TMM_EUNSUPPORTED without cooperative launch; TMM_EDEVICE if a wait gave up.
 * Synchronises. */
int tmm_probe_exchange(tmm_handle h, int rounds, double *out);

/* Static text for a status code. */
const char *tmm_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
