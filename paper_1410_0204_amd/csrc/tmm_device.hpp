// Device code of libtmm: float64 kernels for gfx950.
//
// Method: Piwonski & Slawig, "The Idea and Concept of Metos3D" (arXiv
// 1410.0204).  One time step (section 3)
//     z = Ae(t_j) y_j + dt_d q(y_j, u),   y_{j+1} = Ai(t_j) z
// with Ae, Ai linear interpolations of monthly matrices and q the PO4-DOP
// model of section 2.2.1 (or the PO4-DOP-PHY model of section 2.2.2)
// evaluated per water column (section 5).
//
// Data layout on the device (built by the host code at creation):
//  * Ae, Ae^T: ELL, slot-major: val[month][slot][npad], col[slot][npad].
//    Lanes of a wavefront own consecutive rows, so every slot is one
//    coalesced 512-byte read of values and a 256-byte read of indices.
//  * Ai: one dense n_c x n_c block per water column (the implicit operator
//    acts within columns only, section 3), stored column-major ("cm", lanes
//    = rows of the forward product) and row-major ("rm", lanes = rows of the
//    transposed product).
//  * States: row-major n x W (W = members * tracers), so the W values of a
//    grid point are contiguous.
//  * Tiles: a tile is a run of whole water columns; one workgroup owns one
//    tile, stages z (or the adjoint lambda) of its rows in LDS and applies
//    the column blocks from there.
#pragma once

#include <hip/hip_runtime.h>

namespace tmm {

constexpr int kMaxLayers = 64;
constexpr double kPi = 3.14159265358979323846;
constexpr double kSigmaPar = 0.4;       // photosynthetically available fraction of I_SWR
constexpr double kSigmaIce = 0.0;       // no ice in the synthetic forcing
constexpr double kSolarConstant = 1361.0;
constexpr double kDaysPerYear = 360.0;  // section 5.1

enum { MODEL_N = 1, MODEL_NDOP = 2, MODEL_NDOPPHY = 3 };

// alpha is mu_1 in PO4-DOP-PHY; lam3, kap3, lam3p, sig3 exist only there.
struct BgcParams {
    double alpha, kw, k1, ki, lam, sig, b;
    double lam3, kap3, lam3p, sig3;
};

}  // namespace tmm

#include "tmm_substep.hpp"

namespace tmm {

// Parameter i of member m at u[m * sm + i * sp]: the member-major table
// (sm = nparam, sp = 1) or its member-fastest copy (sm = 1, sp = members).
__device__ __forceinline__ BgcParams load_params_at(const double* __restrict__ u, int model, size_t sm, size_t sp,
                                                    int m) {
    const double* q = u + (size_t)m * sm;
    auto p = [&](int i) { return q[(size_t)i * sp]; };
    BgcParams r;
    r.alpha = p(0);
    r.kw = p(1);
    r.k1 = p(2);
    r.ki = p(3);
    r.lam3 = r.kap3 = r.lam3p = r.sig3 = 0.0;
    if (model == MODEL_NDOPPHY) {
        r.lam = p(4);
        r.sig = p(5);
        r.lam3 = p(6);
        r.kap3 = p(7);
        r.lam3p = p(8);
        r.sig3 = p(9);
        r.b = p(10);
    } else if (model == MODEL_NDOP) {
        r.lam = p(4);
        r.sig = p(5);
        r.b = p(6);
    } else {
        r.lam = 0.0;
        r.sig = 0.0;
        r.b = p(4);
    }
    return r;
}

__device__ __forceinline__ BgcParams load_params(const double* __restrict__ u, int model, int nparam, int m) {
    return load_params_at(u, model, (size_t)nparam, 1, m);
}

// Month pair and weight of step j: monthly matrices sit at mid-month and the
// year is periodic (section 3).  Integer arithmetic, one exact division.
__device__ __forceinline__ void step_phase(int j, int nstep, int nmat, int& k0, int& k1, double& w) {
    const int spm = nstep / nmat;
    int jj = j % nstep;
    if (jj < 0) jj += nstep;
    int tau = jj - spm / 2;
    int kk = tau >= 0 ? tau / spm : -((-tau + spm - 1) / spm);
    int r = tau - kk * spm;
    kk %= nmat;
    if (kk < 0) kk += nmat;
    k0 = kk;
    k1 = kk + 1 == nmat ? 0 : kk + 1;
    w = (double)r / (double)spm;
}

// Daily-mean top-of-atmosphere short-wave radiation at latitude lat (deg) and
// time t (fraction of the 360-day year): I_SWR of section 2.2.1.
__device__ __forceinline__ double insolation(double lat_deg, double t) {
    const double decl = -23.44 * kPi / 180.0 * cos(2.0 * kPi * (t + 10.0 / kDaysPerYear));
    const double phi = lat_deg * kPi / 180.0;
    const double x = -tan(phi) * tan(decl);
    double h0;
    if (x >= 1.0) h0 = 0.0;
    else if (x <= -1.0) h0 = kPi;
    else h0 = acos(x);
    const double q = kSolarConstant / kPi * (h0 * sin(phi) * sin(decl) + cos(phi) * cos(decl) * sin(h0));
    return q > 0.0 ? q : 0.0;
}

// Insolation table ins[j][l] = I_SWR(lat_l, j/nstep) for every step of the year
// and every distinct latitude of the grid (computed once per handle).
__global__ void k_insolation_table(int nstep, int nlat, const double* __restrict__ lat_u,
                                   double* __restrict__ ins) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nstep * nlat) return;
    const int j = idx / nlat, l = idx % nlat;
    ins[idx] = insolation(lat_u[l], (double)j / (double)nstep);
}

// Production f = alpha N+/(N+ + K_1) * I/(I + K_I) (section 2.2.1) and
// derivatives.  I = I_SWR sigma_PAR (1 - sigma_ice) exp(-z K_H2O); the
// exponential factor comes from the per-member light table.
struct Production {
    double f, dfdN, limN, limI, I;
};

__device__ __forceinline__ Production production(const BgcParams& p, double N, double Q, double light) {
    Production r;
    r.I = Q * kSigmaPar * (1.0 - kSigmaIce) * light;
    const double Np = N > 0.0 ? N : 0.0;
    r.limN = Np / (Np + p.k1);
    r.limI = r.I / (r.I + p.ki);
    r.f = p.alpha * r.limN * r.limI;
    r.dfdN = N > 0.0 ? p.alpha * p.k1 / ((N + p.k1) * (N + p.k1)) * r.limI : 0.0;
    return r;
}

// ---------------------------------------------------------------------------
// Per-member tables: light attenuation exp(-z_k K_H2O) at layer centres and
// the Martin-curve remineralisation fractions rho_k (per metre) with
// d rho_k / d b, for every column depth n_c.
// Layout: light[m][k], rho[(m*(nlayer+1) + n_c)*nlayer + k]; the
// member-fastest copies lightT[k][m] and rhoT[n_c*nlayer + k][m] (member
// stride nbm) serve the member-parallel kernel, whose lanes are members.
// ---------------------------------------------------------------------------
__global__ void k_param_tables(int nbatch, int model, int nparam, int nlayer, int neu,
                               const double* __restrict__ u, const double* __restrict__ dz,
                               double* __restrict__ light, double* __restrict__ rho,
                               double* __restrict__ drho, int nbm, double* __restrict__ lightT,
                               double* __restrict__ rhoT) {
    const int per_member = (nlayer + 1) * nlayer;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nbatch * per_member) return;
    const int m = idx / per_member;
    const int rem = idx % per_member;
    const int nc = rem / nlayer;
    const int k = rem % nlayer;
    const BgcParams p = load_params(u, model, nparam, m);

    auto bottom = [&](int kk) {
        double d = 0.0;
        for (int i = 0; i <= kk; ++i) d += dz[i];
        return d;
    };
    if (nc == 0) {
        const double z = bottom(k) - 0.5 * dz[k];
        const double l = exp(-z * p.kw);
        light[(size_t)m * nlayer + k] = l;
        lightT[(size_t)k * nbm + m] = l;
    }
    double r = 0.0, dr = 0.0;
    if (nc >= 1 && k < nc) {
        if (nc <= neu) {
            r = k == nc - 1 ? 1.0 / dz[k] : 0.0;
        } else if (k >= neu) {
            const double lp = bottom(neu - 1);
            const double ztop = bottom(k - 1);
            const double mtop = pow(ztop / lp, -p.b);
            const double dmtop = -log(ztop / lp) * mtop;
            double mbot = 0.0, dmbot = 0.0;
            if (k < nc - 1) {
                const double zbot = bottom(k);
                mbot = pow(zbot / lp, -p.b);
                dmbot = -log(zbot / lp) * mbot;
            }
            r = (mtop - mbot) / dz[k];
            dr = (dmtop - dmbot) / dz[k];
        }
    }
    rho[idx] = r;
    drho[idx] = dr;
    rhoT[(size_t)rem * nbm + m] = r;
}

// ---------------------------------------------------------------------------
// Arguments shared by the step kernels.
// ---------------------------------------------------------------------------
struct Grid {
    int n, npad, nlayer, neu, nstep, nmat;
    const int* tile_col;     // [ntile+1] first column of each tile
    const int* col_start;    // [ncol+1]
    const int* blk_off;      // [ncol] offset of each column's Ai block
    const double* lat;       // [ncol]
    const double* area;      // [ncol]
    const double* dz;        // [nlayer]
    const double* ins;       // [nstep][nlat] insolation per step and distinct latitude
    const int* col_lat;      // [ncol] row of each column in the insolation table
    int nlat;
};

struct Model {
    int model, ntr, nparam;
    const double* u;         // [members][nparam]
    const double* light;     // [members][nlayer]
    const double* rho;       // [members][nlayer+1][nlayer]
    const double* drho;
    const int* member;       // [slots] parameter row of each state slot
    // member-fastest copies for the member-parallel kernel (lane = member):
    // uT[i][m], lightT[k][m], rhoT[n_c*nlayer + k][m], member stride nbm
    const double* uT;
    const double* lightT;
    const double* rhoT;
    int nbm;
    int nsub;                // internal BGC steps per ocean step (section 7)
    double hsub;             // their length dt_d / nsub, days
};

struct Mats {
    int ew;                  // ELL width of Ae
    int etw;                 // ELL width of Ae^T
    size_t ae_month;         // values per month of the ELL array (ew*npad)
    size_t aet_month;
    size_t ai_month;         // values per month of the block array
    const double* ae;        // [nmat][ew][npad]
    const int* ae_col;       // [ew][npad]; slot 0 of every row reads the row itself
    const double* aet;       // [nmat][etw][npad]
    const int* aet_col;
    const double* ai_cm;     // [nmat][blocks] column-major blocks
    const double* ai_rm;     // [nmat][blocks] row-major blocks
};

// LDS map of a tile: for every local row its local column and layer, and per
// column its first local row, depth and insolation at the current step.
struct TileMap {
    int c0, r0, nrows, ncols;
};

template <int MAXR, int MAXC>
struct TileLds {
    short row_col[MAXR];
    short row_k[MAXR];
    short col_r0[MAXC];
    short col_nc[MAXC];
    double Q[MAXC];
};

template <int MAXR, int MAXC>
__device__ __forceinline__ TileMap build_tile(const Grid& g, TileLds<MAXR, MAXC>& L, int jstep) {
    TileMap tm;
    tm.c0 = g.tile_col[blockIdx.x];
    const int c1 = g.tile_col[blockIdx.x + 1];
    tm.ncols = c1 - tm.c0;
    tm.r0 = g.col_start[tm.c0];
    tm.nrows = g.col_start[c1] - tm.r0;
    for (int lc = threadIdx.x; lc < tm.ncols; lc += blockDim.x) {
        const int c = tm.c0 + lc;
        const int s = g.col_start[c] - tm.r0;
        const int nc = g.col_start[c + 1] - g.col_start[c];
        L.col_r0[lc] = (short)s;
        L.col_nc[lc] = (short)nc;
        L.Q[lc] = jstep >= 0 ? g.ins[(size_t)jstep * g.nlat + g.col_lat[c]] : 0.0;
        for (int k = 0; k < nc; ++k) {
            L.row_col[s + k] = (short)lc;
            L.row_k[s + k] = (short)k;
        }
    }
    __syncthreads();
    return tm;
}

// Biogeochemistry of one (row, member) of the PO4-DOP / N model (sections
// 2.2.1 and 5): q for both tracers, from the member's state in the rows of
// the row's water column.  Production runs in the euphotic layers, the export
// Phi = sum_k h_k f_k is remineralised below by the Martin curve, DOP decays
// with rate lambda'_2.
struct ColumnRef {
    int rs;       // global first row of the column
    int nc;       // depth
    int k;        // layer of this row
    double Q;     // insolation
};

__device__ __forceinline__ void bgc_q(const Grid& g, const Model& md, const double* __restrict__ y, int W,
                                      const ColumnRef& c, int slot, double& q1, double& q2) {
    const int m = md.member[slot];
    const BgcParams p = load_params(md.u, md.model, md.nparam, m);
    const double* light = md.light + (size_t)m * g.nlayer;
    const int ne = c.nc < g.neu ? c.nc : g.neu;
    double Phi = 0.0, fk = 0.0;
    for (int e = 0; e < ne; ++e) {
        const double N = y[(size_t)(c.rs + e) * W + slot * md.ntr];
        const double f = production(p, N, c.Q, light[e]).f;
        Phi += g.dz[e] * f;
        if (e == c.k) fk = f;
    }
    const double rho = md.rho[((size_t)m * (g.nlayer + 1) + c.nc) * g.nlayer + c.k];
    const double dop = md.ntr > 1 ? y[(size_t)(c.rs + c.k) * W + slot * md.ntr + 1] : 0.0;
    q1 = -fk + p.lam * dop + (1.0 - p.sig) * Phi * rho;
    q2 = p.sig * fk - p.lam * dop;
}

// PO4-DOP-PHY (section 2.2.2) for one (row, member): f_1 = mu_1 PHY N+/(N+ + K_1)
// I/(I + K_I), f_3 = sigma_3 f_1, export Phi = sum_e h_e f_3,e; the losses
// lambda_3 PHY + kappa_3 PHY^2 act in the euphotic zone only.  q[3].
__device__ __forceinline__ void bgc_q_phy(const Grid& g, const Model& md, const double* __restrict__ y, int W,
                                          const ColumnRef& c, int slot, double* q) {
    const int m = md.member[slot];
    const BgcParams p = load_params(md.u, md.model, md.nparam, m);
    const double* light = md.light + (size_t)m * g.nlayer;
    const int ne = c.nc < g.neu ? c.nc : g.neu;
    double Phi = 0.0, fk = 0.0;
    for (int e = 0; e < ne; ++e) {
        const size_t at = (size_t)(c.rs + e) * W + slot * 3;
        const double f = production(p, y[at], c.Q, light[e]).f * y[at + 2];
        Phi += g.dz[e] * (p.sig3 * f);
        if (e == c.k) fk = f;
    }
    const double rho = md.rho[((size_t)m * (g.nlayer + 1) + c.nc) * g.nlayer + c.k];
    const size_t ak = (size_t)(c.rs + c.k) * W + slot * 3;
    const double D = y[ak + 1], P = y[ak + 2];
    const double loss = c.k < ne ? p.lam3 * P + p.kap3 * P * P : 0.0;
    q[0] = -fk + p.lam * D + (1.0 - p.sig) * Phi * rho;
    q[1] = p.sig * (p.sig3 * fk) + loss - p.lam * D + p.lam3p * P;
    q[2] = (1.0 - p.sig3) * fk - loss - p.lam3p * P;
}

__device__ __forceinline__ void bgc_q_phy_tangent(const Grid& g, const Model& md, const double* __restrict__ y,
                                                  const double* __restrict__ v, int W, const ColumnRef& c, int slot,
                                                  double* qd) {
    const int m = md.member[slot];
    const BgcParams p = load_params(md.u, md.model, md.nparam, m);
    const double* light = md.light + (size_t)m * g.nlayer;
    const int ne = c.nc < g.neu ? c.nc : g.neu;
    double Phid = 0.0, fdk = 0.0;
    for (int e = 0; e < ne; ++e) {
        const size_t at = (size_t)(c.rs + e) * W + slot * 3;
        const Production pr = production(p, y[at], c.Q, light[e]);
        const double fd = pr.dfdN * v[at] * y[at + 2] + pr.f * v[at + 2];
        Phid += g.dz[e] * (p.sig3 * fd);
        if (e == c.k) fdk = fd;
    }
    const double rho = md.rho[((size_t)m * (g.nlayer + 1) + c.nc) * g.nlayer + c.k];
    const size_t ak = (size_t)(c.rs + c.k) * W + slot * 3;
    const double P = y[ak + 2], Dd = v[ak + 1], Pd = v[ak + 2];
    const double lossd = c.k < ne ? (p.lam3 + 2.0 * p.kap3 * P) * Pd : 0.0;
    qd[0] = -fdk + p.lam * Dd + (1.0 - p.sig) * Phid * rho;
    qd[1] = p.sig * (p.sig3 * fdk) + lossd - p.lam * Dd + p.lam3p * Pd;
    qd[2] = (1.0 - p.sig3) * fdk - lossd - p.lam3p * Pd;
}

// Reverse mode of bgc_q_phy for one (row, member): lam += dtd (dq/dy)^T mu for
// the row's three tracers and contrib += (dq/du)^T mu (unscaled), parameters
// in the order of the table of section 2.2.2.
__device__ __forceinline__ void bgc_q_phy_adjoint(const Grid& g, const Model& md, const double* __restrict__ yj,
                                                  const double* __restrict__ mu, int W, const ColumnRef& c, int slot,
                                                  double dtd, double* lam, double* contrib) {
    const int m = md.member[slot];
    const BgcParams p = load_params(md.u, md.model, md.nparam, m);
    const double* light = md.light + (size_t)m * g.nlayer;
    const size_t tab = ((size_t)m * (g.nlayer + 1) + c.nc) * g.nlayer;
    const int ne = c.nc < g.neu ? c.nc : g.neu;
    double Phi = 0.0, Phibar = 0.0;
    for (int e = 0; e < ne; ++e) {
        const size_t at = (size_t)(c.rs + e) * W + slot * 3;
        Phi += g.dz[e] * (p.sig3 * (production(p, yj[at], c.Q, light[e]).f * yj[at + 2]));
    }
    for (int kk = 0; kk < c.nc; ++kk)
        Phibar += (1.0 - p.sig) * md.rho[tab + kk] * mu[(size_t)(c.rs + kk) * W + slot * 3];
    const size_t ak = (size_t)(c.rs + c.k) * W + slot * 3;
    const double m1 = mu[ak], m2 = mu[ak + 1], m3 = mu[ak + 2];
    const double D = yj[ak + 1], P = yj[ak + 2];
    const double rho = md.rho[tab + c.k], drho = md.drho[tab + c.k];
    double b0 = 0.0, b2 = 0.0;
    if (c.k < ne) {
        const Production pr = production(p, yj[ak], c.Q, light[c.k]);
        const double f = pr.f * P;
        // f_1 enters q_1 (-1), q_2 (sigma_2 sigma_3), q_3 (1 - sigma_3) and Phi (h_k sigma_3)
        const double fbar = -m1 + p.sig * p.sig3 * m2 + (1.0 - p.sig3) * m3 + p.sig3 * g.dz[c.k] * Phibar;
        const double dloss = p.lam3 + 2.0 * p.kap3 * P;
        b0 = fbar * pr.dfdN * P;
        b2 = fbar * pr.f + dloss * (m2 - m3);
        const double Np = yj[ak] > 0.0 ? yj[ak] : 0.0;
        double zc = 0.0;
        for (int i = 0; i <= c.k; ++i) zc += g.dz[i];
        zc -= 0.5 * g.dz[c.k];
        const double IKI2 = (pr.I + p.ki) * (pr.I + p.ki);
        contrib[0] += fbar * pr.limN * pr.limI * P;
        contrib[1] += fbar * p.alpha * pr.limN * p.ki / IKI2 * (-zc * pr.I) * P;
        contrib[2] += fbar * (-p.alpha * Np / ((Np + p.k1) * (Np + p.k1)) * pr.limI) * P;
        contrib[3] += fbar * (-p.alpha * pr.limN * pr.I / IKI2) * P;
        contrib[5] += p.sig3 * f * m2;
        contrib[6] += P * (m2 - m3);
        contrib[7] += P * P * (m2 - m3);
        contrib[9] += f * (p.sig * m2 - m3 + g.dz[c.k] * Phibar);
    }
    b2 += p.lam3p * (m2 - m3);
    contrib[4] += D * (m1 - m2);
    contrib[5] += -Phi * rho * m1;
    contrib[8] += P * (m2 - m3);
    contrib[10] += (1.0 - p.sig) * Phi * drho * m1;
    lam[0] += dtd * b0;
    lam[1] += dtd * (p.lam * (m1 - m2));
    lam[2] += dtd * b2;
}

// Tangent of bgc_q in direction v.
__device__ __forceinline__ void bgc_q_tangent(const Grid& g, const Model& md, const double* __restrict__ y,
                                              const double* __restrict__ v, int W, const ColumnRef& c,
                                              int slot, double& q1, double& q2) {
    const int m = md.member[slot];
    const BgcParams p = load_params(md.u, md.model, md.nparam, m);
    const double* light = md.light + (size_t)m * g.nlayer;
    const int ne = c.nc < g.neu ? c.nc : g.neu;
    double Phid = 0.0, fdk = 0.0;
    for (int e = 0; e < ne; ++e) {
        const size_t at = (size_t)(c.rs + e) * W + slot * md.ntr;
        const double fd = production(p, y[at], c.Q, light[e]).dfdN * v[at];
        Phid += g.dz[e] * fd;
        if (e == c.k) fdk = fd;
    }
    const double rho = md.rho[((size_t)m * (g.nlayer + 1) + c.nc) * g.nlayer + c.k];
    const double dopd = md.ntr > 1 ? v[(size_t)(c.rs + c.k) * W + slot * md.ntr + 1] : 0.0;
    q1 = -fdk + p.lam * dopd + (1.0 - p.sig) * Phid * rho;
    q2 = p.sig * fdk - p.lam * dopd;
}

// Euphotic constants of one (column, member) gathered from memory; loads of
// layers beyond the euphotic zone are clamped to layer 0 and ignored.
template <int NEU>
__device__ __forceinline__ Euphotic<NEU> euphotic_from_memory(const Grid& g, const Model& md, const BgcParams& p, int m,
                                                              int nc, double Q, int& ne) {
    ne = nc < g.neu ? nc : g.neu;
    const double* light = md.light + (size_t)m * g.nlayer;
    const double* rho = md.rho + ((size_t)m * (g.nlayer + 1) + nc) * g.nlayer;
    double le[NEU], hz[NEU], re[NEU];
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const int ee = e < ne ? e : 0;
        le[e] = light[ee];
        hz[e] = g.dz[ee];
        re[e] = rho[ee];
    }
    return make_euphotic<NEU>(p, Q, ne, le, hz, re);
}

// Source of one (row, member) over one ocean step with md.nsub internal BGC
// steps (section 7), from the state in memory: out = inc_nsub of the row's
// NTR tracers; with TANGENT also its tangent in direction v.
template <int NTR, bool TANGENT>
__device__ __forceinline__ void bgc_inc(const Grid& g, const Model& md, const double* __restrict__ y,
                                        const double* __restrict__ v, int W, const ColumnRef& c, int slot,
                                        double* out, double* outd) {
    constexpr int NEU = kSubNeuMax;
    const int m = md.member[slot];
    const BgcParams p = load_params(md.u, md.model, md.nparam, m);
    int ne;
    const Euphotic<NEU> E = euphotic_from_memory<NEU>(g, md, p, m, c.nc, c.Q, ne);
    const double rho_k = md.rho[((size_t)m * (g.nlayer + 1) + c.nc) * g.nlayer + c.k];
    double ye[NEU][NTR], ve[NEU][NTR], yk[NTR], vk[NTR];
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const size_t at = (size_t)(c.rs + (e < ne ? e : 0)) * W + slot * NTR;
#pragma unroll
        for (int t = 0; t < NTR; ++t) {
            ye[e][t] = e < ne ? y[at + t] : 0.0;
            ve[e][t] = (TANGENT && e < ne) ? v[at + t] : 0.0;
        }
    }
    const size_t ak = (size_t)(c.rs + c.k) * W + slot * NTR;
#pragma unroll
    for (int t = 0; t < NTR; ++t) {
        yk[t] = y[ak + t];
        vk[t] = TANGENT ? v[ak + t] : 0.0;
    }
    double o[NTR], od[NTR];
    if (TANGENT) {
        row_source_tangent<NTR, NEU>(p, E, c.k, ye, ve, yk, vk, rho_k, md.hsub, md.nsub, o, od);
    } else {
        row_source<NTR, NEU>(p, E, c.k, ye, yk, rho_k, md.hsub, md.nsub, o);
    }
#pragma unroll
    for (int t = 0; t < NTR; ++t) {
        out[t] = o[t];
        if (TANGENT) outd[t] = od[t];
    }
}

// Reverse mode of bgc_inc for one (row, member) of the tile adjoint: the
// euphotic internal steps are replayed from the ocean step's state for every
// reverse internal step (no storage; quadratic in nsub).  Adds h (dq/dy)^T mu
// to ybar[NTR] and the unscaled (dq/du)^T mu sums to ub[NP].
template <int NTR, int NP>
__device__ __forceinline__ void bgc_inc_adjoint(const Grid& g, const Model& md, const double* __restrict__ yj,
                                                const double* __restrict__ mu, int W, const ColumnRef& c, int slot,
                                                double* ybar, double* ub) {
    constexpr int NEU = kSubNeuMax;
    const int m = md.member[slot];
    const BgcParams p = load_params(md.u, md.model, md.nparam, m);
    int ne;
    const Euphotic<NEU> E = euphotic_from_memory<NEU>(g, md, p, m, c.nc, c.Q, ne);
    const size_t tab = ((size_t)m * (g.nlayer + 1) + c.nc) * g.nlayer;
    const double rho_k = md.rho[tab + c.k];
    const double drho_k = md.drho[tab + c.k];
    const double h = md.hsub;
    double zc = 0.0;
    for (int i = 0; i <= c.k; ++i) zc += g.dz[i];
    zc -= 0.5 * g.dz[c.k];
    double ye[NEU][NTR], ib[NEU][NTR], yk[NTR], mk[NTR], yb[NTR], u[NP];
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const size_t at = (size_t)(c.rs + (e < ne ? e : 0)) * W + slot * NTR;
#pragma unroll
        for (int t = 0; t < NTR; ++t) {
            ye[e][t] = e < ne ? yj[at + t] : 0.0;
            ib[e][t] = e < ne ? mu[at + t] : 0.0;
        }
    }
    const size_t ak = (size_t)(c.rs + c.k) * W + slot * NTR;
#pragma unroll
    for (int t = 0; t < NTR; ++t) {
        yk[t] = yj[ak + t];
        mk[t] = mu[ak + t];
        yb[t] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) u[q] = 0.0;
    double pdeep = 0.0;
    for (int kk = ne; kk < c.nc; ++kk) pdeep += (1.0 - p.sig) * md.rho[tab + kk] * mu[(size_t)(c.rs + kk) * W + slot * NTR];
    double sphi = 0.0;
    EuphoticAdj acc{};
    for (int s = md.nsub - 1; s >= 0; --s) {
        double inc[NEU][NTR], ys[NEU][NTR];
#pragma unroll
        for (int t = 0; t < NTR; ++t)
#pragma unroll
            for (int e = 0; e < NEU; ++e) inc[e][t] = 0.0;
        for (int r = 0; r < s; ++r) euphotic_step<NTR, NEU>(p, E, ye, h, inc);
#pragma unroll
        for (int e = 0; e < NEU; ++e)
#pragma unroll
            for (int t = 0; t < NTR; ++t) ys[e][t] = ye[e][t] + inc[e][t];
        sphi += euphotic_reverse<NTR, NEU>(p, E, c.k, rho_k, pdeep, ys, h, ib, yb, acc);
    }
    if (c.k >= ne) deep_reverse<NTR, NP>(p, deep_factors<NTR>(p, h, md.nsub), md.nsub, h, rho_k, drho_k, sphi, yk, mk, yb, u);
    else euphotic_adj_finish<NTR, NEU, NP>(p, E, c.k, zc, drho_k, acc, u);
#pragma unroll
    for (int t = 0; t < NTR; ++t) ybar[t] += yb[t];
#pragma unroll
    for (int q = 0; q < NP; ++q) ub[q] += u[q];
}

// ---------------------------------------------------------------------------
// Forward step (and its tangent).  One workgroup per tile; thread task =
// (row, group of CW state columns).  Phase A: z = Ae(t_j) y + dt_d q(y) into
// LDS.  Phase B: y_out = Ai(t_j) z from LDS.  SUB: 0 = one BGC evaluation
// per step, 1 = internal BGC steps for one or two tracers, 3 = internal BGC
// steps for PO4-DOP-PHY (separate instances, so that each keeps only the
// registers its own model needs).
// ---------------------------------------------------------------------------
template <int CW, bool TANGENT, int MAXR, int MAXC, int SUB = 0>
__global__ __launch_bounds__(256) void k_step(Grid g, Model md, Mats mt, int W, int tpr, int j, double dtd,
                       const double* __restrict__ y, double* __restrict__ yo,
                       const double* __restrict__ v, double* __restrict__ vo) {
    extern __shared__ double s_dyn[];
    __shared__ TileLds<MAXR, MAXC> L;
    int k0, k1;
    double w;
    step_phase(j, g.nstep, g.nmat, k0, k1, w);
    const TileMap tm = build_tile<MAXR, MAXC>(g, L, j % g.nstep);
    double* s_z = s_dyn;                                   // [nrows][W]
    double* s_zd = s_dyn + (size_t)tm.nrows * W;           // tangent [nrows][W]

    const double* ae0 = mt.ae + (size_t)k0 * mt.ae_month;
    const double* ae1 = mt.ae + (size_t)k1 * mt.ae_month;
    const double om = 1.0 - w;
    const int ntask = tm.nrows * tpr;

    for (int task = threadIdx.x; task < ntask; task += blockDim.x) {
        const int rr = task / tpr;
        const int wc0 = (task % tpr) * CW;
        const int r = tm.r0 + rr;
        const int lc = L.row_col[rr];
        ColumnRef c;
        c.rs = tm.r0 + L.col_r0[lc];
        c.nc = L.col_nc[lc];
        c.k = L.row_k[rr];
        c.Q = L.Q[lc];

        double acc[CW], accd[CW];
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) { acc[cc] = 0.0; accd[cc] = 0.0; }
        for (int s = 0; s < mt.ew; ++s) {
            const size_t e = (size_t)s * g.npad + r;
            const int col = mt.ae_col[e];
            const double a = om * ae0[e] + w * ae1[e];
#pragma unroll
            for (int cc = 0; cc < CW; ++cc) {
                if (wc0 + cc < W) {
                    acc[cc] += a * y[(size_t)col * W + wc0 + cc];
                    if (TANGENT) accd[cc] += a * v[(size_t)col * W + wc0 + cc];
                }
            }
        }
        // sources: one BGC evaluation per member, both tracers
        if (SUB == 3 || (SUB == 0 && md.ntr == 3)) {
            // PO4-DOP-PHY: the sources of each member once, then the thread's columns
            double qs[3] = {0.0, 0.0, 0.0}, qds[3] = {0.0, 0.0, 0.0};
            int cur = -1;
#pragma unroll
            for (int cc = 0; cc < CW; ++cc) {
                const int wc = wc0 + cc;
                if (wc >= W) break;
                const int slot = wc / 3;
                if (slot != cur) {
                    if constexpr (SUB == 3) {
                        bgc_inc<3, TANGENT>(g, md, y, v, W, c, slot, qs, qds);
                    } else {
                        bgc_q_phy(g, md, y, W, c, slot, qs);
                        if (TANGENT) bgc_q_phy_tangent(g, md, y, v, W, c, slot, qds);
                    }
                    cur = slot;
                }
                const int tr = wc % 3;
                const double sc = SUB ? 1.0 : dtd;   // internal steps return the increment itself
                acc[cc] += sc * qs[tr];
                if (TANGENT) accd[cc] += sc * qds[tr];
            }
        } else {
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) {
            const int wc = wc0 + cc;
            if (wc >= W) break;
            const int tr = wc % md.ntr;
            if (tr != 0 && cc != 0) continue;   // computed with its tracer-0 column
            const int slot = wc / md.ntr;
            double q1, q2, qd1 = 0.0, qd2 = 0.0;
            double sc = dtd;      // internal steps return the increment itself
            if constexpr (SUB == 1) {
                double o[2] = {0.0, 0.0}, od[2] = {0.0, 0.0};
                if (md.ntr == 2) bgc_inc<2, TANGENT>(g, md, y, v, W, c, slot, o, od);
                else bgc_inc<1, TANGENT>(g, md, y, v, W, c, slot, o, od);
                q1 = o[0];
                q2 = o[1];
                qd1 = od[0];
                qd2 = od[1];
                sc = 1.0;
            } else {
                bgc_q(g, md, y, W, c, slot, q1, q2);
                if (TANGENT) bgc_q_tangent(g, md, y, v, W, c, slot, qd1, qd2);
            }
            if (tr == 0) {
                acc[cc] += sc * q1;
                if (TANGENT) accd[cc] += sc * qd1;
                if (md.ntr > 1 && cc + 1 < CW && wc + 1 < W) {
                    acc[cc + 1] += sc * q2;
                    if (TANGENT) accd[cc + 1] += sc * qd2;
                }
            } else {   // first column of this thread is tracer 1 of its member
                acc[cc] += sc * q2;
                if (TANGENT) accd[cc] += sc * qd2;
            }
        }
        }
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) {
            if (wc0 + cc < W) {
                s_z[(size_t)rr * W + wc0 + cc] = acc[cc];
                if (TANGENT) s_zd[(size_t)rr * W + wc0 + cc] = accd[cc];
            }
        }
    }
    __syncthreads();

    const double* ai0 = mt.ai_cm + (size_t)k0 * mt.ai_month;
    const double* ai1 = mt.ai_cm + (size_t)k1 * mt.ai_month;
    for (int task = threadIdx.x; task < ntask; task += blockDim.x) {
        const int rr = task / tpr;
        const int wc0 = (task % tpr) * CW;
        const int r = tm.r0 + rr;
        const int lc = L.row_col[rr];
        const int lr0 = L.col_r0[lc];
        const int nc = L.col_nc[lc];
        const int k = L.row_k[rr];
        const size_t blk = (size_t)g.blk_off[tm.c0 + lc];
        double acc[CW], accd[CW];
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) { acc[cc] = 0.0; accd[cc] = 0.0; }
        for (int s = 0; s < nc; ++s) {
            const size_t e = blk + (size_t)s * nc + k;
            const double a = om * ai0[e] + w * ai1[e];
#pragma unroll
            for (int cc = 0; cc < CW; ++cc) {
                if (wc0 + cc < W) {
                    acc[cc] += a * s_z[(size_t)(lr0 + s) * W + wc0 + cc];
                    if (TANGENT) accd[cc] += a * s_zd[(size_t)(lr0 + s) * W + wc0 + cc];
                }
            }
        }
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) {
            if (wc0 + cc < W) {
                yo[(size_t)r * W + wc0 + cc] = acc[cc];
                if (TANGENT) vo[(size_t)r * W + wc0 + cc] = accd[cc];
            }
        }
    }
}


// ---------------------------------------------------------------------------
// Forward step for ensembles: one wavefront per water column and group of up
// to 64 members, lane = member (both tracers).  Each wavefront first stages
// the column's interpolated matrices in its own LDS slice with coalesced loads
// (the Ai block, and the Ae rows: row offsets and values), so that all
// gathers of the state are independent and wave-uniform reads come from LDS.
// A member's parameters, light factors and export Phi are evaluated once per
// column; z of the column stays in registers (KMAX >= column depth).
//
// Wave w of workgroup b takes water column order[b * WAVES + w] (-1: none).
// The host builds the order so that each XCD (workgroups are dispatched to
// the 8 XCDs round-robin) sweeps its own share of the grid in bands of a few
// latitude rows, longitude by longitude: a column's horizontal neighbours are
// then processed by the same XCD within a few dozen columns, while their
// state rows are still in its L2, instead of one latitude row (several MB of
// state at 64 members) later.  Without an order (nullptr) wave w of block b
// takes column b * WAVES + w.
//
// Batches of at most 32 (16) members run with G = 32 (16): a wavefront then
// holds CPW = 64 / G columns, lanes [s * G, (s + 1) * G) on column slot
// b * WAVES * CPW + w * CPW + s of the order, member groups of G lanes, so
// that the step's time follows the member count instead of leaving lanes
// idle.  Each lane computes exactly what it computes with G = 64.
// ---------------------------------------------------------------------------
constexpr int kMembersWaves = 4;      // default wavefronts (columns) per workgroup
constexpr int kMembersEll = 8;        // Ae nonzeros per row supported by k_step_members

template <int NTR, int KMAX, int EL, bool SUB = false, int WAVES = kMembersWaves, int G = 64>
__global__ __launch_bounds__(64 * WAVES) void k_step_members(Grid g, Model md, Mats mt, int ncol, int nb, int j,
                                                             double dtd, const int* __restrict__ order,
                                                             const double* __restrict__ y,
                                                             double* __restrict__ yo, int nt_store) {
    constexpr int NEU = 4;
    constexpr int CPW = 64 / G;                  // water columns per wavefront (G lanes = members each)
    static_assert(G == 64 || G == 32 || G == 16, "members per column group");
    // zero-padded KMAX x KMAX block and KMAX x EL explicit rows, so that every
    // loop below runs to its compile-time bound without branches
    __shared__ double s_ai[WAVES * CPW][KMAX * KMAX];
    __shared__ double s_ae[WAVES * CPW][KMAX * EL];
    __shared__ uint32_t s_off[WAVES * CPW][KMAX * EL];   // byte offset of the row each entry reads (< 2^32)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ml = lane % G;                     // member lane within the column's group
    const int cs = wave * CPW + lane / G;        // column slot within the workgroup (its LDS slice)
    const int slot = blockIdx.x * WAVES * CPW + cs;
    const int craw = order ? order[slot] : (slot < ncol ? slot : -1);
    const bool valid = craw >= 0;                // waves without a column idle but reach the barrier
    const int c = valid ? craw : ncol - 1;
    const int b = blockIdx.y * G + ml;
    const bool act = valid && b < nb;
    const int bb = b < nb ? b : 0;               // idle lanes read member 0 (in bounds) and store nothing
    const int W = nb * NTR;
    const int rs = g.col_start[c];
    const int nc = g.col_start[c + 1] - rs;
    int k0, k1;
    double w;
    step_phase(j, g.nstep, g.nmat, k0, k1, w);
    const double om = 1.0 - w;

    // the member's parameters and light factors, the column's insolation and
    // euphotic state: loaded before the staging below so that their latency
    // overlaps it (a load cannot move across the barrier)
    const double Q = g.ins[(size_t)(j % g.nstep) * g.nlat + g.col_lat[c]];
    const int m = md.member[bb];
    // member tables through their member-fastest copies: the lanes of one
    // load read neighbouring words instead of one cache line each
    const BgcParams p = load_params_at(md.uT, md.model, 1, (size_t)md.nbm, m);
    const double* rhoc = md.rhoT + (size_t)nc * g.nlayer * md.nbm + m;   // rho_k of this depth at [k * nbm]
    const size_t me = (size_t)bb * NTR;
    const int ne = nc < g.neu ? nc : g.neu;
    double Ne[NEU], le[NEU], f[NEU];
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const int re = rs + (e < nc ? e : nc - 1);
        Ne[e] = y[(size_t)re * W + me];
        le[e] = md.lightT[(size_t)(e < g.nlayer ? e : 0) * md.nbm + m];
    }

    // stage the interpolated column matrices (this wavefront's slice only);
    // the loops run to compile-time bounds, so that every load of a lane is
    // issued before the first one is waited for
    {
        const size_t bo = (size_t)g.blk_off[c];
        const double* ai0 = mt.ai_rm + (size_t)k0 * mt.ai_month + bo;
        const double* ai1 = mt.ai_rm + (size_t)k1 * mt.ai_month + bo;
        constexpr int NA = (KMAX * KMAX + G - 1) / G;
#pragma unroll
        for (int it = 0; it < NA; ++it) {
            const int i = it * G + ml;
            const int k = i / KMAX, sl = i % KMAX;
            const bool in = i < KMAX * KMAX && k < nc && sl < nc;
            const int at = in ? k * nc + sl : 0;
            const double v = om * ai0[at] + w * ai1[at];
            if (i < KMAX * KMAX) s_ai[cs][i] = in ? v : 0.0;
        }
        const double* ae0 = mt.ae + (size_t)k0 * mt.ae_month;
        const double* ae1 = mt.ae + (size_t)k1 * mt.ae_month;
        constexpr int NE = (KMAX * EL + G - 1) / G;
#pragma unroll
        for (int it = 0; it < NE; ++it) {
            const int i = it * G + ml;
            const int k = i / EL, sl = i % EL;
            const bool in = i < KMAX * EL && k < nc && sl < mt.ew;
            const size_t e = in ? (size_t)sl * g.npad + rs + k : (size_t)rs;
            const int col = mt.ae_col[e];
            const double v = om * ae0[e] + w * ae1[e];
            if (i < KMAX * EL) {
                s_off[cs][i] = (uint32_t)(in ? col : rs) * (uint32_t)(W * 8);
                s_ae[cs][i] = in ? v : 0.0;
            }
        }
    }
    __syncthreads();

    // production in the euphotic layers and the export Phi
    double Phi = 0.0;
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        f[e] = 0.0;
        if (e < ne) {
            f[e] = production(p, Ne[e], Q, le[e]).f;
            Phi += g.dz[e] * f[e];
        }
    }

    // internal BGC steps (section 7): increments of the euphotic rows, the
    // summed export and the decay factors for the rows below
    double einc[NEU][NTR], sphi = 0.0;
    DeepFactors DF{0.0, 0.0, 1.0};
    if (SUB) {
        static_assert(NEU == kSubNeuMax, "euphotic register width");
        double ye[NEU][NTR], hz[NEU], re[NEU];
#pragma unroll
        for (int e = 0; e < NEU; ++e) {
            const int ee = e < g.nlayer ? e : 0;
            const int rr = rs + (e < nc ? e : nc - 1);
            ye[e][0] = e < ne ? Ne[e] : 0.0;
            if (NTR > 1) ye[e][NTR - 1] = e < ne ? y[(size_t)rr * W + me + NTR - 1] : 0.0;
            hz[e] = g.dz[ee];
            re[e] = rhoc[(size_t)ee * md.nbm];
#pragma unroll
            for (int t = 0; t < NTR; ++t) einc[e][t] = 0.0;
        }
        const Euphotic<NEU> E = make_euphotic<NEU>(p, Q, ne, le, hz, re);
        for (int s = 0; s < md.nsub; ++s) sphi += euphotic_step<NTR, NEU>(p, E, ye, md.hsub, einc);
        DF = deep_factors<NTR>(p, md.hsub, md.nsub);
    }

    // z = Ae(t_j) y + dt_d q for every row of the column, in registers.  Rows
    // past the column's depth (k >= nc) repeat finite work on its rows and
    // meet zero columns of the staged Ai block below.
    // A gather is a 32-bit byte offset (the staged row offset plus the lane's
    // member) on the state's base address.
    const char* ybytes = reinterpret_cast<const char*>(y);
    const uint32_t me8 = (uint32_t)me * 8u;
    double z[KMAX][NTR];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int kk = k < nc ? k : nc - 1;
        double yv[EL][NTR];
#pragma unroll
        for (int sl = 0; sl < EL; ++sl) {
            const double* src =
                reinterpret_cast<const double*>(ybytes + (size_t)(s_off[cs][k * EL + sl] + me8));
            if constexpr (NTR == 2) {
                // both tracers of a member in one 16-byte load (W is even, so the pair is aligned)
                const double2 v = *reinterpret_cast<const double2*>(src);
                yv[sl][0] = v.x;
                yv[sl][1] = v.y;
            } else {
#pragma unroll
                for (int t = 0; t < NTR; ++t) yv[sl][t] = src[t];
            }
        }
        // the row's own DOP: slot 0 of every row reads the row itself
        const double dop = NTR > 1 ? yv[0][NTR - 1] : 0.0;
        const double rho = rhoc[(size_t)kk * md.nbm];
        double acc[NTR];
#pragma unroll
        for (int t = 0; t < NTR; ++t) acc[t] = 0.0;
#pragma unroll
        for (int sl = 0; sl < EL; ++sl) {
            const double a = s_ae[cs][k * EL + sl];
#pragma unroll
            for (int t = 0; t < NTR; ++t) acc[t] += a * yv[sl][t];
        }
        if (SUB) {
            double src[NTR];
            src[0] = md.hsub * (p.lam * dop * DF.G + (1.0 - p.sig) * rho * sphi);
            if (NTR > 1) src[NTR - 1] = dop * DF.pm1;
#pragma unroll
            for (int e = 0; e < NEU; ++e)
                if (e == k && e < ne) {
#pragma unroll
                    for (int t = 0; t < NTR; ++t) src[t] = einc[e][t];
                }
#pragma unroll
            for (int t = 0; t < NTR; ++t) z[k][t] = acc[t] + src[t];
        } else {
            double fk = 0.0;
#pragma unroll
            for (int e = 0; e < NEU; ++e)
                if (e == k) fk = f[e];
            const double q1 = -fk + p.lam * dop + (1.0 - p.sig) * Phi * rho;
            z[k][0] = acc[0] + dtd * q1;
            if (NTR > 1) z[k][NTR - 1] = acc[NTR - 1] + dtd * (p.sig * fk - p.lam * dop);
        }
    }

    // y_out = Ai(t_j) z within the column
    for (int k = 0; k < nc; ++k) {
        double acc[NTR];
#pragma unroll
        for (int t = 0; t < NTR; ++t) acc[t] = 0.0;
#pragma unroll
        for (int sl = 0; sl < KMAX; ++sl) {
            const double a = s_ai[cs][k * KMAX + sl];
#pragma unroll
            for (int t = 0; t < NTR; ++t) acc[t] += a * z[sl][t];
        }
        if (act) {
            double* dst = yo + (size_t)(rs + k) * W + me;
            if constexpr (NTR == 2) {
                if (nt_store) {
                    // non-temporal: a step whose state and matrices outgrow the last-level cache
                    // gains nothing from keeping the new state there (its rows are read again
                    // only in the next step), and the store would evict rows still to be gathered
                    typedef double d2v __attribute__((ext_vector_type(2)));
                    const d2v v = {acc[0], acc[1]};
                    __builtin_nontemporal_store(v, reinterpret_cast<d2v*>(dst));
                } else {
                    *reinterpret_cast<double2*>(dst) = make_double2(acc[0], acc[1]);
                }
            } else {
#pragma unroll
                for (int t = 0; t < NTR; ++t) dst[t] = acc[t];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Forward step for ensembles of two-tracer models, a tile of T water columns
// per workgroup.  Lanes are members as in k_step_members and wavefront w owns
// column order[b * T + w], but the state rows the tile's explicit rows read
// (the explicit operator is horizontal, so for layer k these are the tile's
// own rows at layer k and their horizontal neighbours) are loaded once per
// workgroup into LDS instead of once per reading row.  The host lists, per
// workgroup and layer, the distinct rows to load (at most RMAX) and, per
// column, row and stencil entry, which of them the entry reads.  Layers are
// loaded PF ahead into registers and written to one of two LDS buffers, one
// workgroup barrier per layer.  The loads are buffer loads: an unused slot
// gets an offset past the end of the state, which reads zeros without a
// memory access, so that no load sits under a branch and the compiler can
// keep PF layers in flight.  Results are bitwise those of k_step_members:
// every sum is formed in the same order from the same values.
//
// stage[((b * T + w) * KMAX + k) * QN + q]: row that wave w loads for slot
//     w + q * T of layer k of workgroup b, or -1;
// lidx[(b * T + w) * KMAX * 5 + k * 5 + s]: slot of layer k read by stencil
//     entry s of row k of wave w's column (0 where the entry is padding).
// Requires n * W * 8 < 2^32 (byte offsets of the state in 32 bits).
// ---------------------------------------------------------------------------
template <int KMAX, int T, int RMAX, int PF>
__global__ __launch_bounds__(64 * T) void k_step_member_tiles(Grid g, Model md, Mats mt, int nb, int j, double dtd,
                                                              const int* __restrict__ order,
                                                              const int* __restrict__ stage,
                                                              const unsigned char* __restrict__ lidx,
                                                              const double* __restrict__ y,
                                                              double* __restrict__ yo) {
    constexpr int NTR = 2, EL = 5, NEU = 4;
    constexpr int QN = RMAX / T;                       // slots each wave loads per layer
    constexpr int NSE = (KMAX * QN + 63) / 64;         // registers holding the wave's stage entries
    static_assert(RMAX % T == 0, "slots per layer");
    __shared__ double s_ai[T][KMAX * KMAX];
    __shared__ double s_ae[T][KMAX * EL];
    __shared__ uint32_t s_off[T][KMAX * EL];          // byte offset of the slot within a layer buffer
    __shared__ double2 s_rows[2][RMAX][64];           // two layers of staged state rows
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = blockIdx.x * T + wave;
    const int craw = order[slot];
    const bool valid = craw >= 0;
    const int c = valid ? craw : 0;                   // idle waves stage column 0 and store nothing
    const int b = blockIdx.y * 64 + lane;
    const bool act = valid && b < nb;
    const int bb = b < nb ? b : 0;
    const int W = nb * NTR;
    const int rs = g.col_start[c];
    const int nc = g.col_start[c + 1] - rs;
    int k0, k1;
    double w;
    step_phase(j, g.nstep, g.nmat, k0, k1, w);
    const double om = 1.0 - w;
    const int m = md.member[bb];
    const double* rhoc = md.rhoT + (size_t)nc * g.nlayer * md.nbm + m;   // rho_k of this depth at [k * nbm]

    // this wave's stage entries, lane l holding entry l + 64 * r
    int se[NSE];
    {
        const int* st = stage + (size_t)slot * KMAX * QN;
#pragma unroll
        for (int r = 0; r < NSE; ++r) {
            const int i = r * 64 + lane;
            se[r] = i < KMAX * QN ? st[i] : -1;
        }
    }
    const __amdgpu_buffer_rsrc_t yrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double*>(y), (short)0, (int)(uint32_t)((size_t)g.n * W * 8), 0x00020000);
    const uint32_t me8 = (uint32_t)bb * NTR * 8u, rowb = (uint32_t)W * 8u;
    double2 R[PF][QN];
    double rR[PF];
    // layer k's rows into registers set p (k, q, p compile-time after unrolling)
    auto issue = [&](int k, int p) {
        const int kk = k < nc ? k : nc - 1;
        rR[p] = rhoc[(size_t)kk * md.nbm];
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int i = k * QN + q;
            const int row = __builtin_amdgcn_readlane(se[i / 64], i % 64);
            const uint32_t off = row >= 0 ? (uint32_t)row * rowb + me8 : 0xFFFFFFF0u;
            R[p][q] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(yrs, (int)off, 0, 0));
        }
    };
#pragma unroll
    for (int p = 0; p < PF; ++p)
        if (p < KMAX) issue(p, p);

    const double Q = g.ins[(size_t)(j % g.nstep) * g.nlat + g.col_lat[c]];
    const BgcParams p = load_params_at(md.uT, md.model, 1, (size_t)md.nbm, m);
    const size_t me = (size_t)bb * NTR;
    const int ne = nc < g.neu ? nc : g.neu;
    double Ne[NEU], le[NEU], f[NEU];
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const int re = rs + (e < nc ? e : nc - 1);
        Ne[e] = y[(size_t)re * W + me];
        le[e] = md.lightT[(size_t)(e < g.nlayer ? e : 0) * md.nbm + m];
    }

    // the column's interpolated matrices and stencil slots (this wave's slice)
    {
        const size_t bo = (size_t)g.blk_off[c];
        const double* ai0 = mt.ai_rm + (size_t)k0 * mt.ai_month + bo;
        const double* ai1 = mt.ai_rm + (size_t)k1 * mt.ai_month + bo;
        constexpr int NA = (KMAX * KMAX + 63) / 64;
#pragma unroll
        for (int it = 0; it < NA; ++it) {
            const int i = it * 64 + lane;
            const int k = i / KMAX, sl = i % KMAX;
            const bool in = i < KMAX * KMAX && k < nc && sl < nc;
            const int at = in ? k * nc + sl : 0;
            const double v = om * ai0[at] + w * ai1[at];
            if (i < KMAX * KMAX) s_ai[wave][i] = in ? v : 0.0;
        }
        const double* ae0 = mt.ae + (size_t)k0 * mt.ae_month;
        const double* ae1 = mt.ae + (size_t)k1 * mt.ae_month;
        const unsigned char* li = lidx + (size_t)slot * KMAX * EL;
        constexpr int NE = (KMAX * EL + 63) / 64;
#pragma unroll
        for (int it = 0; it < NE; ++it) {
            const int i = it * 64 + lane;
            const int k = i / EL, sl = i % EL;
            const bool in = i < KMAX * EL && k < nc && sl < mt.ew;
            const size_t e = in ? (size_t)sl * g.npad + rs + k : (size_t)rs;
            const double v = om * ae0[e] + w * ae1[e];
            const int ii = i < KMAX * EL ? i : 0;
            const uint32_t at = (uint32_t)li[ii] * (uint32_t)(64 * sizeof(double2));
            if (i < KMAX * EL) {
                s_off[wave][i] = at;
                s_ae[wave][i] = in ? v : 0.0;
            }
        }
    }

    double Phi = 0.0;
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        f[e] = 0.0;
        if (e < ne) {
            f[e] = production(p, Ne[e], Q, le[e]).f;
            Phi += g.dz[e] * f[e];
        }
    }

    // layer by layer: stage the layer's rows, then z of this column's row k.
    // Rows past the column's depth (k >= nc) form finite values that meet
    // zero columns of the staged Ai block below.
    double z[KMAX][NTR];
    const char* lds_lane = reinterpret_cast<const char*>(&s_rows[0][0][lane]);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
#pragma unroll
        for (int q = 0; q < QN; ++q) s_rows[k & 1][wave + q * T][lane] = R[k % PF][q];
        const double rho = rR[k % PF];
        __syncthreads();
        // after the barrier, whose fence keeps the compiler from hoisting
        // every layer's loads to the top (registers)
        if (k + PF < KMAX) issue(k + PF, k % PF);
        double yv[EL][NTR];
#pragma unroll
        for (int sl = 0; sl < EL; ++sl) {
            const double2 v = *reinterpret_cast<const double2*>(
                lds_lane + (size_t)(k & 1) * RMAX * 64 * sizeof(double2) + s_off[wave][k * EL + sl]);
            yv[sl][0] = v.x;
            yv[sl][1] = v.y;
        }
        const double dop = yv[0][1];          // slot of entry 0: the row itself
        double acc[NTR] = {0.0, 0.0};
#pragma unroll
        for (int sl = 0; sl < EL; ++sl) {
            const double a = s_ae[wave][k * EL + sl];
#pragma unroll
            for (int t = 0; t < NTR; ++t) acc[t] += a * yv[sl][t];
        }
        double fk = 0.0;
#pragma unroll
        for (int e = 0; e < NEU; ++e)
            if (e == k) fk = f[e];
        const double q1 = -fk + p.lam * dop + (1.0 - p.sig) * Phi * rho;
        z[k][0] = acc[0] + dtd * q1;
        z[k][1] = acc[1] + dtd * (p.sig * fk - p.lam * dop);
        // form z here: left alone, the compiler sinks this arithmetic past the
        // remaining layers into the product below and keeps every layer's
        // staged values live instead (spills)
        __asm__ volatile("" : "+v"(z[k][0]), "+v"(z[k][1]));
    }

    // y_out = Ai(t_j) z within the column
    for (int k = 0; k < nc; ++k) {
        double acc[NTR] = {0.0, 0.0};
#pragma unroll
        for (int sl = 0; sl < KMAX; ++sl) {
            const double a = s_ai[wave][k * KMAX + sl];
#pragma unroll
            for (int t = 0; t < NTR; ++t) acc[t] += a * z[sl][t];
        }
        if (act) *reinterpret_cast<double2*>(yo + (size_t)(rs + k) * W + me) = make_double2(acc[0], acc[1]);
    }
}

// ---------------------------------------------------------------------------
// Adjoint step (reverse mode of k_step).  With mu_j the cotangent of z_j:
//   lambda_j = Ae(t_j)^T mu_j + dt_d (dq/dy)(y_j)^T mu_j + s_j
//   mu_{j-1} = Ai(t_{j-1})^T lambda_j
//   ubar    += dt_d (dq/du)(y_j)^T mu_j        (per-tile partial sums)
// s_j is the misfit source at month ends.  use_ae = false starts the sweep
// from the source alone; use_ai = false ends it, writing lambda_0.
// Thread task = (row, member); NTR = tracers per member.
// ---------------------------------------------------------------------------
template <int NTR, int MAXR, int MAXC, bool SUB = false>
__global__ __launch_bounds__(256) void k_adjoint(Grid g, Model md, Mats mt, int W, int nb, int j, double dtd,
                          int use_ae, int use_ai, const double* __restrict__ mu,
                          const double* __restrict__ yj, const double* __restrict__ obs, double src_scale,
                          double* __restrict__ out, double* __restrict__ ubar_tile) {
    extern __shared__ double s_dyn[];
    __shared__ TileLds<MAXR, MAXC> L;
    constexpr int NP = NTR == 3 ? 11 : (NTR == 2 ? 7 : 5);
    const TileMap tm = build_tile<MAXR, MAXC>(g, L, use_ae ? j % g.nstep : -1);
    double* s_lam = s_dyn;                                  // [nrows][W]
    double* s_contrib = s_dyn + (size_t)tm.nrows * W;       // [blockDim][NP]

    int k0, k1;
    double w;
    step_phase(j, g.nstep, g.nmat, k0, k1, w);
    const double om = 1.0 - w;
    const double* aet0 = mt.aet + (size_t)k0 * mt.aet_month;
    const double* aet1 = mt.aet + (size_t)k1 * mt.aet_month;
    const int ntask = tm.nrows * nb;
    const int passes = (ntask + blockDim.x - 1) / blockDim.x;
    // reduction threads: (member, parameter) pairs, accumulate over passes
    double ured = 0.0;

    for (int pass = 0; pass < passes; ++pass) {
        const int task = pass * blockDim.x + threadIdx.x;
        double contrib[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) contrib[p] = 0.0;
        if (task < ntask) {
            const int rr = task / nb;
            const int slot = task % nb;
            const int r = tm.r0 + rr;
            const int lc = L.row_col[rr];
            ColumnRef c;
            c.rs = tm.r0 + L.col_r0[lc];
            c.nc = L.col_nc[lc];
            c.k = L.row_k[rr];
            c.Q = L.Q[lc];
            double lam[NTR];
#pragma unroll
            for (int tr = 0; tr < NTR; ++tr) lam[tr] = 0.0;
            if (use_ae) {
                for (int s = 0; s < mt.etw; ++s) {
                    const size_t e = (size_t)s * g.npad + r;
                    const int col = mt.aet_col[e];
                    const double a = om * aet0[e] + w * aet1[e];
#pragma unroll
                    for (int tr = 0; tr < NTR; ++tr) lam[tr] += a * mu[(size_t)col * W + slot * NTR + tr];
                }
                if constexpr (SUB) {
                    // internal BGC steps: the reverse sweep returns h-weighted sums
                    double yb[NTR];
#pragma unroll
                    for (int tr = 0; tr < NTR; ++tr) yb[tr] = 0.0;
                    bgc_inc_adjoint<NTR, NP>(g, md, yj, mu, W, c, slot, yb, contrib);
#pragma unroll
                    for (int tr = 0; tr < NTR; ++tr) lam[tr] += yb[tr];
                } else if constexpr (NTR == 3) {
                    bgc_q_phy_adjoint(g, md, yj, mu, W, c, slot, dtd, lam, contrib);
                } else {
                    // (dq/dy)^T mu and (dq/du)^T mu for this row
                    const int m = md.member[slot];
                    const BgcParams p = load_params(md.u, md.model, md.nparam, m);
                    const double* light = md.light + (size_t)m * g.nlayer;
                    const size_t tab = ((size_t)m * (g.nlayer + 1) + c.nc) * g.nlayer;
                    const int ne = c.nc < g.neu ? c.nc : g.neu;
                    double Phi = 0.0;
                    for (int e = 0; e < ne; ++e) {
                        const double N = yj[(size_t)(c.rs + e) * W + slot * NTR];
                        Phi += g.dz[e] * production(p, N, c.Q, light[e]).f;
                    }
                    const size_t at = (size_t)r * W + slot * NTR;
                    const double mu1 = mu[at];
                    const double mu2 = NTR > 1 ? mu[at + 1] : 0.0;
                    const double dop = NTR > 1 ? yj[at + 1] : 0.0;
                    const double rho = md.rho[tab + c.k];
                    const double drho = md.drho[tab + c.k];
                    double ybar1 = 0.0, ybar2 = 0.0;
                    if (c.k < g.neu) {
                        double Phibar = 0.0;
                        for (int kk = 0; kk < c.nc; ++kk)
                            Phibar += (1.0 - p.sig) * md.rho[tab + kk] * mu[(size_t)(c.rs + kk) * W + slot * NTR];
                        const Production pr = production(p, yj[at], c.Q, light[c.k]);
                        const double fbar = -mu1 + p.sig * mu2 + g.dz[c.k] * Phibar;
                        ybar1 = fbar * pr.dfdN;
                        // df/dalpha, df/dK_H2O, df/dK_1, df/dK_I
                        const double Np = yj[at] > 0.0 ? yj[at] : 0.0;
                        const double zc = [&] {
                            double d = 0.0;
                            for (int i = 0; i <= c.k; ++i) d += g.dz[i];
                            return d - 0.5 * g.dz[c.k];
                        }();
                        const double IKI2 = (pr.I + p.ki) * (pr.I + p.ki);
                        contrib[0] += fbar * pr.limN * pr.limI;
                        contrib[1] += fbar * p.alpha * pr.limN * p.ki / IKI2 * (-zc * pr.I);
                        contrib[2] += fbar * (-p.alpha * Np / ((Np + p.k1) * (Np + p.k1)) * pr.limI);
                        contrib[3] += fbar * (-p.alpha * pr.limN * pr.I / IKI2);
                        if (NTR > 1) contrib[5] += pr.f * mu2;
                    }
                    if (NTR > 1) {
                        ybar2 = p.lam * (mu1 - mu2);
                        contrib[4] += dop * (mu1 - mu2);
                        contrib[5] += -Phi * rho * mu1;
                        contrib[NP - 1] += (1.0 - p.sig) * Phi * drho * mu1;
                        lam[1] += dtd * ybar2;
                    } else {
                        contrib[NP - 1] += (1.0 - p.sig) * Phi * drho * mu1;
                    }
                    lam[0] += dtd * ybar1;
                }
            }
            if (obs) {
                const int lk = c.k;
                const double V = g.area[tm.c0 + lc] * g.dz[lk];
#pragma unroll
                for (int tr = 0; tr < NTR; ++tr) {
                    const size_t at = (size_t)r * W + slot * NTR + tr;
                    lam[tr] += V * (yj[at] - obs[at]) * src_scale;
                }
            }
#pragma unroll
            for (int tr = 0; tr < NTR; ++tr) s_lam[(size_t)rr * W + slot * NTR + tr] = lam[tr];
        }
        if (ubar_tile) {
#pragma unroll
            for (int p = 0; p < NP; ++p) s_contrib[(size_t)threadIdx.x * NP + p] = contrib[p];
            __syncthreads();
            // thread (slot, p) sums the rows of this pass in a fixed order; task
            // pass*blockDim + tt belongs to slot (pass*blockDim + tt) % nb
            if ((int)threadIdx.x < nb * NP) {
                const int slot = threadIdx.x / NP, p = threadIdx.x % NP;
                const int lim = min((int)blockDim.x, ntask - pass * (int)blockDim.x);
                const int first = (slot - (pass * (int)blockDim.x) % nb + nb) % nb;
                double s = 0.0;
                for (int tt = first; tt < lim; tt += nb) s += s_contrib[(size_t)tt * NP + p];
                ured += s;
            }
            __syncthreads();
        }
    }
    if (ubar_tile && (int)threadIdx.x < nb * NP)
        ubar_tile[(size_t)blockIdx.x * nb * NP + threadIdx.x] += (SUB ? md.hsub : dtd) * ured;
    __syncthreads();

    // mu_{j-1} = Ai(t_{j-1})^T lambda_j, or lambda_j itself at the end
    int q0, q1;
    double wq;
    step_phase(j - 1, g.nstep, g.nmat, q0, q1, wq);
    const double omq = 1.0 - wq;
    const double* ai0 = mt.ai_rm + (size_t)q0 * mt.ai_month;
    const double* ai1 = mt.ai_rm + (size_t)q1 * mt.ai_month;
    for (int task = threadIdx.x; task < ntask; task += blockDim.x) {
        const int rr = task / nb;
        const int slot = task % nb;
        const int r = tm.r0 + rr;
        if (!use_ai) {
#pragma unroll
            for (int tr = 0; tr < NTR; ++tr)
                out[(size_t)r * W + slot * NTR + tr] = s_lam[(size_t)rr * W + slot * NTR + tr];
            continue;
        }
        const int lc = L.row_col[rr];
        const int lr0 = L.col_r0[lc];
        const int nc = L.col_nc[lc];
        const int k = L.row_k[rr];
        const size_t blk = (size_t)g.blk_off[tm.c0 + lc];
        double acc[NTR];
#pragma unroll
        for (int tr = 0; tr < NTR; ++tr) acc[tr] = 0.0;
        for (int s = 0; s < nc; ++s) {   // row s of the block, column k
            const size_t e = blk + (size_t)s * nc + k;
            const double a = omq * ai0[e] + wq * ai1[e];
#pragma unroll
            for (int tr = 0; tr < NTR; ++tr) acc[tr] += a * s_lam[(size_t)(lr0 + s) * W + slot * NTR + tr];
        }
#pragma unroll
        for (int tr = 0; tr < NTR; ++tr) out[(size_t)r * W + slot * NTR + tr] = acc[tr];
    }
}

// ---------------------------------------------------------------------------
// Reductions (deterministic: fixed-order per-tile partial sums, then a fixed-
// order sum over tiles).
// ---------------------------------------------------------------------------

// part[tile][slot] = sum over the tile's rows and the slot's tracers of
// weight_i * (a - b)^2, weight_i = V_i if volume != 0 else 1; b may be NULL.
template <int MAXR, int MAXC>
__global__ void k_tile_sqdiff(Grid g, int W, int ntr, int nb, const double* __restrict__ a,
                              const double* __restrict__ b, int volume, double* __restrict__ part) {
    __shared__ TileLds<MAXR, MAXC> L;
    __shared__ double s_red[256];
    const TileMap tm = build_tile<MAXR, MAXC>(g, L, -1);
    for (int slot = 0; slot < nb; ++slot) {
        double s = 0.0;
        for (int rr = threadIdx.x; rr < tm.nrows; rr += blockDim.x) {
            const int r = tm.r0 + rr;
            double wgt = 1.0;
            if (volume) wgt = g.area[tm.c0 + L.row_col[rr]] * g.dz[L.row_k[rr]];
            for (int tr = 0; tr < ntr; ++tr) {
                const size_t at = (size_t)r * W + slot * ntr + tr;
                const double d = b ? a[at] - b[at] : a[at];
                s += wgt * d * d;
            }
        }
        s_red[threadIdx.x] = s;
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) s_red[threadIdx.x] += s_red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * nb + slot] = s_red[0];
        __syncthreads();
    }
}

// Per-tile cell volume sums (for V_tot).
template <int MAXR, int MAXC>
__global__ void k_tile_volume(Grid g, double* __restrict__ part) {
    __shared__ TileLds<MAXR, MAXC> L;
    __shared__ double s_red[256];
    const TileMap tm = build_tile<MAXR, MAXC>(g, L, -1);
    double s = 0.0;
    for (int rr = threadIdx.x; rr < tm.nrows; rr += blockDim.x)
        s += g.area[tm.c0 + L.row_col[rr]] * g.dz[L.row_k[rr]];
    s_red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s_red[threadIdx.x] += s_red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s_red[0];
}

// out[q] = scale * sum_t part[t*stride + q] (+ out[q] if accumulate); optional sqrt.
__global__ void k_sum_tiles(int ntile, int stride, int nq, const double* __restrict__ part, double scale,
                            int accumulate, int take_sqrt, double* __restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    double s = 0.0;
    for (int t = 0; t < ntile; ++t) s += part[(size_t)t * stride + q];
    s *= scale;
    if (take_sqrt) s = sqrt(s);
    out[q] = accumulate ? out[q] + s : s;
}

__global__ void k_fill(double* __restrict__ x, size_t len, double value) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < len; i += stride) x[i] = value;
}

__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, size_t len) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < len; i += stride) dst[i] = src[i];
}

// flag = 1 if any of x[0 .. len) is not finite (left alone otherwise).
__global__ void k_check_finite(const double* __restrict__ x, size_t len, int* __restrict__ flag) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; i < len; i += stride) bad |= !isfinite(x[i]);
    if (bad) *flag = 1;
}

// FD direction: h_s = 1e-8 ||y_s|| / ||v_s|| per slot from squared norms.
__global__ void k_fd_step(int nb, const double* __restrict__ ny2, const double* __restrict__ nv2,
                          double* __restrict__ h) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nb) return;
    h[s] = nv2[s] > 0.0 ? 1e-8 * sqrt(ny2[s]) / sqrt(nv2[s]) : 0.0;
}

// out = y + h_slot v
__global__ void k_axpy_slots(size_t n, int W, int ntr, const double* __restrict__ h, const double* __restrict__ y,
                             const double* __restrict__ v, double* __restrict__ out) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n * W; i += stride) out[i] = y[i] + h[(i % W) / ntr] * v[i];
}

// jv = (fp - f0)/h_slot  (0 where h = 0)
__global__ void k_fd_quot(size_t n, int W, int ntr, const double* __restrict__ h, const double* __restrict__ fp,
                          const double* __restrict__ f0, double* __restrict__ jv) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n * W; i += stride) {
        const double hh = h[(i % W) / ntr];
        jv[i] = hh > 0.0 ? (fp[i] - f0[i]) / hh : 0.0;
    }
}

// Column gather between state layouts: dst[i*Wd + dcol[s]*ntr + tr] = src[i*Ws + scol[s]*ntr + tr]
// for s < ns (member compaction and scatter of finished members).
__global__ void k_gather_slots(size_t n, int ns, int ntr, int Ws, int Wd, const int* __restrict__ scol,
                               const int* __restrict__ dcol, const double* __restrict__ src,
                               double* __restrict__ dst) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t per_row = (size_t)ns * ntr;
    for (; i < n * per_row; i += stride) {
        const size_t row = i / per_row;
        const int q = (int)(i % per_row);
        const int s = q / ntr, tr = q % ntr;
        dst[row * Wd + (size_t)dcol[s] * ntr + tr] = src[row * Ws + (size_t)scol[s] * ntr + tr];
    }
}

}  // namespace tmm
