// Internal biogeochemical steps per ocean step (section 7 of the paper: the
// biogeochemical models take several time steps within one step of the
// transport).
//
// Over one ocean step of length dt_d the source is the increment of nsub
// explicit Euler steps of length h = dt_d / nsub with that step's forcing
// (insolation) held fixed:
//     inc_0 = 0,   inc_{s+1} = inc_s + h q(y + inc_s),   source = inc_nsub,
// so that nsub = 1 is dt_d q(y).
//
// Structure used here: within a water column the euphotic rows (layers
// e < ne) form a closed system -- production feeds the export Phi, which is
// remineralised below, but nothing below feeds back.  Every thread therefore
// integrates the (at most NEU) euphotic rows of its own column in registers,
// without barriers.  A row below the euphotic zone has
//     q_1 = lambda DOP_k + (1 - sigma) Phi rho_k,   q_2 = -lambda DOP_k
// (PO4-DOP-PHY, section 2.2.2: q_2 gains lambda'_3 PHY_k and q_3 = -lambda'_3
// PHY_k), linear in its own state, so its increment follows from sum_s Phi_s
// and per-member decay factors (DeepFactors below).
//
// Tracers of a row: 0 = PO4 (N), 1 = DOP, 2 = PHY.  In PO4-DOP-PHY the
// production f_1 is proportional to PHY, the export is Phi = sum h_e sigma_3
// f_1,e, and the euphotic rows lose lambda_3 PHY + kappa_3 PHY^2 to DOP.
//
// Reverse mode (adjoint of section 6 applied to the internal steps): with
// ib = mu (cotangent of the source) and s = nsub-1 .. 0,
//     ybar += h J_q(y + inc_s)^T ib,   ubar += h (dq/du)^T ib,   ib += h J_q^T ib.
// Below the euphotic zone d q / d N_k = 0, so those rows' nutrient cotangents
// stay mu_1 and their contribution to the export cotangent is a constant sum;
// their DOP cotangent decays by the same factors as the DOP itself.
//
// Included by tmm_device.hpp after the parameter block (BgcParams and the
// light constants).
#pragma once

namespace tmm {

constexpr int kSubMax = 16;     // internal steps per ocean step supported on the device
constexpr int kSubNeuMax = 4;   // euphotic layers supported with internal steps
constexpr int kDop = 1;         // tracer index of DOP (models with more than one tracer)
constexpr int kPhy = 2;         // tracer index of PHY (PO4-DOP-PHY)

// Constants of q for the euphotic rows of one column and member at one ocean
// step; entries e >= ne are zero.
template <int NEU>
struct Euphotic {
    int ne;
    double I[NEU], limI[NEU], hz[NEU], rho[NEU];
};

// light, hz, rho: NEU entries each (light factor exp(-z K_H2O), layer height
// and remineralisation fraction of each euphotic row), indexed with
// compile-time indices only; entries beyond ne are ignored.
template <int NEU>
__device__ __forceinline__ Euphotic<NEU> make_euphotic(const BgcParams& p, double Q, int ne, const double* light,
                                                       const double* hz, const double* rho) {
    Euphotic<NEU> E;
    E.ne = ne;
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const bool in = e < ne;
        E.I[e] = in ? Q * kSigmaPar * (1.0 - kSigmaIce) * light[e] : 0.0;
        E.limI[e] = in ? E.I[e] / (E.I[e] + p.ki) : 0.0;
        E.hz[e] = in ? hz[e] : 0.0;
        E.rho[e] = in ? rho[e] : 0.0;
    }
    return E;
}

// One Euler step of length h of the euphotic rows at state y + inc; returns
// the export Phi of that state.
template <int NTR, int NEU>
__device__ __forceinline__ double euphotic_step(const BgcParams& p, const Euphotic<NEU>& E, const double (&y)[NEU][NTR],
                                                double h, double (&inc)[NEU][NTR]) {
    double f[NEU];
    double Phi = 0.0;
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const double N = y[e][0] + inc[e][0];
        const double Np = N > 0.0 ? N : 0.0;
        f[e] = e < E.ne ? p.alpha * (Np / (Np + p.k1)) * E.limI[e] : 0.0;
        if constexpr (NTR == 3) {
            f[e] *= y[e][kPhy] + inc[e][kPhy];
            Phi += E.hz[e] * (p.sig3 * f[e]);
        } else {
            Phi += E.hz[e] * f[e];
        }
    }
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        if constexpr (NTR == 3) {
            const bool in = e < E.ne;
            const double D = y[e][kDop] + inc[e][kDop];
            const double P = y[e][kPhy] + inc[e][kPhy];
            const double loss = p.lam3 * P + p.kap3 * P * P;
            const double q1 = -f[e] + p.lam * D + (1.0 - p.sig) * Phi * E.rho[e];
            const double q2 = p.sig * (p.sig3 * f[e]) + loss - p.lam * D + p.lam3p * P;
            const double q3 = (1.0 - p.sig3) * f[e] - loss - p.lam3p * P;
            inc[e][0] += in ? h * q1 : 0.0;
            inc[e][kDop] += in ? h * q2 : 0.0;
            inc[e][kPhy] += in ? h * q3 : 0.0;
        } else {
            const double dop = NTR > 1 ? y[e][NTR - 1] + inc[e][NTR - 1] : 0.0;
            const double q1 = -f[e] + p.lam * dop + (1.0 - p.sig) * Phi * E.rho[e];
            inc[e][0] += e < E.ne ? h * q1 : 0.0;
            if (NTR > 1) inc[e][NTR - 1] += e < E.ne ? h * (p.sig * f[e] - p.lam * dop) : 0.0;
        }
    }
    return Phi;
}

// The same step with its tangent in direction v (incd = tangent of inc).
template <int NTR, int NEU>
__device__ __forceinline__ void euphotic_step_tangent(const BgcParams& p, const Euphotic<NEU>& E,
                                                      const double (&y)[NEU][NTR], const double (&v)[NEU][NTR],
                                                      double h, double (&inc)[NEU][NTR], double (&incd)[NEU][NTR],
                                                      double& Phi, double& Phid) {
    double f[NEU], fd[NEU];
    Phi = 0.0;
    Phid = 0.0;
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const double N = y[e][0] + inc[e][0];
        const double Np = N > 0.0 ? N : 0.0;
        const bool in = e < E.ne;
        f[e] = in ? p.alpha * (Np / (Np + p.k1)) * E.limI[e] : 0.0;
        const double dfdN = (in && N > 0.0) ? p.alpha * p.k1 / ((N + p.k1) * (N + p.k1)) * E.limI[e] : 0.0;
        if constexpr (NTR == 3) {
            // f_1 = f(N) PHY
            const double P = y[e][kPhy] + inc[e][kPhy];
            const double Pd = v[e][kPhy] + incd[e][kPhy];
            fd[e] = dfdN * (v[e][0] + incd[e][0]) * P + f[e] * Pd;
            f[e] *= P;
            Phi += E.hz[e] * (p.sig3 * f[e]);
            Phid += E.hz[e] * (p.sig3 * fd[e]);
        } else {
            fd[e] = dfdN * (v[e][0] + incd[e][0]);
            Phi += E.hz[e] * f[e];
            Phid += E.hz[e] * fd[e];
        }
    }
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const bool in = e < E.ne;
        if constexpr (NTR == 3) {
            const double D = y[e][kDop] + inc[e][kDop], Dd = v[e][kDop] + incd[e][kDop];
            const double P = y[e][kPhy] + inc[e][kPhy], Pd = v[e][kPhy] + incd[e][kPhy];
            const double loss = p.lam3 * P + p.kap3 * P * P;
            const double lossd = (p.lam3 + 2.0 * p.kap3 * P) * Pd;
            const double q1 = -f[e] + p.lam * D + (1.0 - p.sig) * Phi * E.rho[e];
            const double q2 = p.sig * (p.sig3 * f[e]) + loss - p.lam * D + p.lam3p * P;
            const double q3 = (1.0 - p.sig3) * f[e] - loss - p.lam3p * P;
            const double qd1 = -fd[e] + p.lam * Dd + (1.0 - p.sig) * Phid * E.rho[e];
            const double qd2 = p.sig * (p.sig3 * fd[e]) + lossd - p.lam * Dd + p.lam3p * Pd;
            const double qd3 = (1.0 - p.sig3) * fd[e] - lossd - p.lam3p * Pd;
            inc[e][0] += in ? h * q1 : 0.0;
            inc[e][kDop] += in ? h * q2 : 0.0;
            inc[e][kPhy] += in ? h * q3 : 0.0;
            incd[e][0] += in ? h * qd1 : 0.0;
            incd[e][kDop] += in ? h * qd2 : 0.0;
            incd[e][kPhy] += in ? h * qd3 : 0.0;
        } else {
            const double dop = NTR > 1 ? y[e][NTR - 1] + inc[e][NTR - 1] : 0.0;
            const double dopd = NTR > 1 ? v[e][NTR - 1] + incd[e][NTR - 1] : 0.0;
            const double q1 = -f[e] + p.lam * dop + (1.0 - p.sig) * Phi * E.rho[e];
            const double qd1 = -fd[e] + p.lam * dopd + (1.0 - p.sig) * Phid * E.rho[e];
            inc[e][0] += in ? h * q1 : 0.0;
            incd[e][0] += in ? h * qd1 : 0.0;
            if (NTR > 1) {
                inc[e][NTR - 1] += in ? h * (p.sig * f[e] - p.lam * dop) : 0.0;
                incd[e][NTR - 1] += in ? h * (p.sig * fd[e] - p.lam * dopd) : 0.0;
            }
        }
    }
}

// Rows below the euphotic zone: their DOP decays linearly and their nutrient
// only receives the export, so with a_s = (1 - h lambda)^s (advanced by the
// same Euler recursion, a_0 = 1) their increments are
//     inc_1 = h (lambda DOP_0 G + (1 - sigma) rho_k sum_s Phi_s),
//     inc_2 = DOP_0 (a_nsub - 1),          G = sum_{s<nsub} a_s,
// and their reverse mode needs only G, a_nsub - 1 and a_{nsub-1} as well.
//
// PO4-DOP-PHY adds PHY_{s+1} = PHY_s - h lambda'_3 PHY_s, whose loss feeds
// DOP: DOP_s = DOP_0 a_s + PHY_0 c_s with c_0 = 0 and
// c_{s+1} = c_s + h (lambda'_3 b_s - lambda c_s), b_s = (1 - h lambda'_3)^s.
// Then
//     inc_1 = h (lambda (DOP_0 G + PHY_0 GC) + (1 - sigma) rho_k sum_s Phi_s),
//     inc_2 = DOP_0 (a_nsub - 1) + PHY_0 c_nsub,   inc_3 = PHY_0 (b_nsub - 1),
// GC = sum_{s<nsub} c_s.  The parameter derivatives of these sums come from
// the same recursion differentiated (forward mode):
//     r_s = d(lambda GC)/d lambda at step s:  r_{s+1} = r_s (1 - h lambda) + c_s,
//     E_s = (1/h) d c_s / d lambda'_3:       E_{s+1} = E_s (1 - h lambda) + b_s + lambda'_3 beta_s,
//     beta_s = d b_s / d lambda'_3:           beta_{s+1} = beta_s (1 - h lambda'_3) - h b_s,
// and d(lambda'_3 GB)/d lambda'_3 = nsub b_{nsub-1} with GB = sum_{s<nsub} b_s.
struct DeepFactors {
    double G;       // sum_{s<nsub} a_s
    double pm1;     // a_nsub - 1
    double alast;   // a_{nsub-1}
    // PO4-DOP-PHY only
    double GC;      // sum_{s<nsub} c_s
    double cn;      // c_nsub
    double qm1;     // b_nsub - 1
    double GB;      // sum_{s<nsub} b_s
    double blast;   // b_{nsub-1}
    double r;       // d(lambda GC) / d lambda
    double E;       // (1/h) d c_nsub / d lambda'_3
};

template <int NTR = 2>
__device__ __forceinline__ DeepFactors deep_factors(const BgcParams& p, double h, int nsub) {
    DeepFactors d{0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0};
    double beta = 0.0;
    for (int s = 0; s < nsub; ++s) {
        const double a = 1.0 + d.pm1;
        d.G += a;
        d.alast = a;
        if constexpr (NTR == 3) {
            const double b = 1.0 + d.qm1;
            const double c = d.cn;
            d.GC += c;
            d.GB += b;
            d.blast = b;
            d.r = d.r * (1.0 - h * p.lam) + c;
            d.E = d.E * (1.0 - h * p.lam) + b + p.lam3p * beta;
            beta = beta * (1.0 - h * p.lam3p) - h * b;
            d.cn += h * (-(p.lam * c) + p.lam3p * b);
            d.qm1 += h * (-(p.lam3p * b));
        }
        d.pm1 += h * (-(p.lam * a));
    }
    return d;
}

// Source of the row in layer k over one ocean step: out = inc_nsub of that
// row.  ye: state of the column's euphotic rows (zero beyond ne); yk: the
// row's own state; rho_k its remineralisation fraction.
template <int NTR, int NEU>
__device__ __forceinline__ void row_source(const BgcParams& p, const Euphotic<NEU>& E, int k,
                                           const double (&ye)[NEU][NTR], const double (&yk)[NTR], double rho_k,
                                           double h, int nsub, double (&out)[NTR]) {
    double inc[NEU][NTR];
#pragma unroll
    for (int t = 0; t < NTR; ++t)
#pragma unroll
        for (int e = 0; e < NEU; ++e) inc[e][t] = 0.0;
    double sphi = 0.0;
    for (int s = 0; s < nsub; ++s) sphi += euphotic_step<NTR, NEU>(p, E, ye, h, inc);
    const DeepFactors D = deep_factors<NTR>(p, h, nsub);
    if constexpr (NTR == 3) {
        const double dop = yk[kDop], phy = yk[kPhy];
        out[0] = h * (p.lam * (dop * D.G + phy * D.GC) + (1.0 - p.sig) * rho_k * sphi);
        out[kDop] = dop * D.pm1 + phy * D.cn;
        out[kPhy] = phy * D.qm1;
    } else {
        const double dop = NTR > 1 ? yk[NTR - 1] : 0.0;
        out[0] = h * (p.lam * dop * D.G + (1.0 - p.sig) * rho_k * sphi);
        if (NTR > 1) out[NTR - 1] = dop * D.pm1;
    }
#pragma unroll
    for (int e = 0; e < NEU; ++e)
        if (e == k && e < E.ne) {
#pragma unroll
            for (int t = 0; t < NTR; ++t) out[t] = inc[e][t];
        }
}

template <int NTR, int NEU>
__device__ __forceinline__ void row_source_tangent(const BgcParams& p, const Euphotic<NEU>& E, int k,
                                                   const double (&ye)[NEU][NTR], const double (&ve)[NEU][NTR],
                                                   const double (&yk)[NTR], const double (&vk)[NTR], double rho_k,
                                                   double h, int nsub, double (&out)[NTR], double (&outd)[NTR]) {
    double inc[NEU][NTR], incd[NEU][NTR];
#pragma unroll
    for (int t = 0; t < NTR; ++t)
#pragma unroll
        for (int e = 0; e < NEU; ++e) {
            inc[e][t] = 0.0;
            incd[e][t] = 0.0;
        }
    double sphi = 0.0, sphid = 0.0;
    for (int s = 0; s < nsub; ++s) {
        double Phi, Phid;
        euphotic_step_tangent<NTR, NEU>(p, E, ye, ve, h, inc, incd, Phi, Phid);
        sphi += Phi;
        sphid += Phid;
    }
    const DeepFactors D = deep_factors<NTR>(p, h, nsub);
    if constexpr (NTR == 3) {
        const double dop = yk[kDop], phy = yk[kPhy], dopd = vk[kDop], phyd = vk[kPhy];
        out[0] = h * (p.lam * (dop * D.G + phy * D.GC) + (1.0 - p.sig) * rho_k * sphi);
        outd[0] = h * (p.lam * (dopd * D.G + phyd * D.GC) + (1.0 - p.sig) * rho_k * sphid);
        out[kDop] = dop * D.pm1 + phy * D.cn;
        outd[kDop] = dopd * D.pm1 + phyd * D.cn;
        out[kPhy] = phy * D.qm1;
        outd[kPhy] = phyd * D.qm1;
    } else {
        const double dop = NTR > 1 ? yk[NTR - 1] : 0.0;
        const double dopd = NTR > 1 ? vk[NTR - 1] : 0.0;
        out[0] = h * (p.lam * dop * D.G + (1.0 - p.sig) * rho_k * sphi);
        outd[0] = h * (p.lam * dopd * D.G + (1.0 - p.sig) * rho_k * sphid);
        if (NTR > 1) {
            out[NTR - 1] = dop * D.pm1;
            outd[NTR - 1] = dopd * D.pm1;
        }
    }
#pragma unroll
    for (int e = 0; e < NEU; ++e)
        if (e == k && e < E.ne) {
#pragma unroll
            for (int t = 0; t < NTR; ++t) {
                out[t] = inc[e][t];
                outd[t] = incd[e][t];
            }
        }
}

// Sums over the internal steps of the row's own parameter terms while the
// row is euphotic (finished by euphotic_adj_finish).
// In PO4-DOP-PHY the production terms carry the factor PHY, sigma_2 sees
// sigma_3 f, and three more sums collect the PHY parameters.
struct EuphoticAdj {
    double A = 0.0;      // sum fbar limN [PHY]            (alpha, K_H2O, K_I)
    double B = 0.0;      // sum fbar N+ / (N+ + K_1)^2 [PHY] (K_1)
    double lam = 0.0;    // sum DOP (ib_1 - ib_2)          (lambda'_2)
    double sig = 0.0;    // sum [sigma_3] f ib_2 - Phi rho_k ib_1 (sigma_2)
    double phib = 0.0;   // sum Phi ib_1                   (b)
    double l3 = 0.0;     // sum PHY (ib_2 - ib_3)          (lambda_3, lambda'_3; PO4-DOP-PHY)
    double k3 = 0.0;     // sum PHY^2 (ib_2 - ib_3)        (kappa_3; PO4-DOP-PHY)
    double s3 = 0.0;     // sum f (sigma_2 ib_2 - ib_3 + h Phibar) (sigma_3; PO4-DOP-PHY)
};

// Parameter sums kept per euphotic row between the phases of the persistent
// adjoint.
template <int NTR>
__host__ __device__ constexpr int acc_fields() { return NTR == 3 ? 8 : 5; }

template <int NTR>
__device__ __forceinline__ void acc_store(const EuphoticAdj& a, double* dst) {
    dst[0] = a.A;
    dst[1] = a.B;
    dst[2] = a.lam;
    dst[3] = a.sig;
    dst[4] = a.phib;
    if constexpr (NTR == 3) {
        dst[5] = a.l3;
        dst[6] = a.k3;
        dst[7] = a.s3;
    }
}

template <int NTR>
__device__ __forceinline__ EuphoticAdj acc_load(const double* src) {
    EuphoticAdj a;
    a.A = src[0];
    a.B = src[1];
    a.lam = src[2];
    a.sig = src[3];
    a.phib = src[4];
    if constexpr (NTR == 3) {
        a.l3 = src[5];
        a.k3 = src[6];
        a.s3 = src[7];
    }
    return a;
}

// Reverse of one internal step for the euphotic rows of PO4-DOP-PHY at state
// ys (section 2.2.2 differentiated): per row e the h-free cotangent update
// g[e] = (dq/dy)^T ib restricted to the row, and the row's parameter terms
// added to acc[e] when take[e].  Returns Phi of the state.
template <int NEU>
__device__ __forceinline__ double euphotic_reverse_phy(const BgcParams& p, const Euphotic<NEU>& E, double pdeep,
                                                       const double (&ys)[NEU][3], const double (&ib)[NEU][3],
                                                       double (&g)[NEU][3], EuphoticAdj* acc, const bool (&take)[NEU]) {
    double f0[NEU], f[NEU], dfdN[NEU], limN[NEU], w2[NEU];
    double Phi = 0.0, Phibar = pdeep;
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const bool in = e < E.ne;
        const double N = ys[e][0];
        const double Np = N > 0.0 ? N : 0.0;
        const double inv = 1.0 / (Np + p.k1);
        limN[e] = in ? Np * inv : 0.0;
        w2[e] = Np * inv * inv;
        f0[e] = p.alpha * limN[e] * E.limI[e];
        f[e] = f0[e] * ys[e][kPhy];
        dfdN[e] = (in && N > 0.0) ? p.alpha * p.k1 * inv * inv * E.limI[e] : 0.0;
        Phi += E.hz[e] * (p.sig3 * f[e]);
        Phibar += (1.0 - p.sig) * E.rho[e] * ib[e][0];
    }
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const double ib1 = ib[e][0], ib2 = ib[e][kDop], ib3 = ib[e][kPhy];
        const double P = ys[e][kPhy];
        // f_1 enters q_1 (-1), q_2 (sigma_2 sigma_3), q_3 (1 - sigma_3) and Phi (h sigma_3)
        const double fbar = -ib1 + p.sig * p.sig3 * ib2 + (1.0 - p.sig3) * ib3 + p.sig3 * E.hz[e] * Phibar;
        const double dloss = p.lam3 + 2.0 * p.kap3 * P;
        g[e][0] = fbar * dfdN[e] * P;
        g[e][kDop] = p.lam * (ib1 - ib2);
        g[e][kPhy] = fbar * f0[e] + dloss * (ib2 - ib3) + p.lam3p * (ib2 - ib3);
        if (take[e]) {
            acc[e].A += fbar * limN[e] * P;
            acc[e].B += fbar * w2[e] * P;
            acc[e].lam += ys[e][kDop] * (ib1 - ib2);
            acc[e].sig += p.sig3 * f[e] * ib2 - Phi * E.rho[e] * ib1;
            acc[e].phib += Phi * ib1;
            acc[e].l3 += P * (ib2 - ib3);
            acc[e].k3 += P * P * (ib2 - ib3);
            acc[e].s3 += f[e] * (p.sig * ib2 - ib3 + E.hz[e] * Phibar);
        }
    }
    return Phi;
}

// Reverse of internal step s of the euphotic rows, seen from the row in
// layer k.
//   ys:    state of the euphotic rows at internal step s (y + inc_s)
//   pdeep: sum over the column's rows below the euphotic zone of
//          (1 - sigma) rho mu_1 (their nutrient cotangents never change)
//   ib:    cotangents of the euphotic rows
// If the row is euphotic, adds h (dq/dy)^T ib of the row to ybar and its
// parameter terms to acc.  Then advances ib by h J_q^T ib.  Returns the
// export Phi of internal step s.
template <int NTR, int NEU>
__device__ __forceinline__ double euphotic_reverse(const BgcParams& p, const Euphotic<NEU>& E, int k, double rho_k,
                                                   double pdeep, const double (&ys)[NEU][NTR], double h,
                                                   double (&ib)[NEU][NTR], double (&ybar)[NTR], EuphoticAdj& acc) {
    if constexpr (NTR == 3) {
        double g[NEU][3];
        EuphoticAdj a[NEU];
        bool take[NEU];
#pragma unroll
        for (int e = 0; e < NEU; ++e) take[e] = e == k && e < E.ne;
        const double Phi = euphotic_reverse_phy<NEU>(p, E, pdeep, ys, ib, g, a, take);
#pragma unroll
        for (int e = 0; e < NEU; ++e) {
            if (take[e]) {
#pragma unroll
                for (int t = 0; t < 3; ++t) ybar[t] += h * g[e][t];
                acc.A += a[e].A;
                acc.B += a[e].B;
                acc.lam += a[e].lam;
                acc.sig += a[e].sig;
                acc.phib += a[e].phib;
                acc.l3 += a[e].l3;
                acc.k3 += a[e].k3;
                acc.s3 += a[e].s3;
            }
            const bool in = e < E.ne;
#pragma unroll
            for (int t = 0; t < 3; ++t) ib[e][t] += in ? h * g[e][t] : 0.0;
        }
        return Phi;
    }
    double f[NEU], dfdN[NEU], limN[NEU], w2[NEU];
    double Phi = 0.0, Phibar = pdeep;
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const bool in = e < E.ne;
        const double N = ys[e][0];
        const double Np = N > 0.0 ? N : 0.0;
        const double inv = 1.0 / (Np + p.k1);
        limN[e] = in ? Np * inv : 0.0;
        w2[e] = Np * inv * inv;                       // N+ / (N+ + K_1)^2
        f[e] = p.alpha * limN[e] * E.limI[e];
        dfdN[e] = (in && N > 0.0) ? p.alpha * p.k1 * inv * inv * E.limI[e] : 0.0;
        Phi += E.hz[e] * f[e];
        Phibar += (1.0 - p.sig) * E.rho[e] * ib[e][0];
    }
    // the row's own terms, at the cotangents before this step's update
#pragma unroll
    for (int e = 0; e < NEU; ++e)
        if (e == k && e < E.ne) {
            const double ib1 = ib[e][0];
            const double ib2 = NTR > 1 ? ib[e][NTR - 1] : 0.0;
            const double fbar = -ib1 + p.sig * ib2 + E.hz[e] * Phibar;
            ybar[0] += h * (fbar * dfdN[e]);
            acc.A += fbar * limN[e];
            acc.B += fbar * w2[e];
            if (NTR > 1) {
                ybar[NTR - 1] += h * (p.lam * (ib1 - ib2));
                acc.lam += ys[e][NTR - 1] * (ib1 - ib2);
                acc.sig += f[e] * ib2 - Phi * rho_k * ib1;
            }
            acc.phib += Phi * ib1;
        }
    // advance the cotangents of the euphotic rows
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const bool in = e < E.ne;
        const double i2 = NTR > 1 ? ib[e][NTR - 1] : 0.0;
        const double fb = -ib[e][0] + p.sig * i2 + E.hz[e] * Phibar;
        const double y1 = fb * dfdN[e];
        const double y2 = p.lam * (ib[e][0] - i2);
        ib[e][0] += in ? h * y1 : 0.0;
        if (NTR > 1) ib[e][NTR - 1] += in ? h * y2 : 0.0;
    }
    return Phi;
}

// The same reverse step for all euphotic rows of a column at once (one
// thread per column): each row e gets its own terms in ybar[e] and acc[e].
template <int NTR, int NEU>
__device__ __forceinline__ double euphotic_reverse_rows(const BgcParams& p, const Euphotic<NEU>& E, double pdeep,
                                                        const double (&ys)[NEU][NTR], double h,
                                                        double (&ib)[NEU][NTR], double (&ybar)[NEU][NTR],
                                                        EuphoticAdj (&acc)[NEU]) {
    if constexpr (NTR == 3) {
        double g[NEU][3];
        bool take[NEU];
#pragma unroll
        for (int e = 0; e < NEU; ++e) take[e] = true;
        const double Phi = euphotic_reverse_phy<NEU>(p, E, pdeep, ys, ib, g, acc, take);
#pragma unroll
        for (int e = 0; e < NEU; ++e) {
            const bool in = e < E.ne;
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                ybar[e][t] += h * g[e][t];
                ib[e][t] += in ? h * g[e][t] : 0.0;
            }
        }
        return Phi;
    }
    double f[NEU], dfdN[NEU], limN[NEU], w2[NEU];
    double Phi = 0.0, Phibar = pdeep;
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const bool in = e < E.ne;
        const double N = ys[e][0];
        const double Np = N > 0.0 ? N : 0.0;
        const double inv = 1.0 / (Np + p.k1);
        limN[e] = in ? Np * inv : 0.0;
        w2[e] = Np * inv * inv;
        f[e] = p.alpha * limN[e] * E.limI[e];
        dfdN[e] = (in && N > 0.0) ? p.alpha * p.k1 * inv * inv * E.limI[e] : 0.0;
        Phi += E.hz[e] * f[e];
        Phibar += (1.0 - p.sig) * E.rho[e] * ib[e][0];
    }
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const bool in = e < E.ne;
        const double ib1 = ib[e][0];
        const double ib2 = NTR > 1 ? ib[e][NTR - 1] : 0.0;
        const double fbar = -ib1 + p.sig * ib2 + E.hz[e] * Phibar;
        const double y1 = fbar * dfdN[e];
        const double y2 = p.lam * (ib1 - ib2);
        ybar[e][0] += h * y1;
        acc[e].A += fbar * limN[e];
        acc[e].B += fbar * w2[e];
        if (NTR > 1) {
            ybar[e][NTR - 1] += h * y2;
            acc[e].lam += ys[e][NTR - 1] * (ib1 - ib2);
            acc[e].sig += f[e] * ib2 - Phi * E.rho[e] * ib1;
        }
        acc[e].phib += Phi * ib1;
        ib[e][0] += in ? h * y1 : 0.0;
        if (NTR > 1) ib[e][NTR - 1] += in ? h * y2 : 0.0;
    }
    return Phi;
}

// Adds the euphotic row's summed parameter terms (unscaled) to ub, in the
// order alpha, K_H2O, K_1, K_I, [lambda'_2, sigma_2,] b; zc is the row's
// centre depth.  The light factors are constant over the ocean step.
template <int NTR, int NEU, int NP>
__device__ __forceinline__ void euphotic_adj_finish(const BgcParams& p, const Euphotic<NEU>& E, int k, double zc,
                                                    double drho_k, const EuphoticAdj& acc, double (&ub)[NP]) {
    double Ik = 0.0, limIk = 0.0;
#pragma unroll
    for (int e = 0; e < NEU; ++e)
        if (e == k) {
            Ik = E.I[e];
            limIk = E.limI[e];
        }
    const double IKI2 = (Ik + p.ki) * (Ik + p.ki);
    ub[0] += acc.A * limIk;
    ub[1] += acc.A * (p.alpha * p.ki / IKI2 * (-zc * Ik));
    ub[2] += acc.B * (-p.alpha * limIk);
    ub[3] += acc.A * (-p.alpha * Ik / IKI2);
    if (NTR > 1) {
        ub[4] += acc.lam;
        ub[5] += acc.sig;
    }
    if constexpr (NTR == 3) {
        ub[6] += acc.l3;
        ub[7] += acc.k3;
        ub[8] += acc.l3;
        ub[9] += acc.s3;
    }
    ub[NP - 1] += (1.0 - p.sig) * drho_k * acc.phib;
}

// Reverse mode of a row below the euphotic zone over all internal steps:
// y0: its state at the ocean step, mu: the cotangent of its source, sphi:
// sum_s Phi_s of its column.  Adds h (dq/dy)^T contributions to ybar and
// unscaled (dq/du)^T sums to ub.
template <int NTR, int NP>
__device__ __forceinline__ void deep_reverse(const BgcParams& p, const DeepFactors& D, int nsub, double h,
                                             double rho_k, double drho_k, double sphi, const double (&y0)[NTR],
                                             const double (&mu)[NTR], double (&ybar)[NTR], double (&ub)[NP]) {
    if constexpr (NTR == 3) {
        // the PHY column of the row's linear map (DeepFactors)
        const double dmu = mu[0] - mu[kDop], dmu3 = mu[kDop] - mu[kPhy];
        const double nb = nsub * D.blast;
        ybar[kDop] += h * (p.lam * dmu * D.G);
        ybar[kPhy] += h * (p.lam * D.GC * dmu + p.lam3p * D.GB * dmu3);
        ub[4] += dmu * (y0[kDop] * (nsub * D.alast) + y0[kPhy] * D.r);
        ub[5] += -sphi * rho_k * mu[0];
        ub[8] += y0[kPhy] * (dmu * (nb - D.E) + dmu3 * nb);
    } else if (NTR > 1) {
        const double dmu = mu[0] - mu[NTR - 1];
        ybar[NTR - 1] += h * (p.lam * dmu * D.G);
        ub[4] += y0[NTR - 1] * dmu * (nsub * D.alast);
        ub[5] += -sphi * rho_k * mu[0];
    }
    ub[NP - 1] += (1.0 - p.sig) * sphi * drho_k * mu[0];
}

}  // namespace tmm
