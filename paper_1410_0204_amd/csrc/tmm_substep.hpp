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
//     q_1 = lambda DOP_k + (1 - sigma) Phi rho_k,   q_2 = -lambda DOP_k,
// linear in its own state, so its increment follows from sum_s Phi_s and
// per-member decay factors (DeepFactors below).
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
        Phi += E.hz[e] * f[e];
    }
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const double dop = NTR > 1 ? y[e][NTR - 1] + inc[e][NTR - 1] : 0.0;
        const double q1 = -f[e] + p.lam * dop + (1.0 - p.sig) * Phi * E.rho[e];
        inc[e][0] += e < E.ne ? h * q1 : 0.0;
        if (NTR > 1) inc[e][NTR - 1] += e < E.ne ? h * (p.sig * f[e] - p.lam * dop) : 0.0;
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
        fd[e] = dfdN * (v[e][0] + incd[e][0]);
        Phi += E.hz[e] * f[e];
        Phid += E.hz[e] * fd[e];
    }
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const bool in = e < E.ne;
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

// Rows below the euphotic zone: their DOP decays linearly and their nutrient
// only receives the export, so with a_s = (1 - h lambda)^s (advanced by the
// same Euler recursion, a_0 = 1) their increments are
//     inc_1 = h (lambda DOP_0 G + (1 - sigma) rho_k sum_s Phi_s),
//     inc_2 = DOP_0 (a_nsub - 1),          G = sum_{s<nsub} a_s,
// and their reverse mode needs only G, a_nsub - 1 and a_{nsub-1} as well.
struct DeepFactors {
    double G;       // sum_{s<nsub} a_s
    double pm1;     // a_nsub - 1
    double alast;   // a_{nsub-1}
};

__device__ __forceinline__ DeepFactors deep_factors(const BgcParams& p, double h, int nsub) {
    DeepFactors d{0.0, 0.0, 1.0};
    for (int s = 0; s < nsub; ++s) {
        const double a = 1.0 + d.pm1;
        d.G += a;
        d.alast = a;
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
    const DeepFactors D = deep_factors(p, h, nsub);
    const double dop = NTR > 1 ? yk[NTR - 1] : 0.0;
    out[0] = h * (p.lam * dop * D.G + (1.0 - p.sig) * rho_k * sphi);
    if (NTR > 1) out[NTR - 1] = dop * D.pm1;
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
    const DeepFactors D = deep_factors(p, h, nsub);
    const double dop = NTR > 1 ? yk[NTR - 1] : 0.0;
    const double dopd = NTR > 1 ? vk[NTR - 1] : 0.0;
    out[0] = h * (p.lam * dop * D.G + (1.0 - p.sig) * rho_k * sphi);
    outd[0] = h * (p.lam * dopd * D.G + (1.0 - p.sig) * rho_k * sphid);
    if (NTR > 1) {
        out[NTR - 1] = dop * D.pm1;
        outd[NTR - 1] = dopd * D.pm1;
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
struct EuphoticAdj {
    double A;      // sum fbar limN            (alpha, K_H2O, K_I)
    double B;      // sum fbar N+ / (N+ + K_1)^2 (K_1)
    double lam;    // sum DOP (ib_1 - ib_2)      (lambda'_2)
    double sig;    // sum f ib_2 - Phi rho_k ib_1 (sigma_2)
    double phib;   // sum Phi ib_1               (b)
};

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
    if (NTR > 1) {
        const double dmu = mu[0] - mu[NTR - 1];
        ybar[NTR - 1] += h * (p.lam * dmu * D.G);
        ub[4] += y0[NTR - 1] * dmu * (nsub * D.alast);
        ub[5] += -sphi * rho_k * mu[0];
    }
    ub[NP - 1] += (1.0 - p.sig) * sphi * drho_k * mu[0];
}

}  // namespace tmm
