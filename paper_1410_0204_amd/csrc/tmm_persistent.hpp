// Persistent model-year kernel: all nstep time steps of one model year in a
// single cooperative launch.
//
// The time step is the one of section 3 of the paper,
//     y_{j+1} = Ai(t_j) (Ae(t_j) y_j + dt_d q(y_j, u)),
// iterated over a model year (section 4).  On the global 2.8-degree grid one
// step moves ~20 MB of matrix values but takes only a few microseconds of
// arithmetic, so a kernel per step is bound by launch and memory latency.
// Here instead:
//
//  * Every workgroup owns a fixed "domain" of whole water columns (at most
//    one row per thread) for the whole year.
//  * The two monthly matrices in use -- the thread's row of Ae and its row of
//    the column block of Ai, for months k0 and k1 -- live in VGPRs and are
//    reloaded only when the month pair changes (12 times a year).  Across the
//    chip the register file holds the interpolation bracket of the whole
//    matrix set, so no step streams matrix values from memory.
//  * The implicit operator acts within a water column (section 3), so the
//    vertical product and the biogeochemistry (section 5: one column at a
//    time) only touch the domain's own rows, kept in LDS.
//  * Only the explicit (horizontal) product reads rows of other domains.
//    Each state y_t of the launch is published to its own slot of a ring of
//    2K slots (K = kRingK) that holds only the sentinel (all bits set, a NaN
//    that a published value never has: NaNs are stored in canonical form)
//    until the owner writes the value (slot 0 holds the launch's initial
//    state and slots 1 .. K-1 the sentinel, written before the launch).  A
//    thread reads a neighbour's value
//    with relaxed agent-scope loads until it is not the sentinel: an aligned
//    8-byte access is single-copy atomic, so the value read is the published
//    one, with no flag and no fence between producer and consumer.
//  * Each domain reads the rows of other domains that its stencil touches
//    (its halo, sorted and without repeats) once per step, consecutive threads
//    taking consecutive halo rows, into LDS beside its own rows; the explicit
//    product then reads only LDS.  Device-scope loads bypass the L1 and L2
//    caches, so fetching each halo row once instead of once per reference
//    cuts the requests that reach the device's point of coherence by about
//    an order of magnitude.  A thread issues the loads of all its halo rows
//    before it checks any of them, so a step waits for one round trip.
//  * Slot reuse is ordered by a hand-over every K steps: before step pK each
//    domain publishes the phase counter p with an agent-scope release store and
//    waits (relaxed polls, then one acquire fence) for the counters of every
//    domain its Ae rows touch and every domain that touches it.  In step jj a
//    domain resets its own rows of the slot of state jj + K: for jj in phase
//    p that is a state of phase p+1, whose slot's previous state jj - K (phase
//    p-1) every neighbour read before hand-over p, and hand-over p+1 orders
//    the reset before any read of it.  One slot per step spreads the resets
//    (resetting a whole phase of slots at the hand-over made every domain
//    write tens of MB at once).
//  * Waits are bounded: after spin_limit polls a workgroup sets a global
//    abort flag and returns; every other workgroup sees the flag and returns
//    too, so the grid always drains.  Cooperative launch guarantees that all
//    workgroups are resident.
//  * The reverse sweep (k_adjoint_persistent) exchanges the cotangent the
//    same way, with the halo of the transposed stencil.
#pragma once

#include "tmm_device.hpp"

namespace tmm {

constexpr int kPersistThreadsMax = 512;   // rows per domain (one per thread), at most
constexpr int kNeuMax = 4;             // euphotic layers supported by this kernel
constexpr int kEllMax = 8;             // Ae nonzeros per row supported by this kernel
constexpr int kHaloPerThread = 2;      // halo rows per thread (a domain's halo is at most 2 TPB rows)
constexpr int kRingK = 64;             // steps between hand-overs; the ring has 2 kRingK slots
constexpr int kRing = 2 * kRingK;
// a step resets the slot of state jj + K after publishing state jj + 1
static_assert(kRingK >= 2, "the per-step reset needs a phase of at least two steps");

// The ring's empty-slot marker and the canonical NaN that replaces any NaN
// before it is published.
constexpr long long kSentinelBits = -1LL;
__device__ __forceinline__ bool is_sentinel(double x) { return __double_as_longlong(x) == kSentinelBits; }
__device__ __forceinline__ double publishable(double x) {
    return x == x ? x : __longlong_as_double(0x7FF8000000000000LL);
}

struct Persist {
    const int* block_dom;   // [G] domain of each workgroup
    const int* dom_col;     // [G+1] first water column of each domain
    const int* dep_ptr;     // [G+1]
    const int* dep_idx;     // domains each domain waits for
    int* flags;             // [G] hand-overs each domain has published
    int* abort_flag;        // non-zero once any wait gave up
    long long spin_limit;
    double* ring;           // [kRing][NTR][n] published states of the forward kernel, sentinel-filled
    double* vring;          // [kRing][NTR][n] the same for the tangent (nullable)
    const int* halo_ptr;    // [G+1]
    const int* halo_row;    // rows of other domains each domain reads, ascending per domain
    int halo_max;           // largest halo (rows); sizes the dynamic LDS of the forward kernel
    const int* ahalo_ptr;   // the same for the transposed stencil of the reverse sweep
    const int* ahalo_row;
    int ahalo_max;
    const int* qlat;        // [G][1 + kInsLat]: number of distinct latitude rows of the domain's
                            // columns, then those rows (indices into the insolation table)
    int qlat_max;           // largest such number over the domains
    const int* col_slot;    // [ncol] thread of the forward kernels that holds the first row of
                            // each water column, within its domain's workgroup
    int wave_local;         // 1: no water column spans two wavefronts (see k_year_persistent)
};

// Distinct latitude rows a domain may span for its insolation table in LDS.
constexpr int kInsLat = 8;

// Dynamic LDS of the forward kernel: own rows then halo rows, for y (and v),
// twice (states of even and odd steps), then the insolation of the domain's
// latitude rows for every step of the year.
__host__ __device__ inline size_t year_kernel_dyn_lds(int tpb, int halo_max, int ntr, bool tangent, int qlat_max,
                                                      int nstep) {
    return (size_t)(tpb + halo_max) * ntr * 8 * 2 * (tangent ? 2 : 1) + (size_t)qlat_max * nstep * 8;
}

// LDS written by lanes of a wavefront and then read by other lanes of the
// same wavefront: the LDS executes a wavefront's operations in order, so
// this only keeps the compiler from moving them across.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Steps j0 .. j1-1 of the year for one launch, with optional state storage
// (y_j of own rows at slot (j - j0)/store_every when (j - j0) % store_every == 0)
// and month-end misfit partial sums against obs.
struct StepRange {
    int j0, j1;
    double* store;          // nullable, [slots][n*NTR]
    int store_every;
    const double* obs;      // nullable, [nmat][n*NTR]
    double* jpart;          // [nmat][G] per-domain sums of V_i (y - obs)^2
};

// A slot holds one state tracer by tracer ([NTR][n]): the threads of a
// wavefront own consecutive rows, so each of its stores (one tracer of 64
// rows) covers whole cache lines.
__device__ __forceinline__ size_t ring_at(size_t slot_base, int n, int row, int t) {
    return slot_base + (size_t)t * n + row;
}

// Ring set-up before a launch: slot 0 = the initial state (NaNs in canonical
// form, so that no value equals the sentinel), slots 1 .. K-1 the sentinel.
// Slots K .. 2K-1 are reset by the kernel itself (step t - K resets the slot
// of state t) before any read, so whatever they hold from earlier launches
// is never read.  y is row-major n x ntr.
__global__ void k_ring_init(double* __restrict__ ring, const double* __restrict__ y, int n, int ntr, size_t total) {
    const double sent = __longlong_as_double(kSentinelBits);
    const size_t slen = (size_t)n * ntr;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        if (i < slen) {
            const int t = (int)(i / n), row = (int)(i % n);
            ring[i] = publishable(y[(size_t)row * ntr + t]);
        } else {
            ring[i] = sent;
        }
    }
}

template <int KMAX>
struct RowMats {
    int col[kEllMax];       // LDS row of each Ae entry: own rows first, then the halo
    double e0[kEllMax], e1[kEllMax];   // Ae row, months k0 and k1
    double a0[KMAX], a1[KMAX];         // row of the Ai block, months k0 and k1
};

template <int KMAX>
__device__ __forceinline__ void load_month(const Mats& mt, const Grid& g, int m, int r, size_t blk, int nc, int k,
                                           double* e, double* a) {
#pragma unroll
    for (int s = 0; s < kEllMax; ++s)
        e[s] = s < mt.ew ? mt.ae[(size_t)m * mt.ae_month + (size_t)s * g.npad + r] : 0.0;
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
        a[s] = s < nc ? mt.ai_rm[(size_t)m * mt.ai_month + blk + (size_t)k * nc + s] : 0.0;
}

// Source of the thread's row over one ocean step with md.nsub internal BGC
// steps (section 7), from the domain's state in LDS: q = inc_nsub (and its
// tangent qd).  light, hz, rho_e: the column's euphotic constants (at least
// NEU entries, zero beyond ne).
template <int NTR, bool TANGENT, int NEU, int TV>
__device__ __forceinline__ void sub_source_lds(const Model& md, const BgcParams& p, double Q, int ne, int k, int lr0,
                                               const double* light, const double* hz, const double* rho_e,
                                               double rho_k, const double* s_y, const double* s_v,
                                               const double (&yr)[NTR], const double (&vr)[TV], double (&q)[NTR],
                                               double (&qd)[TV]) {
    const Euphotic<NEU> E = make_euphotic<NEU>(p, Q, ne, light, hz, rho_e);
    double ye[NEU][NTR], ve[NEU][NTR], vk[NTR];
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const int le = lr0 + (e < ne ? e : 0);
#pragma unroll
        for (int t = 0; t < NTR; ++t) {
            ye[e][t] = e < ne ? s_y[le * NTR + t] : 0.0;
            ve[e][t] = (TANGENT && e < ne) ? s_v[le * TV + t % TV] : 0.0;
        }
    }
    if (TANGENT) {
        double o[NTR];
#pragma unroll
        for (int t = 0; t < NTR; ++t) vk[t] = vr[t % TV];
        row_source_tangent<NTR, NEU>(p, E, k, ye, ve, yr, vk, rho_k, md.hsub, md.nsub, q, o);
#pragma unroll
        for (int t = 0; t < NTR; ++t) qd[t % TV] = o[t];
    } else {
        row_source<NTR, NEU>(p, E, k, ye, yr, rho_k, md.hsub, md.nsub, q);
    }
}

// Euphotic-layer constants of one water column (light factors, layer heights,
// Martin fractions; entries beyond the euphotic depth repeat layer 0) and its
// latitude row: loaded once per launch.
template <int NEU>
struct ColConsts {
    double light[NEU], hz[NEU], rho[NEU];
    int lat;
};

template <int NEU>
__device__ __forceinline__ ColConsts<NEU> load_col_consts(const Grid& g, const Model& md, int m, int c, int nc) {
    ColConsts<NEU> r;
    const int ne = nc < g.neu ? nc : g.neu;
    const size_t tab = ((size_t)m * (g.nlayer + 1) + nc) * g.nlayer;
#pragma unroll
    for (int e = 0; e < NEU; ++e) {
        const int ee = e < ne ? e : 0;
        r.light[e] = md.light[(size_t)m * g.nlayer + ee];
        r.hz[e] = g.dz[ee];
        r.rho[e] = md.rho[tab + ee];
    }
    r.lat = g.col_lat[c];
    return r;
}

// Reverse of the internal BGC steps (section 7 with the adjoint of section
// 6) for the domain's rows.  Phase 1, one thread per water column: the
// column's euphotic rows are run forward over the internal steps (their
// states kept in s_traj, [nsub][TPB][NTR] by row, dynamic LDS) and then
// reversed; each euphotic row's h-weighted (dq/dy)^T mu goes to s_yb, its
// parameter sums to s_acc, the column's summed export to s_sphi.  Phase 2,
// one thread per row: a euphotic row takes its results, a row below the
// euphotic zone uses the summed export and the decay factors.  Only about
// one wavefront works in phase 1, instead of every row thread repeating its
// column's internal steps.  Returns ybar of the thread's row and adds its
// unscaled (dq/du)^T mu to ub.  Every thread of the workgroup must call this.
template <int NTR, int NEU, int NP, int TPB>
__device__ __forceinline__ void sub_adjoint_lds(const Grid& g, const Model& md, const BgcParams& p, int m, int j,
                                                int c0, int ncols, const short* s_colr0, const short* s_colnc,
                                                int tid, int k, int ne, int lc, size_t tab, double zc, double rho_k,
                                                double drho_k, const double* s_y, const double* s_mu,
                                                const double* s_rhoc, double* s_traj, double* s_yb,
                                                double* s_acc, double* s_sphi, const ColConsts<NEU>& cc,
                                                const ColConsts<NEU>& oc, double Q_own,
                                                const double (&yj)[NTR], const double (&mr)[NTR],
                                                double (&ybar)[NTR], double (&ub)[NP]) {
    const double h = md.hsub;
    const int nsub = md.nsub;
    if (tid < ncols) {
        const int r0q = s_colr0[tid];
        const int ncq = s_colnc[tid];
        const int neq = ncq < g.neu ? ncq : g.neu;
        const double Q = g.ins[(size_t)j * g.nlat + cc.lat];
        const Euphotic<NEU> E = make_euphotic<NEU>(p, Q, neq, cc.light, cc.hz, cc.rho);
        double ye[NEU][NTR], ib[NEU][NTR], yb[NEU][NTR];
        EuphoticAdj acc[NEU];
#pragma unroll
        for (int e = 0; e < NEU; ++e) {
            const int le = r0q + (e < neq ? e : 0);
#pragma unroll
            for (int t = 0; t < NTR; ++t) {
                ye[e][t] = e < neq ? s_y[le * NTR + t] : 0.0;
                ib[e][t] = e < neq ? s_mu[le * NTR + t] : 0.0;
                yb[e][t] = 0.0;
            }
            acc[e] = EuphoticAdj{};
        }
        {
            double inc[NEU][NTR];
#pragma unroll
            for (int e = 0; e < NEU; ++e)
#pragma unroll
                for (int t = 0; t < NTR; ++t) inc[e][t] = 0.0;
            for (int s = 0; s < nsub; ++s) {
#pragma unroll
                for (int e = 0; e < NEU; ++e)
                    if (e < neq) {
#pragma unroll
                        for (int t = 0; t < NTR; ++t)
                            s_traj[((size_t)s * TPB + r0q + e) * NTR + t] = ye[e][t] + inc[e][t];
                    }
                euphotic_step<NTR, NEU>(p, E, ye, h, inc);
            }
        }
        double pdeep = 0.0;
        for (int kk = neq; kk < ncq; ++kk) pdeep += s_rhoc[r0q + kk] * s_mu[(r0q + kk) * NTR];
        double sphi = 0.0;
        for (int s = nsub - 1; s >= 0; --s) {
            double ys[NEU][NTR];
#pragma unroll
            for (int e = 0; e < NEU; ++e) {
                const int le = r0q + (e < neq ? e : 0);
#pragma unroll
                for (int t = 0; t < NTR; ++t) ys[e][t] = e < neq ? s_traj[((size_t)s * TPB + le) * NTR + t] : 0.0;
            }
            sphi += euphotic_reverse_rows<NTR, NEU>(p, E, pdeep, ys, h, ib, yb, acc);
        }
#pragma unroll
        for (int e = 0; e < NEU; ++e)
            if (e < neq) {
                const int le = r0q + e;
#pragma unroll
                for (int t = 0; t < NTR; ++t) s_yb[le * NTR + t] = yb[e][t];
                acc_store<NTR>(acc[e], s_acc + le * acc_fields<NTR>());
            }
        s_sphi[tid] = sphi;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NTR; ++t) ybar[t] = 0.0;
    if (k < ne) {
#pragma unroll
        for (int t = 0; t < NTR; ++t) ybar[t] = s_yb[tid * NTR + t];
        const EuphoticAdj acc = acc_load<NTR>(s_acc + tid * acc_fields<NTR>());
        const Euphotic<NEU> E = make_euphotic<NEU>(p, Q_own, ne, oc.light, oc.hz, oc.rho);
        euphotic_adj_finish<NTR, NEU, NP>(p, E, k, zc, drho_k, acc, ub);
    } else {
        deep_reverse<NTR, NP>(p, deep_factors<NTR>(p, h, nsub), nsub, h, rho_k, drho_k, s_sphi[lc], yj, mr, ybar, ub);
    }
}

// NTR tracers of one member; TANGENT also steps v = phi'(y) direction; TPB
// threads per workgroup = maximum rows per domain; SN = 0 for one BGC
// evaluation per step, else internal BGC steps with SN >= neu euphotic rows
// held in registers; QL: the insolation of the domain's latitude rows for the
// whole year in LDS (else loaded from the global table every step).
//
// Thread t of a workgroup holds the row at slot t of its domain: the host
// places each water column at a start slot (ps.col_slot).  With
// ps.wave_local, no column spans two wavefronts (a column that would is moved
// to the next wavefront's first slot), so the column product and the sources,
// which read only rows of the thread's own column, need no workgroup barrier:
// per step one barrier (after the halo has arrived) remains, and the LDS
// state alternates between two buffers (state j in buffer j % 2) so that a
// wavefront that has finished step j may write state j + 1 while another
// still reads state j.  Without it the columns are packed and two more
// workgroup barriers per step order the same accesses.
template <int NTR, bool TANGENT, int KMAX, int TPB, int SN = 0, bool QL = false>
__global__ __launch_bounds__(TPB, 1) void k_year_persistent(
    Grid g, Model md, Mats mt, Persist ps, StepRange sr, double dtd, const double* __restrict__ y_in,
    double* __restrict__ y_out, const double* __restrict__ v_in, double* __restrict__ v_out) {
    constexpr int TV = TANGENT ? NTR : 1;
    constexpr bool SUB = SN > 0;
    __shared__ double s_red[TPB];
    __shared__ short s_rowcol[TPB];      // per slot: the domain's column held there (-1: none)
    __shared__ short s_rowk[TPB];
    __shared__ short s_rowslot[TPB];     // per row of the domain (from its first): its slot
    __shared__ short s_colr0[TPB];       // per column of the domain: its first slot
    __shared__ short s_colnc[TPB];
    // z (and its tangent) of the own slots; without internal steps with zero
    // rows past the domain: the column product then reads KMAX rows from the
    // column's first slot with fixed offsets, and the rows past the column's
    // depth (other columns, padding slots or the zero rows) meet zero
    // coefficients
    constexpr int ZPAD = SUB ? 0 : KMAX;
    __shared__ double s_z[(TPB + ZPAD) * NTR];
    __shared__ double s_zd[(TPB + ZPAD) * TV];
    __shared__ int s_fail;
    // per buffer: own slots [0, TPB) and halo rows [TPB, TPB + halo_max) of y (and v)
    extern __shared__ double s_dyn[];
    const size_t buf_len = (size_t)(TPB + ps.halo_max) * NTR;
    double* const s_y0 = s_dyn;
    double* const s_v0 = s_dyn + 2 * buf_len;
    const bool wave_local = ps.wave_local != 0;

    const int tid = threadIdx.x;
    const int d = ps.block_dom[blockIdx.x];
    const int c0 = ps.dom_col[d], c1 = ps.dom_col[d + 1];
    const int r0 = g.col_start[c0];
    const int nrows = g.col_start[c1] - r0;
    for (int i = tid; i < TPB; i += blockDim.x) s_rowcol[i] = -1;
    if constexpr (!SUB) {
        for (int i = tid; i < (TPB + ZPAD) * NTR; i += blockDim.x) s_z[i] = 0.0;
        for (int i = tid; i < (TPB + ZPAD) * TV; i += blockDim.x) s_zd[i] = 0.0;
    }
    if (tid == 0) s_fail = 0;
    __syncthreads();
    for (int lc = tid; lc < c1 - c0; lc += blockDim.x) {
        const int s = ps.col_slot[c0 + lc];
        const int lrow = g.col_start[c0 + lc] - r0;
        const int nc = g.col_start[c0 + lc + 1] - g.col_start[c0 + lc];
        s_colr0[lc] = (short)s;
        s_colnc[lc] = (short)nc;
        for (int k = 0; k < nc; ++k) {
            s_rowcol[s + k] = (short)lc;
            s_rowk[s + k] = (short)k;
            s_rowslot[lrow + k] = (short)(s + k);
        }
    }
    __syncthreads();

    const bool own = s_rowcol[tid] >= 0;
    const int lc = own ? s_rowcol[tid] : 0;
    const int r = own ? g.col_start[c0 + lc] + s_rowk[tid] : r0;
    const int k = own ? s_rowk[tid] : 0;
    const int nc = own ? s_colnc[lc] : 1;
    const int lr0 = own ? s_colr0[lc] : 0;
    const int c = c0 + lc;
    const size_t blk = (size_t)g.blk_off[c];
    const int latrow = g.col_lat[c];

    // biogeochemical constants of this row (member 0 of the state)
    const int m = md.member[0];
    const BgcParams p = load_params(md.u, md.model, md.nparam, m);
    const double rho = md.rho[((size_t)m * (g.nlayer + 1) + nc) * g.nlayer + k];
    const int ne = nc < g.neu ? nc : g.neu;
    double light[kNeuMax], hz[kNeuMax], rho_e[kNeuMax];
#pragma unroll
    for (int e = 0; e < kNeuMax; ++e) {
        light[e] = e < ne ? md.light[(size_t)m * g.nlayer + e] : 0.0;
        hz[e] = e < ne ? g.dz[e] : 0.0;
        rho_e[e] = (SUB && e < ne) ? md.rho[((size_t)m * (g.nlayer + 1) + nc) * g.nlayer + e] : 0.0;
    }

    RowMats<KMAX> R;
    // the row's Ae entries as LDS rows: an own row at its place in the domain,
    // another domain's row after the own rows, at its place in the halo
    const int h0 = ps.halo_ptr[d], nh = ps.halo_ptr[d + 1] - h0;
#pragma unroll
    for (int s = 0; s < kEllMax; ++s) {
        const int cg = s < mt.ew ? mt.ae_col[(size_t)s * g.npad + r] : r;
        if ((unsigned)(cg - r0) < (unsigned)nrows) {
            R.col[s] = s_rowslot[cg - r0];
        } else {
            int lo = 0, hi = nh - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ps.halo_row[h0 + mid] < cg) lo = mid + 1;
                else hi = mid;
            }
            R.col[s] = TPB + (lo < nh ? lo : 0);
        }
    }
    // the halo rows this thread fetches each step (-1: none)
    int hrow[kHaloPerThread];
#pragma unroll
    for (int i = 0; i < kHaloPerThread; ++i) {
        const int hq = tid + i * TPB;
        hrow[i] = hq < nh ? ps.halo_row[h0 + hq] : -1;
    }

    // own state
    double yr[NTR], vr[TV];
#pragma unroll
    for (int t = 0; t < NTR; ++t) {
        yr[t] = own ? y_in[(size_t)r * NTR + t] : 0.0;
        s_y0[tid * NTR + t] = yr[t];
        if (TANGENT) {
            vr[t % TV] = own ? v_in[(size_t)r * NTR + t] : 0.0;
            s_v0[tid * TV + t % TV] = vr[t % TV];
        }
    }
    const int dep0 = ps.dep_ptr[d], ndep = ps.dep_ptr[d + 1] - dep0;
    int m0 = -1, m1 = -1;
    // QL: the insolation of the domain's latitude rows at every step of the
    // year, staged once: read from LDS, the sources of a step wait for no
    // global memory operation (an insolation load carried from one step to the
    // next made the compiler wait there for all outstanding memory operations,
    // the previous step's write-through ring stores included)
    const double* s_insq = nullptr;
    if constexpr (QL) {
        double* const s_ins = s_dyn + 2 * buf_len * (TANGENT ? 2 : 1);
        const int* const dlat = ps.qlat + (size_t)d * (1 + kInsLat);
        const int nq = dlat[0];
        for (int i = tid; i < nq * g.nstep; i += blockDim.x) {
            const int l = i / g.nstep, jx = i - l * g.nstep;
            s_ins[i] = g.ins[(size_t)jx * g.nlat + dlat[1 + l]];
        }
        int ql = 0;
        for (int l = 0; l < nq; ++l)
            if (dlat[1 + l] == latrow) ql = l;
        s_insq = s_ins + (size_t)ql * g.nstep;
    }
    __syncthreads();

    const int nsteps = sr.j1 - sr.j0;
    const size_t state_len = (size_t)g.n * NTR;
    const int spm = g.nstep / g.nmat;
    const double vol = g.area[c] * g.dz[k];
    // month pair and weight of the coming step, prepared at the end of the
    // step before (off the neighbours' critical path); the month pair and
    // the month-end counter advance by one step at a time, without divisions
    int k0, k1, pr_r, me_cnt;
    double w;
    step_phase(sr.j0, g.nstep, g.nmat, k0, k1, w);
    {
        int jm0 = sr.j0 % g.nstep;
        pr_r = (jm0 - spm / 2) - ((jm0 - spm / 2) >= 0 ? (jm0 - spm / 2) / spm
                                                      : -((spm / 2 - jm0 + spm - 1) / spm)) * spm;
        me_cnt = (sr.j0 + 1) % spm;
    }
    int jm = sr.j0 % g.nstep;
    double Qg = QL ? 0.0 : g.ins[(size_t)jm * g.nlat + latrow];
    for (int jj = 0; jj < nsteps; ++jj) {
        const int j = sr.j0 + jj;
        const double Q = QL ? s_insq[jm] : Qg;
        // state jj in buffer jj % 2 (both buffers alike without wave_local)
        const size_t cur = wave_local ? (size_t)(jj & 1) * buf_len : 0;
        const size_t nxt = wave_local ? (size_t)((jj + 1) & 1) * buf_len : 0;
        double* const s_y = s_y0 + cur;
        double* const s_v = s_v0 + cur;          // (used with TANGENT only, where TV = NTR)
        double* const s_yn = s_y0 + nxt;
        double* const s_vn = s_v0 + nxt;
        if (sr.store && own && jj % sr.store_every == 0) {
#pragma unroll
            for (int t = 0; t < NTR; ++t)
                sr.store[(size_t)(jj / sr.store_every) * state_len + (size_t)r * NTR + t] = yr[t];
        }
        if (k0 != m0 || k1 != m1) {
            if (own) {
                if (k0 == m1) {
#pragma unroll
                    for (int s = 0; s < kEllMax; ++s) R.e0[s] = R.e1[s];
#pragma unroll
                    for (int s = 0; s < KMAX; ++s) R.a0[s] = R.a1[s];
                } else {
                    load_month<KMAX>(mt, g, k0, r, blk, nc, k, R.e0, R.a0);
                }
                load_month<KMAX>(mt, g, k1, r, blk, nc, k, R.e1, R.a1);
            }
            m0 = k0;
            m1 = k1;
        }
        const double om = 1.0 - w;

        // sources from the domain's own rows (no wait needed)
        double q[NTR], qd[TV];
        double sc = dtd;        // internal steps return the increment itself
        if constexpr (SUB) {
            sc = 1.0;
            sub_source_lds<NTR, TANGENT, (SUB ? SN : 1), TV>(md, p, Q, ne, k, lr0, light, hz, rho_e, rho, s_y, s_v,
                                                             yr, vr, q, qd);
        } else if constexpr (NTR == 3) {
            // PO4-DOP-PHY (section 2.2.2): f_1 grows with PHY, f_3 = sigma_3 f_1 is
            // exported, PHY losses in the euphotic zone only
            double Phi = 0.0, fk = 0.0, Phid = 0.0, fdk = 0.0;
#pragma unroll
            for (int e = 0; e < kNeuMax; ++e) {
                if (e < ne) {
                    const int le = lr0 + e;
                    const Production pr = production(p, s_y[le * 3], Q, light[e]);
                    const double f = pr.f * s_y[le * 3 + 2];
                    Phi += hz[e] * (p.sig3 * f);
                    if (e == k) fk = f;
                    if (TANGENT) {
                        const double fd = pr.dfdN * s_v[le * TV] * s_y[le * 3 + 2] + pr.f * s_v[le * TV + TV - 1];
                        Phid += hz[e] * (p.sig3 * fd);
                        if (e == k) fdk = fd;
                    }
                }
            }
            const double D = yr[1], P = yr[2];
            const double loss = k < ne ? p.lam3 * P + p.kap3 * P * P : 0.0;
            q[0] = -fk + p.lam * D + (1.0 - p.sig) * Phi * rho;
            q[1] = p.sig * (p.sig3 * fk) + loss - p.lam * D + p.lam3p * P;
            q[2] = (1.0 - p.sig3) * fk - loss - p.lam3p * P;
            if (TANGENT) {
                const double Dd = vr[1 % TV], Pd = vr[TV - 1];
                const double lossd = k < ne ? (p.lam3 + 2.0 * p.kap3 * P) * Pd : 0.0;
                qd[0] = -fdk + p.lam * Dd + (1.0 - p.sig) * Phid * rho;
                qd[1 % TV] = p.sig * (p.sig3 * fdk) + lossd - p.lam * Dd + p.lam3p * Pd;
                qd[TV - 1] = (1.0 - p.sig3) * fdk - lossd - p.lam3p * Pd;
            }
        } else {
            double Phi = 0.0, fk = 0.0, Phid = 0.0, fdk = 0.0;
#pragma unroll
            for (int e = 0; e < kNeuMax; ++e) {
                if (e < ne) {
                    const double N = s_y[(lr0 + e) * NTR];
                    const Production pr = production(p, N, Q, light[e]);
                    Phi += hz[e] * pr.f;
                    if (e == k) fk = pr.f;
                    if (TANGENT) {
                        const double fd = pr.dfdN * s_v[(lr0 + e) * TV];
                        Phid += hz[e] * fd;
                        if (e == k) fdk = fd;
                    }
                }
            }
            const double dop = NTR > 1 ? yr[NTR - 1] : 0.0;
            q[0] = -fk + p.lam * dop + (1.0 - p.sig) * Phi * rho;
            if (NTR > 1) q[NTR - 1] = p.sig * fk - p.lam * dop;
            if (TANGENT) {
                const double dopd = NTR > 1 ? vr[TV - 1] : 0.0;
                qd[0] = -fdk + p.lam * dopd + (1.0 - p.sig) * Phid * rho;
                if (NTR > 1) qd[TV - 1] = p.sig * fdk - p.lam * dopd;
            }
        }

        // without the table, the coming step's insolation is loaded here
        // (after this step's last use of it, before the halo polls) rather
        // than at the end of the step, where it would still be in flight at the
        // next step's sources
        const int jn = jm + 1 == g.nstep ? 0 : jm + 1;
        const double Qn = QL ? 0.0 : g.ins[(size_t)jn * g.nlat + latrow];

        // hand-over every kRingK steps: publish the phase counter and wait for
        // the neighbours' counters
        if (jj % kRingK == 0) {
            const int ph = jj / kRingK;
            if (ph > 0) {
                // every thread's ring stores of the phase (the sentinel resets of
                // slots its neighbours read in the next phase included) before
                // the counter
                __syncthreads();
                if (tid == 0) __hip_atomic_store(&ps.flags[d], ph, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                for (int qi = tid; qi < ndep; qi += blockDim.x) {
                    const int e = ps.dep_idx[dep0 + qi];
                    long long it = 0;
                    while (__hip_atomic_load(&ps.flags[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < ph) {
                        ++it;
                        if (it > ps.spin_limit || ((it & 63) == 0 && __hip_atomic_load(ps.abort_flag, __ATOMIC_RELAXED,
                                                                                       __HIP_MEMORY_SCOPE_AGENT))) {
                            __hip_atomic_store(ps.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            s_fail = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                if (tid < ndep) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __syncthreads();
                if (s_fail) return;
            }
        }

        // the halo of state jj (ring slot jj; slot 0 holds y_in) into LDS: every
        // pass issues the loads of all the lane's halo rows together, and only
        // then checks them (a check inside a row's branch would make the loads
        // of the next row wait for those of this one: one round trip per row),
        // until none is the sentinel
        {
            const size_t sb = (size_t)(jj % kRing) * state_len;
            double hv[kHaloPerThread][NTR], hd[kHaloPerThread][NTR];
#pragma unroll
            for (int i = 0; i < kHaloPerThread; ++i)
#pragma unroll
                for (int t = 0; t < NTR; ++t) {
                    hv[i][t] = 0.0;
                    hd[i][t] = 0.0;
                }
            long long it = 0;
            for (;;) {
#pragma unroll
                for (int i = 0; i < kHaloPerThread; ++i) {
                    if (hrow[i] < 0) continue;
#pragma unroll
                    for (int t = 0; t < NTR; ++t) {
                        const size_t o = ring_at(sb, g.n, hrow[i], t);
                        hv[i][t] = __hip_atomic_load(&ps.ring[o], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (TANGENT)
                            hd[i][t] = __hip_atomic_load(&ps.vring[o], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                bool miss = false;
#pragma unroll
                for (int i = 0; i < kHaloPerThread; ++i)
#pragma unroll
                    for (int t = 0; t < NTR; ++t) {
                        miss |= is_sentinel(hv[i][t]);
                        if (TANGENT) miss |= is_sentinel(hd[i][t]);
                    }
                if (!miss) break;
                ++it;
                if (it > ps.spin_limit ||
                    ((it & 63) == 0 && __hip_atomic_load(ps.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                    __hip_atomic_store(ps.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_fail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
#pragma unroll
            for (int i = 0; i < kHaloPerThread; ++i) {
                if (hrow[i] < 0) continue;
                const int lh = TPB + tid + i * TPB;
#pragma unroll
                for (int t = 0; t < NTR; ++t) {
                    s_y[lh * NTR + t] = hv[i][t];
                    if (TANGENT) s_v[lh * TV + t % TV] = hd[i][t];
                }
            }
        }
        __syncthreads();
        if (s_fail) return;

        // z = Ae(t_j) y_j + dt_d q, from LDS
        if (own) {
            double acc[NTR], accd[TV];
#pragma unroll
            for (int t = 0; t < NTR; ++t) acc[t] = 0.0;
#pragma unroll
            for (int t = 0; t < TV; ++t) accd[t] = 0.0;
            double yy[kEllMax][NTR], vv[kEllMax][TV];
#pragma unroll
            for (int s = 0; s < kEllMax; ++s)
#pragma unroll
                for (int t = 0; t < NTR; ++t) {
                    yy[s][t] = s_y[R.col[s] * NTR + t];
                    if (TANGENT) vv[s][t % TV] = s_v[R.col[s] * TV + t % TV];
                }
            // one or two tracers without internal steps: every gather issued
            // before the first multiply (the compiler kept four in flight)
            if constexpr (!SUB && NTR <= 2) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < kEllMax; ++s) {
                const double a = om * R.e0[s] + w * R.e1[s];
#pragma unroll
                for (int t = 0; t < NTR; ++t) {
                    acc[t] += a * yy[s][t];
                    if (TANGENT) accd[t % TV] += a * vv[s][t % TV];
                }
            }
#pragma unroll
            for (int t = 0; t < NTR; ++t) {
                s_z[tid * NTR + t] = acc[t] + sc * q[t];
                if (TANGENT) s_zd[tid * TV + t % TV] = accd[t % TV] + sc * qd[t % TV];
            }
        }
        if (wave_local) wave_lds_sync();       // the column's z: written by this wavefront
        else __syncthreads();

        // y_{j+1} = Ai(t_j) z, within the water column
        const bool last = jj == nsteps - 1;
        const size_t wb = (size_t)((jj + 1) % kRing) * state_len;
        if (own) {
            double acc[NTR], accd[TV];
#pragma unroll
            for (int t = 0; t < NTR; ++t) acc[t] = 0.0;
#pragma unroll
            for (int t = 0; t < TV; ++t) accd[t] = 0.0;
            // coefficients beyond the column depth are zero, and so is every
            // product with the (finite) rows read there.  How the KMAX rows are
            // read is chosen per instance (same-box timings of each): one base
            // address with fixed offsets, all reads issued before the first
            // product for one or two tracers, interleaved with the products for
            // PO4-DOP-PHY; with internal BGC steps (whose sources hold more
            // registers) a row index clamped to the column
            [[maybe_unused]] const double* const zc = s_z + (size_t)lr0 * NTR;
            [[maybe_unused]] const double* const zdc = s_zd + (size_t)lr0 * TV;
            if constexpr (!SUB && NTR <= 2) {
                double zz[KMAX][NTR], zzd[KMAX][TV];
#pragma unroll
                for (int s = 0; s < KMAX; ++s)
#pragma unroll
                    for (int t = 0; t < NTR; ++t) {
                        zz[s][t] = zc[s * NTR + t];
                        if (TANGENT) zzd[s][t % TV] = zdc[s * TV + t % TV];
                    }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s = 0; s < KMAX; ++s) {
                    const double a = om * R.a0[s] + w * R.a1[s];
#pragma unroll
                    for (int t = 0; t < NTR; ++t) {
                        acc[t] += a * zz[s][t];
                        if (TANGENT) accd[t % TV] += a * zzd[s][t % TV];
                    }
                }
            } else if constexpr (!SUB) {
#pragma unroll
                for (int s = 0; s < KMAX; ++s) {
                    const double a = om * R.a0[s] + w * R.a1[s];
#pragma unroll
                    for (int t = 0; t < NTR; ++t) {
                        acc[t] += a * zc[s * NTR + t];
                        if (TANGENT) accd[t % TV] += a * zdc[s * TV + t % TV];
                    }
                }
            } else {
#pragma unroll
                for (int s = 0; s < KMAX; ++s) {
                    const double a = om * R.a0[s] + w * R.a1[s];
                    const int ls = lr0 + (s < nc ? s : nc - 1);
#pragma unroll
                    for (int t = 0; t < NTR; ++t) {
                        acc[t] += a * s_z[ls * NTR + t];
                        if (TANGENT) accd[t % TV] += a * s_zd[ls * TV + t % TV];
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < NTR; ++t) {
                yr[t] = acc[t];
                s_yn[tid * NTR + t] = acc[t];
                // agent-scope stores write through the XCD's L2 to the point
                // where every domain's loads see them
                if (last) y_out[(size_t)r * NTR + t] = acc[t];
                else __hip_atomic_store(&ps.ring[ring_at(wb, g.n, r, t)], publishable(acc[t]), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
                if (TANGENT) {
                    vr[t % TV] = accd[t % TV];
                    s_vn[tid * TV + t % TV] = accd[t % TV];
                    if (last) v_out[(size_t)r * NTR + t] = accd[t % TV];
                    else __hip_atomic_store(&ps.vring[ring_at(wb, g.n, r, t)], publishable(accd[t % TV]),
                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            // reset the own rows of the slot of state jj + K (phase after next
            // for the first step of a phase, spread over the phase's steps):
            // its previous state jj - K was read before this phase's hand-over
            const double sent = __longlong_as_double(kSentinelBits);
            const size_t rb = (size_t)((jj + kRingK) % kRing) * state_len;
#pragma unroll
            for (int t = 0; t < NTR; ++t) {
                __hip_atomic_store(&ps.ring[ring_at(rb, g.n, r, t)], sent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (TANGENT)
                    __hip_atomic_store(&ps.vring[ring_at(rb, g.n, r, t)], sent, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        const bool month_end = me_cnt == 0;
        // the coming step's month pair, weight and insolation
        if (++pr_r == spm) {
            pr_r = 0;
            k0 = k1;
            k1 = k1 + 1 == g.nmat ? 0 : k1 + 1;
        }
        w = (double)pr_r / (double)spm;
        // an empty asm with w as its operand keeps the division here, at the
        // end of the step; the compiler would otherwise sink it to the first
        // use, after the halo has arrived, on the path to the next publish
        asm volatile("" : "+v"(w));
        me_cnt = me_cnt + 1 == spm ? 0 : me_cnt + 1;
        jm = jn;
        Qg = Qn;
        // the next step's sources read the new state of the thread's own
        // column; its neighbours' rows are read after the next halo barrier
        if (wave_local) wave_lds_sync();
        else __syncthreads();
        // month-end misfit partial sums (after publishing, off the neighbours' critical path)
        if (sr.obs && month_end) {
            const int mo = (j + 1) / spm - 1;
            double cval = 0.0;
            if (own) {
#pragma unroll
                for (int t = 0; t < NTR; ++t) {
                    const double dd = yr[t] - sr.obs[(size_t)mo * state_len + (size_t)r * NTR + t];
                    cval += vol * dd * dd;
                }
            }
            s_red[tid] = cval;
            __syncthreads();
            for (int hh = TPB / 2; hh > 0; hh >>= 1) {
                if (tid < hh) s_red[tid] += s_red[tid + hh];
                __syncthreads();
            }
            if (tid == 0) sr.jpart[(size_t)mo * gridDim.x + d] = s_red[0];
        }
    }
}

// Sum of v over the rows [lr0, lr0 + nc) of a column, in row order.  v has
// KMAX readable entries past the last row, so the loop runs to the block width
// with fixed offsets from one base address and the LDS reads are issued
// together; the terms past the column's depth are exact zeros.
template <int KMAX>
__device__ __forceinline__ double column_sum(const double* v, int lr0, int nc) {
    double acc = 0.0;
#pragma unroll
    for (int kk = 0; kk < KMAX; ++kk) {
        const double x = v[lr0 + kk];
        acc += kk < nc ? x : 0.0;
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Persistent reverse sweep over steps j_hi-1 down to j_lo (one checkpoint
// segment), for one member.  With mu_j the cotangent of z_j (the argument
// of Ai in step j):
//   lambda_j = Ae(t_j)^T mu_j + dt_d (dq/dy)(y_j)^T mu_j + s_j
//   mu_{j-1} = Ai(t_{j-1})^T lambda_j        (lambda_0 itself when j = 0)
//   ubar    += dt_d (dq/du)(y_j)^T mu_j
// s_j is the misfit source at month ends (j > 0).  Each thread keeps its
// row of Ae^T (months of step j) and column of its Ai block (months of step
// j-1) in registers.  mu crosses domains like the forward state: through
// the sentinel-filled ring (slot 0 holds mu_in) with a hand-over every
// kRingK steps, each domain staging its halo of the transposed stencil in
// LDS once per step.
// y_j of the segment comes from ystore (slot j - j_lo).  Parameter-gradient
// sums are reduced per domain at the end and added to ubar_dom[domain][p].
// ---------------------------------------------------------------------------
template <int NTR, int KMAX, int TPB, int SN = 0>
__global__ __launch_bounds__(TPB, 1) void k_adjoint_persistent(
    Grid g, Model md, Mats mt, Persist ps, double dtd, int j_lo, int j_hi,
    const double* __restrict__ ystore, const double* __restrict__ obs, double src_scale,
    const double* __restrict__ mu_in, double* __restrict__ mu_out, double* __restrict__ ubar_dom) {
    constexpr int NP = NTR == 3 ? 11 : (NTR == 2 ? 7 : 5);
    constexpr bool SUB = SN > 0;
    __shared__ short s_rowcol[TPB];
    __shared__ short s_rowk[TPB];
    __shared__ short s_colr0[TPB];
    __shared__ short s_colnc[TPB];
    constexpr int TS = SUB ? TPB : 1;
    __shared__ double s_y[TS * NTR];       // y_j of the own rows, read by the column's internal steps (SUB only)
    // s_lam, s_rmu and s_hf have readable rows past the domain (zero, or
    // values of other columns), so that per-column loops address them with
    // fixed offsets; rows of no own thread are zero
    __shared__ double s_lam[(TPB + KMAX) * NTR];
    __shared__ double s_red[TPB];
    __shared__ double s_rhoc[TPB];   // (1 - sigma_2) rho of each own row (per member, fixed)
    __shared__ double s_rmu[TPB + KMAX];    // (1 - sigma_2) rho_k mu_k (first tracer) of each own row
    __shared__ double s_hf[TPB + kNeuMax];  // h_k times the export production of a euphotic row, per step
    __shared__ int s_fail;
    // dynamic: mu of the own rows [0, TPB) and of the halo [TPB, TPB + ahalo_max),
    // then the internal-step states [nsub][TPB][NTR] (SUB only)
    extern __shared__ double s_dyn[];
    double* const s_mu = s_dyn;
    double* const s_traj = s_dyn + (size_t)(TPB + ps.ahalo_max) * NTR;
    __shared__ double s_yb[TS * NTR];      // internal-step results per euphotic row (SUB only)
    __shared__ double s_acc[TS * acc_fields<NTR>()];
    __shared__ double s_sphi[TS];

    const int tid = threadIdx.x;
    const int d = ps.block_dom[blockIdx.x];
    const int c0 = ps.dom_col[d], c1 = ps.dom_col[d + 1];
    const int r0 = g.col_start[c0];
    const int nrows = g.col_start[c1] - r0;
    for (int lc = tid; lc < c1 - c0; lc += blockDim.x) {
        const int s = g.col_start[c0 + lc] - r0;
        const int nc = g.col_start[c0 + lc + 1] - g.col_start[c0 + lc];
        s_colr0[lc] = (short)s;
        s_colnc[lc] = (short)nc;
        for (int k = 0; k < nc; ++k) {
            s_rowcol[s + k] = (short)lc;
            s_rowk[s + k] = (short)k;
        }
    }
    if (tid == 0) s_fail = 0;
    __syncthreads();

    const bool own = tid < nrows;
    const int r = r0 + (own ? tid : 0);
    const int lc = own ? s_rowcol[tid] : 0;
    const int k = own ? s_rowk[tid] : 0;
    const int nc = own ? s_colnc[lc] : 1;
    const int lr0 = own ? s_colr0[lc] : 0;
    const int c = c0 + lc;
    const size_t blk = (size_t)g.blk_off[c];
    const int latrow = g.col_lat[c];
    const size_t state_len = (size_t)g.n * NTR;
    const int spm = g.nstep / g.nmat;
    const double vol = g.area[c] * g.dz[k];

    const int m = md.member[0];
    const BgcParams p = load_params(md.u, md.model, md.nparam, m);
    const size_t tab = ((size_t)m * (g.nlayer + 1) + nc) * g.nlayer;
    const double rho = md.rho[tab + k];
    const double drho = md.drho[tab + k];
    const int ne = nc < g.neu ? nc : g.neu;
    const double lk = (own && k < ne) ? md.light[(size_t)m * g.nlayer + k] : 0.0;   // light factor of a euphotic row
    double zc = 0.0;   // centre depth of the row's layer
    for (int i = 0; i <= k; ++i) zc += g.dz[i];
    zc -= 0.5 * g.dz[k];
    const double hk = g.dz[k];
    const double rhoc = own ? (1.0 - p.sig) * rho : 0.0;
    s_rhoc[tid] = rhoc;
    for (int i = tid; i < (TPB + KMAX) * NTR; i += blockDim.x) s_lam[i] = 0.0;
    for (int i = tid; i < TPB + KMAX; i += blockDim.x) s_rmu[i] = 0.0;
    for (int i = tid; i < TPB + kNeuMax; i += blockDim.x) s_hf[i] = 0.0;
    __syncthreads();
    // internal steps: constants of the column this thread integrates (thread
    // index = column of the domain) and of the thread's own column
    constexpr int SNE = SUB ? SN : 1;
    ColConsts<SNE> col_cc{}, own_cc{};
    if constexpr (SUB) {
        if (tid < c1 - c0) col_cc = load_col_consts<SNE>(g, md, m, c0 + tid, s_colnc[tid]);
        own_cc = load_col_consts<SNE>(g, md, m, c, nc);
    }

    // row r of Ae^T and column k of the row's Ai block; the entries of Ae^T as
    // LDS rows (own rows first, then the halo)
    int col[kEllMax];
    double e0[kEllMax], e1[kEllMax], a0[KMAX], a1[KMAX];
    const int h0 = ps.ahalo_ptr[d], nh = ps.ahalo_ptr[d + 1] - h0;
#pragma unroll
    for (int s = 0; s < kEllMax; ++s) {
        const int cg = s < mt.etw ? mt.aet_col[(size_t)s * g.npad + r] : r;
        if ((unsigned)(cg - r0) < (unsigned)nrows) {
            col[s] = cg - r0;
        } else {
            int lo = 0, hi = nh - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ps.ahalo_row[h0 + mid] < cg) lo = mid + 1;
                else hi = mid;
            }
            col[s] = TPB + (lo < nh ? lo : 0);
        }
    }
    int hrow[kHaloPerThread];
#pragma unroll
    for (int i = 0; i < kHaloPerThread; ++i) {
        const int hq = tid + i * TPB;
        hrow[i] = hq < nh ? ps.ahalo_row[h0 + hq] : -1;
    }
    auto load_ae = [&](int mo, double* e) {
#pragma unroll
        for (int s = 0; s < kEllMax; ++s)
            e[s] = s < mt.etw ? mt.aet[(size_t)mo * mt.aet_month + (size_t)s * g.npad + r] : 0.0;
    };
    auto load_ai = [&](int mo, double* a) {
#pragma unroll
        for (int s = 0; s < KMAX; ++s)
            a[s] = s < nc ? mt.ai_cm[(size_t)mo * mt.ai_month + blk + (size_t)k * nc + s] : 0.0;
    };

    double mr[NTR];
#pragma unroll
    for (int t = 0; t < NTR; ++t) {
        mr[t] = own ? mu_in[(size_t)r * NTR + t] : 0.0;
        s_mu[tid * NTR + t] = mr[t];
    }
    s_rmu[tid] = rhoc * mr[0];
    double ub[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) ub[q] = 0.0;
    const int dep0 = ps.dep_ptr[d], ndep = ps.dep_ptr[d + 1] - dep0;
    int me0 = -1, me1 = -1, ma0 = -1, ma1 = -1;
    const int nsteps = j_hi - j_lo;
    // y_j of the own rows (also in s_y for the internal steps)
    double ycur[NTR];
#pragma unroll
    for (int t = 0; t < NTR; ++t) {
        ycur[t] = (own && nsteps > 0) ? ystore[(size_t)(j_hi - 1 - j_lo) * state_len + (size_t)r * NTR + t] : 0.0;
        if constexpr (SUB) s_y[tid * NTR + t] = ycur[t];
    }
    __syncthreads();

    // month pairs of steps j and j-1 and the insolation of step j, prepared at
    // the end of the step before
    int k0, k1, q0, q1;
    double w, wq;
    step_phase(j_hi - 1, g.nstep, g.nmat, k0, k1, w);
    step_phase(j_hi - 2, g.nstep, g.nmat, q0, q1, wq);
    double Q = g.ins[(size_t)(j_hi - 1) * g.nlat + latrow];
    for (int jj = 0; jj < nsteps; ++jj) {
        const int j = j_hi - 1 - jj;
        if (own && (k0 != me0 || k1 != me1)) {
            if (k1 == me0) {          // stepping backwards: the old k0 becomes the new k1
#pragma unroll
                for (int s = 0; s < kEllMax; ++s) e1[s] = e0[s];
            } else {
                load_ae(k1, e1);
            }
            load_ae(k0, e0);
        }
        me0 = k0;
        me1 = k1;
        if (own && j > 0 && (q0 != ma0 || q1 != ma1)) {
            if (q1 == ma0) {
#pragma unroll
                for (int s = 0; s < KMAX; ++s) a1[s] = a0[s];
            } else {
                load_ai(q1, a1);
            }
            load_ai(q0, a0);
        }
        if (j > 0) {
            ma0 = q0;
            ma1 = q1;
        }
        const double om = 1.0 - w;

        // y_j of the own rows (in s_y since the end of the step before)
        double yj[NTR];
#pragma unroll
        for (int t = 0; t < NTR; ++t) yj[t] = ycur[t];

        // (dq/dy)^T mu_j and (dq/du)^T mu_j from the own water column
        double ybar[NTR];
        double hf = 0.0;
        if constexpr (SUB) {
            sub_adjoint_lds<NTR, (SUB ? SN : 1), NP, TPB>(g, md, p, m, j, c0, c1 - c0, s_colr0, s_colnc, tid, k, ne,
                                                          lc, tab, zc, rho, drho, s_y, s_mu, s_rhoc, s_traj, s_yb,
                                                          s_acc, s_sphi, col_cc, own_cc, Q, yj, mr, ybar, ub);
        } else if constexpr (NTR == 3) {
            // PO4-DOP-PHY (section 2.2.2)
            const double m1 = mr[0], m2 = mr[1], m3 = mr[2];
            const double D = yj[1], P = yj[2];
            ybar[0] = 0.0;
            ybar[2] = 0.0;
            if (k < g.neu) {
                const double Phibar = column_sum<KMAX>(s_rmu, lr0, nc);
                const Production pr = production(p, yj[0], Q, lk);
                const double f = pr.f * P;
                hf = hk * (p.sig3 * f);
                // f_1 enters q_1 (-1), q_2 (sigma_2 sigma_3), q_3 (1 - sigma_3) and Phi (h_k sigma_3)
                const double fbar = -m1 + p.sig * p.sig3 * m2 + (1.0 - p.sig3) * m3 + p.sig3 * hk * Phibar;
                const double dloss = p.lam3 + 2.0 * p.kap3 * P;
                ybar[0] = fbar * pr.dfdN * P;
                ybar[2] = fbar * pr.f + dloss * (m2 - m3);
                const double Np = yj[0] > 0.0 ? yj[0] : 0.0;
                const double rIKI2 = 1.0 / ((pr.I + p.ki) * (pr.I + p.ki));
                ub[0] += fbar * pr.limN * pr.limI * P;
                ub[1] += fbar * p.alpha * pr.limN * p.ki * rIKI2 * (-zc * pr.I) * P;
                ub[2] += fbar * (-p.alpha * Np / ((Np + p.k1) * (Np + p.k1)) * pr.limI) * P;
                ub[3] += fbar * (-p.alpha * pr.limN * pr.I * rIKI2) * P;
                ub[5] += p.sig3 * f * m2;
                ub[6] += P * (m2 - m3);
                ub[7] += P * P * (m2 - m3);
                ub[9] += f * (p.sig * m2 - m3 + hk * Phibar);
            }
            ybar[1] = p.lam * (m1 - m2);
            ybar[2] += p.lam3p * (m2 - m3);
            ub[4] += D * (m1 - m2);
            ub[8] += P * (m2 - m3);
        } else {
            const double mu1 = mr[0];
            const double mu2 = NTR > 1 ? mr[NTR - 1] : 0.0;
            const double dop = NTR > 1 ? yj[NTR - 1] : 0.0;
            ybar[0] = 0.0;
            if (k < g.neu) {
                const double Phibar = column_sum<KMAX>(s_rmu, lr0, nc);
                const Production pr = production(p, yj[0], Q, lk);
                hf = hk * pr.f;
                const double fbar = -mu1 + p.sig * mu2 + hk * Phibar;
                ybar[0] = fbar * pr.dfdN;
                const double Np = yj[0] > 0.0 ? yj[0] : 0.0;
                const double rIKI2 = 1.0 / ((pr.I + p.ki) * (pr.I + p.ki));
                ub[0] += fbar * pr.limN * pr.limI;
                ub[1] += fbar * p.alpha * pr.limN * p.ki * rIKI2 * (-zc * pr.I);
                ub[2] += fbar * (-p.alpha * Np / ((Np + p.k1) * (Np + p.k1)) * pr.limI);
                ub[3] += fbar * (-p.alpha * pr.limN * pr.I * rIKI2);
                if (NTR > 1) ub[5] += pr.f * mu2;
            }
            if (NTR > 1) {
                ybar[NTR - 1] = p.lam * (mu1 - mu2);
                ub[4] += dop * (mu1 - mu2);
            }
        }
        // the export Phi of the column is the sum of its euphotic rows' h_k f_k,
        // read back after the halo barrier
        if (!SUB && own) s_hf[tid] = hf;

        // hand-over every kRingK steps
        if (jj % kRingK == 0) {
            const int ph = jj / kRingK;
            if (ph > 0) {
                if (tid == 0) __hip_atomic_store(&ps.flags[d], ph, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                for (int qi = tid; qi < ndep; qi += blockDim.x) {
                    const int e = ps.dep_idx[dep0 + qi];
                    long long it = 0;
                    while (__hip_atomic_load(&ps.flags[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < ph) {
                        ++it;
                        if (it > ps.spin_limit || ((it & 63) == 0 && __hip_atomic_load(ps.abort_flag, __ATOMIC_RELAXED,
                                                                                       __HIP_MEMORY_SCOPE_AGENT))) {
                            __hip_atomic_store(ps.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            s_fail = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                if (tid < ndep) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __syncthreads();
                if (s_fail) return;
            }
        }

        // the halo of mu_j (ring slot jj) into LDS, all of the lane's rows per
        // pass, loaded together and then checked (as in the forward kernel)
        {
            const size_t sb = (size_t)(jj % kRing) * state_len;
            double hv[kHaloPerThread][NTR];
#pragma unroll
            for (int i = 0; i < kHaloPerThread; ++i)
#pragma unroll
                for (int t = 0; t < NTR; ++t) hv[i][t] = 0.0;
            long long it = 0;
            for (;;) {
#pragma unroll
                for (int i = 0; i < kHaloPerThread; ++i) {
                    if (hrow[i] < 0) continue;
#pragma unroll
                    for (int t = 0; t < NTR; ++t)
                        hv[i][t] = __hip_atomic_load(&ps.ring[ring_at(sb, g.n, hrow[i], t)], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                }
                bool miss = false;
#pragma unroll
                for (int i = 0; i < kHaloPerThread; ++i)
#pragma unroll
                    for (int t = 0; t < NTR; ++t) miss |= is_sentinel(hv[i][t]);
                if (!miss) break;
                ++it;
                if (it > ps.spin_limit ||
                    ((it & 63) == 0 && __hip_atomic_load(ps.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                    __hip_atomic_store(ps.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_fail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
#pragma unroll
            for (int i = 0; i < kHaloPerThread; ++i) {
                if (hrow[i] < 0) continue;
                const int lh = TPB + tid + i * TPB;
#pragma unroll
                for (int t = 0; t < NTR; ++t) s_mu[lh * NTR + t] = hv[i][t];
            }
        }
        __syncthreads();
        if (s_fail) return;

        // y_{j-1} of the own rows for the next step, loaded after the halo
        // polls (whose waits would include it) and used at the end of the step;
        // at the segment's last step its first state stands in, and threads
        // without a row read the domain's first row
        double ynx[NTR];
        {
            const int jn = j - 1 >= j_lo ? j - 1 : j_lo;
#pragma unroll
            for (int t = 0; t < NTR; ++t) ynx[t] = ystore[(size_t)(jn - j_lo) * state_len + (size_t)r * NTR + t];
        }

        // lambda_j = Ae^T mu_j + dt_d ybar + s_j
        const int mo = (j > 0 && j % spm == 0 && obs) ? j / spm - 1 : -1;
        if (own) {
            double lam[NTR];
#pragma unroll
            for (int t = 0; t < NTR; ++t) lam[t] = 0.0;
            double mm[kEllMax][NTR];
#pragma unroll
            for (int s = 0; s < kEllMax; ++s)
#pragma unroll
                for (int t = 0; t < NTR; ++t) mm[s][t] = s_mu[col[s] * NTR + t];
#pragma unroll
            for (int s = 0; s < kEllMax; ++s) {
                const double a = om * e0[s] + w * e1[s];
#pragma unroll
                for (int t = 0; t < NTR; ++t) lam[t] += a * mm[s][t];
            }
            if constexpr (!SUB) {
                // the export terms of the sigma_2 and b gradients
                double Phi = 0.0;
#pragma unroll
                for (int e = 0; e < kNeuMax; ++e) {
                    const double x = s_hf[lr0 + e];
                    Phi += e < ne ? x : 0.0;
                }
                if (NTR > 1) ub[5] += -Phi * rho * mr[0];
                ub[NP - 1] += (1.0 - p.sig) * Phi * drho * mr[0];
            }
#pragma unroll
            for (int t = 0; t < NTR; ++t) {
                lam[t] += (SUB ? 1.0 : dtd) * ybar[t];
                if (mo >= 0) lam[t] += vol * (yj[t] - obs[(size_t)mo * state_len + (size_t)r * NTR + t]) * src_scale;
                s_lam[tid * NTR + t] = lam[t];
            }
        }
        __syncthreads();

        // mu_{j-1} = Ai(t_{j-1})^T lambda_j within the column, or lambda_0
        const bool last = jj == nsteps - 1;
        const size_t wb = (size_t)((jj + 1) % kRing) * state_len;
        if (own) {
            double out[NTR];
            if (j > 0) {
                const double omq = 1.0 - wq;
#pragma unroll
                for (int t = 0; t < NTR; ++t) out[t] = 0.0;
                // a0, a1 are zero past the column's depth; the rows read there
                // (other columns, or the zero rows) are finite
#pragma unroll
                for (int s = 0; s < KMAX; ++s) {
                    const double a = omq * a0[s] + wq * a1[s];
#pragma unroll
                    for (int t = 0; t < NTR; ++t) out[t] += a * s_lam[(lr0 + s) * NTR + t];
                }
            } else {
#pragma unroll
                for (int t = 0; t < NTR; ++t) out[t] = s_lam[tid * NTR + t];
            }
            s_rmu[tid] = rhoc * out[0];
#pragma unroll
            for (int t = 0; t < NTR; ++t) {
                mr[t] = out[t];
                s_mu[tid * NTR + t] = out[t];
                if (last) mu_out[(size_t)r * NTR + t] = out[t];
                else __hip_atomic_store(&ps.ring[ring_at(wb, g.n, r, t)], publishable(out[t]), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
            }
            // reset of the slot of the cotangent jj + K, as in the forward kernel
            const double sent = __longlong_as_double(kSentinelBits);
            const size_t rb = (size_t)((jj + kRingK) % kRing) * state_len;
#pragma unroll
            for (int t = 0; t < NTR; ++t)
                __hip_atomic_store(&ps.ring[ring_at(rb, g.n, r, t)], sent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // y_{j-1} for the next step (into s_y with internal steps: this step's
        // reads of s_y all came before the halo barrier)
        if (!last) {
#pragma unroll
            for (int t = 0; t < NTR; ++t) {
                ycur[t] = ynx[t];
                if constexpr (SUB) s_y[tid * NTR + t] = ycur[t];
            }
            step_phase(j - 1, g.nstep, g.nmat, k0, k1, w);
            step_phase(j - 2, g.nstep, g.nmat, q0, q1, wq);
            Q = g.ins[(size_t)(j - 1) * g.nlat + latrow];
        }
        __syncthreads();
    }

    // per-domain parameter-gradient sums (fixed-order tree)
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        s_red[tid] = own ? ub[q] : 0.0;
        __syncthreads();
        for (int hh = TPB / 2; hh > 0; hh >>= 1) {
            if (tid < hh) s_red[tid] += s_red[tid + hh];
            __syncthreads();
        }
        if (tid == 0) ubar_dom[(size_t)d * NP + q] += (SUB ? md.hsub : dtd) * s_red[0];
        __syncthreads();
    }
}

__global__ void k_fill_int(int* __restrict__ x, int len, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) x[i] = value;
}

}  // namespace tmm
