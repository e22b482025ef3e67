// libtmm host code: descriptor validation, device formats, launches, and the
// C ABI declared in include/tmm.h.
//
// The library allocates no device memory.  Everything lives in the caller's
// workspace, laid out by plan_workspace().

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "tmm.h"
#include "tmm_device.hpp"
#include "tmm_persistent.hpp"
#include "tmm_probe.hpp"

// Scratch of tmm_year_noalloc: a fixed device array instead of workspace or
// allocations (a ping-pong state, a copy of the year's start state, residual
// partial sums and the non-finite flag).  Each device that loads the library
// holds its own copy until the process ends.  Host code never uses the name
// itself (on the host it is only a stand-in for the symbol): it uses the
// device address from hipGetSymbolAddress, taken once per device at
// tmm_create with that device current.
constexpr size_t kNoAllocBytes = 32ull << 20;
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return TMM_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TMM_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TMM_OK;
}

constexpr int kMaxTileRows = 256;          // rows per tile (LDS maps are sized for this)
constexpr int kLdsBudget = 48 * 1024;      // dynamic LDS per workgroup
constexpr size_t kAlign = 256;

#define TMM_TRY(expr)                                   \
    do {                                                \
        if ((expr) != hipSuccess) return TMM_EDEVICE;   \
    } while (0)

#define TMM_LAUNCHED()                                  \
    do {                                                \
        if (hipGetLastError() != hipSuccess) return TMM_EDEVICE; \
    } while (0)

int ntracer_of(int model) {
    return model == TMM_MODEL_N ? 1 : model == TMM_MODEL_NDOP ? 2 : model == TMM_MODEL_NDOPPHY ? 3 : -1;
}
int nparam_of(int model) {
    return model == TMM_MODEL_N ? 5 : model == TMM_MODEL_NDOP ? 7 : model == TMM_MODEL_NDOPPHY ? 11 : -1;
}

// One partition of the water columns into tiles of at most max_rows rows.
struct Tiling {
    int max_rows = 0;
    int ntile = 0;
    std::vector<int> tile_col;   // host copy
    int* d_tile_col = nullptr;
};

std::vector<int> make_tiles(const std::vector<int>& col_start, int max_rows) {
    std::vector<int> t{0};
    const int ncol = (int)col_start.size() - 1;
    int rows = 0, cols = 0;
    for (int c = 0; c < ncol; ++c) {
        const int nc = col_start[c + 1] - col_start[c];
        if (cols > 0 && (rows + nc > max_rows || cols == kMaxTileRows)) {
            t.push_back(c);
            rows = 0;
            cols = 0;
        }
        rows += nc;
        cols += 1;
    }
    t.push_back(ncol);
    return t;
}

std::vector<int> tiling_sizes(int nlayer) {
    std::vector<int> s;
    for (int r : {std::max(nlayer, 32), 64, 128, 256})
        if (r >= nlayer && r <= kMaxTileRows && std::find(s.begin(), s.end(), r) == s.end()) s.push_back(r);
    return s;
}

// Host-side summary of a validated descriptor.
struct Plan {
    int n = 0, ncol = 0, nlayer = 0, nmat = 0, nstep = 0, model = 0, neu = 0;
    int nbatch_max = 0, adj_nb = 0, ckpt = 0, ntr = 0, nparam = 0;
    int nsub = 1;                          // internal BGC steps per ocean step
    int npad = 0, ew = 0, etw = 0;
    size_t nblk = 0;                       // sum of n_c^2
    std::vector<int> col_start, tiles_sizes;
    int ntile_max = 0;
    // workspace offsets (bytes)
    size_t o_ae, o_aecol, o_aet, o_aetcol, o_aicm, o_airm, o_colstart, o_blk, o_lat, o_area, o_dz;
    std::vector<size_t> o_tiles;
    size_t o_u, o_light, o_rho, o_drho, o_member, o_scol, o_dcol;
    size_t o_uT, o_lightT, o_rhoT;   // member-fastest copies (member-parallel kernel)
    size_t o_ybuf[3], o_vbuf[2], o_part, o_vec, o_ubt, o_jpart, o_ckpt, o_seg, o_final, o_mu[2];
    size_t o_pubar, o_pjpart;       // per-domain adjoint partial sums (persistent path)
    size_t vec_stride;
    // insolation table over distinct latitudes
    std::vector<double> lat_u;
    std::vector<int> col_lat;
    std::vector<double> lon;        // [ncol] or empty (descriptor's optional longitudes)
    size_t o_morder;                // column order of the member-parallel kernel
    size_t o_morderp[2];            // ... of its packed forms (2 and 4 columns per wavefront)
    size_t o_mstage, o_mlidx;       // tables of the tiled member kernel (0: none)
    size_t o_ins, o_collat, o_latu;
    // persistent-kernel tables (sized for up to kMaxDomains domains)
    size_t o_pblock, o_pdomcol, o_pdepptr, o_pdepidx, o_pflags, o_pabort;
    size_t o_finite;                // set by the per-year non-finite check
    size_t o_probe;                 // words, results and load chain of tmm_probe_exchange
    size_t o_ring, o_vring;         // state rings of the persistent forward kernel (0: none)
    size_t o_phaloptr, o_phalo;     // halo rows of each domain
    size_t o_pqlat;                 // latitude rows of each domain (insolation table in LDS)
    size_t o_pcolslot;              // first slot (thread) of each water column in its domain
    size_t o_pahaloptr, o_pahalo;   // ... for the transposed stencil (reverse sweep)
    size_t dep_capacity, halo_capacity;
    size_t total;
};

constexpr int kMaxDomains = 4096;
// grids up to this many rows get the persistent kernel's state rings
// (2 x kRing x n x ntr doubles); larger ones cannot be resident anyway
constexpr int kMaxPersistentRows = 256 * tmm::kPersistThreadsMax;
constexpr int kDefaultDomainRows = 256;     // rows per persistent workgroup unless set by option (tuned on MI355X)
constexpr int kMembersWavesMax = 8;         // wavefronts per workgroup of the member kernel, at most
constexpr int kDefaultBandRows = 16;        // latitude rows per band of the member kernel's column order
constexpr double kLastLevelCacheBytes = 256.0 * 1024 * 1024;   // MI355X Infinity Cache
constexpr int kTileKmax = 24;               // deepest columns of the tiled member kernel
constexpr int kTileQnMax = 4;               // staged rows per wavefront and layer, at most (4 columns x 16 rows)
constexpr int kProbeLines = 4096;           // 256-byte lines of the probe's load chain (1 MiB)
constexpr size_t kProbeBytes = 4096 + (size_t)kProbeLines * 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int validate(const tmm_desc* d, Plan& P) {
    if (!d) return TMM_EINVAL;
    if (d->n < 1 || d->ncol < 1 || d->nlayer < 1 || d->nlayer > tmm::kMaxLayers) return TMM_EINVAL;
    if (!d->col_start || !d->lat || !d->area || !d->dz) return TMM_EINVAL;
    if (ntracer_of(d->model) < 0) return TMM_EINVAL;
    if (d->nmat < 1 || d->nstep < 1 || d->nstep % d->nmat || (d->nstep / d->nmat) % 2) return TMM_EINVAL;
    if (d->neuphotic < 1 || d->neuphotic > d->nlayer) return TMM_EINVAL;
    if (d->nbgc < 0 || d->nbgc > tmm::kSubMax) return TMM_EINVAL;
    if (d->nbgc > 1 && d->neuphotic > tmm::kSubNeuMax) return TMM_EUNSUPPORTED;
    if (d->nbatch_max < 1 || d->adjoint_nbatch_max < 0 || d->adjoint_nbatch_max > d->nbatch_max) return TMM_EINVAL;
    if (d->adjoint_nbatch_max > 0 && (d->ckpt_every < 1 || d->nstep % d->ckpt_every)) return TMM_EINVAL;
    if (d->adjoint_nbatch_max * nparam_of(d->model) > 128) return TMM_EINVAL;
    if (d->ae_nnz < d->n || !d->ae_rowptr || !d->ae_colidx || !d->ae_val) return TMM_EINVAL;
    if (d->ai_nnz < d->n || !d->ai_rowptr || !d->ai_colidx || !d->ai_val) return TMM_EINVAL;
    if (d->col_start[0] != 0 || d->col_start[d->ncol] != d->n) return TMM_EINVAL;
    for (int c = 0; c < d->ncol; ++c) {
        const int nc = d->col_start[c + 1] - d->col_start[c];
        if (nc < 1 || nc > d->nlayer) return TMM_EINVAL;
    }
    for (int c = 0; c < d->ncol; ++c)
        if (!std::isfinite(d->lat[c]) || !std::isfinite(d->area[c]) || d->area[c] <= 0.0) return TMM_EINVAL;
    for (int k = 0; k < d->nlayer; ++k)
        if (!std::isfinite(d->dz[k]) || d->dz[k] <= 0.0) return TMM_EINVAL;
    if (d->lon)
        for (int c = 0; c < d->ncol; ++c)
            if (!std::isfinite(d->lon[c])) return TMM_EINVAL;
    auto check_csr = [&](const int* rp, const int* ci, int nnz) {
        if (rp[0] != 0 || rp[d->n] != nnz) return false;
        for (int i = 0; i < d->n; ++i)
            if (rp[i + 1] < rp[i]) return false;
        for (int e = 0; e < nnz; ++e)
            if (ci[e] < 0 || ci[e] >= d->n) return false;
        return true;
    };
    if (!check_csr(d->ae_rowptr, d->ae_colidx, d->ae_nnz)) return TMM_EINVAL;
    if (!check_csr(d->ai_rowptr, d->ai_colidx, d->ai_nnz)) return TMM_EINVAL;
    // implicit matrices act within water columns only
    std::vector<int> row_col(d->n);
    for (int c = 0; c < d->ncol; ++c)
        for (int r = d->col_start[c]; r < d->col_start[c + 1]; ++r) row_col[r] = c;
    for (int i = 0; i < d->n; ++i)
        for (int e = d->ai_rowptr[i]; e < d->ai_rowptr[i + 1]; ++e)
            if (row_col[d->ai_colidx[e]] != row_col[i]) return TMM_EINVAL;

    P.n = d->n; P.ncol = d->ncol; P.nlayer = d->nlayer; P.nmat = d->nmat; P.nstep = d->nstep;
    P.model = d->model; P.neu = d->neuphotic; P.nbatch_max = d->nbatch_max;
    P.nsub = d->nbgc > 1 ? d->nbgc : 1;
    P.adj_nb = d->adjoint_nbatch_max; P.ckpt = P.adj_nb > 0 ? d->ckpt_every : 0;
    P.ntr = ntracer_of(d->model); P.nparam = nparam_of(d->model);
    P.npad = (d->n + 63) / 64 * 64;
    P.col_start.assign(d->col_start, d->col_start + d->ncol + 1);
    // ELL width of Ae: slot 0 of every row reads the row itself (its diagonal
    // entry, else a zero padding entry), so a row without a diagonal counts
    // one more
    int ew = 0;
    std::vector<int> tcount(d->n, 0);
    for (int i = 0; i < d->n; ++i) {
        bool diag = false;
        for (int e = d->ae_rowptr[i]; e < d->ae_rowptr[i + 1]; ++e) {
            tcount[d->ae_colidx[e]]++;
            diag = diag || d->ae_colidx[e] == i;
        }
        ew = std::max(ew, d->ae_rowptr[i + 1] - d->ae_rowptr[i] + (diag ? 0 : 1));
    }
    P.ew = ew;
    P.etw = *std::max_element(tcount.begin(), tcount.end());
    if (P.etw < 1) P.etw = 1;
    P.nblk = 0;
    for (int c = 0; c < d->ncol; ++c) {
        const size_t nc = d->col_start[c + 1] - d->col_start[c];
        P.nblk += nc * nc;
    }
    if (P.nblk > (size_t)INT32_MAX) return TMM_EUNSUPPORTED;
    P.tiles_sizes = tiling_sizes(d->nlayer);
    P.ntile_max = 0;
    for (int r : P.tiles_sizes)
        P.ntile_max = std::max(P.ntile_max, (int)make_tiles(P.col_start, r).size() - 1);

    // workspace layout
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    const size_t nm = d->nmat, npad = P.npad;
    P.o_ae = take(nm * P.ew * npad * 8);
    P.o_aecol = take((size_t)P.ew * npad * 4);
    P.o_aet = take(nm * P.etw * npad * 8);
    P.o_aetcol = take((size_t)P.etw * npad * 4);
    P.o_aicm = take(nm * P.nblk * 8);
    P.o_airm = take(nm * P.nblk * 8);
    P.o_colstart = take((size_t)(d->ncol + 1) * 4);
    P.o_blk = take((size_t)d->ncol * 4);
    P.o_lat = take((size_t)d->ncol * 8);
    P.o_area = take((size_t)d->ncol * 8);
    P.o_dz = take((size_t)d->nlayer * 8);
    P.o_tiles.clear();
    for (size_t t = 0; t < P.tiles_sizes.size(); ++t) P.o_tiles.push_back(take((size_t)(d->ncol + 1) * 4));
    const size_t nbm = d->nbatch_max;
    P.o_u = take(nbm * P.nparam * 8);
    P.o_light = take(nbm * d->nlayer * 8);
    P.o_rho = take(nbm * (d->nlayer + 1) * d->nlayer * 8);
    P.o_drho = take(nbm * (d->nlayer + 1) * d->nlayer * 8);
    P.o_member = take(nbm * 4);
    P.o_uT = take(nbm * P.nparam * 8);
    P.o_lightT = take(nbm * d->nlayer * 8);
    P.o_rhoT = take(nbm * (d->nlayer + 1) * d->nlayer * 8);
    P.o_scol = take(nbm * 4);
    P.o_dcol = take(nbm * 4);
    const size_t state = (size_t)d->n * nbm * P.ntr * 8;
    for (auto& b : P.o_ybuf) b = take(state);
    for (auto& b : P.o_vbuf) b = take(state);
    const size_t nq = std::max<size_t>(nbm, (size_t)P.adj_nb * P.nparam);
    P.o_part = take((size_t)P.ntile_max * nq * 8);
    P.vec_stride = std::max<size_t>(std::max<size_t>(nbm, (size_t)P.adj_nb * P.nparam), 8);
    P.o_vec = take(16 * P.vec_stride * 8);
    if (P.adj_nb > 0) {
        const size_t astate = (size_t)d->n * P.adj_nb * P.ntr * 8;
        P.o_ubt = take((size_t)P.ntile_max * P.adj_nb * P.nparam * 8);
        P.o_jpart = take(nm * P.ntile_max * P.adj_nb * 8);
        P.o_ckpt = take((size_t)(d->nstep / P.ckpt) * astate);
        P.o_seg = take((size_t)P.ckpt * astate);
        P.o_final = take(astate);
        P.o_mu[0] = take(astate);
        P.o_mu[1] = take(astate);
        P.o_pubar = take((size_t)kMaxDomains * 8 * 8);
        P.o_pjpart = take(nm * kMaxDomains * 8);
    } else {
        P.o_pubar = P.o_pjpart = 0;
        P.o_ubt = P.o_jpart = P.o_ckpt = P.o_seg = P.o_final = P.o_mu[0] = P.o_mu[1] = 0;
    }
    // distinct latitudes (exact values) for the insolation table
    P.lat_u.clear();
    P.col_lat.assign(d->ncol, 0);
    {
        std::vector<double> l(d->lat, d->lat + d->ncol);
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
        P.lat_u = l;
        for (int c = 0; c < d->ncol; ++c)
            P.col_lat[c] = (int)(std::lower_bound(l.begin(), l.end(), d->lat[c]) - l.begin());
    }
    P.o_ins = take((size_t)d->nstep * P.lat_u.size() * 8);
    if (d->lon) P.lon.assign(d->lon, d->lon + d->ncol);
    else P.lon.clear();
    P.o_morder = take(((size_t)d->ncol + 8 * kMembersWavesMax) * 4);
    for (auto& o_p : P.o_morderp) o_p = take(((size_t)d->ncol + 8 * kMembersWavesMax) * 4);
    if (P.ntr == 2 && d->nlayer <= kTileKmax) {
        const size_t slots = (size_t)d->ncol + 8 * kMembersWavesMax;
        P.o_mstage = take(slots * kTileKmax * kTileQnMax * 4);
        P.o_mlidx = take(slots * kTileKmax * 5);
    } else {
        P.o_mstage = P.o_mlidx = 0;
    }
    P.o_collat = take((size_t)d->ncol * 4);
    P.o_latu = take(P.lat_u.size() * 8);
    P.dep_capacity = 2 * (size_t)d->ae_nnz + 1;
    P.o_pblock = take((size_t)kMaxDomains * 4);
    P.o_pdomcol = take((size_t)(kMaxDomains + 1) * 4);
    P.o_pdepptr = take((size_t)(kMaxDomains + 1) * 4);
    P.o_pdepidx = take(P.dep_capacity * 4);
    P.o_pflags = take((size_t)kMaxDomains * 4);
    P.o_pabort = take(64);
    P.o_finite = take(64);
    P.o_probe = take(kProbeBytes);
    P.o_phaloptr = take((size_t)(kMaxDomains + 1) * 4);
    P.halo_capacity = (size_t)d->ae_nnz + 1;
    P.o_phalo = take(P.halo_capacity * 4);
    P.o_pahaloptr = take((size_t)(kMaxDomains + 1) * 4);
    P.o_pahalo = take(P.halo_capacity * 4);
    P.o_pqlat = take((size_t)kMaxDomains * (1 + tmm::kInsLat) * 4);
    P.o_pcolslot = take((size_t)d->ncol * 4);
    if (d->n <= kMaxPersistentRows) {
        P.o_ring = take((size_t)tmm::kRing * d->n * P.ntr * 8);
        P.o_vring = take((size_t)tmm::kRing * d->n * P.ntr * 8);
    } else {
        P.o_ring = P.o_vring = 0;
    }
    P.total = o;
    return TMM_OK;
}

}  // namespace

struct tmm_ctx {
    Plan P;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    std::vector<Tiling> tilings;
    int nbatch = 0;            // members set by tmm_set_params
    double vtot = 0.0;         // total wet volume
    std::vector<int> h_member, h_scol, h_dcol;
    std::vector<double> h_vec;
    // persistent year kernel
    bool pers_ok = false;          // tables built and the launch fits the device
    bool pers_adj_ok = false;      // ... and so does the persistent adjoint
    bool pers_enabled = true;      // option TMM_OPT_PERSISTENT
    long long spin_limit = 1ll << 22;   // option TMM_OPT_SPIN_LIMIT
    int pers_G = 0;
    int pers_kmax = 16;
    int pers_tpb = 256;            // threads (= maximum rows) per domain
    int pers_hmax = 0;             // largest domain halo (rows)
    int pers_ahmax = 0;            // ... of the transposed stencil
    int pers_qmax = 0;             // most latitude rows a domain spans (its insolation table in LDS)
    bool pers_ql[2] = {false, false};   // the forward kernels keep that table in LDS (state
                                        // only, with the tangent)
    bool pers_wave_local = false;  // no water column spans two wavefronts of the forward kernels
    bool wave_local_enabled = true;    // option TMM_OPT_WAVE_LOCAL
    int pers_target = 0;           // option TMM_OPT_DOMAIN_ROWS as last set
    int wide_min_members = -1;     // batches of at least this many members use k_step_members
                                   // (-1: 2 where the packed forms run, else 6)
    int mem_waves = tmm::kMembersWaves;   // option TMM_OPT_MEMBER_WAVES
    int mem_band = kDefaultBandRows;      // option TMM_OPT_MEMBER_BAND_ROWS (0: natural column order)
    int mem_blocks = 0;            // workgroups of one member-kernel launch (per member group)
    bool mem_ordered = false;      // the order table in the workspace is in use
    bool mem_pack = true;          // option TMM_OPT_MEMBER_PACK
    int mem_blocks_p[2] = {0, 0};  // workgroups of the packed member kernels (32, 16 members per column)
    int mem_tile = 0;              // option TMM_OPT_MEMBER_TILE: columns per workgroup of the tiled
                                   // member kernel (0: k_step_members)
    std::vector<int> ell_col;      // Ae's ELL columns [ew][npad] (host copy, for the tile tables)
    // captured model years of the launch-per-step path, keyed by their arguments
    struct YearGraph {
        int nb;
        const void* ptrs[4];
        hipGraphExec_t exec;
        unsigned long long used;
    };
    std::vector<YearGraph> graphs;
    unsigned long long graph_clock = 0;
    bool graphs_enabled = true;
    hipStream_t capture_stream = nullptr;
    bool capturing = false;
    hipStream_t launch_stream() const { return capturing ? capture_stream : stream; }
    int num_cu = 0;
    bool pers_used = false;        // a persistent launch happened since the last abort check
    bool check_finite = true;      // option TMM_OPT_CHECK_FINITE
    double* noalloc = nullptr;     // device address of the static scratch on the handle's device
    int tile_rows_cap = 0;         // option TMM_OPT_TILE_ROWS (0: by width)
    std::vector<int> ae_rowptr, ae_colidx;   // explicit-matrix pattern (domain dependencies)

    template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }

    tmm::Grid grid(const Tiling& t) const {
        tmm::Grid g;
        g.n = P.n; g.npad = P.npad; g.nlayer = P.nlayer; g.neu = P.neu; g.nstep = P.nstep; g.nmat = P.nmat;
        g.tile_col = t.d_tile_col;
        g.col_start = at<int>(P.o_colstart);
        g.blk_off = at<int>(P.o_blk);
        g.lat = at<double>(P.o_lat);
        g.area = at<double>(P.o_area);
        g.dz = at<double>(P.o_dz);
        g.ins = at<double>(P.o_ins);
        g.col_lat = at<int>(P.o_collat);
        g.nlat = (int)P.lat_u.size();
        return g;
    }
    tmm::Model model() const {
        tmm::Model m;
        m.model = P.model; m.ntr = P.ntr; m.nparam = P.nparam;
        m.u = at<double>(P.o_u);
        m.light = at<double>(P.o_light);
        m.rho = at<double>(P.o_rho);
        m.drho = at<double>(P.o_drho);
        m.member = at<int>(P.o_member);
        m.uT = at<double>(P.o_uT);
        m.lightT = at<double>(P.o_lightT);
        m.rhoT = at<double>(P.o_rhoT);
        m.nbm = P.nbatch_max;
        m.nsub = P.nsub;
        m.hsub = tmm::kDaysPerYear / P.nstep / P.nsub;
        return m;
    }
    tmm::Mats mats() const {
        tmm::Mats m;
        m.ew = P.ew; m.etw = P.etw;
        m.ae_month = (size_t)P.ew * P.npad;
        m.aet_month = (size_t)P.etw * P.npad;
        m.ai_month = P.nblk;
        m.ae = at<double>(P.o_ae);
        m.ae_col = at<int>(P.o_aecol);
        m.aet = at<double>(P.o_aet);
        m.aet_col = at<int>(P.o_aetcol);
        m.ai_cm = at<double>(P.o_aicm);
        m.ai_rm = at<double>(P.o_airm);
        return m;
    }
    double* ybuf(int i) const { return at<double>(P.o_ybuf[i]); }
    double* vbuf(int i) const { return at<double>(P.o_vbuf[i]); }
    double* part() const { return at<double>(P.o_part); }
    // small vectors: 16 rows of vec_stride doubles (per slot, or per slot and parameter)
    double* vec(int row) const { return at<double>(P.o_vec) + (size_t)row * P.vec_stride; }

    // Largest tiling whose rows fit the LDS budget for width W and mult buffers.
    // (capped by option TMM_OPT_TILE_ROWS when set)
    const Tiling& tiling_for(int W, int mult, int extra_bytes = 0) const {
        const Tiling* best = &tilings.front();
        const int cap = tile_rows_cap > 0 ? tile_rows_cap : (W <= 4 ? 128 : kMaxTileRows);
        for (const Tiling& t : tilings) {
            const size_t lds = (size_t)t.max_rows * W * 8 * mult + extra_bytes;
            if (lds <= (size_t)kLdsBudget && t.max_rows <= cap) best = &t;
        }
        return *best;
    }
};

namespace {

int launch_blocks(size_t work, int block = 256) {
    size_t b = (work + block - 1) / block;
    return (int)std::min<size_t>(std::max<size_t>(b, 1), 4096);
}

int upload(tmm_ctx* h, void* dst, const void* src, size_t bytes) {
    TMM_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
    return TMM_OK;
}

int fill(tmm_ctx* h, double* x, size_t len, double v) {
    hipLaunchKernelGGL(tmm::k_fill, dim3(launch_blocks(len)), dim3(256), 0, h->stream, x, len, v);
    TMM_LAUNCHED();
    return TMM_OK;
}

int copy(tmm_ctx* h, double* dst, const double* src, size_t len) {
    hipLaunchKernelGGL(tmm::k_copy, dim3(launch_blocks(len)), dim3(256), 0, h->stream, dst, src, len);
    TMM_LAUNCHED();
    return TMM_OK;
}

// Whether the tiled member kernel can run on this handle: two tracers, one
// BGC evaluation per step, a five-point explicit stencil, columns of at most
// kTileKmax layers, and longitudes to build compact tiles from.
bool member_tiles_possible(const Plan& P) {
    return P.ntr == 2 && P.nsub == 1 && P.ew <= 5 && P.nlayer <= kTileKmax && P.o_mstage != 0 && !P.lon.empty();
}

// Tables of k_step_member_tiles for the column order `order` (T columns per
// workgroup): per workgroup and layer the distinct state rows that the
// explicit rows of its columns read, in order of first use, dealt to the
// wavefronts round-robin; per column, layer and stencil entry the slot it
// reads.  Fails if a layer needs more than RMAX rows.
int build_member_tiles(tmm_ctx* h, const std::vector<int>& order, int T, int rmax) {
    const Plan& P = h->P;
    const int nblk = (int)(order.size() / T);
    const int qn = rmax / T;
    const int KM = kTileKmax, EL = 5;
    std::vector<int> stage((size_t)order.size() * KM * qn, -1);
    std::vector<unsigned char> lidx((size_t)order.size() * KM * EL, 0);
    std::vector<int> rows;
    for (int b = 0; b < nblk; ++b) {
        int kt = 0;
        for (int w = 0; w < T; ++w) {
            const int c = order[(size_t)b * T + w];
            if (c >= 0) kt = std::max(kt, P.col_start[c + 1] - P.col_start[c]);
        }
        for (int k = 0; k < kt; ++k) {
            rows.clear();
            for (int w = 0; w < T; ++w) {
                const int c = order[(size_t)b * T + w];
                if (c < 0) continue;
                const int rs = P.col_start[c], nc = P.col_start[c + 1] - rs;
                if (k >= nc) continue;
                for (int sl = 0; sl < P.ew; ++sl) {
                    const int r = h->ell_col[(size_t)sl * P.npad + rs + k];
                    int at = (int)(std::find(rows.begin(), rows.end(), r) - rows.begin());
                    if (at == (int)rows.size()) rows.push_back(r);
                    if (at >= rmax) return TMM_EUNSUPPORTED;
                    lidx[((size_t)b * T + w) * KM * EL + (size_t)k * EL + sl] = (unsigned char)at;
                }
            }
            for (int i = 0; i < (int)rows.size(); ++i)
                stage[(((size_t)b * T + i % T) * KM + k) * qn + i / T] = rows[i];
        }
    }
    if (upload(h, h->at<int>(P.o_mstage), stage.data(), stage.size() * 4) ||
        upload(h, h->at<unsigned char>(P.o_mlidx), lidx.data(), lidx.size()))
        return TMM_EDEVICE;
    TMM_TRY(hipStreamSynchronize(h->stream));
    return TMM_OK;
}

// Rows per layer that one workgroup of the tiled member kernel stages.
int member_tile_rows(int T) { return T == 8 ? 24 : 16; }

// Column order of the member-parallel kernels (see k_step_members).  With the
// columns' longitudes known and band > 0: the columns sorted by (band of
// `band` latitude rows, longitude, latitude row), cut into 8 runs of equal
// length, run x on the workgroups b with b % 8 == x (the XCD they are
// dispatched to), each workgroup taking `waves` consecutive columns of its
// run (T of them for the tiled kernel, whose tables are built here too).
// Otherwise the natural order.  Written to the workspace; results do not
// depend on it.  Not called during graph capture.
int build_member_order(tmm_ctx* h) {
    const Plan& P = h->P;
    const int waves = h->mem_tile > 0 ? h->mem_tile : h->mem_waves;
    // columns per workgroup of the packed member kernels (two wavefronts of 2 or 4 columns)
    const int pcols[2] = {2 * 2, 2 * 4};
    if (P.lon.empty() || h->mem_band <= 0) {
        if (h->mem_tile > 0) return TMM_EUNSUPPORTED;
        h->mem_ordered = false;
        h->mem_blocks = (P.ncol + waves - 1) / waves;
        for (int i = 0; i < 2; ++i) h->mem_blocks_p[i] = (P.ncol + pcols[i] - 1) / pcols[i];
        return TMM_OK;
    }
    std::vector<int> cols(P.ncol);
    for (int c = 0; c < P.ncol; ++c) cols[c] = c;
    const int band = h->mem_band;
    std::stable_sort(cols.begin(), cols.end(), [&](int a, int b) {
        const int ba = P.col_lat[a] / band, bb = P.col_lat[b] / band;
        if (ba != bb) return ba < bb;
        if (P.lon[a] != P.lon[b]) return P.lon[a] < P.lon[b];
        return P.col_lat[a] < P.col_lat[b];
    });
    // the sorted columns cut into 8 runs, run x on the workgroups b with
    // b % 8 == x, each workgroup taking `per` consecutive columns of its run
    const int runs = 8;
    const int q = (P.ncol + runs - 1) / runs;          // columns per run
    auto make = [&](int per, int& blocks) {
        const int m = (q + per - 1) / per;             // workgroups per run
        std::vector<int> order((size_t)runs * m * per, -1);
        for (int x = 0; x < runs; ++x)
            for (int i = 0; i < m; ++i)
                for (int w = 0; w < per; ++w) {
                    const int pos = x * q + i * per + w;
                    if (i * per + w < q && pos < P.ncol) order[((size_t)i * runs + x) * per + w] = cols[pos];
                }
        blocks = runs * m;
        return order;
    };
    int blocks = 0;
    std::vector<int> order = make(waves, blocks);
    if (order.size() > (size_t)P.ncol + 8 * kMembersWavesMax) return TMM_EUNSUPPORTED;
    if (h->mem_tile > 0) {
        const int rc = build_member_tiles(h, order, waves, member_tile_rows(waves));
        if (rc) return rc;
    }
    if (upload(h, h->at<int>(P.o_morder), order.data(), order.size() * 4)) return TMM_EDEVICE;
    int pblocks[2];
    for (int i = 0; i < 2; ++i) {
        std::vector<int> po = make(pcols[i], pblocks[i]);
        if (po.size() > (size_t)P.ncol + 8 * kMembersWavesMax) return TMM_EUNSUPPORTED;
        if (upload(h, h->at<int>(P.o_morderp[i]), po.data(), po.size() * 4)) return TMM_EDEVICE;
    }
    TMM_TRY(hipStreamSynchronize(h->stream));
    h->mem_blocks = blocks;
    for (int i = 0; i < 2; ++i) h->mem_blocks_p[i] = pblocks[i];
    h->mem_ordered = true;
    return TMM_OK;
}

// Forward step j for nb state slots (W = nb*ntr); tangent when v != nullptr.
int launch_step(tmm_ctx* h, int j, int nb, const double* y, double* yo, const double* v, double* vo) {
    const int W = nb * h->P.ntr;
    const bool tangent = v != nullptr;
    const bool sub = h->P.nsub > 1;
    // measured crossovers with the tile kernel (50k and 500k points): 2 members
    // for the packed member kernel, 6 for one column per wavefront
    const bool packed = h->P.ntr == 2 && !sub && h->P.ew <= 5 && h->mem_pack && h->mem_tile == 0 &&
                        h->P.nlayer <= 24;
    const int min_nb = h->wide_min_members >= 0 ? h->wide_min_members : (packed ? 2 : 6);
    if (!tangent && nb >= min_nb && h->P.ntr <= 2 && h->P.nlayer <= 32 &&
        h->P.ew <= tmm::kMembersEll && (size_t)h->P.npad * W * 8 <= UINT32_MAX) {
        // member-parallel kernel: one wavefront per column and 64 members
        const int kmax = h->P.nlayer <= 16 ? 16 : h->P.nlayer <= 24 ? 24 : 32;
        const double dtd = tmm::kDaysPerYear / h->P.nstep;
        tmm::Grid g = h->grid(h->tilings.front());
        tmm::Model md = h->model();
        tmm::Mats mt = h->mats();
        // the wave count is an option for the two-tracer, five-point case (the ensemble's);
        // every other variant runs with the default
        const bool wave_opt = h->P.ntr == 2 && !sub && h->P.ew <= 5;
        const int waves = wave_opt ? h->mem_waves : tmm::kMembersWaves;
        const int nblk = wave_opt ? h->mem_blocks : (h->P.ncol + waves - 1) / waves;
        const int* order = (wave_opt && h->mem_ordered) ? h->at<int>(h->P.o_morder) : nullptr;
        dim3 grid(nblk, (nb + 63) / 64), blk(64 * waves);
        // non-temporal stores of the new state where a step's state (read and written) and
        // matrices exceed the last-level cache (measured: 3-6 % faster on 500000 points,
        // 10-30 % slower where everything fits, 52749 points)
        const double step_bytes = 2.0 * h->P.n * W * 8 + 16.0 * (double)h->P.nblk + 20.0 * h->P.ew * h->P.npad;
        const int nt = step_bytes > kLastLevelCacheBytes ? 1 : 0;
        if (wave_opt && h->mem_tile == 0 && h->mem_pack && nb <= 32 && kmax <= 24) {
            // packed: 2 (4) columns per wavefront, 32 (16) members each
            const int pi = nb <= 16 ? 1 : 0;
            const int* porder = h->mem_ordered ? h->at<int>(h->P.o_morderp[pi]) : nullptr;
            dim3 pgrid(h->mem_blocks_p[pi], 1), pblk(128);
            if (pi == 0 && kmax == 16)
                hipLaunchKernelGGL((tmm::k_step_members<2, 16, 5, false, 2, 32>), pgrid, pblk, 0, h->launch_stream(),
                                   g, md, mt, h->P.ncol, nb, j, dtd, porder, y, yo, nt);
            else if (pi == 0)
                hipLaunchKernelGGL((tmm::k_step_members<2, 24, 5, false, 2, 32>), pgrid, pblk, 0, h->launch_stream(),
                                   g, md, mt, h->P.ncol, nb, j, dtd, porder, y, yo, nt);
            else if (kmax == 16)
                hipLaunchKernelGGL((tmm::k_step_members<2, 16, 5, false, 2, 16>), pgrid, pblk, 0, h->launch_stream(),
                                   g, md, mt, h->P.ncol, nb, j, dtd, porder, y, yo, nt);
            else
                hipLaunchKernelGGL((tmm::k_step_members<2, 24, 5, false, 2, 16>), pgrid, pblk, 0, h->launch_stream(),
                                   g, md, mt, h->P.ncol, nb, j, dtd, porder, y, yo, nt);
            TMM_LAUNCHED();
            return TMM_OK;
        }
        if (wave_opt && h->mem_tile > 0 && h->mem_ordered && kmax <= kTileKmax) {
            const int* stage = h->at<int>(h->P.o_mstage);
            const unsigned char* lidx = h->at<unsigned char>(h->P.o_mlidx);
            dim3 tgrid(h->mem_blocks, (nb + 63) / 64), tblk(64 * h->mem_tile);
            if (h->mem_tile == 8)
                hipLaunchKernelGGL((tmm::k_step_member_tiles<kTileKmax, 8, 24, 3>), tgrid, tblk, 0, h->launch_stream(),
                                   g, md, mt, nb, j, dtd, order, stage, lidx, y, yo);
            else
                hipLaunchKernelGGL((tmm::k_step_member_tiles<kTileKmax, 4, 16, 3>), tgrid, tblk, 0, h->launch_stream(),
                                   g, md, mt, nb, j, dtd, order, stage, lidx, y, yo);
            TMM_LAUNCHED();
            return TMM_OK;
        }
#define TMM_MEMBERS(NT, KM)                                                                                  \
    do {                                                                                                     \
        if (sub)                                                                                             \
            hipLaunchKernelGGL((tmm::k_step_members<NT, KM, tmm::kMembersEll, true>), grid, blk, 0,          \
                               h->launch_stream(), g, md, mt, h->P.ncol, nb, j, dtd, order, y, yo, nt);          \
        else if (h->P.ew <= 5)                                                                               \
            hipLaunchKernelGGL((tmm::k_step_members<NT, KM, 5>), grid, blk, 0, h->launch_stream(), g, md, mt, h->P.ncol,  \
                               nb, j, dtd, order, y, yo, nt);                                                    \
        else                                                                                                 \
            hipLaunchKernelGGL((tmm::k_step_members<NT, KM, tmm::kMembersEll>), grid, blk, 0, h->launch_stream(), g, md,  \
                               mt, h->P.ncol, nb, j, dtd, order, y, yo, nt);                                     \
    } while (0)
#define TMM_MEMBERS_W(KM, WV)                                                                                \
    hipLaunchKernelGGL((tmm::k_step_members<2, KM, 5, false, WV>), grid, blk, 0, h->launch_stream(), g, md, mt, \
                       h->P.ncol, nb, j, dtd, order, y, yo, nt)
        if (wave_opt && waves != tmm::kMembersWaves) {
            if (waves == 2) {
                if (kmax == 16) TMM_MEMBERS_W(16, 2);
                else if (kmax == 24) TMM_MEMBERS_W(24, 2);
                else TMM_MEMBERS_W(32, 2);
            } else {
                if (kmax == 16) TMM_MEMBERS_W(16, 8);
                else if (kmax == 24) TMM_MEMBERS_W(24, 8);
                else TMM_MEMBERS_W(32, 8);
            }
        } else if (h->P.ntr == 2) {
            if (kmax == 16) TMM_MEMBERS(2, 16);
            else if (kmax == 24) TMM_MEMBERS(2, 24);
            else TMM_MEMBERS(2, 32);
        } else {
            if (kmax == 16) TMM_MEMBERS(1, 16);
            else if (kmax == 24) TMM_MEMBERS(1, 24);
            else TMM_MEMBERS(1, 32);
        }
#undef TMM_MEMBERS
#undef TMM_MEMBERS_W
        TMM_LAUNCHED();
        return TMM_OK;
    }
    const Tiling& t = h->tiling_for(W, tangent ? 2 : 1);
    const int CW = W == 1 ? 1 : 2;
    const int tpr = (W + CW - 1) / CW;
    const int block = W <= 4 ? 128 : 256;
    const size_t lds = (size_t)t.max_rows * W * 8 * (tangent ? 2 : 1);
    const double dtd = tmm::kDaysPerYear / h->P.nstep;
    tmm::Grid g = h->grid(t);
    tmm::Model md = h->model();
    tmm::Mats mt = h->mats();
    dim3 grid(t.ntile), blk(block);
    // PO4-DOP-PHY has W >= 3, so its internal-step instance exists for CW = 2 only
    const bool sub_phy = sub && h->P.ntr == 3;
    if (sub_phy && CW != 2) return TMM_EUNSUPPORTED;
#define TMM_STEP(C, T)                                                                                       \
    do {                                                                                                     \
        if (sub_phy)                                                                                         \
            hipLaunchKernelGGL((tmm::k_step<C, T, kMaxTileRows, kMaxTileRows, (C == 2 ? 3 : 1)>), grid, blk, \
                               lds, h->launch_stream(), g, md, mt, W, tpr, j, dtd, y, yo, v, vo);            \
        else if (sub)                                                                                        \
            hipLaunchKernelGGL((tmm::k_step<C, T, kMaxTileRows, kMaxTileRows, 1>), grid, blk, lds,          \
                               h->launch_stream(), g, md, mt, W, tpr, j, dtd, y, yo, v, vo);                 \
        else                                                                                                 \
            hipLaunchKernelGGL((tmm::k_step<C, T, kMaxTileRows, kMaxTileRows>), grid, blk, lds,             \
                               h->launch_stream(), g, md, mt, W, tpr, j, dtd, y, yo, v, vo);                 \
    } while (0)
    if (CW == 1 && !tangent) TMM_STEP(1, false);
    else if (CW == 1) TMM_STEP(1, true);
    else if (!tangent) TMM_STEP(2, false);
    else TMM_STEP(2, true);
#undef TMM_STEP
    TMM_LAUNCHED();
    return TMM_OK;
}

// Persistent kernels by tracers, tangent, block-row bound and internal BGC
// steps (sn = 0: one evaluation per step; else the euphotic register width);
// 512-thread workgroups exist for 16-row blocks only.
template <int NTR, int KMAX, int TPB>
const void* persistent_kernel_of(bool tangent, int sn, bool ql) {
    if (sn == 0 && ql) return tangent ? (const void*)&tmm::k_year_persistent<NTR, true, KMAX, TPB, 0, true>
                                      : (const void*)&tmm::k_year_persistent<NTR, false, KMAX, TPB, 0, true>;
    if (sn == 2) return tangent ? (const void*)&tmm::k_year_persistent<NTR, true, KMAX, TPB, 2>
                                : (const void*)&tmm::k_year_persistent<NTR, false, KMAX, TPB, 2>;
    if (sn == 4) return tangent ? (const void*)&tmm::k_year_persistent<NTR, true, KMAX, TPB, 4>
                                : (const void*)&tmm::k_year_persistent<NTR, false, KMAX, TPB, 4>;
    return tangent ? (const void*)&tmm::k_year_persistent<NTR, true, KMAX, TPB>
                   : (const void*)&tmm::k_year_persistent<NTR, false, KMAX, TPB>;
}

const void* persistent_kernel(int ntr, bool tangent, int kmax, int tpb, int sn, bool ql = false) {
    if (ntr == 3) {    // PO4-DOP-PHY
        if (tpb == 512) return persistent_kernel_of<3, 16, 512>(tangent, sn, ql);
        if (kmax == 16) return persistent_kernel_of<3, 16, 256>(tangent, sn, ql);
        return persistent_kernel_of<3, 32, 256>(tangent, sn, ql);
    }
    if (tpb == 512)
        return ntr == 1 ? persistent_kernel_of<1, 16, 512>(tangent, sn, ql)
                        : persistent_kernel_of<2, 16, 512>(tangent, sn, ql);
    if (kmax == 16)
        return ntr == 1 ? persistent_kernel_of<1, 16, 256>(tangent, sn, ql)
                        : persistent_kernel_of<2, 16, 256>(tangent, sn, ql);
    return ntr == 1 ? persistent_kernel_of<1, 32, 256>(tangent, sn, ql) : persistent_kernel_of<2, 32, 256>(tangent, sn, ql);
}

template <int NTR, int KMAX, int TPB>
const void* adjoint_kernel_of(int sn) {
    if (sn == 2) return (const void*)&tmm::k_adjoint_persistent<NTR, KMAX, TPB, 2>;
    if (sn == 4) return (const void*)&tmm::k_adjoint_persistent<NTR, KMAX, TPB, 4>;
    return (const void*)&tmm::k_adjoint_persistent<NTR, KMAX, TPB>;
}

const void* adjoint_kernel(int ntr, int kmax, int tpb, int sn) {
    if (ntr == 3)
        return tpb == 512 ? adjoint_kernel_of<3, 16, 512>(sn)
                          : kmax == 16 ? adjoint_kernel_of<3, 16, 256>(sn) : adjoint_kernel_of<3, 32, 256>(sn);
    if (tpb == 512) return ntr == 1 ? adjoint_kernel_of<1, 16, 512>(sn) : adjoint_kernel_of<2, 16, 512>(sn);
    if (kmax == 16) return ntr == 1 ? adjoint_kernel_of<1, 16, 256>(sn) : adjoint_kernel_of<2, 16, 256>(sn);
    return ntr == 1 ? adjoint_kernel_of<1, 32, 256>(sn) : adjoint_kernel_of<2, 32, 256>(sn);
}

// Internal-step variant of the persistent kernels for a plan.
int persistent_sn(const Plan& P) { return P.nsub > 1 ? (P.neu <= 2 ? 2 : 4) : 0; }

// Dynamic LDS of the persistent adjoint: mu of the own rows and of the halo,
// then the internal-step states of every row.
size_t adjoint_dyn_lds(const Plan& P, int tpb, int halo_max) {
    return (size_t)(tpb + halo_max) * P.ntr * 8 + (P.nsub > 1 ? (size_t)P.nsub * tpb * P.ntr * 8 : 0);
}

tmm::Persist persist_args(tmm_ctx* h) {
    const Plan& P = h->P;
    tmm::Persist ps;
    ps.block_dom = h->at<int>(P.o_pblock);
    ps.dom_col = h->at<int>(P.o_pdomcol);
    ps.dep_ptr = h->at<int>(P.o_pdepptr);
    ps.dep_idx = h->at<int>(P.o_pdepidx);
    ps.flags = h->at<int>(P.o_pflags);
    ps.abort_flag = h->at<int>(P.o_pabort);
    ps.spin_limit = h->spin_limit;
    ps.ring = h->at<double>(P.o_ring);
    ps.vring = h->at<double>(P.o_vring);
    ps.halo_ptr = h->at<int>(P.o_phaloptr);
    ps.halo_row = h->at<int>(P.o_phalo);
    ps.halo_max = h->pers_hmax;
    ps.ahalo_ptr = h->at<int>(P.o_pahaloptr);
    ps.ahalo_row = h->at<int>(P.o_pahalo);
    ps.ahalo_max = h->pers_ahmax;
    ps.qlat = h->at<int>(P.o_pqlat);
    ps.qlat_max = h->pers_qmax;
    ps.col_slot = h->at<int>(P.o_pcolslot);
    ps.wave_local = h->pers_wave_local ? 1 : 0;
    return ps;
}

int reset_flags(tmm_ctx* h) {
    hipLaunchKernelGGL(tmm::k_fill_int, dim3((h->pers_G + 255) / 256), dim3(256), 0, h->stream,
                       h->at<int>(h->P.o_pflags), h->pers_G, 0);
    TMM_LAUNCHED();
    return TMM_OK;
}

// Steps sr.j0 .. sr.j1-1 in one cooperative launch (one member).
int launch_persistent(tmm_ctx* h, tmm::StepRange sr, const double* y, double* out, const double* v = nullptr,
                      double* vout = nullptr) {
    const Plan& P = h->P;
    int rc = reset_flags(h);
    if (rc) return rc;
    // ring slot 0 = the initial state, the others the sentinel
    const size_t slen = (size_t)P.n * P.ntr, ring_len = (size_t)tmm::kRingK * slen;   // slots 0 .. K-1
    hipLaunchKernelGGL(tmm::k_ring_init, dim3(launch_blocks(ring_len)), dim3(256), 0, h->stream,
                       h->at<double>(P.o_ring), y, P.n, P.ntr, ring_len);
    TMM_LAUNCHED();
    if (v) {
        hipLaunchKernelGGL(tmm::k_ring_init, dim3(launch_blocks(ring_len)), dim3(256), 0, h->stream,
                           h->at<double>(P.o_vring), v, P.n, P.ntr, ring_len);
        TMM_LAUNCHED();
    }
    tmm::Grid g = h->grid(h->tilings.front());
    tmm::Model md = h->model();
    tmm::Mats mt = h->mats();
    tmm::Persist ps = persist_args(h);
    double dtd = tmm::kDaysPerYear / P.nstep;
    void* args[] = {&g, &md, &mt, &ps, &sr, &dtd, &y, &out, &v, &vout};
    const bool ql = h->pers_ql[v != nullptr ? 1 : 0];
    TMM_TRY(hipLaunchCooperativeKernel(persistent_kernel(P.ntr, v != nullptr, h->pers_kmax, h->pers_tpb, persistent_sn(P),
                                                         ql),
                                       dim3(h->pers_G), dim3(h->pers_tpb), args,
                                       tmm::year_kernel_dyn_lds(h->pers_tpb, h->pers_hmax, P.ntr, v != nullptr,
                                                                ql ? h->pers_qmax : 0, P.nstep),
                                       h->stream));
    h->pers_used = true;
    return TMM_OK;
}

int launch_persistent_year(tmm_ctx* h, const double* y, double* out, const double* v, double* vout) {
    tmm::StepRange sr{0, h->P.nstep, nullptr, 1, nullptr, nullptr};
    return launch_persistent(h, sr, y, out, v, vout);
}

// Reverse sweep over steps j_hi-1 .. j_lo in one cooperative launch.
int launch_adjoint_persistent(tmm_ctx* h, int j_lo, int j_hi, const double* ystore, const double* obs,
                              double src_scale, const double* mu_in, double* mu_out, double* ubar_dom) {
    const Plan& P = h->P;
    int rc = reset_flags(h);
    if (rc) return rc;
    // the cotangent uses the forward kernel's ring (launches never overlap)
    const size_t slen = (size_t)P.n * P.ntr, ring_len = (size_t)tmm::kRingK * slen;   // slots 0 .. K-1
    hipLaunchKernelGGL(tmm::k_ring_init, dim3(launch_blocks(ring_len)), dim3(256), 0, h->stream,
                       h->at<double>(P.o_ring), mu_in, P.n, P.ntr, ring_len);
    TMM_LAUNCHED();
    tmm::Grid g = h->grid(h->tilings.front());
    tmm::Model md = h->model();
    tmm::Mats mt = h->mats();
    tmm::Persist ps = persist_args(h);
    double dtd = tmm::kDaysPerYear / P.nstep;
    void* args[] = {&g, &md, &mt, &ps, &dtd, &j_lo, &j_hi, &ystore, &obs, &src_scale, &mu_in, &mu_out, &ubar_dom};
    TMM_TRY(hipLaunchCooperativeKernel(adjoint_kernel(P.ntr, h->pers_kmax, h->pers_tpb, persistent_sn(P)),
                                       dim3(h->pers_G), dim3(h->pers_tpb), args,
                                       adjoint_dyn_lds(P, h->pers_tpb, h->pers_ahmax), h->stream));
    h->pers_used = true;
    return TMM_OK;
}

// After the persistent launches of a call: a set abort flag means a wait
// gave up in one of them.  It is reported once and cleared, so the next call
// starts afresh.
int check_abort(tmm_ctx* h) {
    if (!h->pers_used) return TMM_OK;
    int flag = 0;
    TMM_TRY(hipMemcpyAsync(&flag, h->at<int>(h->P.o_pabort), 4, hipMemcpyDeviceToHost, h->stream));
    TMM_TRY(hipStreamSynchronize(h->stream));
    h->pers_used = false;
    if (!flag) return TMM_OK;
    hipLaunchKernelGGL(tmm::k_fill_int, dim3(1), dim3(64), 0, h->stream, h->at<int>(h->P.o_pabort), 16, 0);
    TMM_LAUNCHED();
    TMM_TRY(hipStreamSynchronize(h->stream));
    return TMM_EDEVICE;
}

// After the model years of a call: a set non-finite flag means some year
// ended with a NaN or an infinity in its state.  Reported once and cleared.
int take_nonfinite(tmm_ctx* h) {
    int flag = 0;
    TMM_TRY(hipMemcpyAsync(&flag, h->at<int>(h->P.o_finite), 4, hipMemcpyDeviceToHost, h->stream));
    TMM_TRY(hipStreamSynchronize(h->stream));
    if (!flag) return TMM_OK;
    hipLaunchKernelGGL(tmm::k_fill_int, dim3(1), dim3(64), 0, h->stream, h->at<int>(h->P.o_finite), 16, 0);
    TMM_LAUNCHED();
    TMM_TRY(hipStreamSynchronize(h->stream));
    return TMM_ENONFINITE;
}

// One model year of the launch-per-step path replayed from a hipGraph: the
// 2880 step launches of a given (members, buffers) combination are captured
// once on a private stream and replayed on the handle's stream afterwards.
// The graphs hold kernel nodes only.
constexpr size_t kMaxYearGraphs = 8;

int run_year_graph(tmm_ctx* h, int nb, const double* y, double* out, double* a, double* b) {
    const void* key[4] = {y, out, a, b};
    tmm_ctx::YearGraph* hit = nullptr;
    for (auto& gr : h->graphs)
        if (gr.nb == nb && std::equal(key, key + 4, gr.ptrs)) hit = &gr;
    if (!hit) {
        if (!h->capture_stream) TMM_TRY(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
        if (h->graphs.size() >= kMaxYearGraphs) {     // evict the least recently used
            auto lru = std::min_element(h->graphs.begin(), h->graphs.end(),
                                        [](const tmm_ctx::YearGraph& p, const tmm_ctx::YearGraph& q) {
                                            return p.used < q.used;
                                        });
            TMM_TRY(hipGraphExecDestroy(lru->exec));
            h->graphs.erase(lru);
        }
        TMM_TRY(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
        h->capturing = true;
        int rc = TMM_OK;
        const double* cur = y;
        for (int j = 0; j < h->P.nstep && rc == TMM_OK; ++j) {
            double* nxt = j == h->P.nstep - 1 ? out : (j % 2 == 0 ? a : b);
            rc = launch_step(h, j, nb, cur, nxt, nullptr, nullptr);
            cur = nxt;
        }
        h->capturing = false;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(h->capture_stream, &graph);
        if (rc != TMM_OK || e != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc != TMM_OK ? rc : TMM_EDEVICE;
        }
        tmm_ctx::YearGraph gr;
        gr.nb = nb;
        std::copy(key, key + 4, gr.ptrs);
        e = hipGraphInstantiate(&gr.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return TMM_EDEVICE;
        h->graphs.push_back(gr);
        hit = &h->graphs.back();
    }
    hit->used = ++h->graph_clock;
    TMM_TRY(hipGraphLaunch(hit->exec, h->stream));
    return TMM_OK;
}

// One model year for nb slots from y to out, ping-ponging through a, b.  The
// last step writes out directly.  Tangent when v != nullptr (vout, va, vb).
// One member on a handle with the persistent tables runs as one persistent
// launch; otherwise one launch per step.
int run_year(tmm_ctx* h, int nb, const double* y, double* out, double* a, double* b,
             const double* v = nullptr, double* vout = nullptr, double* va = nullptr, double* vb = nullptr) {
    if (nb == 1 && h->pers_ok && h->pers_enabled) return launch_persistent_year(h, y, out, v, vout);
    if (!v && h->graphs_enabled) return run_year_graph(h, nb, y, out, a, b);
    const double* cur = y;
    const double* vcur = v;
    for (int j = 0; j < h->P.nstep; ++j) {
        const bool last = j == h->P.nstep - 1;
        double* nxt = last ? out : (j % 2 == 0 ? a : b);
        double* vnxt = v ? (last ? vout : (j % 2 == 0 ? va : vb)) : nullptr;
        int rc = launch_step(h, j, nb, cur, nxt, vcur, vnxt);
        if (rc) return rc;
        cur = nxt;
        vcur = vnxt;
    }
    return TMM_OK;
}

// The largest dynamic LDS any handle on a device has needed of a kernel: the
// attribute is a limit of the kernel, shared by every handle, so it only grows
// (a handle never lowers it below what another one launches with).
int ensure_dyn_lds(const void* fk, size_t dyn) {
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, size_t> granted;
    int dev = 0;
    TMM_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    size_t& cur = granted[{dev, fk}];
    if (dyn <= cur) return TMM_OK;
    TMM_TRY(hipFuncSetAttribute(fk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    cur = dyn;
    return TMM_OK;
}

// Domains for the persistent kernel: contiguous runs of water columns with
// about n/G rows each (at most the workgroup size), the domains each one must
// wait for (both directions of every explicit-matrix coupling), and an
// XCD-aware block order (consecutive domains on the same XCD, assuming the
// round-robin dispatch of workgroups over the 8 XCDs).
int build_persistent(tmm_ctx* h, int target_rows) {
    const Plan& P = h->P;
    int dev = 0, coop = 0, ncu = 0;
    TMM_TRY(hipGetDevice(&dev));
    TMM_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    TMM_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    h->num_cu = ncu;
    h->pers_ok = false;
    h->pers_adj_ok = false;
    h->pers_target = target_rows;
    if (!coop || !P.o_ring || P.ew > tmm::kEllMax || P.nlayer > 32 || P.neu > tmm::kNeuMax) return TMM_OK;
    h->pers_kmax = P.nlayer <= 16 ? 16 : 32;
    if (target_rows < 1) target_rows = kDefaultDomainRows;
    // 512-thread workgroups only where the row's Ai block fits the halved register budget
    const int tpb = (target_rows > 256 && h->pers_kmax == 16) ? tmm::kPersistThreadsMax : 256;
    target_rows = std::min(target_rows, tpb);
    // co-residency of the forward kernels (both modes) and, separately, of the adjoint
    const int sn = persistent_sn(P);
    int occ = 0, occ_adj = 0;
    // the forward kernels' dynamic LDS at the largest halo the domains may have
    const size_t halo_cap = (size_t)tmm::kHaloPerThread * tpb;
    int lds_max = 0;
    TMM_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    for (int t = 0; t < 2; ++t) {
        const void* fk = persistent_kernel(P.ntr, t, h->pers_kmax, tpb, sn);
        const size_t dyn = tmm::year_kernel_dyn_lds(tpb, (int)halo_cap, P.ntr, t, 0, 0);
        hipFuncAttributes attr;
        TMM_TRY(hipFuncGetAttributes(&attr, fk));
        if (attr.sharedSizeBytes + dyn > (size_t)lds_max) return TMM_OK;
        TMM_TRY(ensure_dyn_lds(fk, dyn));
        int o = 0;
        TMM_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, fk, tpb, dyn));
        occ = t == 0 ? o : std::min(occ, o);
    }
    {
        // the internal-step store of the adjoint is dynamic LDS beside the static arrays
        const void* fa = adjoint_kernel(P.ntr, h->pers_kmax, tpb, sn);
        const size_t dyn = adjoint_dyn_lds(P, tpb, (int)halo_cap);
        hipFuncAttributes attr;
        TMM_TRY(hipFuncGetAttributes(&attr, fa));
        if (attr.sharedSizeBytes + dyn <= (size_t)lds_max) {
            if (dyn > 0) TMM_TRY(ensure_dyn_lds(fa, dyn));
            TMM_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_adj, fa, tpb, dyn));
        }
    }
    const int maxG = std::min(kMaxDomains, std::min(ncu * occ, P.ncol));
    if (maxG < 1) return TMM_OK;
    int G = std::min(maxG, std::max(1, (P.n + target_rows - 1) / target_rows));
    std::vector<int> dom;
    // slots of a domain's columns with none spanning two wavefronts (a column
    // that would starts the next one); returns the slots used
    std::vector<int> col_slot(P.ncol, 0);
    auto place = [&](int cb, int ce, bool wave_local) {
        int slot = 0;
        for (int c = cb; c < ce; ++c) {
            const int nc = P.col_start[c + 1] - P.col_start[c];
            if (wave_local && slot / 64 != (slot + nc - 1) / 64) slot = (slot / 64 + 1) * 64;
            col_slot[c] = slot;
            slot += nc;
        }
        return slot;
    };
    bool wave_local = false;
    for (;;) {
        dom.assign(1, 0);
        long long rows = 0;
        for (int c = 0; c < P.ncol; ++c) {
            rows += P.col_start[c + 1] - P.col_start[c];
            const long long target = (long long)P.n * (long long)dom.size() / G;
            if (rows >= target && (int)dom.size() < G && c + 1 < P.ncol) dom.push_back(c + 1);
        }
        dom.push_back(P.ncol);
        int maxrows = 0, maxslots = 0;
        for (size_t i = 0; i + 1 < dom.size(); ++i) {
            maxrows = std::max(maxrows, P.col_start[dom[i + 1]] - P.col_start[dom[i]]);
            maxslots = std::max(maxslots, place(dom[i], dom[i + 1], true));
        }
        // wave-aligned columns where the domains allow it (more, smaller
        // domains if needed), else packed columns
        if (h->wave_local_enabled && maxslots <= tpb) {
            wave_local = true;
            break;
        }
        if (G >= maxG || !h->wave_local_enabled) {
            if (maxrows > tpb) {
                if (G >= maxG) return TMM_OK;         // does not fit: per-step path only
            } else {
                break;
            }
        }
        G = std::min(maxG, G + std::max(1, G / 8));
    }
    G = (int)dom.size() - 1;
    for (int q = 0; q < G; ++q) place(dom[q], dom[q + 1], wave_local);
    std::vector<int> row_dom(P.n);
    for (int q = 0; q < G; ++q)
        for (int r = P.col_start[dom[q]]; r < P.col_start[dom[q + 1]]; ++r) row_dom[r] = q;
    std::vector<std::vector<int>> deps(G);
    for (int i = 0; i < P.n; ++i)
        for (int e = h->ae_rowptr[i]; e < h->ae_rowptr[i + 1]; ++e) {
            const int a = row_dom[i], b = row_dom[h->ae_colidx[e]];
            if (a != b) {
                deps[a].push_back(b);
                deps[b].push_back(a);
            }
        }
    std::vector<int> dep_ptr(G + 1, 0), dep_idx;
    for (int q = 0; q < G; ++q) {
        std::sort(deps[q].begin(), deps[q].end());
        deps[q].erase(std::unique(deps[q].begin(), deps[q].end()), deps[q].end());
        dep_idx.insert(dep_idx.end(), deps[q].begin(), deps[q].end());
        dep_ptr[q + 1] = (int)dep_idx.size();
    }
    if (dep_idx.size() > P.dep_capacity) return TMM_OK;
    if (dep_idx.empty()) dep_idx.push_back(0);
    // halo of each domain: the rows of other domains its Ae rows read, ascending
    std::vector<int> halo_ptr(G + 1, 0), halo;
    int hmax = 0;
    for (int q = 0; q < G; ++q) {
        std::vector<int> hq;
        for (int i = P.col_start[dom[q]]; i < P.col_start[dom[q + 1]]; ++i)
            for (int e = h->ae_rowptr[i]; e < h->ae_rowptr[i + 1]; ++e)
                if (row_dom[h->ae_colidx[e]] != q) hq.push_back(h->ae_colidx[e]);
        std::sort(hq.begin(), hq.end());
        hq.erase(std::unique(hq.begin(), hq.end()), hq.end());
        if (hq.size() > halo_cap) return TMM_OK;          // does not fit: per-step path only
        hmax = std::max(hmax, (int)hq.size());
        halo.insert(halo.end(), hq.begin(), hq.end());
        halo_ptr[q + 1] = (int)halo.size();
    }
    if (halo.size() > P.halo_capacity) return TMM_OK;
    if (halo.empty()) halo.push_back(0);
    // halo of the transposed stencil: row i of Ae^T reads mu at the rows whose
    // Ae rows have an entry in column i
    std::vector<std::vector<int>> ah(G);
    for (int i = 0; i < P.n; ++i)
        for (int e = h->ae_rowptr[i]; e < h->ae_rowptr[i + 1]; ++e) {
            const int q = row_dom[h->ae_colidx[e]];
            if (row_dom[i] != q) ah[q].push_back(i);
        }
    std::vector<int> ahalo_ptr(G + 1, 0), ahalo;
    int ahmax = 0;
    bool ahalo_ok = true;
    for (int q = 0; q < G; ++q) {
        std::sort(ah[q].begin(), ah[q].end());
        ah[q].erase(std::unique(ah[q].begin(), ah[q].end()), ah[q].end());
        if (ah[q].size() > halo_cap) ahalo_ok = false;
        ahmax = std::max(ahmax, (int)ah[q].size());
        ahalo.insert(ahalo.end(), ah[q].begin(), ah[q].end());
        ahalo_ptr[q + 1] = (int)ahalo.size();
    }
    if (ahalo.size() > P.halo_capacity) ahalo_ok = false;
    if (!ahalo_ok) {                                      // the reverse sweep falls back to per-step kernels
        ahmax = 0;
        ahalo.assign(1, 0);
        std::fill(ahalo_ptr.begin(), ahalo_ptr.end(), 0);
    }
    if (ahalo.empty()) ahalo.push_back(0);
    // latitude rows of each domain's columns: without internal BGC steps the
    // forward kernels keep the insolation of those rows for the whole year in
    // LDS beside their halo, where it fits (else they load it every step)
    std::vector<int> qlat((size_t)G * (1 + tmm::kInsLat), 0);
    int qmax = 0;
    bool ql = sn == 0;
    for (int q = 0; q < G && ql; ++q) {
        int* e = qlat.data() + (size_t)q * (1 + tmm::kInsLat);
        for (int c = dom[q]; c < dom[q + 1] && ql; ++c) {
            const int l = P.col_lat[c];
            bool seen = false;
            for (int i = 0; i < e[0]; ++i) seen = seen || e[1 + i] == l;
            if (seen) continue;
            if (e[0] == tmm::kInsLat) ql = false;
            else e[1 + e[0]++] = l;
        }
        qmax = std::max(qmax, e[0]);
    }
    // decided per mode: the tangent's larger LDS may not leave room for the
    // table (or for the co-residency of all domains) where the state's does
    bool ql_mode[2] = {ql, ql};
    for (int t = 0; t < 2 && ql; ++t) {
        const void* fk = persistent_kernel(P.ntr, t, h->pers_kmax, tpb, sn, true);
        const size_t dyn = tmm::year_kernel_dyn_lds(tpb, hmax, P.ntr, t, qmax, P.nstep);
        hipFuncAttributes attr;
        TMM_TRY(hipFuncGetAttributes(&attr, fk));
        if (attr.sharedSizeBytes + dyn > (size_t)lds_max) {
            ql_mode[t] = false;
            continue;
        }
        TMM_TRY(ensure_dyn_lds(fk, dyn));
        int o = 0;
        TMM_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, fk, tpb, dyn));
        if ((long long)ncu * o < G) ql_mode[t] = false;
    }
    if (!ql_mode[0] && !ql_mode[1]) qmax = 0;
    std::vector<int> block_dom(G);
    {
        int next = 0;
        for (int x = 0; x < 8; ++x)
            for (int b = x; b < G; b += 8) block_dom[b] = next++;
    }
    if (upload(h, h->at<int>(P.o_pblock), block_dom.data(), (size_t)G * 4) ||
        upload(h, h->at<int>(P.o_pdomcol), dom.data(), dom.size() * 4) ||
        upload(h, h->at<int>(P.o_pdepptr), dep_ptr.data(), dep_ptr.size() * 4) ||
        upload(h, h->at<int>(P.o_pdepidx), dep_idx.data(), dep_idx.size() * 4) ||
        upload(h, h->at<int>(P.o_phaloptr), halo_ptr.data(), halo_ptr.size() * 4) ||
        upload(h, h->at<int>(P.o_phalo), halo.data(), halo.size() * 4) ||
        upload(h, h->at<int>(P.o_pahaloptr), ahalo_ptr.data(), ahalo_ptr.size() * 4) ||
        upload(h, h->at<int>(P.o_pahalo), ahalo.data(), ahalo.size() * 4) ||
        upload(h, h->at<int>(P.o_pqlat), qlat.data(), qlat.size() * 4) ||
        upload(h, h->at<int>(P.o_pcolslot), col_slot.data(), col_slot.size() * 4))
        return TMM_EDEVICE;
    hipLaunchKernelGGL(tmm::k_fill_int, dim3(1), dim3(64), 0, h->stream, h->at<int>(P.o_pabort), 16, 0);
    TMM_LAUNCHED();
    TMM_TRY(hipStreamSynchronize(h->stream));
    h->pers_G = G;
    h->pers_tpb = tpb;
    h->pers_hmax = hmax;
    h->pers_ahmax = ahmax;
    h->pers_qmax = qmax;
    h->pers_ql[0] = ql_mode[0];
    h->pers_ql[1] = ql_mode[1];
    h->pers_wave_local = wave_local;
    h->pers_ok = true;
    h->pers_adj_ok = ahalo_ok && (long long)ncu * occ_adj >= G;
    return TMM_OK;
}

// part[tile][slot] = sum of weight*(a-b)^2 per slot, then out[slot] = scale*sum (sqrt optional).
int sqdiff(tmm_ctx* h, int nb, const double* a, const double* b, int volume, double scale, int take_sqrt,
           double* out, int accumulate = 0, double* part = nullptr, int part_stride_tiles = 0) {
    const Tiling& t = h->tilings.front();
    tmm::Grid g = h->grid(t);
    double* pp = part ? part : h->part();
    hipLaunchKernelGGL((tmm::k_tile_sqdiff<kMaxTileRows, kMaxTileRows>), dim3(t.ntile), dim3(256), 0, h->stream,
                       g, nb * h->P.ntr, h->P.ntr, nb, a, b, volume, pp);
    TMM_LAUNCHED();
    (void)part_stride_tiles;
    if (out) {
        hipLaunchKernelGGL(tmm::k_sum_tiles, dim3(1), dim3(256), 0, h->stream, t.ntile, nb, nb, pp, scale,
                           accumulate, take_sqrt, out);
        TMM_LAUNCHED();
    }
    return TMM_OK;
}



// Checkpointed adjoint of one model year for one member with persistent
// launches: a forward sweep storing y every ckpt steps and the month-end
// misfit sums; the misfit source of the last month and Ai^T for the last
// step; then per segment, last first, a forward replay storing every state
// and a reverse sweep over the segment.  The forward sweep writes the last
// segment's states straight into the segment store, so that segment is not
// replayed; with one segment (ckpt = nstep) nothing is.
int adjoint_persistent(tmm_ctx* h, const double* y0, const double* obs, double* J_host, double* dJdu_host,
                       double* dJdy0) {
    const Plan& P = h->P;
    const int np = P.nparam, G = h->pers_G;
    const size_t len = (size_t)P.n * P.ntr;
    const int K = P.ckpt, nseg = P.nstep / K;
    const double dtd = tmm::kDaysPerYear / P.nstep;
    double* ckpt = h->at<double>(P.o_ckpt);
    double* seg = h->at<double>(P.o_seg);
    double* fin = h->at<double>(P.o_final);
    double* mu[2] = {h->at<double>(P.o_mu[0]), h->at<double>(P.o_mu[1])};
    double* ubar = h->at<double>(P.o_pubar);
    double* jpart = h->at<double>(P.o_pjpart);
    int rc;
    if ((rc = fill(h, ubar, (size_t)G * np, 0.0)) || (rc = fill(h, jpart, (size_t)P.nmat * G, 0.0))) return rc;
    // forward sweep: checkpoints y_{sK} at slot s up to the last segment, whose
    // states y_lo .. y_{nstep-1} go to the segment store; misfit partial sums
    const int lo_last = (nseg - 1) * K;
    const double* ylast = y0;
    if (nseg > 1) {
        tmm::StepRange fw{0, lo_last, ckpt, K, obs, jpart};
        double* yl = ckpt + (size_t)(nseg - 1) * len;
        if ((rc = launch_persistent(h, fw, y0, yl)))
            return rc;
        ylast = yl;
    }
    {
        tmm::StepRange fl{lo_last, P.nstep, seg, 1, obs, jpart};
        if ((rc = launch_persistent(h, fl, ylast, fin)))
            return rc;
    }
    hipLaunchKernelGGL(tmm::k_sum_tiles, dim3(1), dim3(64), 0, h->stream, P.nmat * G, 1, 1, jpart,
                       1.0 / (2.0 * P.nmat * h->vtot), 0, 0, h->vec(4));
    TMM_LAUNCHED();
    // head: lambda_nstep = source of the last month, mu_{nstep-1} = Ai(t_{nstep-1})^T lambda_nstep
    {
        const Tiling& tl = h->tiling_for(P.ntr, 1, 256 * 8 * np);
        tmm::Grid g = h->grid(tl);
        tmm::Model md = h->model();
        tmm::Mats mt = h->mats();
        const size_t lds = (size_t)tl.max_rows * P.ntr * 8 + (size_t)256 * np * 8;
        const double sc = 1.0 / (P.nmat * h->vtot);
        const double* ob = obs + (size_t)(P.nmat - 1) * len;
        if (P.ntr == 3)
            hipLaunchKernelGGL((tmm::k_adjoint<3, kMaxTileRows, kMaxTileRows>), dim3(tl.ntile), dim3(256), lds,
                               h->stream, g, md, mt, P.ntr, 1, P.nstep, dtd, 0, 1, nullptr, fin, ob, sc, mu[0],
                               nullptr);
        else if (P.ntr == 2)
            hipLaunchKernelGGL((tmm::k_adjoint<2, kMaxTileRows, kMaxTileRows>), dim3(tl.ntile), dim3(256), lds,
                               h->stream, g, md, mt, P.ntr, 1, P.nstep, dtd, 0, 1, nullptr, fin, ob, sc, mu[0],
                               nullptr);
        else
            hipLaunchKernelGGL((tmm::k_adjoint<1, kMaxTileRows, kMaxTileRows>), dim3(tl.ntile), dim3(256), lds,
                               h->stream, g, md, mt, P.ntr, 1, P.nstep, dtd, 0, 1, nullptr, fin, ob, sc, mu[0],
                               nullptr);
        TMM_LAUNCHED();
    }
    int im = 0;
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int lo = sg * K, hi = lo + K;
        // replay: y_lo .. y_{hi-1} into the segment store (the forward sweep
        // left the last segment there)
        tmm::StepRange rp{lo, hi, seg, 1, nullptr, nullptr};
        if (sg < nseg - 1 &&
            (rc = launch_persistent(h, rp, ckpt + (size_t)sg * len, h->ybuf(2))))
            return rc;
        double* out = sg == 0 ? (dJdy0 ? dJdy0 : mu[1 - im]) : mu[1 - im];
        if ((rc = launch_adjoint_persistent(h, lo, hi, seg, obs, 1.0 / (P.nmat * h->vtot), mu[im], out, ubar)))
            return rc;
        im = 1 - im;
    }
    hipLaunchKernelGGL(tmm::k_sum_tiles, dim3(1), dim3(64), 0, h->stream, G, np, np, ubar, 1.0, 0, 0, h->vec(5));
    TMM_LAUNCHED();
    double J = 0.0;
    std::vector<double> Gr(np);
    TMM_TRY(hipMemcpyAsync(&J, h->vec(4), 8, hipMemcpyDeviceToHost, h->stream));
    TMM_TRY(hipMemcpyAsync(Gr.data(), h->vec(5), (size_t)np * 8, hipMemcpyDeviceToHost, h->stream));
    TMM_TRY(hipStreamSynchronize(h->stream));
    if ((rc = check_abort(h))) return rc;
    if (!std::isfinite(J)) return TMM_ENONFINITE;
    J_host[0] = J;
    for (int q = 0; q < np; ++q) {
        if (!std::isfinite(Gr[q])) return TMM_ENONFINITE;
        dJdu_host[q] = Gr[q];
    }
    return TMM_OK;
}

}  // namespace

extern "C" {

const char* tmm_strerror(int status) {
    switch (status) {
        case TMM_OK: return "ok";
        case TMM_EINVAL: return "invalid argument or descriptor";
        case TMM_ENOMEM: return "workspace too small";
        case TMM_EDEVICE: return "HIP runtime error";
        case TMM_ESTATE: return "call not valid in the handle's state";
        case TMM_ENONFINITE: return "non-finite value in a result";
        case TMM_EUNSUPPORTED: return "unsupported request";
        case TMM_ETOOBIG: return "request exceeds the fixed scratch of tmm_year_noalloc";
        default: return "unknown status";
    }
}

int tmm_workspace_bytes(const tmm_desc* desc, size_t* bytes) {
    if (!bytes) return TMM_EINVAL;
    Plan P;
    int rc = validate(desc, P);
    if (rc) return rc;
    *bytes = P.total;
    return TMM_OK;
}

int tmm_create(const tmm_desc* d, void* dev_workspace, size_t bytes, void* hip_stream, tmm_handle* out) {
    if (!out || !dev_workspace) return TMM_EINVAL;
    *out = nullptr;
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) return TMM_EINVAL;
    tmm_ctx* h = new (std::nothrow) tmm_ctx();
    if (!h) return TMM_ENOMEM;
    int rc = validate(d, h->P);
    if (rc) { delete h; return rc; }
    if (bytes < h->P.total) { delete h; return TMM_ENOMEM; }
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->ws = static_cast<char*>(dev_workspace);
    const Plan& P = h->P;
    auto fail = [&](int code) { (void)hipStreamSynchronize(h->stream); delete h; return code; };

    // Ae in slot-major ELL; padding entries point at the row itself with value 0.
    // Slot 0 of row i reads row i: the row's entries in their given order, with
    // the one that reads row i (its diagonal entry, else the first padding entry;
    // the width leaves one for every row without a diagonal) swapped to the front.
    {
        std::vector<int> col((size_t)P.ew * P.npad);
        std::vector<int> pos(d->ae_nnz);
        for (int i = 0; i < P.npad; ++i) {
            const int len = i < P.n ? d->ae_rowptr[i + 1] - d->ae_rowptr[i] : 0;
            int own = i < P.n ? -1 : 0;
            for (int s = 0; s < P.ew && own < 0; ++s)
                if (s >= len || d->ae_colidx[d->ae_rowptr[i] + s] == i) own = s;
            if (own < 0) return fail(TMM_EINVAL);
            for (int s = 0; s < P.ew; ++s) {
                const int from = s == 0 ? own : s == own ? 0 : s;
                const size_t at = (size_t)s * P.npad + i;
                if (from < len) {
                    const int e = d->ae_rowptr[i] + from;
                    col[at] = d->ae_colidx[e];
                    pos[e] = (int)at;
                } else {
                    col[at] = i < P.n ? i : 0;
                }
            }
        }
        if (upload(h, h->at<int>(P.o_aecol), col.data(), col.size() * 4)) return fail(TMM_EDEVICE);
        if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(TMM_EDEVICE);
        h->ell_col = col;
        std::vector<double> val((size_t)P.ew * P.npad);
        for (int m = 0; m < P.nmat; ++m) {
            std::fill(val.begin(), val.end(), 0.0);
            const double* src = d->ae_val + (size_t)m * d->ae_nnz;
            for (int e = 0; e < d->ae_nnz; ++e) val[pos[e]] = src[e];
            if (upload(h, h->at<double>(P.o_ae) + (size_t)m * val.size(), val.data(), val.size() * 8))
                return fail(TMM_EDEVICE);
            if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(TMM_EDEVICE);
        }
        // Ae^T: row c of the transpose lists (i, a_ic) in increasing i
        std::vector<int> tlen(P.npad, 0);
        std::vector<int> tcol((size_t)P.etw * P.npad);
        std::vector<int> tpos(d->ae_nnz);
        for (int i = 0; i < P.n; ++i)
            for (int e = d->ae_rowptr[i]; e < d->ae_rowptr[i + 1]; ++e) {
                const int c = d->ae_colidx[e];
                const size_t at = (size_t)tlen[c]++ * P.npad + c;
                tcol[at] = i;
                tpos[e] = (int)at;
            }
        for (int c = 0; c < P.npad; ++c)
            for (int s = tlen[c]; s < P.etw; ++s) tcol[(size_t)s * P.npad + c] = c < P.n ? c : 0;
        if (upload(h, h->at<int>(P.o_aetcol), tcol.data(), tcol.size() * 4)) return fail(TMM_EDEVICE);
        std::vector<double> tval((size_t)P.etw * P.npad);
        for (int m = 0; m < P.nmat; ++m) {
            std::fill(tval.begin(), tval.end(), 0.0);
            const double* src = d->ae_val + (size_t)m * d->ae_nnz;
            for (int e = 0; e < d->ae_nnz; ++e) tval[tpos[e]] = src[e];
            if (upload(h, h->at<double>(P.o_aet) + (size_t)m * tval.size(), tval.data(), tval.size() * 8))
                return fail(TMM_EDEVICE);
            if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(TMM_EDEVICE);
        }
    }
    // Ai as dense per-column blocks, column-major and row-major.
    {
        std::vector<int> blk(P.ncol), row_col(P.n);
        size_t off = 0;
        for (int c = 0; c < P.ncol; ++c) {
            blk[c] = (int)off;
            const size_t nc = P.col_start[c + 1] - P.col_start[c];
            off += nc * nc;
            for (int r = P.col_start[c]; r < P.col_start[c + 1]; ++r) row_col[r] = c;
        }
        if (upload(h, h->at<int>(P.o_blk), blk.data(), blk.size() * 4)) return fail(TMM_EDEVICE);
        std::vector<double> cm(P.nblk), rm(P.nblk);
        for (int m = 0; m < P.nmat; ++m) {
            std::fill(cm.begin(), cm.end(), 0.0);
            std::fill(rm.begin(), rm.end(), 0.0);
            const double* src = d->ai_val + (size_t)m * d->ai_nnz;
            for (int i = 0; i < P.n; ++i) {
                const int c = row_col[i];
                const int nc = P.col_start[c + 1] - P.col_start[c];
                const int k = i - P.col_start[c];
                for (int e = d->ai_rowptr[i]; e < d->ai_rowptr[i + 1]; ++e) {
                    const int s = d->ai_colidx[e] - P.col_start[c];
                    cm[(size_t)blk[c] + (size_t)s * nc + k] += src[e];
                    rm[(size_t)blk[c] + (size_t)k * nc + s] += src[e];
                }
            }
            if (upload(h, h->at<double>(P.o_aicm) + (size_t)m * P.nblk, cm.data(), P.nblk * 8) ||
                upload(h, h->at<double>(P.o_airm) + (size_t)m * P.nblk, rm.data(), P.nblk * 8))
                return fail(TMM_EDEVICE);
            if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(TMM_EDEVICE);
        }
    }
    if (upload(h, h->at<int>(P.o_colstart), P.col_start.data(), P.col_start.size() * 4) ||
        upload(h, h->at<double>(P.o_lat), d->lat, (size_t)P.ncol * 8) ||
        upload(h, h->at<double>(P.o_area), d->area, (size_t)P.ncol * 8) ||
        upload(h, h->at<double>(P.o_dz), d->dz, (size_t)P.nlayer * 8))
        return fail(TMM_EDEVICE);
    for (size_t t = 0; t < P.tiles_sizes.size(); ++t) {
        Tiling tl;
        tl.max_rows = P.tiles_sizes[t];
        tl.tile_col = make_tiles(P.col_start, tl.max_rows);
        tl.ntile = (int)tl.tile_col.size() - 1;
        tl.d_tile_col = h->at<int>(P.o_tiles[t]);
        if (upload(h, tl.d_tile_col, tl.tile_col.data(), tl.tile_col.size() * 4)) return fail(TMM_EDEVICE);
        h->tilings.push_back(std::move(tl));
    }
    // insolation per step and distinct latitude
    if (upload(h, h->at<int>(P.o_collat), P.col_lat.data(), P.col_lat.size() * 4) ||
        upload(h, h->at<double>(P.o_latu), P.lat_u.data(), P.lat_u.size() * 8))
        return fail(TMM_EDEVICE);
    {
        const int tot = P.nstep * (int)P.lat_u.size();
        hipLaunchKernelGGL(tmm::k_insolation_table, dim3((tot + 255) / 256), dim3(256), 0, h->stream, P.nstep,
                           (int)P.lat_u.size(), h->at<double>(P.o_latu), h->at<double>(P.o_ins));
        if (hipGetLastError() != hipSuccess) return fail(TMM_EDEVICE);
    }
    hipLaunchKernelGGL(tmm::k_fill_int, dim3(1), dim3(64), 0, h->stream, h->at<int>(P.o_finite), 16, 0);
    if (hipGetLastError() != hipSuccess) return fail(TMM_EDEVICE);
    h->ae_rowptr.assign(d->ae_rowptr, d->ae_rowptr + P.n + 1);
    h->ae_colidx.assign(d->ae_colidx, d->ae_colidx + d->ae_nnz);
    if (build_persistent(h, 0)) return fail(TMM_EDEVICE);
    if (build_member_order(h)) return fail(TMM_EDEVICE);
    {
        void* sp = nullptr;
        if (scratch_address(&sp)) return fail(TMM_EDEVICE);
        h->noalloc = static_cast<double*>(sp);
    }
    h->h_member.resize(P.nbatch_max);
    h->h_scol.resize(P.nbatch_max);
    h->h_dcol.resize(P.nbatch_max);
    // total wet volume, for the misfit normalisation
    {
        const Tiling& t = h->tilings.front();
        tmm::Grid g = h->grid(t);
        hipLaunchKernelGGL((tmm::k_tile_volume<kMaxTileRows, kMaxTileRows>), dim3(t.ntile), dim3(256), 0,
                           h->stream, g, h->part());
        hipLaunchKernelGGL(tmm::k_sum_tiles, dim3(1), dim3(64), 0, h->stream, t.ntile, 1, 1, h->part(), 1.0, 0, 0,
                           h->vec(15));
        if (hipGetLastError() != hipSuccess) return fail(TMM_EDEVICE);
        if (hipMemcpyAsync(&h->vtot, h->vec(15), 8, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
            return fail(TMM_EDEVICE);
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(TMM_EDEVICE);
    *out = h;
    return TMM_OK;
}

int tmm_destroy(tmm_handle h) {
    if (!h) return TMM_OK;
    int rc = hipStreamSynchronize(h->stream) == hipSuccess ? TMM_OK : TMM_EDEVICE;
    for (auto& gr : h->graphs)
        if (hipGraphExecDestroy(gr.exec) != hipSuccess) rc = TMM_EDEVICE;
    if (h->capture_stream && hipStreamDestroy(h->capture_stream) != hipSuccess) rc = TMM_EDEVICE;
    delete h;
    return rc;
}

int tmm_set_params(tmm_handle h, int nbatch, const double* u) {
    if (!h || !u || nbatch < 1 || nbatch > h->P.nbatch_max) return TMM_EINVAL;
    const int np = h->P.nparam;
    for (int b = 0; b < nbatch; ++b) {
        const double* p = u + (size_t)b * np;
        for (int i = 0; i < np; ++i)
            if (!std::isfinite(p[i])) return TMM_EINVAL;
        if (p[2] <= 0.0 || p[3] <= 0.0) return TMM_EINVAL;
        if (h->P.model != TMM_MODEL_N && (p[5] < 0.0 || p[5] > 1.0)) return TMM_EINVAL;
        if (h->P.model == TMM_MODEL_NDOPPHY && (p[9] < 0.0 || p[9] > 1.0)) return TMM_EINVAL;
    }
    std::vector<double> uu(u, u + (size_t)nbatch * np);
    if (upload(h, h->at<double>(h->P.o_u), uu.data(), uu.size() * 8)) return TMM_EDEVICE;
    const size_t nbm = (size_t)h->P.nbatch_max;
    std::vector<double> ut(nbm * np, 0.0);
    for (int b = 0; b < nbatch; ++b)
        for (int i = 0; i < np; ++i) ut[(size_t)i * nbm + b] = u[(size_t)b * np + i];
    if (upload(h, h->at<double>(h->P.o_uT), ut.data(), ut.size() * 8)) return TMM_EDEVICE;
    for (int b = 0; b < nbatch; ++b) h->h_member[b] = b;
    if (upload(h, h->at<int>(h->P.o_member), h->h_member.data(), (size_t)nbatch * 4)) return TMM_EDEVICE;
    const int total = nbatch * (h->P.nlayer + 1) * h->P.nlayer;
    hipLaunchKernelGGL(tmm::k_param_tables, dim3((total + 255) / 256), dim3(256), 0, h->stream, nbatch, h->P.model,
                       np, h->P.nlayer, h->P.neu, h->at<double>(h->P.o_u), h->at<double>(h->P.o_dz),
                       h->at<double>(h->P.o_light), h->at<double>(h->P.o_rho), h->at<double>(h->P.o_drho),
                       h->P.nbatch_max, h->at<double>(h->P.o_lightT), h->at<double>(h->P.o_rhoT));
    TMM_LAUNCHED();
    TMM_TRY(hipStreamSynchronize(h->stream));
    h->nbatch = nbatch;
    return TMM_OK;
}

int tmm_step(tmm_handle h, int j, const double* y_in, double* y_out) {
    if (!h || !y_in || !y_out || y_in == y_out || j < 0) return TMM_EINVAL;
    if (h->nbatch < 1) return TMM_ESTATE;
    return launch_step(h, j, h->nbatch, y_in, y_out, nullptr, nullptr);
}

// Member map: slot s of the working state holds member h_member[s].
static int push_member_map(tmm_handle h, int na) {
    if (upload(h, h->at<int>(h->P.o_member), h->h_member.data(), (size_t)na * 4)) return TMM_EDEVICE;
    TMM_TRY(hipStreamSynchronize(h->stream));
    return TMM_OK;
}

int tmm_year(tmm_handle h, int nyears, const int* years_per_member, const double* y0, double* y1,
             double* resid_host) {
    if (!h || !y0 || !y1 || nyears < 0) return TMM_EINVAL;
    const int nb = h->nbatch;
    if (nb < 1) return TMM_ESTATE;
    std::vector<int> left(nb, nyears);
    if (years_per_member)
        for (int b = 0; b < nb; ++b) {
            if (years_per_member[b] < 0 || years_per_member[b] > nyears) return TMM_EINVAL;
            left[b] = years_per_member[b];
        }
    const int ntr = h->P.ntr, Wf = nb * ntr;
    const size_t n = h->P.n;
    if (resid_host) std::fill(resid_host, resid_host + (size_t)nyears * nb, 0.0);

    // working state: slot s holds member active[s]
    std::vector<int> active;
    for (int b = 0; b < nb; ++b) active.push_back(b);
    int ib = 0;                    // ybuf index holding the current state
    int rc = copy(h, h->ybuf(0), y0, n * Wf);
    if (rc) return rc;

    auto scatter_finished = [&](const std::vector<int>& slots, int Wc) -> int {
        // copy finished slots of the working state into their member columns of y1
        int k = 0;
        for (int s : slots) {
            h->h_scol[k] = s;
            h->h_dcol[k] = active[s];
            ++k;
        }
        if (!k) return TMM_OK;
        if (upload(h, h->at<int>(h->P.o_scol), h->h_scol.data(), (size_t)k * 4) ||
            upload(h, h->at<int>(h->P.o_dcol), h->h_dcol.data(), (size_t)k * 4))
            return TMM_EDEVICE;
        hipLaunchKernelGGL(tmm::k_gather_slots, dim3(launch_blocks(n * k * ntr)), dim3(256), 0, h->stream, n, k,
                           ntr, Wc, Wf, h->at<int>(h->P.o_scol), h->at<int>(h->P.o_dcol), h->ybuf(ib), y1);
        TMM_LAUNCHED();
        TMM_TRY(hipStreamSynchronize(h->stream));
        return TMM_OK;
    };

    // members with no years at all keep y0
    {
        std::vector<int> done;
        for (size_t s = 0; s < active.size(); ++s)
            if (left[active[s]] == 0) done.push_back((int)s);
        if (!done.empty()) {
            if ((rc = scatter_finished(done, Wf))) return rc;
        }
    }
    std::vector<int> keep;
    for (size_t s = 0; s < active.size(); ++s)
        if (left[active[s]] > 0) keep.push_back((int)s);
    // compact away members with no years
    if (keep.size() != active.size() && !keep.empty()) {
        const int other = (ib + 1) % 3;
        for (size_t k = 0; k < keep.size(); ++k) { h->h_scol[k] = keep[k]; h->h_dcol[k] = (int)k; }
        if (upload(h, h->at<int>(h->P.o_scol), h->h_scol.data(), keep.size() * 4) ||
            upload(h, h->at<int>(h->P.o_dcol), h->h_dcol.data(), keep.size() * 4))
            return TMM_EDEVICE;
        hipLaunchKernelGGL(tmm::k_gather_slots, dim3(launch_blocks(n * keep.size() * ntr)), dim3(256), 0,
                           h->stream, n, (int)keep.size(), ntr, Wf, (int)keep.size() * ntr,
                           h->at<int>(h->P.o_scol), h->at<int>(h->P.o_dcol), h->ybuf(ib), h->ybuf(other));
        TMM_LAUNCHED();
        std::vector<int> na;
        for (int s : keep) na.push_back(active[s]);
        active = na;
        ib = other;
    }
    if (keep.empty()) active.clear();
    for (size_t s = 0; s < active.size(); ++s) h->h_member[s] = active[s];
    if (!active.empty() && (rc = push_member_map(h, (int)active.size()))) return rc;

    for (int yr = 0; yr < nyears && !active.empty(); ++yr) {
        const int na = (int)active.size();
        const int Wc = na * ntr;
        const int ia = (ib + 1) % 3, iout = (ib + 2) % 3;
        // year: ybuf(ib) -> ybuf(iout) via ybuf(ia) and ... ping-pong needs two scratch buffers
        // besides the start: use ia and the v buffers' first slot.
        rc = run_year(h, na, h->ybuf(ib), h->ybuf(iout), h->ybuf(ia), h->vbuf(0));
        if (rc) return rc;
        if (h->check_finite) {
            hipLaunchKernelGGL(tmm::k_check_finite, dim3(launch_blocks(n * Wc)), dim3(256), 0, h->stream,
                               h->ybuf(iout), n * Wc, h->at<int>(h->P.o_finite));
            TMM_LAUNCHED();
        }
        if (resid_host) {
            rc = sqdiff(h, na, h->ybuf(iout), h->ybuf(ib), 0, 1.0, 1, h->vec(0));
            if (rc) return rc;
            std::vector<double> r(na);
            TMM_TRY(hipMemcpyAsync(r.data(), h->vec(0), (size_t)na * 8, hipMemcpyDeviceToHost, h->stream));
            TMM_TRY(hipStreamSynchronize(h->stream));
            for (int s = 0; s < na; ++s) resid_host[(size_t)yr * nb + active[s]] = r[s];
        }
        ib = iout;
        std::vector<int> fin, stay;
        for (int s = 0; s < na; ++s) {
            if (--left[active[s]] == 0) fin.push_back(s);
            else stay.push_back(s);
        }
        if (!fin.empty()) {
            if ((rc = scatter_finished(fin, Wc))) return rc;
            if (!stay.empty()) {
                const int other = (ib + 1) % 3;
                for (size_t k = 0; k < stay.size(); ++k) { h->h_scol[k] = stay[k]; h->h_dcol[k] = (int)k; }
                if (upload(h, h->at<int>(h->P.o_scol), h->h_scol.data(), stay.size() * 4) ||
                    upload(h, h->at<int>(h->P.o_dcol), h->h_dcol.data(), stay.size() * 4))
                    return TMM_EDEVICE;
                hipLaunchKernelGGL(tmm::k_gather_slots, dim3(launch_blocks(n * stay.size() * ntr)), dim3(256), 0,
                                   h->stream, n, (int)stay.size(), ntr, Wc, (int)stay.size() * ntr,
                                   h->at<int>(h->P.o_scol), h->at<int>(h->P.o_dcol), h->ybuf(ib), h->ybuf(other));
                TMM_LAUNCHED();
                std::vector<int> na2;
                for (int s : stay) na2.push_back(active[s]);
                active = na2;
                ib = other;
                for (size_t s = 0; s < active.size(); ++s) h->h_member[s] = active[s];
                if ((rc = push_member_map(h, (int)active.size()))) return rc;
            } else {
                active.clear();
            }
        }
    }
    // restore the identity member map for later calls
    for (int b = 0; b < nb; ++b) h->h_member[b] = b;
    if ((rc = push_member_map(h, nb))) return rc;
    if ((rc = check_abort(h))) return rc;
    return take_nonfinite(h);
}

int tmm_year_jvp(tmm_handle h, int mode, const double* y, const double* v, double* phi_y, double* jv) {
    if (!h || !y || !v || !jv) return TMM_EINVAL;
    if (mode != TMM_JVP_FD && mode != TMM_JVP_TANGENT && mode != TMM_JVP_FD_GIVEN_PHI) return TMM_EINVAL;
    if (mode == TMM_JVP_FD_GIVEN_PHI && !phi_y) return TMM_EINVAL;
    const int nb = h->nbatch;
    if (nb < 1) return TMM_ESTATE;
    const int ntr = h->P.ntr, W = nb * ntr;
    const size_t n = h->P.n;
    double* f0 = phi_y ? phi_y : h->ybuf(2);
    if (mode == TMM_JVP_TANGENT) {
        int rt = run_year(h, nb, y, f0, h->ybuf(0), h->ybuf(1), v, jv, h->vbuf(0), h->vbuf(1));
        return rt ? rt : check_abort(h);
    }
    // finite differences: h_s = 1e-8 ||y_s|| / ||v_s||
    int rc = sqdiff(h, nb, y, nullptr, 0, 1.0, 0, h->vec(1));
    if (!rc) rc = sqdiff(h, nb, v, nullptr, 0, 1.0, 0, h->vec(2));
    if (rc) return rc;
    hipLaunchKernelGGL(tmm::k_fd_step, dim3(1), dim3(64), 0, h->stream, nb, h->vec(1), h->vec(2), h->vec(3));
    TMM_LAUNCHED();
    hipLaunchKernelGGL(tmm::k_axpy_slots, dim3(launch_blocks(n * W)), dim3(256), 0, h->stream, n, W, ntr,
                       h->vec(3), y, v, h->vbuf(0));
    TMM_LAUNCHED();
    if (mode == TMM_JVP_FD && (rc = run_year(h, nb, y, f0, h->ybuf(0), h->ybuf(1)))) return rc;
    if ((rc = run_year(h, nb, h->vbuf(0), jv, h->ybuf(0), h->ybuf(1)))) return rc;
    hipLaunchKernelGGL(tmm::k_fd_quot, dim3(launch_blocks(n * W)), dim3(256), 0, h->stream, n, W, ntr, h->vec(3),
                       jv, f0, jv);
    TMM_LAUNCHED();
    return check_abort(h);
}

static int drop_graphs(tmm_handle h) {
    if (hipStreamSynchronize(h->stream) != hipSuccess) return TMM_EDEVICE;
    for (auto& gr : h->graphs)
        if (hipGraphExecDestroy(gr.exec) != hipSuccess) return TMM_EDEVICE;
    h->graphs.clear();
    return TMM_OK;
}

int tmm_set_option(tmm_handle h, int option, int value) {
    if (!h) return TMM_EINVAL;
    switch (option) {
        case TMM_OPT_PERSISTENT: h->pers_enabled = value != 0; return TMM_OK;
        case TMM_OPT_MEMBER_KERNEL_MIN:
            if (value < -1) return TMM_EINVAL;
            h->wide_min_members = value < 0 ? -1 : (value == 0 ? 1 << 30 : value);
            return drop_graphs(h);
        case TMM_OPT_GRAPH:
            h->graphs_enabled = value != 0;
            return TMM_OK;
        case TMM_OPT_SPIN_LIMIT:
            if (value < 0) return TMM_EINVAL;
            h->spin_limit = value == 0 ? 1ll << 22 : value;
            return TMM_OK;
        case TMM_OPT_CHECK_FINITE:
            h->check_finite = value != 0;
            return TMM_OK;
        case TMM_OPT_TILE_ROWS: {
            if (value != 0 && value != 32 && value != 64 && value != 128 && value != 256) return TMM_EINVAL;
            int rc = drop_graphs(h);
            if (rc) return rc;
            h->tile_rows_cap = value;
            return TMM_OK;
        }
        case TMM_OPT_MEMBER_WAVES: {
            if (value != 0 && value != 2 && value != 4 && value != 8) return TMM_EINVAL;
            int rc = drop_graphs(h);
            if (rc) return rc;
            h->mem_waves = value == 0 ? tmm::kMembersWaves : value;
            return build_member_order(h);
        }
        case TMM_OPT_MEMBER_BAND_ROWS: {
            if (value < -1) return TMM_EINVAL;
            int rc = drop_graphs(h);
            if (rc) return rc;
            const int old = h->mem_band;
            h->mem_band = value == 0 ? kDefaultBandRows : (value < 0 ? 0 : value);
            rc = build_member_order(h);
            if (rc && rc != TMM_EDEVICE) {      // the tiled kernel's tables do not fit this order
                h->mem_band = old;
                if (build_member_order(h)) return TMM_EDEVICE;
            }
            return rc;
        }
        case TMM_OPT_MEMBER_PACK: {
            int rc = drop_graphs(h);
            if (rc) return rc;
            h->mem_pack = value != 0;
            return TMM_OK;
        }
        case TMM_OPT_MEMBER_TILE: {
            if (value != 0 && value != 4 && value != 8) return TMM_EINVAL;
            if (value != 0 && !member_tiles_possible(h->P)) return TMM_EUNSUPPORTED;
            int rc = drop_graphs(h);
            if (rc) return rc;
            const int old = h->mem_tile;
            h->mem_tile = value;
            rc = build_member_order(h);
            if (rc && rc != TMM_EDEVICE) {      // a layer of some tile needs more rows than a workgroup stages
                h->mem_tile = old;
                if (build_member_order(h)) return TMM_EDEVICE;
            }
            return rc;
        }
        case TMM_OPT_DOMAIN_ROWS: {
            if (value < 0) return TMM_EINVAL;
            if (hipStreamSynchronize(h->stream) != hipSuccess) return TMM_EDEVICE;
            return build_persistent(h, value);
        }
        case TMM_OPT_WAVE_LOCAL: {
            if (hipStreamSynchronize(h->stream) != hipSuccess) return TMM_EDEVICE;
            h->wave_local_enabled = value != 0;
            return build_persistent(h, h->pers_target);
        }
        default: return TMM_EINVAL;
    }
}

int tmm_query(tmm_handle h, int what, long long* value) {
    if (!h || !value) return TMM_EINVAL;
    switch (what) {
        case TMM_Q_PERSISTENT: *value = h->pers_ok ? 1 : 0; return TMM_OK;
        case TMM_Q_DOMAINS: *value = h->pers_G; return TMM_OK;
        case TMM_Q_WORKSPACE: *value = (long long)h->P.total; return TMM_OK;
        case TMM_Q_COMPUTE_UNITS: *value = h->num_cu; return TMM_OK;
        case TMM_Q_PERSISTENT_ADJOINT:
            *value = (h->pers_ok && h->pers_adj_ok && h->P.etw <= tmm::kEllMax) ? 1 : 0;
            return TMM_OK;
        case TMM_Q_INSOLATION_LDS: *value = (h->pers_ok && h->pers_ql[0]) ? 1 : 0; return TMM_OK;
        case TMM_Q_WAVE_LOCAL: *value = (h->pers_ok && h->pers_wave_local) ? 1 : 0; return TMM_OK;
        default: return TMM_EINVAL;
    }
}

int tmm_year_noalloc(tmm_handle h, int nyears, const double* y0, double* y1, double* resid_host) {
    if (!h || !y0 || !y1 || nyears < 0) return TMM_EINVAL;
    const int nb = h->nbatch;
    if (nb < 1) return TMM_ESTATE;
    if (!h->noalloc) return TMM_EDEVICE;
    const Plan& P = h->P;
    const int W = nb * P.ntr;
    const size_t L = (size_t)P.n * W;
    const Tiling& tf = h->tilings.front();
    // scratch layout (doubles): ping-pong state, start-state copy, residual
    // partials per tile, residuals, flag
    const size_t o_part = align_up(2 * L * 8) / 8;
    const size_t o_vec = o_part + align_up((size_t)tf.ntile * nb * 8) / 8;
    const size_t o_flag = o_vec + align_up((size_t)nb * 8) / 8;
    if ((o_flag + 32) * 8 > kNoAllocBytes) return TMM_ETOOBIG;
    double* S = h->noalloc;
    double* T = h->noalloc + L;
    double* part = h->noalloc + o_part;
    double* vec = h->noalloc + o_vec;
    int* flag = reinterpret_cast<int*>(h->noalloc + o_flag);
    if (h->check_finite) {
        hipLaunchKernelGGL(tmm::k_fill_int, dim3(1), dim3(64), 0, h->stream, flag, 16, 0);
        TMM_LAUNCHED();
    }
    for (int yr = 0; yr < nyears; ++yr) {
        // the year's start state: y0, then y1; kept in T when it is about to be overwritten
        // and the residual needs it
        const double* in = yr == 0 ? y0 : y1;
        const double* start = in;
        if (resid_host && (yr > 0 || y1 == y0)) {
            int rc = copy(h, T, in, L);
            if (rc) return rc;
            start = T;
        }
        // steps alternate between S and y1 and end in y1 (nstep is even)
        const double* cur = in;
        for (int j = 0; j < P.nstep; ++j) {
            double* nxt = (j % 2 == 0) ? S : y1;
            int rc = launch_step(h, j, nb, cur, nxt, nullptr, nullptr);
            if (rc) return rc;
            cur = nxt;
        }
        if (h->check_finite) {
            hipLaunchKernelGGL(tmm::k_check_finite, dim3(launch_blocks(L)), dim3(256), 0, h->stream, y1, L, flag);
            TMM_LAUNCHED();
        }
        if (resid_host) {
            tmm::Grid g = h->grid(tf);
            hipLaunchKernelGGL((tmm::k_tile_sqdiff<kMaxTileRows, kMaxTileRows>), dim3(tf.ntile), dim3(256), 0,
                               h->stream, g, W, P.ntr, nb, y1, start, 0, part);
            TMM_LAUNCHED();
            hipLaunchKernelGGL(tmm::k_sum_tiles, dim3(1), dim3(256), 0, h->stream, tf.ntile, nb, nb, part, 1.0, 0, 1,
                               vec);
            TMM_LAUNCHED();
            TMM_TRY(hipMemcpyAsync(resid_host + (size_t)yr * nb, vec, (size_t)nb * 8, hipMemcpyDeviceToHost,
                                   h->stream));
        }
    }
    if (nyears == 0 && y1 != y0) {
        int rc = copy(h, y1, y0, L);
        if (rc) return rc;
    }
    if (!resid_host && !h->check_finite) return TMM_OK;       // kernels only, no synchronisation
    int bad = 0;
    if (h->check_finite) TMM_TRY(hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, h->stream));
    TMM_TRY(hipStreamSynchronize(h->stream));
    return bad ? TMM_ENONFINITE : TMM_OK;
}

int tmm_probe_exchange(tmm_handle h, int rounds, double* out) {
    if (!h || !out || rounds < 1 || rounds > 1000000) return TMM_EINVAL;
    int dev = 0, khz = 0, coop = 0;
    TMM_TRY(hipGetDevice(&dev));
    TMM_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    TMM_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (khz <= 0 || !coop) return TMM_EUNSUPPORTED;
    char* base = h->at<char>(h->P.o_probe);
    long long* words = reinterpret_cast<long long*>(base);          // [0, 512): ping-pong words
    long long* res = reinterpret_cast<long long*>(base + 1024);     // [1024, 1152): results
    int* fail = reinterpret_cast<int*>(base + 2048);
    int* chain = reinterpret_cast<int*>(base + 4096);
    int rc = fill(h, reinterpret_cast<double*>(base), 4096 / 8, 0.0);
    if (rc) return rc;
    // the ping-pong pairs: blocks 0 and 8, then blocks 0 and 1 of a 16-block grid (workgroups are
    // dispatched round-robin over the 8 XCDs: the first pair shares one, the second does not; the
    // kernel records where each ran)
    const int pairs[2][2] = {{0, 8}, {0, 1}};
    for (int p = 0; p < 2; ++p) {
        if (p && (rc = fill(h, reinterpret_cast<double*>(words), 512 / 8, 0.0))) return rc;
        int a = pairs[p][0], b = pairs[p][1], nr = rounds;
        long long* o = res + 3 * p;
        void* args[] = {&a, &b, &nr, &words, &o, &fail};
        TMM_TRY(hipLaunchCooperativeKernel((const void*)&tmm::k_probe_pingpong, dim3(16), dim3(64), args, 0,
                                           h->stream));
    }
    hipLaunchKernelGGL((tmm::k_probe_barrier<256>), dim3(1), dim3(256), 0, h->stream, rounds, res + 6);
    TMM_LAUNCHED();
    hipLaunchKernelGGL(tmm::k_probe_chain, dim3((kProbeLines + 255) / 256), dim3(256), 0, h->stream, kProbeLines,
                       1021, chain);
    TMM_LAUNCHED();
    hipLaunchKernelGGL(tmm::k_probe_load, dim3(1), dim3(64), 0, h->stream, rounds, chain, res + 7);
    TMM_LAUNCHED();
    long long r[8];
    int failed = 0;
    TMM_TRY(hipMemcpyAsync(r, res, sizeof(r), hipMemcpyDeviceToHost, h->stream));
    TMM_TRY(hipMemcpyAsync(&failed, fail, 4, hipMemcpyDeviceToHost, h->stream));
    TMM_TRY(hipStreamSynchronize(h->stream));
    if (failed) return TMM_EDEVICE;
    const double us_per_tick = 1e3 / khz;
    out[0] = r[0] * us_per_tick / rounds;
    out[1] = r[3] * us_per_tick / rounds;
    out[2] = r[6] * us_per_tick / rounds;
    out[3] = r[7] * us_per_tick / rounds;
    out[4] = (double)r[1];
    out[5] = (double)r[2];
    out[6] = (double)r[4];
    out[7] = (double)r[5];
    return TMM_OK;
}

int tmm_year_adjoint(tmm_handle h, const double* y0, const double* obs, int ckpt_every, double* J_host,
                     double* dJdu_host, double* dJdy0) {
    if (!h || !y0 || !obs || !J_host || !dJdu_host) return TMM_EINVAL;
    const Plan& P = h->P;
    if (P.adj_nb < 1) return TMM_EUNSUPPORTED;
    if (ckpt_every != P.ckpt) return TMM_EINVAL;
    const int nb = h->nbatch;
    if (nb < 1) return TMM_ESTATE;
    if (nb > P.adj_nb) return TMM_EUNSUPPORTED;
    const int ntr = P.ntr, W = nb * ntr, np = P.nparam;
    const size_t n = P.n, len = n * W;
    const int K = P.ckpt, spm = P.nstep / P.nmat, nseg = P.nstep / K;
    const double dtd = tmm::kDaysPerYear / P.nstep;
    if (nb == 1 && h->pers_ok && h->pers_adj_ok && h->pers_enabled && P.etw <= tmm::kEllMax)
        return adjoint_persistent(h, y0, obs, J_host, dJdu_host, dJdy0);
    const Tiling& tl = h->tiling_for(W, 1, 256 * 8 * np);
    tmm::Grid g = h->grid(tl);
    tmm::Model md = h->model();
    tmm::Mats mt = h->mats();
    double* ckpt = h->at<double>(P.o_ckpt);
    double* seg = h->at<double>(P.o_seg);
    double* fin = h->at<double>(P.o_final);
    double* mu[2] = {h->at<double>(P.o_mu[0]), h->at<double>(P.o_mu[1])};
    double* ubt = h->at<double>(P.o_ubt);
    double* jpart = h->at<double>(P.o_jpart);
    const int ntile_m = h->tilings.front().ntile;   // misfit partials use the first tiling
    int rc;
    if ((rc = fill(h, ubt, (size_t)tl.ntile * nb * np, 0.0))) return rc;

    auto ckpt_ptr = [&](int s) -> const double* { return s == 0 ? y0 : ckpt + (size_t)s * len; };
    // forward sweep with checkpoints and misfit partials; the states of the
    // last segment stay in the segment store, so that segment is not replayed
    const int lo_last = (nseg - 1) * K;
    {
        const double* cur = y0;
        for (int j = 0; j < P.nstep; ++j) {
            const int nj = j + 1;
            double* nxt;
            if (nj == P.nstep) nxt = fin;
            else if (nj % K == 0) nxt = ckpt + (size_t)(nj / K) * len;
            else if (nj > lo_last) nxt = seg + (size_t)(nj - lo_last) * len;
            else nxt = (cur == seg) ? seg + len : seg;          // two scratch slots of the segment store
            if ((rc = launch_step(h, j, nb, cur, nxt, nullptr, nullptr))) return rc;
            if (nj % spm == 0) {
                const int m = nj / spm - 1;
                rc = sqdiff(h, nb, nxt, obs + (size_t)m * len, 1, 1.0, 0, nullptr, 0,
                            jpart + (size_t)m * ntile_m * nb);
                if (rc) return rc;
            }
            cur = nxt;
        }
        hipLaunchKernelGGL(tmm::k_sum_tiles, dim3(1), dim3(256), 0, h->stream, P.nmat * ntile_m, nb, nb, jpart,
                           1.0 / (2.0 * P.nmat * h->vtot), 0, 0, h->vec(4));
        TMM_LAUNCHED();
    }
    const size_t lds = (size_t)tl.max_rows * W * 8 + (size_t)256 * np * 8;
    auto adjoint = [&](int j, int use_ae, int use_ai, const double* mu_in, const double* yj, const double* ob,
                       double* out) -> int {
        const double sc = 1.0 / (P.nmat * h->vtot);
        double* ub = use_ae ? ubt : nullptr;
        if (ntr == 3 && P.nsub > 1)
            hipLaunchKernelGGL((tmm::k_adjoint<3, kMaxTileRows, kMaxTileRows, true>), dim3(tl.ntile), dim3(256), lds,
                               h->stream, g, md, mt, W, nb, j, dtd, use_ae, use_ai, mu_in, yj, ob, sc, out, ub);
        else if (ntr == 3)
            hipLaunchKernelGGL((tmm::k_adjoint<3, kMaxTileRows, kMaxTileRows>), dim3(tl.ntile), dim3(256), lds,
                               h->stream, g, md, mt, W, nb, j, dtd, use_ae, use_ai, mu_in, yj, ob, sc, out, ub);
        else if (ntr == 2 && P.nsub > 1)
            hipLaunchKernelGGL((tmm::k_adjoint<2, kMaxTileRows, kMaxTileRows, true>), dim3(tl.ntile), dim3(256), lds,
                               h->stream, g, md, mt, W, nb, j, dtd, use_ae, use_ai, mu_in, yj, ob, sc, out, ub);
        else if (ntr == 2)
            hipLaunchKernelGGL((tmm::k_adjoint<2, kMaxTileRows, kMaxTileRows>), dim3(tl.ntile), dim3(256), lds,
                               h->stream, g, md, mt, W, nb, j, dtd, use_ae, use_ai, mu_in, yj, ob, sc, out, ub);
        else if (P.nsub > 1)
            hipLaunchKernelGGL((tmm::k_adjoint<1, kMaxTileRows, kMaxTileRows, true>), dim3(tl.ntile), dim3(256), lds,
                               h->stream, g, md, mt, W, nb, j, dtd, use_ae, use_ai, mu_in, yj, ob, sc, out, ub);
        else
            hipLaunchKernelGGL((tmm::k_adjoint<1, kMaxTileRows, kMaxTileRows>), dim3(tl.ntile), dim3(256), lds,
                               h->stream, g, md, mt, W, nb, j, dtd, use_ae, use_ai, mu_in, yj, ob, sc, out, ub);
        TMM_LAUNCHED();
        return TMM_OK;
    };
    // head: lambda_nstep = misfit source of the last snapshot; mu_{nstep-1} = Ai^T lambda
    int im = 0;
    if ((rc = adjoint(P.nstep, 0, 1, nullptr, fin, obs + (size_t)(P.nmat - 1) * len, mu[im]))) return rc;
    for (int s = nseg - 1; s >= 0; --s) {
        const int base = s * K;
        // replay the segment, keeping y_{base+1} .. y_{base+K-1}
        const double* cur = ckpt_ptr(s);
        for (int jj = base; s < nseg - 1 && jj < base + K - 1; ++jj) {
            double* nxt = seg + (size_t)(jj + 1 - base) * len;
            if ((rc = launch_step(h, jj, nb, cur, nxt, nullptr, nullptr))) return rc;
            cur = nxt;
        }
        for (int j = base + K - 1; j >= base && j >= 1; --j) {
            const double* yj = j == base ? ckpt_ptr(s) : seg + (size_t)(j - base) * len;
            const double* ob = (j % spm == 0) ? obs + (size_t)(j / spm - 1) * len : nullptr;
            if ((rc = adjoint(j, 1, 1, mu[im], yj, ob, mu[1 - im]))) return rc;
            im = 1 - im;
        }
    }
    // tail: lambda_0 = Ae(t_0)^T mu_0 + dt_d (dq/dy)(y_0)^T mu_0
    double* l0 = dJdy0 ? dJdy0 : mu[1 - im];
    if ((rc = adjoint(0, 1, 0, mu[im], y0, nullptr, l0))) return rc;
    hipLaunchKernelGGL(tmm::k_sum_tiles, dim3(1), dim3(256), 0, h->stream, tl.ntile, nb * np, nb * np, ubt, 1.0, 0, 0,
                       h->vec(5));
    TMM_LAUNCHED();
    std::vector<double> J(nb), G((size_t)nb * np);
    TMM_TRY(hipMemcpyAsync(J.data(), h->vec(4), (size_t)nb * 8, hipMemcpyDeviceToHost, h->stream));
    TMM_TRY(hipMemcpyAsync(G.data(), h->vec(5), (size_t)nb * np * 8, hipMemcpyDeviceToHost, h->stream));
    TMM_TRY(hipStreamSynchronize(h->stream));
    for (int b = 0; b < nb; ++b) {
        if (!std::isfinite(J[b])) return TMM_ENONFINITE;
        J_host[b] = J[b];
    }
    for (size_t i = 0; i < G.size(); ++i) {
        if (!std::isfinite(G[i])) return TMM_ENONFINITE;
        dJdu_host[i] = G[i];
    }
    return TMM_OK;
}

}  // extern "C"
