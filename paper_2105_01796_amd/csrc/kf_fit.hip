// kf_fit.hip -- kernels and C ABI of the MI355X batched Kalman-filter track fit.
//
// Forward filter + RTS smoother (Sect. 2; Sect. 4.1), one lane per track:
//   * the surface table is staged once per workgroup in LDS, next to a
//     per-lane slot for the filtered covariance carried from hit to hit;
//   * the forward pass writes, per hit, the predicted state and covariance
//     and the transport Jacobian F (Sect. 2: the smoother uses the Jacobians
//     stored in the forward pass) to a tile-major workspace
//     [tile][hit][component][64 lanes]: a wave's 64 lanes store/load 64
//     consecutive doubles (coalesced), and every component sits at a
//     compile-time offset from one per-lane base.  With KF_JAC_RECOMPUTE the
//     Jacobian is not stored: the smoother propagates each filtered state
//     again (27 instead of 52 doubles per hit travel through memory, one more
//     propagation per hit);
//   * the backward pass recomputes each filtered state from the stored
//     prediction and the hit (the same update, bit for bit), solves the RTS
//     gain in FP64 (Cholesky of the predicted covariance, Sect. 4.2.4),
//     applies the smoother and writes the smoothed states to the caller's CSR
//     outputs, and the seed-surface result to tgt_*.
// The two-filter smoother (KF_SMOOTHER_TWO_FILTER; Sect. 2, Fig. 2) replaces
// the RTS pass by a second Kalman filter run from the last hit back to the
// seed surface, propagating against the direction of flight, whose
// predictions combine with the forward filtered states (fused kernel, 27
// doubles per hit in the workspace).
// Schedules: DIRECT (track i on lane i) and SORTED (tracks ordered by hit
// count, longest first; persistent waves pull 64-track tiles from a queue so
// that waves carry tracks of equal length).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <mutex>
#include <map>
#include <limits.h>
#include "kf_fit_kernels.hpp"

namespace {
using namespace kffit;

// Perigee target: one lane per track carries the fitted state on the seed
// surface (tgt_*) to the perigee of the line through a.perigee parallel to z
// and replaces it there, covariance C <- F C F^T.  A track that does not
// reach it fails: status and NaN outputs.
template <int FK>
__global__ void __launch_bounds__(256) k_perigee(FitArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n_tracks || a.status[t] != ST_OK) return;
    const int64_t N = a.n_tracks;
    const int S = a.n_surf, s0 = a.seed_sid;
    double sv[SURF_STRIDE];
#pragma unroll
    for (int f = 0; f < 3; ++f) sv[f] = a.center[f * S + s0];
#pragma unroll
    for (int f = 0; f < 9; ++f) sv[3 + f] = a.rot[f * S + s0];
    sv[12] = a.x0[s0];
    sv[13] = 0.0;                       // the seed surface is a plane
    if (a.align) {
        double al[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) al[c] = a.align[c * S + s0];
        apply_alignment(al, sv);
    }
    double x[6], C[21], xp[6], F[25], Cp[21];
    load_rows(a.tgt_par + t, N, x);
    load_rows(a.tgt_cov + t, N, C);
    int tr = 0;
    const int st = transport_perigee<FK>(a.field, a.cfg, sv, a.perigee, x, xp, F, &tr);
    if (st == ST_OK) {
        transport_cov(F, C, Cp);
        store_rows(a.tgt_par + t, N, xp);
        store_rows(a.tgt_cov + t, N, Cp);
        return;
    }
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    const int64_t H = a.n_hits;
    const int o = a.off[t], n = a.off[t + 1] - o;
    for (int k = 0; k < n; ++k) {
        fill_rows<6>(a.par + o + k, H, nan);
        fill_rows<21>(a.pcov + o + k, H, nan);
    }
    fill_rows<6>(a.tgt_par + t, N, nan);
    fill_rows<21>(a.tgt_cov + t, N, nan);
    a.chi2[t] = nan;
    a.status[t] = (uint8_t)st;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct WsLayout {
    int64_t tile_doubles;
    size_t fit_bytes;     // [tiles][max_hits][NC][64] doubles
    size_t order_off;     // int32 [tiles * 64]
    size_t counts_off;    // int32 [NBINS][sort blocks] histogram / positions
    size_t counter_off;   // int32 tile counter
    size_t total;
};


WsLayout ws_layout(int64_t n_tracks, int max_hits) {
    WsLayout L;
    const int64_t tiles = n_tracks > 0 ? (n_tracks + TILE - 1) / TILE : 1;
    L.tile_doubles = (int64_t)max_hits * NC * TILE;
    L.fit_bytes = (size_t)tiles * L.tile_doubles * sizeof(double);
    L.order_off = align_up(L.fit_bytes, 256);
    L.counts_off = align_up(L.order_off + (size_t)tiles * TILE * 4, 256);
    L.counter_off = align_up(L.counts_off + (size_t)sort_count_entries((int)n_tracks) * 4, 256);
    L.total = align_up(L.counter_off + SORT_HEADS * 4, 256);
    return L;
}

int validate(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field, const kf_measurements* meas,
             const kf_seeds* seeds, const kf_outputs* out) {
    if (!cfg || !surf || !field || !meas || !seeds || !out) return KF_E_NULL;
    const int rc = validate_inputs(cfg, surf, field, meas, seeds);
    if (rc != KF_OK || meas->n_tracks == 0) return rc;
    if (!out->par && meas->n_hits > 0) return KF_E_NULL;
    if (!out->cov && meas->n_hits > 0) return KF_E_NULL;
    if (!out->tgt_par || !out->tgt_cov || !out->chi2 || !out->ndf || !out->status) return KF_E_NULL;
    if ((out->filt_par == nullptr) != (out->filt_cov == nullptr)) return KF_E_NULL;
    // cylinders and lines: the kernels are built for one wave per SIMD only
    if (surf->type && surf->radius && cfg->occupancy != 0 && cfg->occupancy != 1) return KF_E_VALUE;
    return KF_OK;
}

// The split smoother's kernel, after the filter kernel on the same stream
// (SORTED: up to 8 persistent waves per CU pull the tiles again).
hipError_t launch_bwd(const FitArgs& a, int sched, int block, bool curved, hipStream_t stream) {
    const size_t shm = (size_t)(block / TILE) * a.wave_lds * sizeof(double);
    const int need = (a.n_tiles * TILE + block - 1) / block;
    int grid = need;
    if (sched == KF_SCHED_SORTED) {
        grid = num_cu() * 8 * TILE / block;
        grid = grid > need ? need : (grid < 1 ? 1 : grid);
    }
    hipError_t e = hipSuccess;
    if (sched == KF_SCHED_SORTED) {
        if (curved) {
            if ((e = allow_lds(k_bwd<true, true>, shm)) != hipSuccess) return e;
            hipLaunchKernelGGL((k_bwd<true, true>), dim3(grid), dim3(block), shm, stream, a);
        } else {
            if ((e = allow_lds(k_bwd<true, false>, shm)) != hipSuccess) return e;
            hipLaunchKernelGGL((k_bwd<true, false>), dim3(grid), dim3(block), shm, stream, a);
        }
    } else {
        if (curved) {
            if ((e = allow_lds(k_bwd<false, true>, shm)) != hipSuccess) return e;
            hipLaunchKernelGGL((k_bwd<false, true>), dim3(grid), dim3(block), shm, stream, a);
        } else {
            if ((e = allow_lds(k_bwd<false, false>, shm)) != hipSuccess) return e;
            hipLaunchKernelGGL((k_bwd<false, false>), dim3(grid), dim3(block), shm, stream, a);
        }
    }
    return hipGetLastError();
}

// Enqueue one fit with every launch setting resolved (no AUTO fields).
int enqueue_fit(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field, const kf_measurements* meas,
                const kf_seeds* seeds, const kf_outputs* out, void* workspace, hipStream_t stream) {
    const WsLayout L = ws_layout(meas->n_tracks, meas->max_hits);
    char* wsb = (char*)workspace;

    FitArgs a;
    memset(&a, 0, sizeof(a));
    a.n_tracks = meas->n_tracks;
    a.n_surf = surf->n;
    a.seed_sid = seeds->surface_id;
    a.max_hits = meas->max_hits;
    a.n_hits = meas->n_hits;
    // the workspace is sized for stored Jacobians; without them a tile packs tighter
    const bool twof = cfg->smoother == KF_SMOOTHER_TWO_FILTER;
    a.tile_doubles = (cfg->jacobians == KF_JAC_RECOMPUTE || twof) ? (int64_t)meas->max_hits * NC_RECOMPUTE * TILE
                                                                  : L.tile_doubles;
    a.bwd_scale = cfg->bwd_scale > 0.0 ? cfg->bwd_scale : 1e3;
    for (int i = 0; i < 3; ++i) a.perigee[i] = cfg->perigee[i];
    a.off = meas->hit_offsets;
    a.sid = meas->surface_id;
    a.loc = meas->loc;
    a.cov = meas->cov;
    a.center = surf->center;
    a.rot = surf->rot;
    a.x0 = surf->x_over_X0;
    a.align = surf->align;
    a.stype = surf->type;
    // cylinders and lines: the kernels built for every surface type
    const bool curved = surf->type && surf->radius;
    a.radius = curved ? surf->radius : nullptr;
    a.seed = seeds->par;
    a.seed_cov = seeds->cov;
    a.field = field_def(field);
    a.cfg = cfg_def(cfg);
    a.bnz = (field->kind != KF_FIELD_UNIFORM) || field->b0[0] != 0.0 || field->b0[1] != 0.0 || field->b0[2] != 0.0;
    a.par = out->par;
    a.pcov = out->cov;
    a.tgt_par = out->tgt_par;
    a.tgt_cov = out->tgt_cov;
    a.chi2 = out->chi2;
    a.ndf = out->ndf;
    a.status = out->status;
    a.trials = out->trials;
    a.filt_par = out->filt_par;
    a.filt_cov = out->filt_cov;
    a.ws = (double*)wsb;
    a.order = (const int32_t*)(wsb + L.order_off);
    a.tile_counter = (int32_t*)(wsb + L.counter_off);
    a.n_tiles = (int)((a.n_tracks + TILE - 1) / TILE);

    const int sched = cfg->schedule;
    const int block = cfg->block;
    const int wpc = cfg->waves_per_cu;
    // the kernels for cylinders and lines are built for one wave per SIMD only
    if (curved && cfg->occupancy != 1) return KF_E_VALUE;
    // LDS per wave: the output transpose of the two-filter smoother and of
    // KF_OUT_SLOTS, or the RTS smoother's output stage (KF_OUT_STAGED) of two
    // steps where the workgroups of a CU at the kernel's occupancy (4 x
    // occupancy waves) still fit beside their surface tables, else of one step
    if (twof || cfg->output == KF_OUT_SLOTS) {
        a.stage_hits = 0;
        a.wave_lds = WAVE_LDS_DOUBLES;
    } else {
        const int wgs = 4 * cfg->occupancy / (block / TILE) > 0 ? 4 * cfg->occupancy / (block / TILE) : 1;
        const size_t two = (size_t)wgs * fwd_lds_bytes(surf->n, block, wave_lds_doubles(STAGE_MAX_HITS));
        a.stage_hits = two <= lds_cap() ? STAGE_MAX_HITS : 1;
        a.wave_lds = wave_lds_doubles(a.stage_hits);
    }

    hipError_t e = hipSuccess;
    if (sched == KF_SCHED_SORTED) {
        e = enqueue_length_sort(a.off, a.n_tracks, a.max_hits, (int32_t*)(wsb + L.counts_off), (int32_t*)a.order,
                                a.tile_counter, stream);
        if (e != hipSuccess) return KF_E_HIP;
    }
    const bool mixed = cfg->precision == KF_PREC_MIXED;
    const int occ = cfg->occupancy;
    const bool split = cfg->split_smoother != 0;
    const bool storef = cfg->jacobians != KF_JAC_RECOMPUTE && !twof;
    if ((!storef || twof) && split) return KF_E_VALUE;
    if (field->kind == KF_FIELD_UNIFORM)
        e = mixed ? launch_fwd_uniform_mixed(a, sched, block, wpc, occ, split, storef, twof, curved, stream)
                  : launch_fwd_uniform_fp64(a, sched, block, wpc, occ, split, storef, twof, curved, stream);
    else if (field->kind == KF_FIELD_SOLENOID)
        e = mixed ? launch_fwd_solenoid_mixed(a, sched, block, wpc, occ, split, storef, twof, curved, stream)
                  : launch_fwd_solenoid_fp64(a, sched, block, wpc, occ, split, storef, twof, curved, stream);
    else
        e = mixed ? launch_fwd_map_mixed(a, sched, block, wpc, occ, split, storef, twof, curved, stream)
                  : launch_fwd_map_fp64(a, sched, block, wpc, occ, split, storef, twof, curved, stream);
    if (e == hipSuccess && split) e = launch_bwd(a, sched, block, curved, stream);
    // a workgroup needing more LDS than the device has, or an occupancy the
    // kernels for cylinders and lines are not built for
    if (e == hipErrorInvalidValue) return KF_E_VALUE;
    if (e == hipSuccess && cfg->target == KF_TARGET_PERIGEE) {
        const dim3 grid((unsigned)((a.n_tracks + 255) / 256));
        if (field->kind == KF_FIELD_UNIFORM)
            hipLaunchKernelGGL(k_perigee<FIELD_UNIFORM>, grid, dim3(256), 0, stream, a);
        else if (field->kind == KF_FIELD_SOLENOID)
            hipLaunchKernelGGL(k_perigee<FIELD_SOLENOID>, grid, dim3(256), 0, stream, a);
        else
            hipLaunchKernelGGL(k_perigee<FIELD_MAP>, grid, dim3(256), 0, stream, a);
        e = hipGetLastError();
    }
    return e == hipSuccess ? KF_OK : KF_E_HIP;
}


// ---- autotuned launch settings ----
// Key: precision, field kind, smoother, surfaces with cylinders or lines,
// max hits per track, track count rounded to a power of two.  Filled by
// kf_autotune, read when a setting is AUTO (0).
struct TuneKey {
    int precision, field_kind, smoother, curved, max_hits, log2n;
    bool operator<(const TuneKey& o) const {
        if (curved != o.curved) return curved < o.curved;
        if (precision != o.precision) return precision < o.precision;
        if (field_kind != o.field_kind) return field_kind < o.field_kind;
        if (smoother != o.smoother) return smoother < o.smoother;
        if (max_hits != o.max_hits) return max_hits < o.max_hits;
        return log2n < o.log2n;
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, kf_config> g_tune;

TuneKey tune_key(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field, const kf_measurements* meas) {
    int l = 0;
    while ((1LL << (l + 1)) <= (long long)meas->n_tracks) ++l;
    const int curved = surf->type && surf->radius ? 1 : 0;
    return TuneKey{cfg->precision, field->kind, cfg->smoother, curved, meas->max_hits, l};
}

// Fill AUTO (0) launch settings from the tuning table, else the defaults
// (length-sorted persistent schedule, 64-thread groups, one wave per SIMD,
// 8 resident waves per CU, smoother fused into the filter kernel).
kf_config resolve(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field, const kf_measurements* meas) {
    kf_config r = *cfg;
    kf_config d = r;
    d.schedule = KF_SCHED_SORTED;
    d.block = 64;
    d.occupancy = 1;
    d.waves_per_cu = 8;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(tune_key(cfg, surf, field, meas));
        if (it != g_tune.end()) d = it->second;
    }
    if (r.schedule == KF_SCHED_AUTO) {
        r.schedule = d.schedule;
        r.split_smoother = r.smoother == KF_SMOOTHER_TWO_FILTER ? 0 : d.split_smoother;
        r.jacobians = d.jacobians;
    }
    if (r.output == KF_OUT_AUTO) r.output = d.output == KF_OUT_AUTO ? KF_OUT_STAGED : d.output;
    if (r.block == 0) r.block = d.block;
    if (r.occupancy == 0) r.occupancy = d.occupancy;
    if (r.waves_per_cu == 0) r.waves_per_cu = d.waves_per_cu;
    return r;
}

int check_ws(const kf_measurements* meas, void* workspace, size_t workspace_bytes) {
    if (!workspace) return KF_E_WS;
    if (workspace_bytes < ws_layout(meas->n_tracks, meas->max_hits).total) return KF_E_WS;
    return KF_OK;
}

// ---- host-staged chunked fit ----
// CSR offsets of a chunk copied from the host start at the chunk's first hit;
// the fit wants them to start at 0.
__global__ void k_rebase(int32_t* off, int n1, int32_t base) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n1) off[i] -= base;
}

struct StagedLayout {
    int n_chunks;
    int64_t max_nc, max_hc;                 // largest chunk in tracks and in hits
    size_t off, sid, loc, cov, seed, seed_cov, par, pcov, tgt_par, tgt_cov, chi2, ndf, status, fit;
    size_t slot_bytes;
};

inline int64_t chunk_begin(int64_t N, int n_chunks, int i) { return (int64_t)i * N / n_chunks; }

StagedLayout staged_layout(const kf_measurements* meas, int n_chunks) {
    StagedLayout L;
    const int64_t N = meas->n_tracks;
    L.n_chunks = (int)(n_chunks > N ? (N > 0 ? N : 1) : n_chunks);
    L.max_nc = 0;
    L.max_hc = 0;
    for (int i = 0; i < L.n_chunks; ++i) {
        const int64_t t0 = chunk_begin(N, L.n_chunks, i), t1 = chunk_begin(N, L.n_chunks, i + 1);
        const int64_t nc = t1 - t0;
        const int64_t hc = N > 0 ? (int64_t)meas->hit_offsets[t1] - meas->hit_offsets[t0] : 0;
        L.max_nc = nc > L.max_nc ? nc : L.max_nc;
        L.max_hc = hc > L.max_hc ? hc : L.max_hc;
    }
    const size_t nc = (size_t)(L.max_nc > 0 ? L.max_nc : 1), hc = (size_t)(L.max_hc > 0 ? L.max_hc : 1);
    size_t p = 0;
    auto take = [&](size_t bytes) { const size_t at = p; p = align_up(p + bytes, 256); return at; };
    L.off = take((nc + 1) * 4);
    L.sid = take(hc * 4);
    L.loc = take(2 * hc * 8);
    L.cov = take(3 * hc * 8);
    L.seed = take(6 * nc * 8);
    L.seed_cov = take(21 * nc * 8);
    L.par = take(6 * hc * 8);
    L.pcov = take(21 * hc * 8);
    L.tgt_par = take(6 * nc * 8);
    L.tgt_cov = take(21 * nc * 8);
    L.chi2 = take(nc * 8);
    L.ndf = take(nc * 4);
    L.status = take(nc);
    L.fit = take(ws_layout((int64_t)nc, meas->max_hits).total);
    L.slot_bytes = p;
    return L;
}

// rows r of a component-major [R][len] array: elements [at, at + n) of every
// row, between host (row stride len) and a compact device block (row stride n)
hipError_t copy_rows(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t rows,
                     hipMemcpyKind kind, hipStream_t stream) {
    if (width == 0 || rows == 0) return hipSuccess;
    return hipMemcpy2DAsync(dst, dpitch, src, spitch, width, rows, kind, stream);
}

}  // namespace

// ---- the workspace of kf_fit_tracks_noalloc ----
// A static device array: every device the library runs on holds its own copy
// until the process ends.  In host code the name `scratch` is only a handle
// for the runtime; the device address comes from hipGetSymbolAddress, looked
// up once per device with that device current (noalloc_scratch), and only
// that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[KF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES];

// Device address of the current device's scratch (nullptr on a HIP error).
void* noalloc_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

const char* kf_version(void) { return "kfmi 0.1 (gfx950, fp64 + mixed)"; }

const char* kf_status_string(int code) {
    switch (code) {
        case KF_OK: return "ok";
        case KF_E_NULL: return "required pointer is NULL";
        case KF_E_SIZE: return "count negative, too large or inconsistent";
        case KF_E_ENUM: return "unknown enum value";
        case KF_E_WS: return "workspace missing or too small";
        case KF_E_HIP: return "HIP runtime error";
        case KF_E_VALUE: return "configuration value out of range";
        case KF_E_SCRATCH: return "batch needs more workspace than the static scratch of kf_fit_tracks_noalloc";
        case KF_ST_NO_INTERSECT: return "track: no intersection with a surface";
        case KF_ST_STEP_CAP: return "track: step cap reached";
        case KF_ST_NOT_SPD: return "track: covariance not positive definite";
        case KF_ST_BAD_INPUT: return "track: invalid input";
        case KF_ST_TOO_FEW: return "track: fewer than 3 hits";
        default: return "unknown code";
    }
}

size_t kf_workspace_bytes(const kf_config* cfg, const kf_measurements* meas, int32_t n_surfaces) {
    (void)cfg;
    if (!meas || meas->n_tracks < 0 || meas->max_hits < 1 || meas->max_hits > KF_MAX_HITS || n_surfaces < 1)
        return 0;
    return ws_layout(meas->n_tracks, meas->max_hits).total;
}

int kf_fit_tracks(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field,
                  const kf_measurements* meas, const kf_seeds* seeds, const kf_outputs* out, void* workspace,
                  size_t workspace_bytes, void* stream) {
    int rc = validate(cfg, surf, field, meas, seeds, out);
    if (rc != KF_OK) return rc;
    if (meas->n_tracks == 0) return KF_OK;
    rc = check_ws(meas, workspace, workspace_bytes);
    if (rc != KF_OK) return rc;
    num_cu();
    const kf_config r = resolve(cfg, surf, field, meas);
    return enqueue_fit(&r, surf, field, meas, seeds, out, workspace, (hipStream_t)stream);
}

int kf_fit_tracks_noalloc(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field,
                          const kf_measurements* meas, const kf_seeds* seeds, const kf_outputs* out, void* stream) {
    int rc = validate(cfg, surf, field, meas, seeds, out);
    if (rc != KF_OK) return rc;
    if (meas->n_tracks == 0) return KF_OK;
    if (ws_layout(meas->n_tracks, meas->max_hits).total > KF_NOALLOC_SCRATCH_BYTES) return KF_E_SCRATCH;
    void* ws = noalloc_scratch();
    if (!ws) return KF_E_HIP;
    num_cu();
    const kf_config r = resolve(cfg, surf, field, meas);
    return enqueue_fit(&r, surf, field, meas, seeds, out, ws, (hipStream_t)stream);
}

struct kf_plan {
    hipStream_t capture;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int empty;
};

int kf_plan_create(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field,
                   const kf_measurements* meas, const kf_seeds* seeds, const kf_outputs* out, void* workspace,
                   size_t workspace_bytes, kf_plan** plan) {
    if (!plan) return KF_E_NULL;
    *plan = nullptr;
    int rc = validate(cfg, surf, field, meas, seeds, out);
    if (rc != KF_OK) return rc;
    kf_plan* p = new kf_plan();
    p->empty = meas->n_tracks == 0;
    if (p->empty) { *plan = p; return KF_OK; }
    rc = check_ws(meas, workspace, workspace_bytes);
    if (rc != KF_OK) { delete p; return rc; }
    num_cu();
    const kf_config r = resolve(cfg, surf, field, meas);
    if (hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess) { delete p; return KF_E_HIP; }
    if (hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(p->capture);
        delete p;
        return KF_E_HIP;
    }
    rc = enqueue_fit(&r, surf, field, meas, seeds, out, workspace, p->capture);
    hipGraph_t g = nullptr;
    const hipError_t e1 = hipStreamEndCapture(p->capture, &g);
    if (rc != KF_OK || e1 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(p->capture);
        delete p;
        return rc != KF_OK ? rc : KF_E_HIP;
    }
    p->graph = g;
    if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(p->capture);
        delete p;
        return KF_E_HIP;
    }
    *plan = p;
    return KF_OK;
}

int kf_plan_launch(kf_plan* plan, void* stream) {
    if (!plan) return KF_E_NULL;
    if (plan->empty) return KF_OK;
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? KF_OK : KF_E_HIP;
}

void kf_plan_destroy(kf_plan* plan) {
    if (!plan) return;
    if (!plan->empty) {
        (void)hipGraphExecDestroy(plan->exec);
        (void)hipGraphDestroy(plan->graph);
        (void)hipStreamDestroy(plan->capture);
    }
    delete plan;
}

int kf_autotune(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field, const kf_measurements* meas,
                const kf_seeds* seeds, const kf_outputs* out, void* workspace, size_t workspace_bytes,
                void* stream_, kf_config* best, float* best_ms) {
    if (!best) return KF_E_NULL;
    int rc = validate(cfg, surf, field, meas, seeds, out);
    if (rc != KF_OK) return rc;
    *best = resolve(cfg, surf, field, meas);
    if (best_ms) *best_ms = 0.0f;
    if (meas->n_tracks == 0) return KF_OK;
    rc = check_ws(meas, workspace, workspace_bytes);
    if (rc != KF_OK) return rc;
    num_cu();
    hipStream_t stream = (hipStream_t)stream_;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return KF_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return KF_E_HIP; }
    static const int scheds[] = {KF_SCHED_DIRECT, KF_SCHED_SORTED};
    static const int blocks[] = {64, 256};
    static const int occs[] = {1, 2, 3};
    static const int splits[] = {0, 1, 2};     // 2: fused smoother recomputing the Jacobians
    static const int wpcs[] = {4, 8};
    static const int outputs[] = {KF_OUT_STAGED, KF_OUT_SLOTS};
    const bool twof = cfg->smoother == KF_SMOOTHER_TWO_FILTER;
    float best_t = 1e30f;
    kf_config win = *best;
    for (int sc : scheds)
        for (int bl : blocks)
            for (int oc : occs)
                for (int sp : splits)
                    for (int wp : wpcs)
                        for (int op : outputs) {
                        if (sc == KF_SCHED_DIRECT && wp != wpcs[0]) continue;   // unused by DIRECT
                        if (twof && (sp != 0 || op != outputs[0])) continue;   // fused, through its slots
                        if (!twof && cfg->output != KF_OUT_AUTO && op != cfg->output) continue;   // fixed
                        kf_config c = *cfg;
                        c.schedule = sc;
                        c.block = bl;
                        c.occupancy = oc;
                        c.split_smoother = sp == 1;
                        c.jacobians = sp == 2 ? KF_JAC_RECOMPUTE : KF_JAC_STORE;
                        c.waves_per_cu = wp;
                        c.output = op;
                        rc = enqueue_fit(&c, surf, field, meas, seeds, out, workspace, stream);   // warm-up
                        if (rc == KF_E_VALUE) { rc = KF_OK; continue; }   // does not fit this device
                        if (rc != KF_OK) break;
                        (void)hipEventRecord(e0, stream);
                        for (int rep = 0; rep < 3 && rc == KF_OK; ++rep)
                            rc = enqueue_fit(&c, surf, field, meas, seeds, out, workspace, stream);
                        (void)hipEventRecord(e1, stream);
                        if (hipEventSynchronize(e1) != hipSuccess) rc = KF_E_HIP;
                        if (rc != KF_OK) break;
                        float ms = 0.0f;
                        (void)hipEventElapsedTime(&ms, e0, e1);
                        ms /= 3.0f;
                        if (ms < best_t) { best_t = ms; win = c; }
                    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != KF_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(cfg, surf, field, meas)] = win;
    }
    *best = win;
    if (best_ms) *best_ms = best_t;
    return KF_OK;
}

size_t kf_staged_workspace_bytes(const kf_config* cfg, const kf_measurements* meas, int32_t n_surfaces,
                                 int32_t n_chunks, int32_t n_streams) {
    (void)cfg;
    if (!meas || !meas->hit_offsets || meas->n_tracks < 0 || meas->max_hits < 1 || meas->max_hits > KF_MAX_HITS ||
        n_surfaces < 1 || n_chunks < 1 || n_streams < 1)
        return 0;
    return staged_layout(meas, n_chunks).slot_bytes * (size_t)n_streams;
}

int kf_fit_tracks_staged(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field,
                         const kf_measurements* meas, const kf_seeds* seeds, const kf_outputs* out, void* workspace,
                         size_t workspace_bytes, int32_t n_chunks, void* const* streams, int32_t n_streams) {
    int rc = validate(cfg, surf, field, meas, seeds, out);
    if (rc != KF_OK) return rc;
    if (n_chunks < 1 || n_streams < 1) return KF_E_VALUE;
    if (!streams) return KF_E_NULL;
    for (int i = 0; i < n_streams; ++i)
        if (!streams[i]) return KF_E_NULL;
    if (out->trials || out->filt_par || out->filt_cov) return KF_E_VALUE;
    const int64_t N = meas->n_tracks, H = meas->n_hits;
    if (N == 0) return KF_OK;
    if (!meas->hit_offsets || meas->hit_offsets[0] != 0 || meas->hit_offsets[N] != H) return KF_E_SIZE;
    const StagedLayout L = staged_layout(meas, n_chunks);
    if (!workspace || workspace_bytes < L.slot_bytes * (size_t)n_streams) return KF_E_WS;
    num_cu();
    for (int i = 0; i < L.n_chunks; ++i) {
        hipStream_t st = (hipStream_t)streams[i % n_streams];
        char* slot = (char*)workspace + (size_t)(i % n_streams) * L.slot_bytes;
        const int64_t t0 = chunk_begin(N, L.n_chunks, i), t1 = chunk_begin(N, L.n_chunks, i + 1);
        const int64_t nc = t1 - t0;
        const int32_t h0 = meas->hit_offsets[t0];
        const int64_t hc = (int64_t)meas->hit_offsets[t1] - h0;
        if (hc < 0) return KF_E_SIZE;
        const size_t hb = (size_t)hc * 8, nb = (size_t)nc * 8;
        const hipMemcpyKind in = hipMemcpyHostToDevice, outk = hipMemcpyDeviceToHost;
        hipError_t e = hipMemcpyAsync(slot + L.off, meas->hit_offsets + t0, (size_t)(nc + 1) * 4, in, st);
        if (e == hipSuccess && hc > 0)
            e = hipMemcpyAsync(slot + L.sid, meas->surface_id + h0, (size_t)hc * 4, in, st);
        if (e == hipSuccess) e = copy_rows(slot + L.loc, hb, meas->loc + h0, (size_t)H * 8, hb, 2, in, st);
        if (e == hipSuccess) e = copy_rows(slot + L.cov, hb, meas->cov + h0, (size_t)H * 8, hb, 3, in, st);
        if (e == hipSuccess) e = copy_rows(slot + L.seed, nb, seeds->par + t0, (size_t)N * 8, nb, 6, in, st);
        if (e == hipSuccess) e = copy_rows(slot + L.seed_cov, nb, seeds->cov + t0, (size_t)N * 8, nb, 21, in, st);
        if (e != hipSuccess) return KF_E_HIP;
        hipLaunchKernelGGL(k_rebase, dim3((unsigned)((nc + 1 + 255) / 256)), dim3(256), 0, st, (int32_t*)(slot + L.off),
                           (int)(nc + 1), h0);
        if (hipGetLastError() != hipSuccess) return KF_E_HIP;
        kf_measurements mc = *meas;
        mc.n_tracks = (int32_t)nc;
        mc.n_hits = hc;
        mc.hit_offsets = (const int32_t*)(slot + L.off);
        mc.surface_id = (const int32_t*)(slot + L.sid);
        mc.loc = (const double*)(slot + L.loc);
        mc.cov = (const double*)(slot + L.cov);
        kf_seeds sc = *seeds;
        sc.par = (const double*)(slot + L.seed);
        sc.cov = (const double*)(slot + L.seed_cov);
        kf_outputs oc;
        memset(&oc, 0, sizeof(oc));
        oc.par = (double*)(slot + L.par);
        oc.cov = (double*)(slot + L.pcov);
        oc.tgt_par = (double*)(slot + L.tgt_par);
        oc.tgt_cov = (double*)(slot + L.tgt_cov);
        oc.chi2 = (double*)(slot + L.chi2);
        oc.ndf = (int32_t*)(slot + L.ndf);
        oc.status = (uint8_t*)(slot + L.status);
        const kf_config r = resolve(cfg, surf, field, &mc);
        rc = enqueue_fit(&r, surf, field, &mc, &sc, &oc, slot + L.fit, st);
        if (rc != KF_OK) return rc;
        e = copy_rows(out->par + h0, (size_t)H * 8, slot + L.par, hb, hb, 6, outk, st);
        if (e == hipSuccess) e = copy_rows(out->cov + h0, (size_t)H * 8, slot + L.pcov, hb, hb, 21, outk, st);
        if (e == hipSuccess) e = copy_rows(out->tgt_par + t0, (size_t)N * 8, slot + L.tgt_par, nb, nb, 6, outk, st);
        if (e == hipSuccess) e = copy_rows(out->tgt_cov + t0, (size_t)N * 8, slot + L.tgt_cov, nb, nb, 21, outk, st);
        if (e == hipSuccess) e = hipMemcpyAsync(out->chi2 + t0, slot + L.chi2, nb, outk, st);
        if (e == hipSuccess) e = hipMemcpyAsync(out->ndf + t0, slot + L.ndf, (size_t)nc * 4, outk, st);
        if (e == hipSuccess) e = hipMemcpyAsync(out->status + t0, slot + L.status, (size_t)nc, outk, st);
        if (e != hipSuccess) return KF_E_HIP;
    }
    return KF_OK;
}

}  // extern "C"
