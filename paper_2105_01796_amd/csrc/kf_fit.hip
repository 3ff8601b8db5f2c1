// kf_fit.hip -- kernels and C ABI of the MI355X batched Kalman-filter track fit.
//
// Forward filter + RTS smoother (Sect. 2; Sect. 4.1), one lane per track:
//   * the surface table is staged once per workgroup in LDS;
//   * the forward pass writes, per hit, the predicted state, the filtered
//     state and the RTS gain of the previous state (computed as soon as the
//     predicted covariance exists, with the FP64 Cholesky solve) to a
//     tile-major workspace [tile][hit][component][64 lanes]: a wave's 64
//     lanes store/load 64 consecutive doubles (coalesced), and every
//     component sits at a compile-time offset from one per-lane base, so the
//     addressing costs neither scalar nor vector registers per component;
//   * the backward pass is then a light streaming pass: it reads them back,
//     applies the smoother and writes the smoothed states to the caller's CSR
//     outputs, and the seed-surface result to tgt_*.
// Schedules: DIRECT (track i on lane i) and SORTED (tracks ordered by hit
// count, longest first; persistent waves pull 64-track tiles from a queue so
// that waves carry tracks of equal length).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <mutex>
#include "kf_device.hpp"
#include "kf.h"

using namespace kfm;

namespace {

// workspace doubles per hit: filtered state xf 6, Cf 21; smoother gain of the
// previous state A 36 (row-major); predicted state xp 6, Cp 21
constexpr int NC = 90;
constexpr int OFF_XF = 0, OFF_CF = 6, OFF_A = 27, OFF_XP = 63, OFF_CP = 69;
constexpr int TILE = 64;

struct FitArgs {
    int n_tracks;
    int n_surf;
    int seed_sid;
    int max_hits;
    int64_t n_hits;
    int64_t tile_doubles;       // workspace doubles per 64-track tile = max_hits * NC * 64
    const int32_t* off;
    const int32_t* sid;
    const double* loc;
    const double* cov;
    const double* center;
    const double* rot;
    const double* x0;
    const double* seed;
    const double* seed_cov;
    FieldDef field;
    Cfg cfg;
    int bnz;                    // field is not identically zero
    double* par;
    double* pcov;
    double* tgt_par;
    double* tgt_cov;
    double* chi2;
    int32_t* ndf;
    uint8_t* status;
    int32_t* trials;
    double* filt_par;
    double* filt_cov;
    double* ws;
    const int32_t* order;       // slot -> track (SORTED) or NULL
    int32_t* tile_counter;      // SORTED queue head
    int n_tiles;
};

__device__ inline bool finite(double v) { return isfinite(v); }

// Store v[0..N) at p, p + H, p + 2H, ...: the running pointer is kept opaque
// so the compiler adds H per row instead of materialising N scalar offsets.
template <int N>
__device__ inline void store_rows(double* p, int64_t H, const double (&v)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        *p = v[i];
        p += H;
        __asm__ volatile("" : "+v"(p));
    }
}

// Fit the track held by workspace slot `slot` (track index t).
template <class P, int FK>
__device__ void fit_one(const FitArgs& a, const double* __restrict__ sm, int64_t slot, int t) {
    const int o = a.off[t];
    int n = a.off[t + 1] - o;
    const int64_t H = a.n_hits;
    int status = ST_OK;
    if (o < 0 || n < 0 || (int64_t)o + n > H) { status = ST_BAD_INPUT; n = 0; }   // corrupt CSR: touch no hit
    else if (n < 3) status = ST_TOO_FEW;
    else if (n > a.max_hits) status = ST_BAD_INPUT;
    double x[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) x[i] = a.seed[i * a.n_tracks + t];
    if (status == ST_OK) {
        double C[21];
#pragma unroll
        for (int q = 0; q < 21; ++q) C[q] = a.seed_cov[q * a.n_tracks + t];
        bool ok = true;
#pragma unroll
        for (int i = 0; i < 6; ++i) ok = ok && finite(x[i]);
#pragma unroll
        for (int q = 0; q < 21; ++q) ok = ok && finite(C[q]);
        // seed covariance must be SPD (Cholesky pivots)
        if (ok) {
            double L[6][6];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                double s = C[sy(j, j)];
#pragma unroll
                for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
                ok = ok && (s > 0.0);
                const double l = sqrt(s > 0.0 ? s : 1.0);
                L[j][j] = l;
#pragma unroll
                for (int i = j + 1; i < 6; ++i) {
                    double tt = C[sy(i, j)];
#pragma unroll
                    for (int k = 0; k < j; ++k) tt -= L[i][k] * L[j][k];
                    L[i][j] = tt / l;
                }
            }
        }
        for (int k = 0; k < n && ok; ++k) {
            const int s = a.sid[o + k];
            const double m0 = a.loc[o + k], m1 = a.loc[H + o + k];
            const double v0 = a.cov[o + k], v1 = a.cov[H + o + k], v2 = a.cov[2 * H + o + k];
            ok = (s >= 0 && s < a.n_surf) && finite(m0) && finite(m1) && finite(v0) && finite(v1) && finite(v2) &&
                 (v0 > 0.0) && (v0 * v2 - v1 * v1 > 0.0);
        }
        if (!ok) status = ST_BAD_INPUT;
    }
    Field<P, FK> fl;
    fl.init(a.field);
    // this lane's column of its tile: component c of hit k at wl[(k * NC + c) * TILE]
    double* wl = a.ws + (slot / TILE) * a.tile_doubles + (slot % TILE);
    double chi2 = 0.0;
    // ---- forward filter ----
    int prev = a.seed_sid;
    for (int k = 0; k < n && status == ST_OK; ++k) {
        const int s = a.sid[o + k];
        const double* sa = sm + prev * SURF_STRIDE;
        const double* sb = sm + s * SURF_STRIDE;
        double q22 = 0.0, q33 = 0.0;
        if (a.cfg.ms) highland(sa, x, a.cfg.mass, &q22, &q33);
        double xp[6], F[25];
        int tr = 0;
        status = transport<P, FK>(fl, a.field, a.cfg, sa, sb, x, xp, F, &tr);
        if (a.trials) a.trials[o + k] = tr;
        if (status != ST_OK) break;
        phase_boundary();
        // the previous filtered covariance is not kept live across the
        // propagation: it is re-read from the slot written one step earlier
        double CQ[21];
        if (k == 0) {
#pragma unroll
            for (int q = 0; q < 21; ++q) CQ[q] = a.seed_cov[q * a.n_tracks + t];
        } else {
            const double* wprev = wl + (k - 1) * (NC * TILE);
#pragma unroll
            for (int q = 0; q < 21; ++q) CQ[q] = wprev[(OFF_CF + q) * TILE];
        }
        CQ[sy(2, 2)] += q22;
        CQ[sy(3, 3)] += q33;
        phase_boundary();
        double* w = wl + k * (NC * TILE);
        {
            double Cp[21];
            transport_cov(F, CQ, Cp);
#pragma unroll
            for (int i = 0; i < 6; ++i) w[(OFF_XP + i) * TILE] = xp[i];
#pragma unroll
            for (int q = 0; q < 21; ++q) w[(OFF_CP + q) * TILE] = Cp[q];
            phase_boundary();
            // RTS gain of the previous state, A = C F^T Cp^-1 (C without the noise)
            double L[21], id[6];
            const bool spd = chol6(Cp, L, id);
            CQ[sy(2, 2)] -= q22;
            CQ[sy(3, 3)] -= q33;
            phase_boundary();
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                double g[6];
                smoother_gain_row(F, CQ, L, id, c, g);
                // g is column c of A^T = row c of A
#pragma unroll
                for (int i = 0; i < 6; ++i) w[(OFF_A + 6 * c + i) * TILE] = g[i];
                phase_boundary();
            }
            if (!spd) { status = ST_NOT_SPD; break; }
        }
        // the update reads the predicted covariance back (L1/L2 hit) rather
        // than holding it across the gain solve
        double Cp[21];
#pragma unroll
        for (int q = 0; q < 21; ++q) Cp[q] = w[(OFF_CP + q) * TILE];
        const double m[2] = {a.loc[o + k], a.loc[H + o + k]};
        const double V[3] = {a.cov[o + k], a.cov[H + o + k], a.cov[2 * H + o + k]};
        double ck, C[21];
        phase_boundary();
        status = kalman_update(xp, Cp, m, V, x, C, &ck);
        if (status != ST_OK) break;
        phase_boundary();
        chi2 += ck;
#pragma unroll
        for (int i = 0; i < 6; ++i) w[(OFF_XF + i) * TILE] = x[i];
#pragma unroll
        for (int q = 0; q < 21; ++q) w[(OFF_CF + q) * TILE] = C[q];
        if (a.filt_par) {
            store_rows(a.filt_par + o + k, H, x);
            store_rows(a.filt_cov + o + k, H, C);
        }
        prev = s;
    }
    // ---- RTS smoother ----
    double C[21];
    if (status == ST_OK) {
        // last hit: smoothed = filtered (re-read, so the covariance is not kept
        // live in registers across the forward loop)
        {
            const double* w = wl + (n - 1) * (NC * TILE);
#pragma unroll
            for (int i = 0; i < 6; ++i) x[i] = w[(OFF_XF + i) * TILE];
#pragma unroll
            for (int q = 0; q < 21; ++q) C[q] = w[(OFF_CF + q) * TILE];
        }
        store_rows(a.par + o + n - 1, H, x);
        store_rows(a.pcov + o + n - 1, H, C);
        for (int k = n - 2; k >= -1; --k) {
            const double* w1 = wl + (k + 1) * (NC * TILE);
            double xf[6], Cf[21], A[36], xp1[6], Cp1[21];
            if (k >= 0) {
                const double* w = wl + k * (NC * TILE);
#pragma unroll
                for (int i = 0; i < 6; ++i) xf[i] = w[(OFF_XF + i) * TILE];
#pragma unroll
                for (int q = 0; q < 21; ++q) Cf[q] = w[(OFF_CF + q) * TILE];
            } else {
#pragma unroll
                for (int i = 0; i < 6; ++i) xf[i] = a.seed[i * a.n_tracks + t];
#pragma unroll
                for (int q = 0; q < 21; ++q) Cf[q] = a.seed_cov[q * a.n_tracks + t];
            }
#pragma unroll
            for (int q = 0; q < 36; ++q) A[q] = w1[(OFF_A + q) * TILE];
#pragma unroll
            for (int i = 0; i < 6; ++i) xp1[i] = w1[(OFF_XP + i) * TILE];
#pragma unroll
            for (int q = 0; q < 21; ++q) Cp1[q] = w1[(OFF_CP + q) * TILE];
            rts_apply(xf, Cf, A, xp1, Cp1, x, C);
            if (k >= 0) {
                store_rows(a.par + o + k, H, x);
                store_rows(a.pcov + o + k, H, C);
            }
        }
    }
    if (status == ST_OK) {
#pragma unroll
        for (int i = 0; i < 6; ++i) a.tgt_par[i * a.n_tracks + t] = x[i];
#pragma unroll
        for (int q = 0; q < 21; ++q) a.tgt_cov[q * a.n_tracks + t] = C[q];
        a.chi2[t] = chi2;
    } else {
        const double nan = __longlong_as_double(0x7ff8000000000000LL);
        for (int k = 0; k < n; ++k) {
#pragma unroll
            for (int i = 0; i < 6; ++i) a.par[i * H + o + k] = nan;
#pragma unroll
            for (int q = 0; q < 21; ++q) a.pcov[q * H + o + k] = nan;
            if (a.filt_par) {
#pragma unroll
                for (int i = 0; i < 6; ++i) a.filt_par[i * H + o + k] = nan;
#pragma unroll
                for (int q = 0; q < 21; ++q) a.filt_cov[q * H + o + k] = nan;
            }
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) a.tgt_par[i * a.n_tracks + t] = nan;
#pragma unroll
        for (int q = 0; q < 21; ++q) a.tgt_cov[q * a.n_tracks + t] = nan;
        a.chi2[t] = nan;
    }
    a.ndf[t] = 2 * n - (a.bnz ? 5 : 4);
    a.status[t] = (uint8_t)status;
}

__device__ inline void stage_surfaces(const FitArgs& a, double* sm) {
    const int S = a.n_surf;
    for (int i = threadIdx.x; i < S * SURF_STRIDE; i += blockDim.x) {
        const int s = i / SURF_STRIDE, f = i - s * SURF_STRIDE;
        double v;
        if (f < 3) v = a.center[f * S + s];
        else if (f < 12) v = a.rot[(f - 3) * S + s];
        else v = a.x0[s];
        sm[i] = v;
    }
    __syncthreads();
}

// SORTED selects the schedule at compile time (one inlined copy of the fit
// per kernel); OCC is the occupancy target in waves per SIMD, which caps the
// registers per lane.
template <class P, int FK, int OCC, bool SORTED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
k_fit(FitArgs a) {
    extern __shared__ double sm[];
    stage_surfaces(a, sm);
    if (!SORTED) {
        const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (i < a.n_tracks) fit_one<P, FK>(a, sm, i, (int)i);
        return;
    }
    const int lane = threadIdx.x & (TILE - 1);
    for (;;) {
        int tile = 0;
        if (lane == 0) tile = atomicAdd(a.tile_counter, 1);
        tile = __shfl(tile, 0, TILE);
        if (tile >= a.n_tiles) break;
        const int64_t i = (int64_t)tile * TILE + lane;
        if (i < a.n_tracks) fit_one<P, FK>(a, sm, i, a.order[i]);
    }
}

// ---- sorted schedule: order tracks by hit count, longest first ----
// counts[b] for b = 0..KF_MAX_HITS+1 (bin of n clipped), then positions.
__global__ void k_zero_i32(int32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__device__ inline int len_bin(const int32_t* off, int t, int max_hits) {
    int n = off[t + 1] - off[t];
    n = n < 0 ? 0 : n;
    n = n > max_hits + 1 ? max_hits + 1 : n;
    return (max_hits + 1) - n;      // longest first
}

// Each workgroup builds its histogram in LDS and adds it to the global one
// with one atomic per non-empty bin (equal lengths would otherwise serialise
// every track on one address).
constexpr int NBINS = KF_MAX_HITS + 2;

__global__ void __launch_bounds__(256) k_hist(const int32_t* off, int N, int max_hits, int32_t* counts) {
    __shared__ int32_t h[NBINS];
    for (int i = threadIdx.x; i < NBINS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N) atomicAdd(&h[len_bin(off, t, max_hits)], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < NBINS; i += blockDim.x)
        if (h[i]) atomicAdd(&counts[i], h[i]);
}

// exclusive scan of the NBINS (<= 256) bins by one workgroup of 256 threads
__global__ void __launch_bounds__(256) k_scan(int32_t* counts) {
    __shared__ int32_t s[256];
    const int i = threadIdx.x;
    const int own = i < NBINS ? counts[i] : 0;
    s[i] = own;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int v = i >= d ? s[i - d] : 0;
        __syncthreads();
        s[i] += v;
        __syncthreads();
    }
    if (i < NBINS) counts[i] = s[i] - own;
}

// each workgroup reserves one range per bin, then places its tracks
__global__ void __launch_bounds__(256) k_scatter(const int32_t* off, int N, int max_hits, int32_t* pos,
                                                 int32_t* order) {
    __shared__ int32_t h[NBINS], base[NBINS];
    for (int i = threadIdx.x; i < NBINS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int b = 0, local = 0;
    if (t < N) {
        b = len_bin(off, t, max_hits);
        local = atomicAdd(&h[b], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NBINS; i += blockDim.x)
        if (h[i]) base[i] = atomicAdd(&pos[i], h[i]);
    __syncthreads();
    if (t < N) order[base[b] + local] = t;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct WsLayout {
    int64_t tile_doubles;
    size_t fit_bytes;     // [tiles][max_hits][NC][64] doubles
    size_t order_off;     // int32 [tiles * 64]
    size_t counts_off;    // int32 [NBINS] histogram / positions
    size_t counter_off;   // int32 tile counter
    size_t total;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

WsLayout ws_layout(int64_t n_tracks, int max_hits) {
    WsLayout L;
    const int64_t tiles = n_tracks > 0 ? (n_tracks + TILE - 1) / TILE : 1;
    L.tile_doubles = (int64_t)max_hits * NC * TILE;
    L.fit_bytes = (size_t)tiles * L.tile_doubles * sizeof(double);
    L.order_off = align_up(L.fit_bytes, 256);
    L.counts_off = align_up(L.order_off + (size_t)tiles * TILE * 4, 256);
    L.counter_off = align_up(L.counts_off + NBINS * 4, 256);
    L.total = align_up(L.counter_off + 256, 256);
    return L;
}

int g_num_cu = 0;
std::once_flag g_cu_once;

int num_cu() {
    std::call_once(g_cu_once, [] {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            g_num_cu = p.multiProcessorCount;
        if (g_num_cu <= 0) g_num_cu = 256;
    });
    return g_num_cu;
}

int validate(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field, const kf_measurements* meas,
             const kf_seeds* seeds, const kf_outputs* out) {
    if (!cfg || !surf || !field || !meas || !seeds || !out) return KF_E_NULL;
    if (cfg->precision != KF_PREC_FP64 && cfg->precision != KF_PREC_MIXED) return KF_E_ENUM;
    if (cfg->schedule != KF_SCHED_AUTO && cfg->schedule != KF_SCHED_DIRECT && cfg->schedule != KF_SCHED_SORTED)
        return KF_E_ENUM;
    if (field->kind != KF_FIELD_UNIFORM && field->kind != KF_FIELD_SOLENOID) return KF_E_ENUM;
    if (cfg->block != 0 && cfg->block != 64 && cfg->block != 128 && cfg->block != 256) return KF_E_VALUE;
    if (cfg->waves_per_cu < 0 || cfg->waves_per_cu > 32) return KF_E_VALUE;
    if (cfg->occupancy < 0 || cfg->occupancy > 3) return KF_E_VALUE;
    if (!(cfg->rk_tol > 0.0) || !(cfg->land_tol > 0.0) || !(cfg->mass >= 0.0) || cfg->max_steps < 1)
        return KF_E_VALUE;
    if (!isfinite(field->b0[0]) || !isfinite(field->b0[1]) || !isfinite(field->b0[2]) || !isfinite(field->a))
        return KF_E_VALUE;
    if (meas->n_tracks < 0 || meas->n_hits < 0 || meas->max_hits < 1 || meas->max_hits > KF_MAX_HITS)
        return KF_E_SIZE;
    if (surf->n < 1 || surf->n > KF_MAX_SURFACES) return KF_E_SIZE;
    if (seeds->surface_id < 0 || seeds->surface_id >= surf->n) return KF_E_SIZE;
    if (meas->n_tracks == 0) return KF_OK;
    if (!surf->center || !surf->rot || !surf->x_over_X0) return KF_E_NULL;
    if (!meas->hit_offsets || !seeds->par || !seeds->cov) return KF_E_NULL;
    if (meas->n_hits > 0 && (!meas->surface_id || !meas->loc || !meas->cov)) return KF_E_NULL;
    if (!out->par && meas->n_hits > 0) return KF_E_NULL;
    if (!out->cov && meas->n_hits > 0) return KF_E_NULL;
    if (!out->tgt_par || !out->tgt_cov || !out->chi2 || !out->ndf || !out->status) return KF_E_NULL;
    if ((out->filt_par == nullptr) != (out->filt_cov == nullptr)) return KF_E_NULL;
    return KF_OK;
}

template <class P, int FK, int OCC>
hipError_t launch_fit_occ(const FitArgs& a, int sched, int block, int waves_per_cu, hipStream_t stream) {
    const size_t shm = (size_t)a.n_surf * SURF_STRIDE * sizeof(double);
    int grid;
    if (sched == KF_SCHED_SORTED) {
        grid = num_cu() * waves_per_cu * TILE / block;
        const int need = (a.n_tiles * TILE + block - 1) / block;
        if (grid > need) grid = need;
        if (grid < 1) grid = 1;
    } else {
        grid = (int)((a.n_tracks + block - 1) / block);
    }
    if (sched == KF_SCHED_SORTED)
        hipLaunchKernelGGL((k_fit<P, FK, OCC, true>), dim3(grid), dim3(block), shm, stream, a);
    else
        hipLaunchKernelGGL((k_fit<P, FK, OCC, false>), dim3(grid), dim3(block), shm, stream, a);
    return hipGetLastError();
}

template <class P, int FK>
hipError_t launch_fit(const FitArgs& a, int sched, int block, int waves_per_cu, int occ, hipStream_t stream) {
    switch (occ) {
        case 1: return launch_fit_occ<P, FK, 1>(a, sched, block, waves_per_cu, stream);
        case 3: return launch_fit_occ<P, FK, 3>(a, sched, block, waves_per_cu, stream);
        default: return launch_fit_occ<P, FK, 2>(a, sched, block, waves_per_cu, stream);
    }
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
                  size_t workspace_bytes, void* stream_) {
    int rc = validate(cfg, surf, field, meas, seeds, out);
    if (rc != KF_OK) return rc;
    if (meas->n_tracks == 0) return KF_OK;
    const WsLayout L = ws_layout(meas->n_tracks, meas->max_hits);
    if (!workspace) return KF_E_WS;
    if (workspace_bytes < L.total) return KF_E_WS;
    hipStream_t stream = (hipStream_t)stream_;
    char* wsb = (char*)workspace;

    FitArgs a;
    memset(&a, 0, sizeof(a));
    a.n_tracks = meas->n_tracks;
    a.n_surf = surf->n;
    a.seed_sid = seeds->surface_id;
    a.max_hits = meas->max_hits;
    a.n_hits = meas->n_hits;
    a.tile_doubles = L.tile_doubles;
    a.off = meas->hit_offsets;
    a.sid = meas->surface_id;
    a.loc = meas->loc;
    a.cov = meas->cov;
    a.center = surf->center;
    a.rot = surf->rot;
    a.x0 = surf->x_over_X0;
    a.seed = seeds->par;
    a.seed_cov = seeds->cov;
    a.field.kind = field->kind;
    for (int i = 0; i < 3; ++i) a.field.b0[i] = field->b0[i];
    a.field.a = field->a;
    a.cfg.ms = cfg->multiple_scattering ? 1 : 0;
    a.cfg.mass = cfg->mass;
    a.cfg.tol = cfg->rk_tol;
    a.cfg.land_tol = cfg->land_tol;
    a.cfg.max_steps = cfg->max_steps;
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

    int sched = cfg->schedule;
    if (sched == KF_SCHED_AUTO) sched = KF_SCHED_SORTED;
    int block = cfg->block ? cfg->block : 64;
    int wpc = cfg->waves_per_cu ? cfg->waves_per_cu : 8;

    hipError_t e = hipSuccess;
    if (sched == KF_SCHED_SORTED) {
        const int nb = NBINS;
        int32_t* counts = (int32_t*)(wsb + L.counts_off);
        const int N = a.n_tracks;
        const int tb = 256, tg = (N + tb - 1) / tb;
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(128), 0, stream, counts, nb);
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, stream, a.tile_counter, 1);
        hipLaunchKernelGGL(k_hist, dim3(tg), dim3(tb), 0, stream, a.off, N, a.max_hits, counts);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(256), 0, stream, counts);
        hipLaunchKernelGGL(k_scatter, dim3(tg), dim3(tb), 0, stream, a.off, N, a.max_hits, counts,
                           (int32_t*)a.order);
        e = hipGetLastError();
        if (e != hipSuccess) return KF_E_HIP;
    }
    const bool mixed = cfg->precision == KF_PREC_MIXED;
    const int occ = cfg->occupancy ? cfg->occupancy : 1;
    if (field->kind == KF_FIELD_UNIFORM)
        e = mixed ? launch_fit<float, FIELD_UNIFORM>(a, sched, block, wpc, occ, stream)
                  : launch_fit<double, FIELD_UNIFORM>(a, sched, block, wpc, occ, stream);
    else
        e = mixed ? launch_fit<float, FIELD_SOLENOID>(a, sched, block, wpc, occ, stream)
                  : launch_fit<double, FIELD_SOLENOID>(a, sched, block, wpc, occ, stream);
    return e == hipSuccess ? KF_OK : KF_E_HIP;
}

}  // extern "C"
