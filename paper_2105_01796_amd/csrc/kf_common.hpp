// kf_common.hpp -- pieces shared by the fit and the adjoint translation units:
// per-lane workspace row helpers, track validation, the LDS surface table
// (with optional alignment corrections), the tile queue of the persistent
// schedule and the length sort that feeds it.
//
// Everything here has internal linkage (anonymous namespace): each .hip file
// gets its own copy of these kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <limits.h>
#include <mutex>
#include "kf_device.hpp"
#include "kf.h"

namespace {

using namespace kfm;

constexpr int TILE = 64;    // tracks per tile = lanes per wave

__device__ inline bool finite(double v) { return isfinite(v); }

// Component-major rows: v[i] lives at p + i * stride.  The running pointer
// is kept opaque so the compiler adds the stride per row at the point of use
// instead of computing all N per-lane addresses once and keeping them live
// across the whole fit (27 64-bit addresses would otherwise occupy 54
// registers for the track's lifetime).
template <int N>
__device__ inline void store_rows(double* p0, int64_t stride, const double (&v)[N]) {
    auto p = gbl(p0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        *p = v[i];
        p += stride;
        __asm__ volatile("" : "+v"(p));
    }
}

template <int N>
__device__ inline void load_rows(const double* p0, int64_t stride, double (&v)[N]) {
    auto p = gbl(p0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        v[i] = *p;
        p += stride;
        __asm__ volatile("" : "+v"(p));
    }
}

template <int N>
__device__ inline void fill_rows(double* p0, int64_t stride, double val) {
    auto p = gbl(p0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        *p = val;
        p += stride;
        __asm__ volatile("" : "+v"(p));
    }
}

// One hit is usable: a known surface of a measuring type (plane or disc;
// stype NULL: all planes), finite coordinates, an SPD covariance.
__device__ inline bool hit_ok(int s, int n_surf, const double m[2], const double V[3],
                              const int32_t* stype = nullptr) {
    return (s >= 0 && s < n_surf) && (!stype || stype[s] == 0 || stype[s] == 1) && finite(m[0]) &&
           finite(m[1]) && finite(V[0]) && finite(V[1]) && finite(V[2]) && (V[0] > 0.0) &&
           (V[0] * V[2] - V[1] * V[1] > 0.0);
}

// The per-track checks that need no hit: CSR range, hit count, a finite seed
// with an SPD covariance.  On a corrupt CSR range n is set to 0 so no hit is
// touched.
__device__ inline int check_head(const int32_t* off, const double* seed, const double* seed_cov, int64_t H,
                                 int64_t N, int max_hits, int t, int& o, int& n) {
    o = off[t];
    n = off[t + 1] - o;
    if (o < 0 || n < 0 || (int64_t)o + n > H) { n = 0; return ST_BAD_INPUT; }
    if (n < 3) return ST_TOO_FEW;
    if (n > max_hits) return ST_BAD_INPUT;
    double x[6], C[21];
    load_rows(seed + t, N, x);
    load_rows(seed_cov + t, N, C);
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
    return ok ? ST_OK : ST_BAD_INPUT;
}

// Some hit in [k0, n) of the track at CSR offset o is unusable.
__device__ inline bool any_bad_hit(const int32_t* sid, const double* loc, const double* cov, int64_t H, int n_surf,
                                   int o, int k0, int n, const int32_t* stype = nullptr) {
    for (int k = k0; k < n; ++k) {
        double m[2], V[3];
        load_rows(loc + o + k, H, m);
        load_rows(cov + o + k, H, V);
        if (!hit_ok(sid[o + k], n_surf, m, V, stype)) return true;
    }
    return false;
}

// Every input check of one track, as the CPU reference applies them before
// fitting (all of them report ST_BAD_INPUT except the hit count).
__device__ inline int check_track(const int32_t* off, const int32_t* sid, const double* loc, const double* cov,
                                  const double* seed, const double* seed_cov, int64_t H, int64_t N, int n_surf,
                                  int max_hits, int t, int& o, int& n) {
    const int st = check_head(off, seed, seed_cov, H, N, max_hits, t, o, n);
    if (st != ST_OK) return st;
    return any_bad_hit(sid, loc, cov, H, n_surf, o, 0, n) ? ST_BAD_INPUT : ST_OK;
}

// The seed surface is a plane (the transports start from plane coordinates there)
__device__ inline bool seed_surface_ok(const int32_t* stype, int seed_sid) {
    return !stype || stype[seed_sid] == 0;
}

// Surface s with an alignment correction a = (dx, dy, dz, alpha, beta, gamma):
// centre c + (dx, dy, dz), rotation R Rx(alpha) Ry(beta) Rz(gamma), i.e. the
// plane turned about its own u, v, n axes.
__device__ inline void apply_alignment(const double al[6], double s[SURF_STRIDE]) {
    double sa, ca, sb, cb, sg, cg;
    angle_sincos(al[3], &sa, &ca);
    angle_sincos(al[4], &sb, &cb);
    angle_sincos(al[5], &sg, &cg);
    const double Rx[3][3] = {{1.0, 0.0, 0.0}, {0.0, ca, -sa}, {0.0, sa, ca}};
    const double Ry[3][3] = {{cb, 0.0, sb}, {0.0, 1.0, 0.0}, {-sb, 0.0, cb}};
    const double Rz[3][3] = {{cg, -sg, 0.0}, {sg, cg, 0.0}, {0.0, 0.0, 1.0}};
    double T1[3][3], T2[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += s[3 + 3 * i + k] * Rx[k][j];
            T1[i][j] = acc;
        }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += T1[i][k] * Ry[k][j];
            T2[i][j] = acc;
        }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += T2[i][k] * Rz[k][j];
            s[3 + 3 * i + j] = acc;
        }
#pragma unroll
    for (int i = 0; i < 3; ++i) s[i] += al[i];
}

// Surface table in LDS: c[3], R[9] row-major, x/X0, type per surface (14
// doubles).  Type slot: 1 for a disc, else 0; with `radius` given (the
// kernels built for cylinders and lines) also 3 for a line and minus the
// radius for a cylinder.
__device__ inline double table_type_slot(const int32_t* stype, const double* radius, int s) {
    if (!stype) return 0.0;
    const int ty = stype[s];
    if (ty == 1) return 1.0;
    if (radius && ty == 3) return 3.0;
    if (radius && ty == 2) return -radius[s];
    return 0.0;
}

__device__ inline void stage_surfaces(int S, const double* center, const double* rot, const double* x0,
                                      const double* align, const int32_t* stype, double* sm,
                                      const double* radius = nullptr) {
    if (!align) {
        for (int i = threadIdx.x; i < S * SURF_STRIDE; i += blockDim.x) {
            const int s = i / SURF_STRIDE, f = i - s * SURF_STRIDE;
            double v;
            if (f < 3) v = center[f * S + s];
            else if (f < 12) v = rot[(f - 3) * S + s];
            else if (f == 12) v = x0[s];
            else v = table_type_slot(stype, radius, s);
            sm[i] = v;
        }
    } else {
        for (int s = threadIdx.x; s < S; s += blockDim.x) {
            double v[SURF_STRIDE], al[6];
#pragma unroll
            for (int f = 0; f < 3; ++f) v[f] = center[f * S + s];
#pragma unroll
            for (int f = 0; f < 9; ++f) v[3 + f] = rot[f * S + s];
            v[12] = x0[s];
            v[13] = table_type_slot(stype, radius, s);
#pragma unroll
            for (int c = 0; c < 6; ++c) al[c] = align[c * S + s];
            apply_alignment(al, v);
#pragma unroll
            for (int f = 0; f < SURF_STRIDE; ++f) sm[s * SURF_STRIDE + f] = v[f];
        }
    }
    __syncthreads();
}

// Tile source: DIRECT maps workgroups to tiles in order; SORTED makes every
// wave pull tiles (64 tracks of equal length, longest first) from a queue
// until it is empty.
template <bool SORTED>
__device__ inline int next_tile(int32_t* counter, int& iter) {
    if (!SORTED) return iter++ == 0 ? (int)((blockIdx.x * blockDim.x + threadIdx.x) / TILE) : INT_MAX;
    int tile = 0;
    if ((threadIdx.x & (TILE - 1)) == 0) tile = atomicAdd(counter, 1);
    return __shfl(tile, 0, TILE);
}

// ---- sorted schedule: order tracks by hit count, longest first ----
// A stable counting sort: tracks of equal length keep their input order, so a
// tile holds consecutive tracks (their CSR outputs are neighbours in memory)
// and the order is the same on every run.
//   k_hist:     per-block histogram over the block's 256 tracks -> counts[bin][block],
//               and the per-bin totals (integer sums: order-independent)
//   k_bin_scan: one workgroup per bin: exclusive scan of the bin's per-block
//               counts, offset by the totals of the earlier bins -> first slot
//               per (bin, block)
//   k_scatter:  rank of each track among the block's tracks of its bin (wave ballots)
constexpr int NBINS = KF_MAX_HITS + 2;
constexpr int SORT_BLOCK = 256;

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

__global__ void __launch_bounds__(SORT_BLOCK) k_hist(const int32_t* off, int N, int max_hits, int n_blocks,
                                                     int32_t* counts, int32_t* totals) {
    __shared__ int32_t h[NBINS];
    for (int i = threadIdx.x; i < NBINS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N) atomicAdd(&h[len_bin(off, t, max_hits)], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < NBINS; i += blockDim.x) {
        counts[(int64_t)i * n_blocks + blockIdx.x] = h[i];
        if (h[i]) atomicAdd(&totals[i], h[i]);
    }
}

__global__ void __launch_bounds__(SORT_BLOCK) k_bin_scan(int32_t* counts, const int32_t* totals, int n_blocks) {
    __shared__ int32_t sc[SORT_BLOCK];
    __shared__ int32_t base;
    const int bin = blockIdx.x, i = threadIdx.x;
    if (i == 0) {
        int b = 0;
        for (int k = 0; k < bin; ++k) b += totals[k];
        base = b;
    }
    __syncthreads();
    int32_t carry = base;
    int32_t* row = counts + (int64_t)bin * n_blocks;
    for (int c0 = 0; c0 < n_blocks; c0 += SORT_BLOCK) {
        const int k = c0 + i;
        const int32_t own = k < n_blocks ? row[k] : 0;
        sc[i] = own;
        __syncthreads();
        for (int d = 1; d < SORT_BLOCK; d <<= 1) {
            const int32_t v = i >= d ? sc[i - d] : 0;
            __syncthreads();
            sc[i] += v;
            __syncthreads();
        }
        if (k < n_blocks) row[k] = carry + sc[i] - own;
        carry += sc[SORT_BLOCK - 1];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(SORT_BLOCK) k_scatter(const int32_t* off, int N, int max_hits, int n_blocks,
                                                        const int32_t* pos, int32_t* order) {
    constexpr int W = SORT_BLOCK / 64;
    __shared__ int32_t wc[W][NBINS];
    for (int i = threadIdx.x; i < W * NBINS; i += blockDim.x) wc[i / NBINS][i % NBINS] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool valid = t < N;
    const int b = valid ? len_bin(off, t, max_hits) : -1;
    // rank among the earlier lanes of this wave with the same bin
    int rank = 0;
    unsigned long long todo = __ballot(valid);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int bl = __shfl(b, leader);
        const unsigned long long m = __ballot(valid && b == bl);
        if (valid && b == bl) rank = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == leader) wc[w][bl] = __popcll(m);
        todo &= ~m;
    }
    __syncthreads();
    if (valid) {
        for (int v = 0; v < w; ++v) rank += wc[v][b];
        order[pos[(int64_t)b * n_blocks + blockIdx.x] + rank] = t;
    }
}

inline int sort_blocks(int N) { return N > 0 ? (N + SORT_BLOCK - 1) / SORT_BLOCK : 1; }

// int32 entries of the sort's count table for N tracks
inline int64_t sort_count_entries(int N) { return (int64_t)NBINS * sort_blocks(N); }

// Enqueue the length sort: order[] receives the track indices, longest
// first, equal lengths in input order.  heads: the two tile-queue heads
// followed by the NBINS per-bin totals (all cleared here).
constexpr int SORT_HEADS = 2 + NBINS;

inline hipError_t enqueue_length_sort(const int32_t* off, int N, int max_hits, int32_t* counts, int32_t* order,
                                      int32_t* heads, hipStream_t stream) {
    const int nb = sort_blocks(N);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(128), 0, stream, heads, SORT_HEADS);
    hipLaunchKernelGGL(k_hist, dim3(nb), dim3(SORT_BLOCK), 0, stream, off, N, max_hits, nb, counts, heads + 2);
    hipLaunchKernelGGL(k_bin_scan, dim3(NBINS), dim3(SORT_BLOCK), 0, stream, counts, (const int32_t*)(heads + 2), nb);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(SORT_BLOCK), 0, stream, off, N, max_hits, nb,
                       (const int32_t*)counts, order);
    return hipGetLastError();
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline int num_cu() {
    static int n = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            n = p.multiProcessorCount;
        if (n <= 0) n = 256;
    });
    return n;
}

// LDS one workgroup may use on this device (160 KB on gfx950).
inline size_t lds_cap() {
    static size_t v = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            v = p.maxSharedMemoryPerMultiProcessor > p.sharedMemPerBlock ? p.maxSharedMemoryPerMultiProcessor
                                                                        : p.sharedMemPerBlock;
        if (v == 0) v = 65536;
    });
    return v;
}

// Let `kernel` take `bytes` of dynamic LDS: beyond 64 KB the limit is raised
// explicitly; beyond the device's LDS it is refused (no launch).
template <class K>
inline hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes > lds_cap()) return hipErrorInvalidValue;
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Host-side checks shared by every entry point (everything but the outputs).
inline int validate_inputs(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field,
                           const kf_measurements* meas, const kf_seeds* seeds) {
    if (!cfg || !surf || !field || !meas || !seeds) return KF_E_NULL;
    if (cfg->precision != KF_PREC_FP64 && cfg->precision != KF_PREC_MIXED) return KF_E_ENUM;
    if (cfg->schedule != KF_SCHED_AUTO && cfg->schedule != KF_SCHED_DIRECT && cfg->schedule != KF_SCHED_SORTED)
        return KF_E_ENUM;
    if (field->kind != KF_FIELD_UNIFORM && field->kind != KF_FIELD_SOLENOID && field->kind != KF_FIELD_MAP)
        return KF_E_ENUM;
    if (field->kind == KF_FIELD_MAP) {
        if (!field->map) return KF_E_NULL;
        for (int i = 0; i < 3; ++i)
            if (field->map_n[i] < 2 || !(field->map_spacing[i] > 0.0) || !isfinite(field->map_spacing[i]) ||
                !isfinite(field->map_origin[i]))
                return KF_E_VALUE;
        if ((double)field->map_n[0] * field->map_n[1] * field->map_n[2] > 2.0e9) return KF_E_SIZE;
    }
    if (cfg->block != 0 && cfg->block != 64 && cfg->block != 128 && cfg->block != 256) return KF_E_VALUE;
    if (cfg->waves_per_cu < 0 || cfg->waves_per_cu > 32) return KF_E_VALUE;
    if (cfg->occupancy < 0 || cfg->occupancy > 3) return KF_E_VALUE;
    if (cfg->split_smoother < 0 || cfg->split_smoother > 1) return KF_E_VALUE;
    if (cfg->jacobians != KF_JAC_STORE && cfg->jacobians != KF_JAC_RECOMPUTE) return KF_E_VALUE;
    if (cfg->jacobians == KF_JAC_RECOMPUTE && cfg->split_smoother) return KF_E_VALUE;
    if (cfg->smoother != KF_SMOOTHER_RTS && cfg->smoother != KF_SMOOTHER_TWO_FILTER) return KF_E_VALUE;
    if (cfg->smoother == KF_SMOOTHER_TWO_FILTER &&
        (cfg->split_smoother || !(cfg->bwd_scale == 0.0 || (cfg->bwd_scale > 1.0 && isfinite(cfg->bwd_scale)))))
        return KF_E_VALUE;
    if (cfg->target != KF_TARGET_SEED_SURFACE && cfg->target != KF_TARGET_PERIGEE) return KF_E_VALUE;
    if (cfg->output != KF_OUT_AUTO && cfg->output != KF_OUT_STAGED && cfg->output != KF_OUT_SLOTS) return KF_E_VALUE;
    if (cfg->target == KF_TARGET_PERIGEE &&
        !(isfinite(cfg->perigee[0]) && isfinite(cfg->perigee[1]) && isfinite(cfg->perigee[2])))
        return KF_E_VALUE;
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
    return KF_OK;
}

inline FieldDef field_def(const kf_field* field) {
    FieldDef f;
    f.kind = field->kind;
    for (int i = 0; i < 3; ++i) f.b0[i] = field->b0[i];
    f.a = field->a;
    f.map = field->kind == KF_FIELD_MAP ? field->map : nullptr;
    for (int i = 0; i < 3; ++i) {
        f.mo[i] = field->map_origin[i];
        f.mih[i] = field->kind == KF_FIELD_MAP ? 1.0 / field->map_spacing[i] : 0.0;
        f.mn[i] = field->map_n[i];
    }
    return f;
}

inline Cfg cfg_def(const kf_config* cfg) {
    Cfg c;
    c.ms = cfg->multiple_scattering ? 1 : 0;
    c.mass = cfg->mass;
    c.tol = cfg->rk_tol;
    c.land_tol = cfg->land_tol;
    c.max_steps = cfg->max_steps;
    return c;
}

}  // namespace
