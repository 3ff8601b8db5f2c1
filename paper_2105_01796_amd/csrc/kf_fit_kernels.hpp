// kf_fit_kernels.hpp -- device code of the fit: the forward filter, the RTS
// and two-filter smoothers, the tile flush and the fit kernels, with their
// launch templates.  Each kf_fit_<field>_<precision>.hip translation unit
// instantiates the kernels of one field kind and one stepping precision
// (so the library's kernels compile in parallel); kf_fit.hip holds the host
// side, the split smoother's kernel and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <math.h>
#include "kf_common.hpp"
#include "kf_curved.hpp"

namespace kffit {
using namespace kfm;
// workspace doubles per hit: predicted state xp 6, Cp 21; transport Jacobian
// F into this hit (25 stored entries) unless the smoother recomputes it
constexpr int NC = 52;
constexpr int NC_RECOMPUTE = 27;
constexpr int OFF_XP = 0, OFF_CP = 6, OFF_F = 27;
template <bool STOREF>
constexpr int nc_of() { return STOREF ? NC : NC_RECOMPUTE; }
// LDS per wave: the carried filtered covariance [21][64 lanes] during the
// filter; after the smoother the same area holds the output transpose of
// flush_tile (FLUSH_GROUP components x FLUSH_HITS hits x 64 lanes doubles,
// then two int lists of FLUSH_HITS x 64 entries)
constexpr int CARRY = 21;
constexpr int FLUSH_HITS = 4;
constexpr int FLUSH_GROUP = 5;
constexpr int FLUSH_DOUBLES = FLUSH_GROUP * FLUSH_HITS * TILE + FLUSH_HITS * TILE;
constexpr int WAVE_LDS_DOUBLES = CARRY * TILE > FLUSH_DOUBLES ? CARRY * TILE : FLUSH_DOUBLES;
// The RTS smoother's output stage (smooth_staged): sh smoother steps of the
// wave's 64 smoothed states [27][sh][64] doubles, then the (lane, row) list
// and the CSR indices of one write-out (2 x sh x 64 ints); sh is 2 where the
// LDS holds it, else 1.
constexpr int STAGE_MAX_HITS = 2;
__host__ __device__ constexpr int stage_doubles(int sh) { return 27 * sh * TILE + sh * TILE; }
__host__ __device__ constexpr int wave_lds_doubles(int sh) {
    return stage_doubles(sh) > WAVE_LDS_DOUBLES ? stage_doubles(sh) : WAVE_LDS_DOUBLES;
}

struct FitArgs {
    int n_tracks;
    int n_surf;
    int seed_sid;
    int max_hits;
    int64_t n_hits;
    int64_t tile_doubles;       // workspace doubles per 64-track tile = max_hits * (NC or NC_RECOMPUTE) * 64
    const int32_t* off;
    const int32_t* sid;
    const double* loc;
    const double* cov;
    const double* center;
    const double* rot;
    const double* x0;
    const double* align;        // [6][S] alignment corrections or NULL
    const int32_t* stype;       // [S] surface types (0 plane, 1 disc, 2 cylinder, 3 line) or NULL
    const double* radius;       // [S] cylinder radii: set for the kernels built for cylinders and lines, else NULL
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
    int32_t* tile_counter;      // SORTED queue heads: [0] forward pass, [1] backward pass
    int n_tiles;
    double bwd_scale;           // two-filter smoother: inflation of the backward filter's start
    double perigee[3];          // perigee target: a point of the line (parallel to z)
    int stage_hits;             // RTS smoother: steps staged in LDS per write-out (1 or 2; 0: through the slots)
    int wave_lds;               // doubles of LDS per wave (carry, stage or flush area)
};

// Hit k of the track at CSR offset o lies on a disc (its azimuth wraps).
__device__ inline bool disc_hit(const FitArgs& a, int o, int k) {
    return a.stype && a.stype[a.sid[o + k]] == 1;
}

// The kernels built for cylinders and lines (CV) read a hit's surface type
// (0 plane, 1 disc, 2 cylinder, 3 line) where the plane/disc kernels ask
// whether it is a disc; `ang`: its loc1 is an azimuth.
template <bool CV>
__device__ inline int hit_kind(const FitArgs& a, int o, int k) {
    if (CV) return a.stype[a.sid[o + k]];
    return disc_hit(a, o, k) ? 1 : 0;
}
template <bool CV>
__device__ inline bool kind_ang(int kind) { return CV ? (kind == 1 || kind == 2) : kind == 1; }
template <bool CV>
__device__ inline int update_kind(int kind, const double xp[6], const double Cp[21], const double m[2],
                                  const double V[3], double xf[6], double Cf[21], double* chi2) {
    if (CV) return update_typed(kind, xp, Cp, m, V, xf, Cf, chi2);
    return kalman_update(xp, Cp, m, V, xf, Cf, chi2, kind == 1);
}
// surface-table entry -> kind
template <bool CV>
__device__ inline int table_kind(const double* __restrict__ s) { return CV ? table_type(s) : (is_disc(s) ? 1 : 0); }
template <bool CV, class P, int FK>
__device__ inline int transport_any(const Field<P, FK>& fl, const FieldDef& fd, const Cfg& cfg,
                                    const double* __restrict__ sa, const double* __restrict__ sb,
                                    const double x[6], double xp[6], double F[25], int* trials) {
    if (CV) return transport_c<P, FK>(fl, fd, cfg, sa, sb, x, xp, F, trials);
    return transport<P, FK>(fl, fd, cfg, sa, sb, x, xp, F, trials);
}
template <bool CV>
__device__ inline void highland_any(const double* __restrict__ s, const double x[6], double mass, double* q22,
                                    double* q33) {
    if (CV) highland_c(s, x, mass, q22, q33);
    else highland(s, x, mass, q22, q33);
}

// The input checks of one hit when surfaces may be cylinders or lines: the
// surface id in range and of a known type, a cylinder's radius > 0; a line
// hit has loc0 and v00 only (finite, v00 > 0; the rest is not read); the
// other types as hit_ok.
__device__ inline bool hit_ok_typed(int s, int n_surf, const double m[2], const double V[3], const int32_t* stype,
                                    const double* radius) {
    if (!(s >= 0 && s < n_surf)) return false;
    const int ty = stype[s];
    if (ty < 0 || ty > 3) return false;
    if (ty == 2 && !(radius[s] > 0.0)) return false;
    if (ty == 3) return isfinite(m[0]) && isfinite(V[0]) && V[0] > 0.0;
    return isfinite(m[0]) && isfinite(m[1]) && isfinite(V[0]) && isfinite(V[1]) && isfinite(V[2]) && (V[0] > 0.0) &&
           (V[0] * V[2] - V[1] * V[1] > 0.0);
}

template <bool CV>
__device__ inline bool hit_ok_any(const FitArgs& a, int s, const double m[2], const double V[3]) {
    if (CV) return hit_ok_typed(s, a.n_surf, m, V, a.stype, a.radius);
    return hit_ok(s, a.n_surf, m, V, a.stype);
}

template <bool CV>
__device__ inline bool any_bad_hit_any(const FitArgs& a, int o, int k0, int n) {
    if (!CV) return any_bad_hit(a.sid, a.loc, a.cov, a.n_hits, a.n_surf, o, k0, n, a.stype);
    for (int k = k0; k < n; ++k) {
        double m[2], V[3];
        load_rows(a.loc + o + k, a.n_hits, m);
        load_rows(a.cov + o + k, a.n_hits, V);
        if (!hit_ok_typed(a.sid[o + k], a.n_surf, m, V, a.stype, a.radius)) return true;
    }
    return false;
}

// Degrees of freedom: the measured coordinates (two per hit, one on a line)
// less the five fitted parameters (four without a field: q/p is then not
// measured).
template <bool CV>
__device__ inline int track_ndf(const FitArgs& a, int o, int n) {
    int dims = 2 * n;
    if (CV) {
        for (int k = 0; k < n; ++k) {
            const int s = a.sid[o + k];
            if (s >= 0 && s < a.n_surf && a.stype[s] == 3) --dims;
        }
    }
    return dims - (a.bnz ? 5 : 4);
}

// Forward filter of the track held by workspace slot `slot` (track index t):
// per hit propagation, covariance transport and the gain-matrix update.
// Each hit is checked when the loop reaches it, with its surface id and
// measurement loaded one hit ahead so the loads overlap the propagation; if
// the filter fails before the last hit, the remaining hits are checked too,
// so that a bad input anywhere wins over a filter failure (the CPU reference
// checks every hit before it fits).  `cl` is this lane's LDS slot for the
// filtered covariance between hits (component c at cl[c * 64]).  Writes
// chi2, ndf and status; a failed track gets NaN outputs here (the backward
// pass skips it).  STOREF: store the transport Jacobians for the smoother.
// CV: surfaces of every type (the kernels built for cylinders and lines).
template <class P, int FK, bool STOREF, bool CV>
__device__ void fwd_one(const FitArgs& a, const double* __restrict__ sm, double* cl, int64_t slot, int t) {
    constexpr int NW = nc_of<STOREF>();
    const int64_t H = a.n_hits;
    const int64_t N = a.n_tracks;
    int o, n;
    int status = check_head(a.off, a.seed, a.seed_cov, H, N, a.max_hits, t, o, n);
    if (status == ST_OK && !seed_surface_ok(a.stype, a.seed_sid)) status = ST_BAD_INPUT;
    double x[6];
    load_rows(a.seed + t, N, x);
    Field<P, FK> fl;
    fl.init(a.field);
    // this lane's column of its tile: component c of hit k at wl[(k * NW + c) * TILE]
    double* wl = a.ws + (slot / TILE) * a.tile_doubles + (slot % TILE);
    double chi2 = 0.0;
    // hit k's surface and measurement, loaded during hit k-1
    int s_nx = 0;
    double m_nx[2] = {0.0, 0.0}, V_nx[3] = {0.0, 0.0, 0.0};
    if (status == ST_OK) {
        s_nx = a.sid[o];
        load_rows(a.loc + o, H, m_nx);
        load_rows(a.cov + o, H, V_nx);
    }
    // ---- forward filter ----
    int prev = a.seed_sid;
    int k = 0;
    for (; k < n && status == ST_OK; ++k) {
        const int s = s_nx;
        const double m[2] = {m_nx[0], m_nx[1]};
        const double V[3] = {V_nx[0], V_nx[1], V_nx[2]};
        if (!hit_ok_any<CV>(a, s, m, V)) { status = ST_BAD_INPUT; break; }
        if (k + 1 < n) {
            s_nx = a.sid[o + k + 1];
            load_rows(a.loc + o + k + 1, H, m_nx);
            load_rows(a.cov + o + k + 1, H, V_nx);
        }
        phase_boundary();
        const double* sa = sm + prev * SURF_STRIDE;
        const double* sb = sm + s * SURF_STRIDE;
        double q22 = 0.0, q33 = 0.0;
        if (a.cfg.ms) highland_any<CV>(sa, x, a.cfg.mass, &q22, &q33);
        double xp[6], F[25];
        int tr = 0;
        status = transport_any<CV>(fl, a.field, a.cfg, sa, sb, x, xp, F, &tr);
        if (a.trials) a.trials[o + k] = tr;
        if (status != ST_OK) break;
        phase_boundary();
        double* w = wl + k * (NW * TILE);
#pragma unroll
        for (int i = 0; i < 6; ++i) w[(OFF_XP + i) * TILE] = xp[i];
        if (STOREF) {
#pragma unroll
            for (int q = 0; q < 25; ++q) w[(OFF_F + q) * TILE] = F[q];
        }
        // the previous filtered covariance waits in LDS during the propagation
        double Cp[21];
        {
            double CQ[21];
            if (k == 0) {
                load_rows(a.seed_cov + t, N, CQ);
            } else {
#pragma unroll
                for (int q = 0; q < 21; ++q) CQ[q] = cl[q * TILE];
            }
            CQ[sy(2, 2)] += q22;
            CQ[sy(3, 3)] += q33;
            phase_boundary();
            transport_cov(F, CQ, Cp);
        }
#pragma unroll
        for (int q = 0; q < 21; ++q) w[(OFF_CP + q) * TILE] = Cp[q];
        double ck, C[21];
        phase_boundary();
        status = update_kind<CV>(table_kind<CV>(sb), xp, Cp, m, V, x, C, &ck);
        if (status != ST_OK) break;
        phase_boundary();
        chi2 += ck;
#pragma unroll
        for (int q = 0; q < 21; ++q) cl[q * TILE] = C[q];
        if (a.filt_par) {
            store_rows(a.filt_par + o + k, H, x);
            store_rows(a.filt_cov + o + k, H, C);
        }
        prev = s;
    }
    if (status != ST_OK && status != ST_BAD_INPUT && status != ST_TOO_FEW && any_bad_hit_any<CV>(a, o, k + 1, n))
        status = ST_BAD_INPUT;
    if (status == ST_OK) {
        a.chi2[t] = chi2;
    } else {
        const double nan = __longlong_as_double(0x7ff8000000000000LL);
        for (int k = 0; k < n; ++k) {
            fill_rows<6>(a.par + o + k, H, nan);
            fill_rows<21>(a.pcov + o + k, H, nan);
            if (a.filt_par) {
                fill_rows<6>(a.filt_par + o + k, H, nan);
                fill_rows<21>(a.filt_cov + o + k, H, nan);
            }
        }
        fill_rows<6>(a.tgt_par + t, N, nan);
        fill_rows<21>(a.tgt_cov + t, N, nan);
        a.chi2[t] = nan;
    }
    a.ndf[t] = track_ndf<CV>(a, o, n);
    a.status[t] = (uint8_t)status;
}

// RTS smoother of one track (Sect. 2), fused after the forward pass or run by
// a separate streaming kernel: the smoothed state of the last hit is its
// filtered state; every earlier state, and finally the seed/target state,
// follows from the next hit's stored prediction and Jacobian with the gain
// A = Cf F^T Cp^-1 solved in FP64.  The smoothed state of hit k replaces the
// prediction in slot k once that has been read for the last time; flush_tile
// then writes the tile's CSR outputs (output path KF_OUT_SLOTS; smooth_staged
// is the same smoother with KF_OUT_STAGED).  Without stored Jacobians (STOREF
// false; fused only, sm is the surface table) F of the gap k -> k+1 comes from
// propagating the recomputed filtered state of hit k (or the seed) again with
// the forward pass's routine.  Returns true if the track's smoothed states are
// in its slots (false: not fitted, or failed here with NaN outputs).
// CV: surfaces of every type.
template <class P, int FK, bool STOREF, bool CV>
__device__ bool bwd_one(const FitArgs& a, const double* __restrict__ sm, int64_t slot, int t) {
    constexpr int NW = nc_of<STOREF>();
    if (a.status[t] != ST_OK) return false;
    const int o = a.off[t];
    const int n = a.off[t + 1] - o;
    const int64_t H = a.n_hits;
    const int64_t N = a.n_tracks;
    double* wl = a.ws + (slot / TILE) * a.tile_doubles + (slot % TILE);
    Field<P, FK> fl;
    if (!STOREF) fl.init(a.field);
    // prediction of hit k+1 (carried from one step to the next)
    double xp1[6], Cp1[21];
    double x[6], C[21];
    {
        const double* w = wl + (n - 1) * (NW * TILE);
        double m[2], V[3], ck;
#pragma unroll
        for (int i = 0; i < 6; ++i) xp1[i] = w[(OFF_XP + i) * TILE];
#pragma unroll
        for (int q = 0; q < 21; ++q) Cp1[q] = w[(OFF_CP + q) * TILE];
        load_rows(a.loc + o + n - 1, H, m);
        load_rows(a.cov + o + n - 1, H, V);
        update_kind<CV>(hit_kind<CV>(a, o, n - 1), xp1, Cp1, m, V, x, C, &ck);
    }
    bool ang1 = kind_ang<CV>(hit_kind<CV>(a, o, n - 1));   // loc1 of hit k+1 is an azimuth
    bool spd = true;
    int fail = ST_OK;
    int s1 = STOREF ? 0 : a.sid[o + n - 1];          // surface of hit k+1
    for (int k = n - 2; k >= -1; --k) {
        double* w1 = wl + (k + 1) * (NW * TILE);
        // every load of this step at once: F of hit k+1 (if stored), the
        // prediction and measurement of hit k (or the seed)
        double F[25], xp[6], Cp[21], m[2], V[3], xf[6], Cf[21];
        if (STOREF) {
#pragma unroll
            for (int q = 0; q < 25; ++q) F[q] = w1[(OFF_F + q) * TILE];
        }
        int s0 = a.seed_sid;
        if (k >= 0) {
            const double* w = wl + k * (NW * TILE);
#pragma unroll
            for (int i = 0; i < 6; ++i) xp[i] = w[(OFF_XP + i) * TILE];
#pragma unroll
            for (int q = 0; q < 21; ++q) Cp[q] = w[(OFF_CP + q) * TILE];
            load_rows(a.loc + o + k, H, m);
            load_rows(a.cov + o + k, H, V);
            if (!STOREF) s0 = a.sid[o + k];
        } else {
            load_rows(a.seed + t, N, xf);
            load_rows(a.seed_cov + t, N, Cf);
        }
        // slot k+1 is done: it now keeps the smoothed state of hit k+1
#pragma unroll
        for (int i = 0; i < 6; ++i) w1[(OFF_XP + i) * TILE] = x[i];
#pragma unroll
        for (int q = 0; q < 21; ++q) w1[(OFF_CP + q) * TILE] = C[q];
        double dx[6], L[21], id[6];
        spd = chol6(Cp1, L, id) && spd;
        rts_diff(x, C, xp1, Cp1, dx, ang1);              // C now holds D = Cs1 - Cp1
        const int kind0 = k >= 0 ? hit_kind<CV>(a, o, k) : 0;
        const bool ang0 = kind_ang<CV>(kind0);
        if (k >= 0) {
            double ck;
            update_kind<CV>(kind0, xp, Cp, m, V, xf, Cf, &ck);   // filtered state of hit k, as in the forward pass
#pragma unroll
            for (int i = 0; i < 6; ++i) xp1[i] = xp[i];
#pragma unroll
            for (int q = 0; q < 21; ++q) Cp1[q] = Cp[q];
        }
        if (!STOREF) {
            // F of the gap from hit k (or the seed) to hit k+1, as the forward pass propagated it
            phase_boundary();
            double xq[6];
            int tr = 0;
            const int st = transport_any<CV>(fl, a.field, a.cfg, sm + s0 * SURF_STRIDE, sm + s1 * SURF_STRIDE, xf,
                                             xq, F, &tr);
            if (st != ST_OK && fail == ST_OK) fail = st;
            s1 = s0;
        }
        phase_boundary();
        double A[36];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double g[6];
            smoother_gain_row(F, Cf, L, id, c, g);
#pragma unroll
            for (int i = 0; i < 6; ++i) A[6 * c + i] = g[i];
        }
        phase_boundary();
        rts_mean(xf, A, dx, x, ang0);
        rts_cov(A, C, Cf);
        ang1 = ang0;
#pragma unroll
        for (int q = 0; q < 21; ++q) C[q] = Cf[q];
        phase_boundary();
    }
    if (spd && fail == ST_OK) {
        store_rows(a.tgt_par + t, N, x);
        store_rows(a.tgt_cov + t, N, C);
        return true;
    }
    // a predicted covariance that is not positive definite (or a propagation
    // that did not repeat): the track fails
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    for (int k = 0; k < n; ++k) {
        fill_rows<6>(a.par + o + k, H, nan);
        fill_rows<21>(a.pcov + o + k, H, nan);
    }
    fill_rows<6>(a.tgt_par + t, N, nan);
    fill_rows<21>(a.tgt_cov + t, N, nan);
    a.chi2[t] = nan;
    a.status[t] = (uint8_t)(fail != ST_OK ? fail : ST_NOT_SPD);
    return false;
}

// All lanes of the wave, in step: LDS written by one lane is then visible to
// the others (the waves of a workgroup run different tiles, so no workgroup
// barrier may be used here).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Write-out of the smoothing stage: every lane's entries of the last `rows`
// steps (steps it - rows + 1 .. it; step i holds the smoothed state of hit
// n - 1 - i of the lane's track, from row i % sh) go to the CSR outputs.  The
// wave lists the (lane, row) pairs in the order of their CSR indices (a
// lane's entries are consecutive hits), then for each component consecutive
// lanes store consecutive entries of that list.  Every lane of the wave calls
// it (fitted: the lane's track has smoothed states; o, n: its CSR range).
__device__ inline void stage_write(const FitArgs& a, double* stg, int sh, int rows, int it, bool fitted, int o,
                                   int n) {
    const int lane = threadIdx.x & (TILE - 1);
    int32_t* own = (int32_t*)(stg + 27 * sh * TILE);      // [sh * 64]: lane | row << 6
    int32_t* dst = own + sh * TILE;                        // [sh * 64]: CSR index
    const int i0 = it - rows + 1;
    const int i1 = it < n - 1 ? it : n - 1;
    const int cnt = fitted && i1 >= i0 ? i1 - i0 + 1 : 0;
    int inc = cnt;
#pragma unroll
    for (int d = 1; d < TILE; d <<= 1) {
        const int u = __shfl_up(inc, d, TILE);
        if (lane >= d) inc += u;
    }
    const int start = inc - cnt;
    const int total = __shfl(inc, TILE - 1, TILE);
    for (int e = 0; e < cnt; ++e) {
        const int i = i1 - e;                              // ascending hit index
        own[start + e] = lane | ((i % sh) << 6);
        dst[start + e] = o + n - 1 - i;
    }
    wave_sync();
    const int64_t H = a.n_hits;
    for (int g = lane; g < total; g += TILE) {
        const int e = own[g];
        const int64_t d = dst[g];
        const double* src = stg + (e >> 6) * TILE + (e & 63);
#pragma unroll
        for (int c = 0; c < 27; ++c) {
            double* out = c < 6 ? a.par + (int64_t)c * H : a.pcov + (int64_t)(c - 6) * H;
            out[d] = src[c * sh * TILE];
        }
    }
    wave_sync();
}

// RTS smoother of the wave's tracks (Sect. 2), fused after the forward pass
// or run by a separate streaming kernel: the smoothed state of the last hit
// is its filtered state; every earlier state, and finally the seed/target
// state, follows from the next hit's stored prediction and Jacobian with the
// gain A = Cf F^T Cp^-1 solved in FP64.  Without stored Jacobians (STOREF
// false; fused only, sm is the surface table) F of the gap k -> k+1 comes from
// propagating the recomputed filtered state of hit k (or the seed) again with
// the forward pass's routine.  The lanes step together (step `it` smooths
// hit n - 1 - it of each lane's track), each lane puts its smoothed state
// into the wave's LDS stage, and every `sh` steps the wave writes the stage to
// the CSR outputs (stage_write): the states never travel through the
// workspace.  Every lane of the wave calls it (have: the lane holds track t
// in workspace slot `slot`; lw: the wave's LDS area).  Returns true if the
// track was smoothed (false: not fitted, or failed here with NaN outputs).
// CV: surfaces of every type.
template <class P, int FK, bool STOREF, bool CV>
__device__ bool smooth_staged(const FitArgs& a, const double* __restrict__ sm, double* lw, int64_t slot, int t,
                              bool have) {
    constexpr int NW = nc_of<STOREF>();
    const int lane = threadIdx.x & (TILE - 1);
    const int sh = a.stage_hits;
    const int64_t H = a.n_hits;
    const int64_t N = a.n_tracks;
    const bool fitted = have && a.status[t] == ST_OK;
    int o = 0, n = 0;
    if (fitted) {
        o = a.off[t];
        n = a.off[t + 1] - o;
    }
    int nmax = n;
#pragma unroll
    for (int d = 1; d < TILE; d <<= 1) {
        const int v = __shfl_xor(nmax, d, TILE);
        nmax = v > nmax ? v : nmax;
    }
    double* wl = a.ws + (slot / TILE) * a.tile_doubles + (slot % TILE);
    Field<P, FK> fl;
    if (!STOREF) fl.init(a.field);
    // prediction of hit k+1 (carried from one step to the next)
    double xp1[6], Cp1[21];
    double x[6], C[21];
    bool ang1 = false;
    int s1 = 0;                                         // surface of hit k+1
    if (fitted) {
        const double* w = wl + (n - 1) * (NW * TILE);
        double m[2], V[3], ck;
#pragma unroll
        for (int i = 0; i < 6; ++i) xp1[i] = w[(OFF_XP + i) * TILE];
#pragma unroll
        for (int q = 0; q < 21; ++q) Cp1[q] = w[(OFF_CP + q) * TILE];
        load_rows(a.loc + o + n - 1, H, m);
        load_rows(a.cov + o + n - 1, H, V);
        const int kind1 = hit_kind<CV>(a, o, n - 1);
        update_kind<CV>(kind1, xp1, Cp1, m, V, x, C, &ck);
        ang1 = kind_ang<CV>(kind1);
        if (!STOREF) s1 = a.sid[o + n - 1];
    }
    bool spd = true;
    int fail = ST_OK;
    // step `it` smooths hit k = n - 1 - it (k = -1: the seed/target surface);
    // step 0 is the last hit, whose smoothed state is its filtered state
    for (int it = 0; it <= nmax; ++it) {
        const int k = n - 1 - it;
        if (fitted && it > 0 && k >= -1) {
            double* w1 = wl + (k + 1) * (NW * TILE);
            // every load of this step at once: F of hit k+1 (if stored), the
            // prediction and measurement of hit k (or the seed)
            double F[25], xp[6], Cp[21], m[2], V[3], xf[6], Cf[21];
            if (STOREF) {
#pragma unroll
                for (int q = 0; q < 25; ++q) F[q] = w1[(OFF_F + q) * TILE];
            }
            int s0 = a.seed_sid;
            if (k >= 0) {
                const double* w = wl + k * (NW * TILE);
#pragma unroll
                for (int i = 0; i < 6; ++i) xp[i] = w[(OFF_XP + i) * TILE];
#pragma unroll
                for (int q = 0; q < 21; ++q) Cp[q] = w[(OFF_CP + q) * TILE];
                load_rows(a.loc + o + k, H, m);
                load_rows(a.cov + o + k, H, V);
                if (!STOREF) s0 = a.sid[o + k];
            } else {
                load_rows(a.seed + t, N, xf);
                load_rows(a.seed_cov + t, N, Cf);
            }
            double dx[6], L[21], id[6];
            spd = chol6(Cp1, L, id) && spd;
            rts_diff(x, C, xp1, Cp1, dx, ang1);              // C now holds D = Cs1 - Cp1
            const int kind0 = k >= 0 ? hit_kind<CV>(a, o, k) : 0;
            const bool ang0 = kind_ang<CV>(kind0);
            if (k >= 0) {
                double ck;
                update_kind<CV>(kind0, xp, Cp, m, V, xf, Cf, &ck);   // filtered state of hit k, as in the forward pass
#pragma unroll
                for (int i = 0; i < 6; ++i) xp1[i] = xp[i];
#pragma unroll
                for (int q = 0; q < 21; ++q) Cp1[q] = Cp[q];
            }
            if (!STOREF) {
                // F of the gap from hit k (or the seed) to hit k+1, as the forward pass propagated it
                phase_boundary();
                double xq[6];
                int tr = 0;
                const int st = transport_any<CV>(fl, a.field, a.cfg, sm + s0 * SURF_STRIDE, sm + s1 * SURF_STRIDE,
                                                 xf, xq, F, &tr);
                if (st != ST_OK && fail == ST_OK) fail = st;
                s1 = s0;
            }
            phase_boundary();
            double A[36];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                double g[6];
                smoother_gain_row(F, Cf, L, id, c, g);
#pragma unroll
                for (int i = 0; i < 6; ++i) A[6 * c + i] = g[i];
            }
            phase_boundary();
            rts_mean(xf, A, dx, x, ang0);
            rts_cov(A, C, Cf);
            ang1 = ang0;
#pragma unroll
            for (int q = 0; q < 21; ++q) C[q] = Cf[q];
            phase_boundary();
        }
        // the smoothed state of hit k into this step's row of the stage
        const int row = it % sh;
        if (fitted && k >= 0) {
#pragma unroll
            for (int i = 0; i < 6; ++i) lw[(i * sh + row) * TILE + lane] = x[i];
#pragma unroll
            for (int q = 0; q < 21; ++q) lw[((6 + q) * sh + row) * TILE + lane] = C[q];
        }
        if (row == sh - 1 || it == nmax) stage_write(a, lw, sh, row + 1, it, fitted, o, n);
    }
    if (!fitted) return false;
    if (spd && fail == ST_OK) {
        store_rows(a.tgt_par + t, N, x);
        store_rows(a.tgt_cov + t, N, C);
        return true;
    }
    // a predicted covariance that is not positive definite (or a propagation
    // that did not repeat): the track fails
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    for (int k = 0; k < n; ++k) {
        fill_rows<6>(a.par + o + k, H, nan);
        fill_rows<21>(a.pcov + o + k, H, nan);
    }
    fill_rows<6>(a.tgt_par + t, N, nan);
    fill_rows<21>(a.tgt_cov + t, N, nan);
    a.chi2[t] = nan;
    a.status[t] = (uint8_t)(fail != ST_OK ? fail : ST_NOT_SPD);
    return false;
}

// Two-filter smoother of one track (Sect. 2, Fig. 2), fused after the forward
// pass (which kept only the predictions: 27 doubles per hit).  The backward
// filter starts at the last hit from the forward filtered state with its
// covariance times bwd_scale and takes in that hit; then for k = n-2 .. 0 and
// finally the seed surface it propagates back to surface k (against the
// direction of flight, the forward pass's transport routine), adds the
// scatterer of surface k as the forward filter evaluated it (at the forward
// filtered state of hit k, or the seed), combines that prediction with the
// forward filtered state of hit k (recomputed from the stored prediction and
// the hit, bit for bit as in the forward pass) into the smoothed state, which
// replaces slot k, and takes in hit k.  The last hit keeps its filtered
// state.  Returns true if the track's smoothed states are in its slots.
// CV: surfaces of every type.
template <class P, int FK, bool CV>
__device__ bool bwd_two_filter(const FitArgs& a, const double* __restrict__ sm, int64_t slot, int t) {
    constexpr int NW = NC_RECOMPUTE;
    if (a.status[t] != ST_OK) return false;
    const int o = a.off[t];
    const int n = a.off[t + 1] - o;
    const int64_t H = a.n_hits;
    const int64_t N = a.n_tracks;
    double* wl = a.ws + (slot / TILE) * a.tile_doubles + (slot % TILE);
    Field<P, FK> fl;
    fl.init(a.field);
    int fail = ST_OK;
    double xb[6], Cb[21];
    // surface types from the LDS table (the azimuth of a disc or cylinder hit wraps)
    const int kind_last = table_kind<CV>(sm + a.sid[o + n - 1] * SURF_STRIDE);
    {
        double* w = wl + (n - 1) * (NW * TILE);
        double xp[6], Cp[21], m[2], V[3], x[6], C[21], ck;
#pragma unroll
        for (int i = 0; i < 6; ++i) xp[i] = w[(OFF_XP + i) * TILE];
#pragma unroll
        for (int q = 0; q < 21; ++q) Cp[q] = w[(OFF_CP + q) * TILE];
        load_rows(a.loc + o + n - 1, H, m);
        load_rows(a.cov + o + n - 1, H, V);
        update_kind<CV>(kind_last, xp, Cp, m, V, x, C, &ck);
#pragma unroll
        for (int i = 0; i < 6; ++i) w[(OFF_XP + i) * TILE] = x[i];
#pragma unroll
        for (int q = 0; q < 21; ++q) w[(OFF_CP + q) * TILE] = C[q];
#pragma unroll
        for (int q = 0; q < 21; ++q) C[q] *= a.bwd_scale;
        if (update_kind<CV>(kind_last, x, C, m, V, xb, Cb, &ck) != ST_OK) fail = ST_NOT_SPD;
    }
    int s1 = a.sid[o + n - 1];
    double xs[6], Cs[21];
    for (int k = n - 2; k >= -1 && fail == ST_OK; --k) {
        double xf[6], Cf[21], m[2], V[3];
        int s0 = a.seed_sid;
        double* w = wl + (k >= 0 ? k : 0) * (NW * TILE);
        const int kind = k >= 0 ? table_kind<CV>(sm + a.sid[o + k] * SURF_STRIDE) : 0;
        const bool ang = kind_ang<CV>(kind);
        if (k >= 0) {
            double xp[6], Cp[21], ck;
#pragma unroll
            for (int i = 0; i < 6; ++i) xp[i] = w[(OFF_XP + i) * TILE];
#pragma unroll
            for (int q = 0; q < 21; ++q) Cp[q] = w[(OFF_CP + q) * TILE];
            load_rows(a.loc + o + k, H, m);
            load_rows(a.cov + o + k, H, V);
            s0 = a.sid[o + k];
            update_kind<CV>(kind, xp, Cp, m, V, xf, Cf, &ck);
        } else {
            load_rows(a.seed + t, N, xf);
            load_rows(a.seed_cov + t, N, Cf);
        }
        double q22 = 0.0, q33 = 0.0;
        if (a.cfg.ms) highland_any<CV>(sm + s0 * SURF_STRIDE, xf, a.cfg.mass, &q22, &q33);
        phase_boundary();
        double xq[6], G[25];
        int tr = 0;
        fail = transport_any<CV>(fl, a.field, a.cfg, sm + s1 * SURF_STRIDE, sm + s0 * SURF_STRIDE, xb, xq, G, &tr);
        if (fail != ST_OK) break;
        phase_boundary();
        double Cq[21];
        transport_cov(G, Cb, Cq);
        Cq[sy(2, 2)] += q22;
        Cq[sy(3, 3)] += q33;
        phase_boundary();
        if (!two_filter_combine(xf, Cf, xq, Cq, xs, Cs, ang)) { fail = ST_NOT_SPD; break; }
        phase_boundary();
        if (k >= 0) {
#pragma unroll
            for (int i = 0; i < 6; ++i) w[(OFF_XP + i) * TILE] = xs[i];
#pragma unroll
            for (int q = 0; q < 21; ++q) w[(OFF_CP + q) * TILE] = Cs[q];
            double ck;
            if (update_kind<CV>(kind, xq, Cq, m, V, xb, Cb, &ck) != ST_OK) { fail = ST_NOT_SPD; break; }
        }
        s1 = s0;
    }
    if (fail == ST_OK) {
        store_rows(a.tgt_par + t, N, xs);
        store_rows(a.tgt_cov + t, N, Cs);
        return true;
    }
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    for (int k = 0; k < n; ++k) {
        fill_rows<6>(a.par + o + k, H, nan);
        fill_rows<21>(a.pcov + o + k, H, nan);
    }
    fill_rows<6>(a.tgt_par + t, N, nan);
    fill_rows<21>(a.tgt_cov + t, N, nan);
    a.chi2[t] = nan;
    a.status[t] = (uint8_t)fail;
    return false;
}


// Write the smoothed states of a tile's tracks (left in their workspace slots
// by the two-filter smoother, or by bwd_one) to the CSR outputs.  One lane per track computed them; a store
// from each lane would touch a different cache line per lane.  Instead, for a
// block of FLUSH_HITS hits: every lane loads its 27 x FLUSH_HITS values at
// once (coalesced: the slots are tile-major), the wave lists which (lane,
// hit) owns each entry of the block's CSR ranges, and then, FLUSH_GROUP
// components at a time, the values pass through LDS so that consecutive
// lanes store consecutive CSR entries.  Every lane of the wave must call it
// (done: this lane's track has results; o, n: its CSR range).  lw: this
// wave's LDS area (free once the smoother has finished).  NW: workspace
// doubles per hit.
template <int NW>
__device__ void flush_tile(const FitArgs& a, double* lw, const double* wtile, bool done, int o, int n) {
    const int lane = threadIdx.x & (TILE - 1);
    double* tb = lw;                                                    // [FLUSH_GROUP][FLUSH_HITS][64]
    int32_t* own = (int32_t*)(lw + FLUSH_GROUP * FLUSH_HITS * TILE);   // [FLUSH_HITS * 64]: lane | hit << 6
    int32_t* dst = own + FLUSH_HITS * TILE;                             // [FLUSH_HITS * 64]: CSR index
    const int nl = done ? n : 0;
    int nmax = nl;
#pragma unroll
    for (int d = 1; d < TILE; d <<= 1) {
        const int v = __shfl_xor(nmax, d, TILE);
        nmax = v > nmax ? v : nmax;
    }
    const int64_t H = a.n_hits;
    for (int hb = 0; hb < nmax; hb += FLUSH_HITS) {
        const int cnt = nl - hb < 0 ? 0 : (nl - hb > FLUSH_HITS ? FLUSH_HITS : nl - hb);
        // every value of this block first: one wait for all of them
        double v[27][FLUSH_HITS];
        const double* src = wtile + (int64_t)hb * (NW * TILE) + OFF_XP * TILE + lane;
#pragma unroll
        for (int c = 0; c < 27; ++c)
#pragma unroll
            for (int h = 0; h < FLUSH_HITS; ++h)
                v[c][h] = h < cnt ? src[(int64_t)h * (NW * TILE) + c * TILE] : 0.0;
        // exclusive prefix of cnt over the wave
        int inc = cnt;
#pragma unroll
        for (int d = 1; d < TILE; d <<= 1) {
            const int u = __shfl_up(inc, d, TILE);
            if (lane >= d) inc += u;
        }
        const int start = inc - cnt;
        const int total = __shfl(inc, TILE - 1, TILE);
#pragma unroll
        for (int h = 0; h < FLUSH_HITS; ++h)
            if (h < cnt) {
                own[start + h] = lane | (h << 6);
                dst[start + h] = o + hb + h;
            }
#pragma unroll
        for (int c0 = 0; c0 < 27; c0 += FLUSH_GROUP) {
#pragma unroll
            for (int c = c0; c < c0 + FLUSH_GROUP && c < 27; ++c)
#pragma unroll
                for (int h = 0; h < FLUSH_HITS; ++h)
                    if (h < cnt) tb[((c - c0) * FLUSH_HITS + h) * TILE + lane] = v[c][h];
            wave_sync();
            for (int g = lane; g < total; g += TILE) {
                const int e = own[g];
                const int64_t d = dst[g];
                const int from = (e >> 6) * TILE + (e & 63);
#pragma unroll
                for (int c = c0; c < c0 + FLUSH_GROUP && c < 27; ++c) {
                    double* out = c < 6 ? a.par + (int64_t)c * H : a.pcov + (int64_t)(c - 6) * H;
                    out[d] = tb[(c - c0) * FLUSH_HITS * TILE + from];
                }
            }
            wave_sync();
        }
    }
}

// Filter (+ smoother).  SORTED selects the schedule at compile time; OCC is
// the occupancy target in waves per SIMD, which caps the registers per lane;
// FUSED runs the smoother for a track right after its forward pass, while
// its workspace column is still cache-hot (otherwise k_bwd does it); STOREF
// (always with a split smoother) stores the transport Jacobians, otherwise the
// fused smoother recomputes them; TWOF (fused, no stored Jacobians) runs the
// two-filter smoother instead of RTS; CV: surfaces of every type (cylinders
// and lines too; built for OCC 1 only).
// Dynamic LDS: the surface table, then per wave the carried covariances.
template <class P, int FK, int OCC, bool SORTED, bool FUSED, bool STOREF, bool TWOF, bool CV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
k_fwd(FitArgs a) {
    static_assert(FUSED || STOREF, "the split smoother reads stored Jacobians");
    static_assert(!TWOF || (FUSED && !STOREF), "the two-filter smoother is fused and stores no Jacobians");
    extern __shared__ double sm[];
    stage_surfaces(a.n_surf, a.center, a.rot, a.x0, a.align, a.stype, sm, CV ? a.radius : nullptr);
    const int lane = threadIdx.x & (TILE - 1);
    double* lw = sm + a.n_surf * SURF_STRIDE + (threadIdx.x / TILE) * a.wave_lds;
    double* cl = lw + lane;
    int iter = 0;
    for (;;) {
        const int tile = next_tile<SORTED>(a.tile_counter, iter);
        if (tile >= a.n_tiles) break;
        const int64_t i = (int64_t)tile * TILE + lane;
        const bool have = i < a.n_tracks;
        const int t = have ? (SORTED ? a.order[i] : (int)i) : 0;
        if (have) fwd_one<P, FK, STOREF, CV>(a, sm, cl, i, t);
        if constexpr (TWOF) {
            bool done = false;
            int o = 0, n = 0;
            if (have) {
                done = bwd_two_filter<P, FK, CV>(a, sm, i, t);
                o = a.off[t];
                n = a.off[t + 1] - o;
            }
            flush_tile<NC_RECOMPUTE>(a, lw, a.ws + (int64_t)tile * a.tile_doubles, done, o, n);
        } else if constexpr (FUSED) {
            if (a.stage_hits > 0) {
                smooth_staged<P, FK, STOREF, CV>(a, sm, lw, i, t, have);
            } else {
                bool done = false;
                int o = 0, n = 0;
                if (have) {
                    done = bwd_one<P, FK, STOREF, CV>(a, sm, i, t);
                    o = a.off[t];
                    n = a.off[t + 1] - o;
                }
                flush_tile<nc_of<STOREF>()>(a, lw, a.ws + (int64_t)tile * a.tile_doubles, done, o, n);
            }
        }
    }
}

// Backward (smoother) pass as its own kernel (launched after k_fwd<..., FUSED
// false, ...>).  Dynamic LDS: per wave the smoother's output stage or the
// output transpose.  CV: hits on surfaces of every type.
template <bool SORTED, bool CV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_bwd(FitArgs a) {
    extern __shared__ double sm[];
    const int lane = threadIdx.x & (TILE - 1);
    double* lw = sm + (threadIdx.x / TILE) * a.wave_lds;
    int iter = 0;
    for (;;) {
        const int tile = next_tile<SORTED>(a.tile_counter + 1, iter);
        if (tile >= a.n_tiles) break;
        const int64_t i = (int64_t)tile * TILE + lane;
        const bool have = i < a.n_tracks;
        const int t = have ? (SORTED ? a.order[i] : (int)i) : 0;
        if (a.stage_hits > 0) {
            smooth_staged<double, FIELD_UNIFORM, true, CV>(a, nullptr, lw, i, t, have);
        } else {
            bool done = false;
            int o = 0, n = 0;
            if (have) {
                done = bwd_one<double, FIELD_UNIFORM, true, CV>(a, nullptr, i, t);
                o = a.off[t];
                n = a.off[t + 1] - o;
            }
            flush_tile<NC>(a, lw, a.ws + (int64_t)tile * a.tile_doubles, done, o, n);
        }
    }
}

// Dynamic LDS of k_fwd: the surface table and one area per wave
inline size_t fwd_lds_bytes(int n_surf, int block, int wave_lds) {
    return ((size_t)n_surf * SURF_STRIDE + (size_t)(block / TILE) * wave_lds) * sizeof(double);
}

// Launch k_fwd for one schedule: SORTED runs min(tiles, CUs x waves_per_cu)
// persistent waves, DIRECT one wave per tile.
template <class P, int FK, int OCC, bool FUSED, bool STOREF, bool TWOF, bool CV>
hipError_t launch_fwd_kernel(const FitArgs& a, int sched, int block, int waves_per_cu, hipStream_t stream) {
    const size_t shm = fwd_lds_bytes(a.n_surf, block, a.wave_lds);
    const int need = (a.n_tiles * TILE + block - 1) / block;
    hipError_t e = hipSuccess;
    if (sched == KF_SCHED_SORTED) {
        int grid = num_cu() * waves_per_cu * TILE / block;
        grid = grid > need ? need : (grid < 1 ? 1 : grid);
        if ((e = allow_lds(k_fwd<P, FK, OCC, true, FUSED, STOREF, TWOF, CV>, shm)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_fwd<P, FK, OCC, true, FUSED, STOREF, TWOF, CV>), dim3(grid), dim3(block), shm, stream,
                           a);
    } else {
        if ((e = allow_lds(k_fwd<P, FK, OCC, false, FUSED, STOREF, TWOF, CV>, shm)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_fwd<P, FK, OCC, false, FUSED, STOREF, TWOF, CV>), dim3(need), dim3(block), shm, stream,
                           a);
    }
    return hipGetLastError();
}

template <class P, int FK, int OCC, bool CV>
hipError_t launch_fwd_occ(const FitArgs& a, int sched, int block, int waves_per_cu, bool split, bool storef,
                          bool twof, hipStream_t stream) {
    if (twof) return launch_fwd_kernel<P, FK, OCC, true, false, true, CV>(a, sched, block, waves_per_cu, stream);
    if (split) return launch_fwd_kernel<P, FK, OCC, false, true, false, CV>(a, sched, block, waves_per_cu, stream);
    return storef ? launch_fwd_kernel<P, FK, OCC, true, true, false, CV>(a, sched, block, waves_per_cu, stream)
                  : launch_fwd_kernel<P, FK, OCC, true, false, false, CV>(a, sched, block, waves_per_cu, stream);
}

// The filter kernel of one fit (with the smoother fused, or, with `split`,
// the filter alone: the caller then launches k_bwd).  Cylinders and lines
// (curved) are built for one wave per SIMD only: any other occupancy is
// refused with hipErrorInvalidValue.
template <class P, int FK>
hipError_t launch_fwd(const FitArgs& a, int sched, int block, int waves_per_cu, int occ, bool split, bool storef,
                      bool twof, bool curved, hipStream_t stream) {
    if (curved) {
        if (occ != 1) return hipErrorInvalidValue;
        return launch_fwd_occ<P, FK, 1, true>(a, sched, block, waves_per_cu, split, storef, twof, stream);
    }
    switch (occ) {
        case 1: return launch_fwd_occ<P, FK, 1, false>(a, sched, block, waves_per_cu, split, storef, twof, stream);
        case 3: return launch_fwd_occ<P, FK, 3, false>(a, sched, block, waves_per_cu, split, storef, twof, stream);
        default: return launch_fwd_occ<P, FK, 2, false>(a, sched, block, waves_per_cu, split, storef, twof, stream);
    }
}

// One translation unit per (field kind, stepping precision) instantiates
// launch_fwd: kf_fit_<field>_<precision>.hip.
#define KF_FWD_ARGS const FitArgs& a, int sched, int block, int waves_per_cu, int occ, bool split, bool storef, \
                    bool twof, bool curved, hipStream_t stream
hipError_t launch_fwd_uniform_fp64(KF_FWD_ARGS);
hipError_t launch_fwd_uniform_mixed(KF_FWD_ARGS);
hipError_t launch_fwd_solenoid_fp64(KF_FWD_ARGS);
hipError_t launch_fwd_solenoid_mixed(KF_FWD_ARGS);
hipError_t launch_fwd_map_fp64(KF_FWD_ARGS);
hipError_t launch_fwd_map_mixed(KF_FWD_ARGS);

}  // namespace kffit
