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
#include "kf_common.hpp"

namespace {

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
    const int32_t* stype;       // [S] surface types (0 plane, 1 disc) or NULL
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
};

// Hit k of the track at CSR offset o lies on a disc (its azimuth wraps).
__device__ inline bool disc_hit(const FitArgs& a, int o, int k) {
    return a.stype && a.stype[a.sid[o + k]] == 1;
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
template <class P, int FK, bool STOREF>
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
        if (!hit_ok(s, a.n_surf, m, V, a.stype)) { status = ST_BAD_INPUT; break; }
        if (k + 1 < n) {
            s_nx = a.sid[o + k + 1];
            load_rows(a.loc + o + k + 1, H, m_nx);
            load_rows(a.cov + o + k + 1, H, V_nx);
        }
        phase_boundary();
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
        status = kalman_update(xp, Cp, m, V, x, C, &ck, is_disc(sb));
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
    if (status != ST_OK && status != ST_BAD_INPUT && status != ST_TOO_FEW &&
        any_bad_hit(a.sid, a.loc, a.cov, H, a.n_surf, o, k + 1, n, a.stype))
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
    a.ndf[t] = 2 * n - (a.bnz ? 5 : 4);
    a.status[t] = (uint8_t)status;
}

// RTS smoother of one track (Sect. 2), fused after the forward pass or run by
// a separate streaming kernel: the smoothed state of the last hit is its
// filtered state; every earlier state, and finally the seed/target state,
// follows from the next hit's stored prediction and Jacobian with the gain
// A = Cf F^T Cp^-1 solved in FP64.  The smoothed state of hit k replaces the
// prediction in slot k once that has been read for the last time; flush_tile
// then writes the tile's CSR outputs.  Without stored Jacobians (STOREF
// false; fused only, sm is the surface table) F of the gap k -> k+1 comes from
// propagating the recomputed filtered state of hit k (or the seed) again with
// the forward pass's routine.  Returns true if the track's smoothed states are
// in its slots (false: not fitted, or failed here with NaN outputs).
template <class P, int FK, bool STOREF>
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
        kalman_update(xp1, Cp1, m, V, x, C, &ck, disc_hit(a, o, n - 1));
    }
    bool ang1 = disc_hit(a, o, n - 1);                 // hit k+1 is on a disc
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
        const bool ang0 = k >= 0 && disc_hit(a, o, k);
        if (k >= 0) {
            double ck;
            kalman_update(xp, Cp, m, V, xf, Cf, &ck, ang0);   // filtered state of hit k, as in the forward pass
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
            const int st = transport<P, FK>(fl, a.field, a.cfg, sm + s0 * SURF_STRIDE, sm + s1 * SURF_STRIDE, xf,
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
template <class P, int FK>
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
    // surface types from the LDS table (the azimuth of a disc hit wraps)
    const bool ang_last = is_disc(sm + a.sid[o + n - 1] * SURF_STRIDE);
    {
        double* w = wl + (n - 1) * (NW * TILE);
        double xp[6], Cp[21], m[2], V[3], x[6], C[21], ck;
#pragma unroll
        for (int i = 0; i < 6; ++i) xp[i] = w[(OFF_XP + i) * TILE];
#pragma unroll
        for (int q = 0; q < 21; ++q) Cp[q] = w[(OFF_CP + q) * TILE];
        load_rows(a.loc + o + n - 1, H, m);
        load_rows(a.cov + o + n - 1, H, V);
        kalman_update(xp, Cp, m, V, x, C, &ck, ang_last);
#pragma unroll
        for (int i = 0; i < 6; ++i) w[(OFF_XP + i) * TILE] = x[i];
#pragma unroll
        for (int q = 0; q < 21; ++q) w[(OFF_CP + q) * TILE] = C[q];
#pragma unroll
        for (int q = 0; q < 21; ++q) C[q] *= a.bwd_scale;
        if (kalman_update(x, C, m, V, xb, Cb, &ck, ang_last) != ST_OK) fail = ST_NOT_SPD;
    }
    int s1 = a.sid[o + n - 1];
    double xs[6], Cs[21];
    for (int k = n - 2; k >= -1 && fail == ST_OK; --k) {
        double xf[6], Cf[21], m[2], V[3];
        int s0 = a.seed_sid;
        double* w = wl + (k >= 0 ? k : 0) * (NW * TILE);
        const bool ang = k >= 0 && is_disc(sm + a.sid[o + k] * SURF_STRIDE);
        if (k >= 0) {
            double xp[6], Cp[21], ck;
#pragma unroll
            for (int i = 0; i < 6; ++i) xp[i] = w[(OFF_XP + i) * TILE];
#pragma unroll
            for (int q = 0; q < 21; ++q) Cp[q] = w[(OFF_CP + q) * TILE];
            load_rows(a.loc + o + k, H, m);
            load_rows(a.cov + o + k, H, V);
            s0 = a.sid[o + k];
            kalman_update(xp, Cp, m, V, xf, Cf, &ck, ang);
        } else {
            load_rows(a.seed + t, N, xf);
            load_rows(a.seed_cov + t, N, Cf);
        }
        double q22 = 0.0, q33 = 0.0;
        if (a.cfg.ms) highland(sm + s0 * SURF_STRIDE, xf, a.cfg.mass, &q22, &q33);
        phase_boundary();
        double xq[6], G[25];
        int tr = 0;
        fail = transport<P, FK>(fl, a.field, a.cfg, sm + s1 * SURF_STRIDE, sm + s0 * SURF_STRIDE, xb, xq, G, &tr);
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
            if (kalman_update(xq, Cq, m, V, xb, Cb, &ck, ang) != ST_OK) { fail = ST_NOT_SPD; break; }
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

// All lanes of the wave, in step: LDS written by one lane is then visible to
// the others (the waves of a workgroup run different tiles, so no workgroup
// barrier may be used here).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Write the smoothed states of a tile's tracks (left in their workspace slots
// by bwd_one) to the CSR outputs.  One lane per track computed them; a store
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
// two-filter smoother instead of RTS.
// Dynamic LDS: the surface table, then per wave the carried covariances.
template <class P, int FK, int OCC, bool SORTED, bool FUSED, bool STOREF, bool TWOF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
k_fwd(FitArgs a) {
    static_assert(FUSED || STOREF, "the split smoother reads stored Jacobians");
    static_assert(!TWOF || (FUSED && !STOREF), "the two-filter smoother is fused and stores no Jacobians");
    extern __shared__ double sm[];
    stage_surfaces(a.n_surf, a.center, a.rot, a.x0, a.align, a.stype, sm);
    const int lane = threadIdx.x & (TILE - 1);
    double* cl = sm + a.n_surf * SURF_STRIDE + (threadIdx.x / TILE) * WAVE_LDS_DOUBLES + lane;
    int iter = 0;
    for (;;) {
        const int tile = next_tile<SORTED>(a.tile_counter, iter);
        if (tile >= a.n_tiles) break;
        const int64_t i = (int64_t)tile * TILE + lane;
        bool done = false;
        int o = 0, n = 0;
        if (i < a.n_tracks) {
            const int t = SORTED ? a.order[i] : (int)i;
            fwd_one<P, FK, STOREF>(a, sm, cl, i, t);
            if constexpr (TWOF) {
                done = bwd_two_filter<P, FK>(a, sm, i, t);
                o = a.off[t];
                n = a.off[t + 1] - o;
            } else if constexpr (FUSED) {
                done = bwd_one<P, FK, STOREF>(a, sm, i, t);
                o = a.off[t];
                n = a.off[t + 1] - o;
            }
        }
        if (FUSED) flush_tile<nc_of<STOREF>()>(a, cl - lane, a.ws + (int64_t)tile * a.tile_doubles, done, o, n);
    }
}

// Backward (smoother) pass as its own kernel.  Dynamic LDS: per wave the
// output transpose.
template <bool SORTED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_bwd(FitArgs a) {
    extern __shared__ double sm[];
    const int lane = threadIdx.x & (TILE - 1);
    double* lw = sm + (threadIdx.x / TILE) * WAVE_LDS_DOUBLES;
    int iter = 0;
    for (;;) {
        const int tile = next_tile<SORTED>(a.tile_counter + 1, iter);
        if (tile >= a.n_tiles) break;
        const int64_t i = (int64_t)tile * TILE + lane;
        bool done = false;
        int o = 0, n = 0;
        if (i < a.n_tracks) {
            const int t = SORTED ? a.order[i] : (int)i;
            done = bwd_one<double, FIELD_UNIFORM, true>(a, nullptr, i, t);
            o = a.off[t];
            n = a.off[t + 1] - o;
        }
        flush_tile<NC>(a, lw, a.ws + (int64_t)tile * a.tile_doubles, done, o, n);
    }
}

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
    return KF_OK;
}

template <class P, int FK, int OCC, bool STOREF, bool TWOF>
hipError_t launch_fit_fused(const FitArgs& a, int sched, int block, int waves_per_cu, size_t shm,
                            hipStream_t stream) {
    const int need = (a.n_tiles * TILE + block - 1) / block;
    hipError_t e = hipSuccess;
    if (sched == KF_SCHED_SORTED) {
        int grid = num_cu() * waves_per_cu * TILE / block;
        grid = grid > need ? need : (grid < 1 ? 1 : grid);
        if ((e = allow_lds(k_fwd<P, FK, OCC, true, true, STOREF, TWOF>, shm)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_fwd<P, FK, OCC, true, true, STOREF, TWOF>), dim3(grid), dim3(block), shm, stream, a);
    } else {
        if ((e = allow_lds(k_fwd<P, FK, OCC, false, true, STOREF, TWOF>, shm)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_fwd<P, FK, OCC, false, true, STOREF, TWOF>), dim3(need), dim3(block), shm, stream,
                           a);
    }
    return hipGetLastError();
}

template <class P, int FK, int OCC>
hipError_t launch_fit_occ(const FitArgs& a, int sched, int block, int waves_per_cu, bool split, bool storef,
                          bool twof, hipStream_t stream) {
    const size_t shm = ((size_t)a.n_surf * SURF_STRIDE + (size_t)(block / TILE) * WAVE_LDS_DOUBLES) * sizeof(double);
    const size_t shm_b = (size_t)(block / TILE) * WAVE_LDS_DOUBLES * sizeof(double);
    const int need = (a.n_tiles * TILE + block - 1) / block;
    hipError_t e = hipSuccess;
    if (twof) return launch_fit_fused<P, FK, OCC, false, true>(a, sched, block, waves_per_cu, shm, stream);
    if (!split)
        return storef ? launch_fit_fused<P, FK, OCC, true, false>(a, sched, block, waves_per_cu, shm, stream)
                      : launch_fit_fused<P, FK, OCC, false, false>(a, sched, block, waves_per_cu, shm, stream);
    if (sched == KF_SCHED_SORTED) {
        int grid = num_cu() * waves_per_cu * TILE / block;
        grid = grid > need ? need : (grid < 1 ? 1 : grid);
        int gridb = num_cu() * 8 * TILE / block;
        gridb = gridb > need ? need : (gridb < 1 ? 1 : gridb);
        if ((e = allow_lds(k_fwd<P, FK, OCC, true, false, true, false>, shm)) != hipSuccess) return e;
        if ((e = allow_lds(k_bwd<true>, shm_b)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_fwd<P, FK, OCC, true, false, true, false>), dim3(grid), dim3(block), shm, stream, a);
        hipLaunchKernelGGL((k_bwd<true>), dim3(gridb), dim3(block), shm_b, stream, a);
    } else {
        if ((e = allow_lds(k_fwd<P, FK, OCC, false, false, true, false>, shm)) != hipSuccess) return e;
        if ((e = allow_lds(k_bwd<false>, shm_b)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_fwd<P, FK, OCC, false, false, true, false>), dim3(need), dim3(block), shm, stream, a);
        hipLaunchKernelGGL((k_bwd<false>), dim3(need), dim3(block), shm_b, stream, a);
    }
    return hipGetLastError();
}

template <class P, int FK>
hipError_t launch_fit(const FitArgs& a, int sched, int block, int waves_per_cu, int occ, bool split, bool storef,
                      bool twof, hipStream_t stream) {
    switch (occ) {
        case 1: return launch_fit_occ<P, FK, 1>(a, sched, block, waves_per_cu, split, storef, twof, stream);
        case 3: return launch_fit_occ<P, FK, 3>(a, sched, block, waves_per_cu, split, storef, twof, stream);
        default: return launch_fit_occ<P, FK, 2>(a, sched, block, waves_per_cu, split, storef, twof, stream);
    }
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
        e = mixed ? launch_fit<float, FIELD_UNIFORM>(a, sched, block, wpc, occ, split, storef, twof, stream)
                  : launch_fit<double, FIELD_UNIFORM>(a, sched, block, wpc, occ, split, storef, twof, stream);
    else if (field->kind == KF_FIELD_SOLENOID)
        e = mixed ? launch_fit<float, FIELD_SOLENOID>(a, sched, block, wpc, occ, split, storef, twof, stream)
                  : launch_fit<double, FIELD_SOLENOID>(a, sched, block, wpc, occ, split, storef, twof, stream);
    else
        e = mixed ? launch_fit<float, FIELD_MAP>(a, sched, block, wpc, occ, split, storef, twof, stream)
                  : launch_fit<double, FIELD_MAP>(a, sched, block, wpc, occ, split, storef, twof, stream);
    if (e == hipErrorInvalidValue) return KF_E_VALUE;     // workgroup needs more LDS than the device has
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
// Key: precision, field kind, max hits per track, track count rounded to a
// power of two.  Filled by kf_autotune, read when a setting is AUTO (0).
struct TuneKey {
    int precision, field_kind, smoother, max_hits, log2n;
    bool operator<(const TuneKey& o) const {
        if (precision != o.precision) return precision < o.precision;
        if (field_kind != o.field_kind) return field_kind < o.field_kind;
        if (smoother != o.smoother) return smoother < o.smoother;
        if (max_hits != o.max_hits) return max_hits < o.max_hits;
        return log2n < o.log2n;
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, kf_config> g_tune;

TuneKey tune_key(const kf_config* cfg, const kf_field* field, const kf_measurements* meas) {
    int l = 0;
    while ((1LL << (l + 1)) <= (long long)meas->n_tracks) ++l;
    return TuneKey{cfg->precision, field->kind, cfg->smoother, meas->max_hits, l};
}

// Fill AUTO (0) launch settings from the tuning table, else the defaults
// (length-sorted persistent schedule, 64-thread groups, one wave per SIMD,
// 8 resident waves per CU, smoother fused into the filter kernel).
kf_config resolve(const kf_config* cfg, const kf_field* field, const kf_measurements* meas) {
    kf_config r = *cfg;
    kf_config d = r;
    d.schedule = KF_SCHED_SORTED;
    d.block = 64;
    d.occupancy = 1;
    d.waves_per_cu = 8;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(tune_key(cfg, field, meas));
        if (it != g_tune.end()) d = it->second;
    }
    if (r.schedule == KF_SCHED_AUTO) {
        r.schedule = d.schedule;
        r.split_smoother = r.smoother == KF_SMOOTHER_TWO_FILTER ? 0 : d.split_smoother;
        r.jacobians = d.jacobians;
    }
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
    const kf_config r = resolve(cfg, field, meas);
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
    const kf_config r = resolve(cfg, field, meas);
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
    const kf_config r = resolve(cfg, field, meas);
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
    *best = resolve(cfg, field, meas);
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
    float best_t = 1e30f;
    kf_config win = *best;
    for (int sc : scheds)
        for (int bl : blocks)
            for (int oc : occs)
                for (int sp : splits)
                    for (int wp : wpcs) {
                        if (sc == KF_SCHED_DIRECT && wp != wpcs[0]) continue;   // unused by DIRECT
                        if (cfg->smoother == KF_SMOOTHER_TWO_FILTER && sp != 0) continue;   // fused only
                        kf_config c = *cfg;
                        c.schedule = sc;
                        c.block = bl;
                        c.occupancy = oc;
                        c.split_smoother = sp == 1;
                        c.jacobians = sp == 2 ? KF_JAC_RECOMPUTE : KF_JAC_STORE;
                        c.waves_per_cu = wp;
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
        g_tune[tune_key(cfg, field, meas)] = win;
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
        const kf_config r = resolve(cfg, field, &mc);
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
