// kf_vjp.hip -- adjoint (vector-Jacobian product) of the batched track fit.
//
// For L = sum_t g_chi2 chi2_t + sum_hits g_par . xs + sum_t g_tgt . x_target,
// one lane per track runs two sweeps over its hits:
//
//   forward  (k = 0 .. n-1): the filter of Sect. 2 / Sect. 4.1 again (in the
//            fit's precision: FP32 stepping on an FP64 anchor for the mixed
//            fit, so the recomputed states are the mixed fit's), storing
//            per hit the predicted state and covariance, the transport
//            Jacobian F_k, the noise terms and the filtered state and
//            covariance.  The reverse of the RTS mean recursion only needs the
//            smoother gains, so it runs here too:
//              xsb_k = g_par_k + u_k,  u_k = A_{k-1}^T xsb_{k-1}
//                    = Cp_k^-1 F_k C_{k-1} xsb_{k-1}   (one FP64 Cholesky solve)
//            with xsb_{-1} = g_tgt.
//   backward (k = n-1 .. 0): the RTS mean recursion xs_{k-1} = xf_{k-1} + A
//            (xs_k - xp_k) (with A dx = C_{k-1} F_k^T Cp_k^-1 dx), and the
//            reverse of the update, the rank-one smoother-gain adjoint, the
//            covariance transport and the propagation.  The propagation of
//            each gap is replayed and reversed by hand, step by step, through
//            the RKN stages, the tangent-column (transport Jacobian) update,
//            the capped step sizes, the final move onto the plane and the
//            local <-> global conversions (kf_gap_reverse.hpp); the small
//            thin-scatterer noise term by its closed-form derivative.
//
// Per-hit alignment contributions go to a [6][H + N] buffer; a deterministic
// two-level reduction (fixed chunks summed in a fixed order, then a
// fixed-order tree per surface)
// sums them per surface and converts the rotation part from the surface's own
// frame to the (alpha, beta, gamma) of its alignment correction.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <type_traits>
#include "kf_common.hpp"
#include "kf_adjoint.hpp"
#include "kf_gap_reverse.hpp"

namespace {

// per-hit adjoint workspace [tile][hit][NCV][64 lanes]
constexpr int NCV = 87;
constexpr int V_XF = 0, V_CF = 6, V_XP = 27, V_CP = 33, V_F = 54, V_Q = 79, V_U = 81;
// Per lane, the backward sweep keeps what one hit's step produces for later in
// the same step in LDS ([SX_N][64 lanes] doubles per wave): in device memory
// every reload would also wait for all earlier stores (one counter covers
// loads and stores), LDS reads do not.
//   SX_XS: xs_{k-1}, SX_XPB: adjoint of xp_k, SX_CB: adjoint of C_{k-1},
//   SX_FB: adjoint of F_k, SX_QB: adjoints of the two noise terms,
//   SX_AV: xsb_{k-1}, SX_X0: the start state of gap k, SX_AA: the alignment
//   contribution of hit k's surface from gap k+1.
constexpr int SX_XS = 0, SX_XPB = 6, SX_CB = 12, SX_FB = 33, SX_QB = 58, SX_AV = 60, SX_X0 = 66, SX_AA = 72,
              SX_N = 78;
// the stash's fields are disjoint and fill [0, SX_N) (6, 6, 21, 25, 2, 6, 6, 6 doubles)
static_assert(SX_XPB == SX_XS + 6 && SX_CB == SX_XPB + 6 && SX_FB == SX_CB + 21 && SX_QB == SX_FB + 25 &&
              SX_AV == SX_QB + 2 && SX_X0 == SX_AV + 6 && SX_AA == SX_X0 + 6 && SX_N == SX_AA + 6,
              "stash layout");
typedef __attribute__((address_space(3))) double ldouble;

struct VjpArgs {
    int n_tracks;
    int n_surf;
    int seed_sid;
    int max_hits;
    int64_t n_hits;
    int64_t tile_doubles;       // max_hits * NCV * 64
    const int32_t* off;
    const int32_t* sid;
    const double* loc;
    const double* cov;
    const double* center;
    const double* rot;
    const double* x0;
    const double* align;
    const double* seed;
    const double* seed_cov;
    FieldDef field;
    Cfg cfg;
    const double* g_chi2;
    const double* g_par;
    const double* g_tgt;
    double* g_meas;
    double* g_seed;
    uint8_t* status;
    double* contrib;            // [6][n_items]: items < H are hits, the rest tracks (seed surface)
    int64_t n_items;
    double* ws;
    const int32_t* order;
    int32_t* tile_counter;
    int n_tiles;
};

template <int N>
__device__ inline void ld(const double* w, int off, double (&v)[N]) {
    auto g = gbl(w);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = g[(off + i) * TILE];
}

template <int N>
__device__ inline void st(double* w, int off, const double (&v)[N]) {
    auto g = gbl(w);
#pragma unroll
    for (int i = 0; i < N; ++i) g[(off + i) * TILE] = v[i];
}

template <int N>
__device__ inline void ldl(const ldouble* x, int off, double (&v)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = x[(off + i) * TILE];
}

template <int N>
__device__ inline void stl(ldouble* x, int off, const double (&v)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[(off + i) * TILE] = v[i];
}

// ---------------------------------------------------------------------------
// forward sweep: filter recompute + reverse RTS mean recursion
// ---------------------------------------------------------------------------
template <class P, int FK>
__device__ __attribute__((always_inline)) int vjp_fwd(const VjpArgs& a, const double* __restrict__ sm, double* wl,
                                                      ldouble* sx, int t, int o, int n) {
    const int64_t H = a.n_hits, N = a.n_tracks;
    Field<P, FK> fl;
    fl.init(a.field);
    double x[6];
    load_rows(a.seed + t, N, x);
    double as[6];                                   // xsb_{k-1}
    if (a.g_tgt) load_rows(a.g_tgt + t, N, as);
    else {
#pragma unroll
        for (int i = 0; i < 6; ++i) as[i] = 0.0;
    }
    // The filtered covariance of the previous hit waits in the (still unused)
    // LDS stash during each propagation, and hit k's surface, measurement and
    // smoothed-state cotangent are loaded during hit k-1: no load of this
    // sweep is issued behind its own workspace stores (on gfx9 one counter
    // covers loads and stores, so such a load would wait for them).
    {
        double C0[21];
        load_rows(a.seed_cov + t, N, C0);
        stl(sx, 0, C0);
    }
    int s_nx = gbl(a.sid)[o];
    double m_nx[2], V_nx[3], gp_nx[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    load_rows(a.loc + o, H, m_nx);
    load_rows(a.cov + o, H, V_nx);
    if (a.g_par) load_rows(a.g_par + o, H, gp_nx);
    int prev = a.seed_sid;
    int status = ST_OK;
    for (int k = 0; k < n; ++k) {
        const int s = s_nx;
        const double m[2] = {m_nx[0], m_nx[1]};
        const double V[3] = {V_nx[0], V_nx[1], V_nx[2]};
        double gp[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) gp[i] = gp_nx[i];
        if (k + 1 < n) {
            s_nx = gbl(a.sid)[o + k + 1];
            load_rows(a.loc + o + k + 1, H, m_nx);
            load_rows(a.cov + o + k + 1, H, V_nx);
            if (a.g_par) load_rows(a.g_par + o + k + 1, H, gp_nx);
        }
        phase_boundary();
        const double* sa = sm + prev * SURF_STRIDE;
        const double* sb = sm + s * SURF_STRIDE;
        double q[2] = {0.0, 0.0};
        if (a.cfg.ms) highland(sa, x, a.cfg.mass, &q[0], &q[1]);
        double xp[6], F[25];
        int tr = 0;
        status = transport<P, FK>(fl, a.field, a.cfg, sa, sb, x, xp, F, &tr);
        if (status != ST_OK) break;
        phase_boundary();
        double* w = wl + k * (NCV * TILE);
        st(w, V_XP, xp);
        st(w, V_F, F);
        st(w, V_Q, q);
        double C[21], Cp[21];
        ldl(sx, 0, C);
        {
            double CQ[21];
#pragma unroll
            for (int i = 0; i < 21; ++i) CQ[i] = C[i];
            CQ[sy(2, 2)] += q[0];
            CQ[sy(3, 3)] += q[1];
            transport_cov(F, CQ, Cp);
            st(w, V_CP, Cp);
        }
        phase_boundary();
        {
            // u = A^T as = Cp^-1 F C as
            double y[6], v[6], L[21], id[6];
            symv(C, as, y);
            fy(F, y, v);
            const bool spd = chol6(Cp, L, id);
            chol_solve6(L, id, v);
            st(w, V_U, v);
            if (!spd) { status = ST_NOT_SPD; break; }
            if (a.g_par) {
#pragma unroll
                for (int i = 0; i < 6; ++i) as[i] = v[i] + gp[i];
            } else {
#pragma unroll
                for (int i = 0; i < 6; ++i) as[i] = v[i];
            }
        }
        phase_boundary();
        {
            double ck;
            status = kalman_update(xp, Cp, m, V, x, C, &ck);
            if (status != ST_OK) break;
            st(w, V_XF, x);
            st(w, V_CF, C);
            stl(sx, 0, C);
        }
        phase_boundary();
        prev = s;
    }
    return status;
}

// Adjoint of the thin-scatterer noise of the start surface (PDG Highland
// width as in highland): q33 = th0^2, q22 = th0^2 / sin^2(theta) with
// th0 = K / (beta p) sqrt(l) (1 + c log(l / beta^2)), l = x/X0 / |n.T|,
// p = 1 / |q/p|, beta = p / sqrt(p^2 + m^2).  Adds to xb (phi, theta, q/p)
// and to the adjoint of surface a's normal n (column 2 of R, entries
// sab[3 + 3 i + 2]).
__device__ inline void noise_vjp(const double* sa, const double x[6], double mass, double q22b, double q33b,
                                 double xb[6], double sab[13]) {
    constexpr double K = 0.0136, c = 0.038;
    const double x0 = sa[12];
    double sp, cp, st, ct;
    angle_sincos(x[2], &sp, &cp);
    angle_sincos(x[3], &st, &ct);
    const double n[3] = {sa[3 + 2], sa[3 + 5], sa[3 + 8]};
    const double T[3] = {cp * st, sp * st, ct};
    const double dTdp[3] = {-sp * st, cp * st, 0.0};
    const double dTdt[3] = {cp * ct, sp * ct, -st};
    const double a = n[0] * T[0] + n[1] * T[1] + n[2] * T[2];
    const double ell = x0 / fabs(a);
    const double p = 1.0 / fabs(x[4]);
    const double E = sqrt(p * p + mass * mass);
    const double beta = p / E;
    const double A = K / (beta * p);
    const double sq = sqrt(ell);
    const double th0 = A * sq * (1.0 + c * log(ell / (beta * beta)));
    const double is2 = 1.0 / (st * st);
    const double th0b = 2.0 * th0 * (q33b + q22b * is2);
    xb[3] += q22b * (-2.0 * th0 * th0 * ct * is2 / st);
    // through the path length l = x0 / |a|, a = n.T
    const double ab = th0b * (th0 / (2.0 * ell) + A * c / sq) * (-ell / a);
    xb[2] += ab * (n[0] * dTdp[0] + n[1] * dTdp[1] + n[2] * dTdp[2]);
    xb[3] += ab * (n[0] * dTdt[0] + n[1] * dTdt[1] + n[2] * dTdt[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) sab[3 + 3 * i + 2] += ab * T[i];
    // through p and beta
    const double dth_dp = -th0 / p;
    const double dth_dbeta = -th0 / beta - 2.0 * A * c * sq / beta;
    const double dbeta_dp = mass * mass / (E * E * E);
    const double dp_dlam = (x[4] < 0.0 ? 1.0 : -1.0) * p * p;
    xb[4] += th0b * (dth_dp + dth_dbeta * dbeta_dp) * dp_dlam;
}

// Reverse of one gap (start state x on surface sa -> predicted state on sb):
// adds d(contracted outputs)/d(x) to xb and the derivatives with respect to
// the alignment of sa and sb to ga and gb.  sx (LDS) holds the start state
// (SX_X0) and the adjoints (SX_XPB, SX_FB, SX_QB).  The propagation is
// reversed by hand (kf_gap_reverse.hpp; it reads the adjoint of F column by
// column, then keeps the surface placement adjoints in those SX_FB slots;
// the replay in the forward pass's stepping precision P), the noise by its
// closed-form derivative.
static_assert(PK_N <= SX_QB - SX_FB, "the placement adjoints fit in the slots of F's adjoint");
template <class P, int FK>
__device__ __attribute__((always_inline)) void gap_vjp(const VjpArgs& a, const double* __restrict__ sa, const double* __restrict__ sb,
                        ldouble* sx, double xb[6], double ga[6], double gb[6]) {
    double xpb[6];
    ldl(sx, SX_XPB, xpb);
    double sab[13], sbb[13];
#pragma unroll
    for (int i = 0; i < 13; ++i) { sab[i] = 0.0; sbb[i] = 0.0; }
    gap_reverse<P, FK>(a.field, a.cfg, sa, sb, sx + SX_X0 * TILE, xpb, sx + SX_FB * TILE, TILE, xb, sab, sbb);
    double x[6];
    ldl(sx, SX_X0, x);
    if (a.cfg.ms && sa[12] > 0.0) noise_vjp(sa, x, a.cfg.mass, sx[SX_QB * TILE], sx[(SX_QB + 1) * TILE], xb, sab);
    double t[6];
    placement_to_alignment(sa, sab, t);
#pragma unroll
    for (int i = 0; i < 6; ++i) ga[i] += t[i];
    placement_to_alignment(sb, sbb, t);
#pragma unroll
    for (int i = 0; i < 6; ++i) gb[i] += t[i];
}

// ---------------------------------------------------------------------------
// backward sweep
// ---------------------------------------------------------------------------
template <class P, int FK>
__device__ __attribute__((always_inline)) void vjp_bwd(const VjpArgs& a, const double* __restrict__ sm, double* wl,
                                                       ldouble* sx, int t, int o, int n) {
    const int64_t H = a.n_hits, N = a.n_tracks;
    const double chi2b = a.g_chi2 ? gbl(a.g_chi2)[t] : 0.0;
    double xs[6], xsb[6], xfb[6], Cfb[21], aab[6];
    {
        const double* w = wl + (n - 1) * (NCV * TILE);
        ld(w, V_XF, xs);
        ld(w, V_U, xsb);
        if (a.g_par) {
            double gp[6];
            load_rows(a.g_par + o + n - 1, H, gp);
#pragma unroll
            for (int i = 0; i < 6; ++i) xsb[i] += gp[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) { xfb[i] = 0.0; aab[i] = 0.0; }
#pragma unroll
    for (int q = 0; q < 21; ++q) Cfb[q] = 0.0;
    // The two per-hit outputs (the hit's gradient and its alignment
    // contribution) are stored at the start of the next iteration, after that
    // iteration's first loads: a load issued behind a store waits for it (on
    // gfx9 one counter covers loads and stores).
    double mb_pend[2], c_pend[6];

    for (int k = n - 1; k >= 0; --k) {
        double* w = wl + k * (NCV * TILE);
        const double* wp = w - NCV * TILE;           // slot k-1 (used only for k > 0)
        const int s = gbl(a.sid)[o + k];
        const int prev = k > 0 ? gbl(a.sid)[o + k - 1] : a.seed_sid;
        double xpb[6], Cpb[21], wv[6], mb[2];
        // ---- update adjoint, and w = Cp^-1 (xs_k - xp_k) ----
        {
            double xp[6], Cp[21], m[2], V[3];
            ld(w, V_XP, xp);
            ld(w, V_CP, Cp);
            ld(w, V_U, xpb);
            load_rows(a.loc + o + k, H, m);
            load_rows(a.cov + o + k, H, V);
            if (k < n - 1) {
                store_rows(a.g_meas + o + k + 1, H, mb_pend);
                store_rows(a.contrib + o + k + 1, a.n_items, c_pend);
            }
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                xpb[i] = -xpb[i];                     // from the smoother: -A^T xsb_{k-1}
                xfb[i] += xsb[i];
                wv[i] = xs[i] - xp[i];
            }
            wv[2] = wrap_phi(wv[2]);
#pragma unroll
            for (int q = 0; q < 21; ++q) Cpb[q] = 0.0;
            update_vjp(xp, Cp, m, V, xfb, Cfb, chi2b, xpb, Cpb, mb);
            double L[21], id[6];
            chol6(Cp, L, id);
            chol_solve6(L, id, wv);
        }
        phase_boundary();
        // ---- xsb_{k-1} ----
        double av[6];
        if (k > 0) {
            ld(wp, V_U, av);
            if (a.g_par) {
                double gp[6];
                load_rows(a.g_par + o + k - 1, H, gp);
#pragma unroll
                for (int i = 0; i < 6; ++i) av[i] += gp[i];
            }
        } else if (a.g_tgt) {
            load_rows(a.g_tgt + t, N, av);
        } else {
#pragma unroll
            for (int i = 0; i < 6; ++i) av[i] = 0.0;
        }
        // ---- smoother-gain adjoint and xs_{k-1} ----
        double C[21], F[25], Cb[21], Fb[25];
        if (k > 0) ld(wp, V_CF, C);
        else load_rows(a.seed_cov + t, N, C);
        ld(w, V_F, F);
#pragma unroll
        for (int q = 0; q < 21; ++q) Cb[q] = 0.0;
#pragma unroll
        for (int q = 0; q < 25; ++q) Fb[q] = 0.0;
        {
            double y[6], z[6], u[6], xn[6], xprev[6];
            symv(C, av, y);
            ftw(F, wv, z);
            ld(w, V_U, u);
            gain_vjp_rank1(av, wv, z, y, u, Cb, Fb, Cpb);
            if (k > 0) ld(wp, V_XF, xprev);
            else load_rows(a.seed + t, N, xprev);
            stl(sx, SX_X0, xprev);                    // start state of gap k
            symv(C, z, xn);
#pragma unroll
            for (int i = 0; i < 6; ++i) xn[i] += xprev[i];
            xn[2] = wrap_phi(xn[2]);
            stl(sx, SX_XS, xn);                       // xs_{k-1}
        }
        phase_boundary();
        // ---- covariance-transport adjoint ----
        {
            double q[2], CQb[21];
            ld(w, V_Q, q);
            C[sy(2, 2)] += q[0];
            C[sy(3, 3)] += q[1];
            covtransport_vjp(F, C, Cpb, Fb, CQb);
#pragma unroll
            for (int i = 0; i < 21; ++i) Cb[i] += CQb[i];
            const double qb[2] = {CQb[sy(2, 2)], CQb[sy(3, 3)]};
            stl(sx, SX_QB, qb);
        }
        stl(sx, SX_XPB, xpb);
        stl(sx, SX_FB, Fb);
        stl(sx, SX_CB, Cb);
        stl(sx, SX_AV, av);
        // hit k's surface receives aab (from gap k+1, where it was the start)
        // and gb (gap k, where it is the target)
        stl(sx, SX_AA, aab);
        phase_boundary();
        // ---- propagation adjoint (reverse mode) ----
        double xb[6], ga[6], gb[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) { xb[i] = 0.0; ga[i] = 0.0; gb[i] = 0.0; }
        gap_vjp<P, FK>(a, sm + prev * SURF_STRIDE, sm + s * SURF_STRIDE, sx, xb, ga, gb);
        {
            double c[6];
            ldl(sx, SX_AA, c);
#pragma unroll
            for (int i = 0; i < 6; ++i) c[i] += gb[i];
#pragma unroll
            for (int i = 0; i < 6; ++i) c_pend[i] = c[i];
            mb_pend[0] = mb[0];
            mb_pend[1] = mb[1];
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            aab[i] = ga[i];
            xfb[i] = xb[i];
        }
        ldl(sx, SX_CB, Cfb);
        ldl(sx, SX_XS, xs);
        ldl(sx, SX_AV, xsb);
        phase_boundary();
    }
    store_rows(a.g_meas + o, H, mb_pend);
    store_rows(a.contrib + o, a.n_items, c_pend);
    if (a.g_seed) {
        double g[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) g[i] = xsb[i] + xfb[i];
        store_rows(a.g_seed + t, N, g);
    }
    store_rows(a.contrib + H + t, a.n_items, aab);
}

// One track's adjoint, a called function that holds the whole per-track
// body (the sweeps above are inlined into it).  At two waves per SIMD (half
// the registers) its spills made the C2 adjoint 1.8x slower (measured), so the
// kernels are built for one wave per SIMD only.
// The kernel arguments reach it by reference in the FP64 kernels and as a
// private copy in the mixed-precision ones.  Through the reference the body
// reads them with flat loads, which count against the LDS wait counter as
// well, so every wait for the LDS stash also waits for them; from the copy
// they are private (scratch) loads, at the price of the copy per track.
// Measured on 1e5 tracks: the copy made the mixed adjoint 2-6 % faster (C2,
// C3, C5) and the FP64 one up to 4 % slower (C2, C3).
template <class P>
using VjpArgsIn = typename std::conditional<std::is_same<P, float>::value, const VjpArgs, const VjpArgs&>::type;

template <class P, int FK>
__device__ __attribute__((noinline)) void vjp_one(VjpArgsIn<P> ag, const ldouble* sml, ldouble* sx, int64_t slot,
                                                  int t) {
    const VjpArgs& a = ag;
    // the surface table is in LDS; a generic pointer derived from an LDS one
    // keeps its reads LDS instructions in the inlined body
    const double* __restrict__ sm = (const double*)sml;
    const int64_t H = a.n_hits, N = a.n_tracks;
    int o, n;
    int status = check_track(a.off, a.sid, a.loc, a.cov, a.seed, a.seed_cov, H, N, a.n_surf, a.max_hits, t, o, n);
    double* wl = a.ws + (slot / TILE) * a.tile_doubles + (slot % TILE);
    if (status == ST_OK) status = vjp_fwd<P, FK>(a, sm, wl, sx, t, o, n);
    if (status == ST_OK) {
        vjp_bwd<P, FK>(a, sm, wl, sx, t, o, n);
    } else {
        const double nan = __longlong_as_double(0x7ff8000000000000LL);
        for (int k = 0; k < n; ++k) fill_rows<2>(a.g_meas + o + k, H, nan);
        if (a.g_seed) fill_rows<6>(a.g_seed + t, N, nan);
    }
    gbl(a.status)[t] = (uint8_t)status;
}

// Dynamic LDS: the surface table, then per wave the backward sweep's stash
// [SX_N][64] doubles.
template <class P, int FK, bool SORTED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) k_vjp(VjpArgs a) {
    extern __shared__ double sm[];
    stage_surfaces(a.n_surf, a.center, a.rot, a.x0, a.align, nullptr, sm);
    const int lane = threadIdx.x & (TILE - 1);
    ldouble* sx = (ldouble*)(sm + a.n_surf * SURF_STRIDE + (threadIdx.x / TILE) * (SX_N * TILE)) + lane;
    int iter = 0;
    for (;;) {
        const int tile = next_tile<SORTED>(a.tile_counter, iter);
        if (tile >= a.n_tiles) break;
        const int64_t i = (int64_t)tile * TILE + lane;
        if (i < a.n_tracks) vjp_one<P, FK>(a, (const ldouble*)sm, sx, i, SORTED ? a.order[i] : (int)i);
    }
}

// ---------------------------------------------------------------------------
// deterministic alignment reduction
// ---------------------------------------------------------------------------
__global__ void k_fill_f64(double* p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ inline double readlane_f64(double v, int j) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), j);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), j);
    return __hiloint2double(hi, lo);
}

// One wave per chunk of items: lanes load 64 items at a time (coalesced),
// then the items are added one after another, in item order, into an LDS
// table [S][6] (lane c < 6 adds component c).  The table is the chunk's
// partial sum.
__global__ void __launch_bounds__(64) k_align_partial(const double* contrib, int64_t n_items, int64_t H,
                                                      const int32_t* sid, int seed_sid, int S, int64_t chunk,
                                                      double* partial) {
    extern __shared__ double tab[];
    const int lane = threadIdx.x;
    for (int i = lane; i < S * 6; i += 64) tab[i] = 0.0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * chunk;
    const int64_t b1 = b0 + chunk < n_items ? b0 + chunk : n_items;
    for (int64_t base = b0; base < b1; base += 64) {
        const int64_t i = base + lane;
        double v[6];
        int s = -1;
        if (i < b1) {
            s = i < H ? sid[i] : seed_sid;
#pragma unroll
            for (int c = 0; c < 6; ++c) v[c] = contrib[c * n_items + i];
        } else {
#pragma unroll
            for (int c = 0; c < 6; ++c) v[c] = 0.0;
        }
        const int cnt = (int)(b1 - base < 64 ? b1 - base : 64);
        for (int j = 0; j < cnt; ++j) {
            const int sj = __builtin_amdgcn_readlane(s, j);
            double vj = 0.0;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double t = readlane_f64(v[c], j);
                vj = lane == c ? t : vj;
            }
            if (lane < 6 && sj >= 0 && sj < S) tab[sj * 6 + lane] += vj;
        }
    }
    __syncthreads();
    for (int i = lane; i < S * 6; i += 64) partial[(int64_t)blockIdx.x * S * 6 + i] = tab[i];
}

// Surfaces up to which k_align_lanes is used: its LDS table of 64 x S x 6
// doubles must fit one workgroup's LDS (160 KB on gfx950).
constexpr int ALIGN_LANES_MAX_S = 53;
constexpr int ALIGN_LANES_CHUNK = 1024;

// One wave per chunk of items, every lane with its own table [S][6] in LDS
// (entry e of lane l at tab[e * 64 + l]): lane l adds the chunk's items l,
// l + 64, l + 128, ... in that order, then the lane owning entry e (e mod 64)
// sums it over the 64 lane tables starting at lane table e mod 64 (a fixed
// order per entry; the rotation keeps the lanes on different LDS banks).  The
// chunk's partial sum is thus a fixed-order sum, and no item waits for the
// previous one.
__global__ void __launch_bounds__(64) k_align_lanes(const double* contrib, int64_t n_items, int64_t H,
                                                    const int32_t* sid, int seed_sid, int S, int64_t chunk,
                                                    double* partial) {
    extern __shared__ double tab[];
    const int lane = threadIdx.x;
    const int E = S * 6;
    for (int e = 0; e < E; ++e) tab[e * TILE + lane] = 0.0;
    const int64_t b0 = (int64_t)blockIdx.x * chunk;
    const int64_t b1 = b0 + chunk < n_items ? b0 + chunk : n_items;
    for (int64_t i = b0 + lane; i < b1; i += TILE) {
        const int s = i < H ? sid[i] : seed_sid;
        if (s < 0 || s >= S) continue;
#pragma unroll
        for (int c = 0; c < 6; ++c) tab[(s * 6 + c) * TILE + lane] += contrib[c * n_items + i];
    }
    __syncthreads();
    for (int e = lane; e < E; e += TILE) {
        double acc = 0.0;
        for (int l = 0; l < TILE; ++l) acc += tab[e * TILE + ((l + e) & (TILE - 1))];
        partial[(int64_t)blockIdx.x * E + e] = acc;
    }
}

// One workgroup per surface: each thread sums a fixed stride of chunks, then
// a fixed tree in LDS.  The rotation part is converted from rotations about
// the aligned surface's own axes (e1, e2, e3) to (alpha, beta, gamma):
//   R(a) = R0 Rx(alpha) Ry(beta) Rz(gamma), R^T dR/dalpha = [Rz^T Ry^T e_x]x,
//   R^T dR/dbeta = [Rz^T e_y]x, R^T dR/dgamma = [e_z]x.
__global__ void __launch_bounds__(256) k_align_final(const double* partial, int n_chunks, int S,
                                                     const double* align, double* g_align) {
    __shared__ double red[6][256];
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = tid; c < n_chunks; c += 256)
#pragma unroll
        for (int q = 0; q < 6; ++q) acc[q] += partial[(int64_t)c * S * 6 + s * 6 + q];
#pragma unroll
    for (int q = 0; q < 6; ++q) red[q][tid] = acc[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
#pragma unroll
            for (int q = 0; q < 6; ++q) red[q][tid] += red[q][tid + h];
        __syncthreads();
    }
    if (tid == 0) {
        double g[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) g[q] = red[q][0];
        if (align) {
            double sb, cb, sg, cg;
            angle_sincos(align[4 * S + s], &sb, &cb);
            angle_sincos(align[5 * S + s], &sg, &cg);
            const double e1 = g[3], e2 = g[4], e3 = g[5];
            g[3] = cg * cb * e1 - sg * cb * e2 + sb * e3;
            g[4] = sg * e1 + cg * e2;
            g[5] = e3;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) g_align[q * S + s] = g[q];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct VjpLayout {
    int64_t tile_doubles;
    int64_t n_items;
    int n_chunks;
    int64_t chunk;
    size_t contrib_off, partial_off, status_off, order_off, counts_off, counter_off, total;
};

VjpLayout vjp_layout(int64_t n_tracks, int64_t n_hits, int max_hits, int n_surf) {
    VjpLayout L;
    const int64_t tiles = n_tracks > 0 ? (n_tracks + TILE - 1) / TILE : 1;
    L.tile_doubles = (int64_t)max_hits * NCV * TILE;
    L.n_items = n_hits + n_tracks;
    // k_align_lanes: chunks of 1024 items.  k_align_partial (wide detectors)
    // adds its chunk serially, so chunks of ~128 items keep that pass short;
    // its partial sums are capped at 32 MiB.
    int64_t nc;
    if (n_surf <= ALIGN_LANES_MAX_S) {
        nc = (L.n_items + ALIGN_LANES_CHUNK - 1) / ALIGN_LANES_CHUNK;
    } else {
        const int64_t nc_cap = ((int64_t)32 << 20) / ((int64_t)n_surf * 6 * sizeof(double));
        nc = (L.n_items + 127) / 128;
        nc = nc > nc_cap ? nc_cap : nc;
    }
    nc = nc < 1 ? 1 : nc;
    L.n_chunks = (int)nc;
    L.chunk = (L.n_items + nc - 1) / nc;
    if (L.chunk < 1) L.chunk = 1;
    size_t p = (size_t)tiles * L.tile_doubles * sizeof(double);
    L.contrib_off = align_up(p, 256);
    p = L.contrib_off + (size_t)6 * L.n_items * sizeof(double);
    L.partial_off = align_up(p, 256);
    p = L.partial_off + (size_t)L.n_chunks * n_surf * 6 * sizeof(double);
    L.status_off = align_up(p, 256);
    p = L.status_off + (size_t)(n_tracks > 0 ? n_tracks : 1);
    L.order_off = align_up(p, 256);
    L.counts_off = align_up(L.order_off + (size_t)tiles * TILE * 4, 256);
    L.counter_off = align_up(L.counts_off + (size_t)sort_count_entries((int)n_tracks) * 4, 256);
    L.total = align_up(L.counter_off + SORT_HEADS * 4, 256);
    return L;
}

// Four waves per workgroup share one surface table while it and their four
// stashes fit the LDS (up to 36 surfaces on gfx950: 160 KiB less four
// 78 x 64-double stashes leaves 4 KiB, 112 bytes per surface); wider detectors run one
// wave per workgroup (fewer resident waves as the table grows).
template <class P, int FK, bool SORTED>
hipError_t launch_vjp(const VjpArgs& a, hipStream_t stream) {
    const size_t stash = (size_t)SX_N * TILE * sizeof(double);
    const size_t table = (size_t)a.n_surf * SURF_STRIDE * sizeof(double);
    const int block = table + 4 * stash <= lds_cap() ? 4 * TILE : TILE;
    const size_t shm = table + (size_t)(block / TILE) * stash;
    hipError_t e = allow_lds(k_vjp<P, FK, SORTED>, shm);
    if (e != hipSuccess) return e;
    const int need = (int)(((int64_t)a.n_tiles * TILE + block - 1) / block);
    int grid = need;
    if (SORTED) {
        const int persistent = num_cu() * 4 * TILE / block;    // one wave per SIMD
        grid = grid < persistent ? grid : persistent;
    }
    hipLaunchKernelGGL((k_vjp<P, FK, SORTED>), dim3(grid), dim3(block), shm, stream, a);
    return hipGetLastError();
}

template <bool SORTED>
hipError_t launch_vjp_prec(const VjpArgs& a, bool mixed, int field_kind, hipStream_t stream) {
    if (mixed)
        return field_kind == KF_FIELD_UNIFORM ? launch_vjp<float, FIELD_UNIFORM, SORTED>(a, stream)
                                              : launch_vjp<float, FIELD_SOLENOID, SORTED>(a, stream);
    return field_kind == KF_FIELD_UNIFORM ? launch_vjp<double, FIELD_UNIFORM, SORTED>(a, stream)
                                          : launch_vjp<double, FIELD_SOLENOID, SORTED>(a, stream);
}

}  // namespace

extern "C" {

size_t kf_vjp_workspace_bytes(const kf_config* cfg, const kf_measurements* meas, int32_t n_surfaces) {
    (void)cfg;
    if (!meas || meas->n_tracks < 0 || meas->n_hits < 0 || meas->max_hits < 1 || meas->max_hits > KF_MAX_HITS ||
        n_surfaces < 1 || n_surfaces > KF_MAX_SURFACES)
        return 0;
    return vjp_layout(meas->n_tracks, meas->n_hits, meas->max_hits, n_surfaces).total;
}

int kf_fit_tracks_vjp(const kf_config* cfg, const kf_surfaces* surf, const kf_field* field,
                      const kf_measurements* meas, const kf_seeds* seeds, const kf_cotangents* cot,
                      const kf_gradients* grad, void* workspace, size_t workspace_bytes, void* stream_) {
    if (!cot || !grad) return KF_E_NULL;
    int rc = validate_inputs(cfg, surf, field, meas, seeds);
    if (rc != KF_OK) return rc;
    if (cfg->smoother != KF_SMOOTHER_RTS) return KF_E_VALUE;     // the reverse pass is that of RTS
    if (cfg->target != KF_TARGET_SEED_SURFACE) return KF_E_VALUE;  // ... ending on the seed surface
    if (field->kind == KF_FIELD_MAP) return KF_E_VALUE;            // analytic fields only
    if (surf->type || surf->radius) return KF_E_VALUE;             // planes only
    if (meas->n_hits > 0 && !grad->meas) return KF_E_NULL;
    const VjpLayout L = vjp_layout(meas->n_tracks, meas->n_hits, meas->max_hits, surf->n);
    if (!workspace) return KF_E_WS;
    if (workspace_bytes < L.total) return KF_E_WS;
    hipStream_t stream = (hipStream_t)stream_;
    char* wsb = (char*)workspace;
    const int S = surf->n;
    if (meas->n_tracks == 0) {
        if (grad->align) {
            hipLaunchKernelGGL(k_fill_f64, dim3((6 * S + 255) / 256), dim3(256), 0, stream, grad->align,
                               (int64_t)6 * S, 0.0);
            if (hipGetLastError() != hipSuccess) return KF_E_HIP;
        }
        return KF_OK;
    }
    num_cu();
    VjpArgs a;
    memset(&a, 0, sizeof(a));
    a.n_tracks = meas->n_tracks;
    a.n_surf = S;
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
    a.align = surf->align;
    a.seed = seeds->par;
    a.seed_cov = seeds->cov;
    a.field = field_def(field);
    a.cfg = cfg_def(cfg);
    a.g_chi2 = cot->chi2;
    a.g_par = cot->par;
    a.g_tgt = cot->tgt_par;
    a.g_meas = grad->meas;
    a.g_seed = grad->seed;
    a.status = grad->status ? grad->status : (uint8_t*)(wsb + L.status_off);
    a.contrib = (double*)(wsb + L.contrib_off);
    a.n_items = L.n_items;
    a.ws = (double*)wsb;
    a.order = (const int32_t*)(wsb + L.order_off);
    a.tile_counter = (int32_t*)(wsb + L.counter_off);
    a.n_tiles = (int)((a.n_tracks + TILE - 1) / TILE);

    const int sched = cfg->schedule == KF_SCHED_DIRECT ? KF_SCHED_DIRECT : KF_SCHED_SORTED;
    {
        const int64_t nc = 6 * L.n_items;
        hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, stream, a.contrib, nc, 0.0);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return KF_E_HIP;
    if (sched == KF_SCHED_SORTED) {
        e = enqueue_length_sort(a.off, a.n_tracks, a.max_hits, (int32_t*)(wsb + L.counts_off), (int32_t*)a.order,
                                a.tile_counter, stream);
        if (e != hipSuccess) return KF_E_HIP;
        e = launch_vjp_prec<true>(a, cfg->precision == KF_PREC_MIXED, field->kind, stream);
    } else {
        e = launch_vjp_prec<false>(a, cfg->precision == KF_PREC_MIXED, field->kind, stream);
    }
    if (e != hipSuccess) return KF_E_HIP;
    if (grad->align) {
        double* partial = (double*)(wsb + L.partial_off);
        if (S <= ALIGN_LANES_MAX_S) {
            const size_t shm = (size_t)S * 6 * TILE * sizeof(double);
            if (allow_lds(k_align_lanes, shm) != hipSuccess) return KF_E_HIP;
            hipLaunchKernelGGL(k_align_lanes, dim3(L.n_chunks), dim3(64), shm, stream, (const double*)a.contrib,
                               L.n_items, (int64_t)meas->n_hits, meas->surface_id, seeds->surface_id, S, L.chunk,
                               partial);
        } else {
            hipLaunchKernelGGL(k_align_partial, dim3(L.n_chunks), dim3(64), (size_t)S * 6 * sizeof(double), stream,
                               (const double*)a.contrib, L.n_items, (int64_t)meas->n_hits, meas->surface_id,
                               seeds->surface_id, S, L.chunk, partial);
        }
        hipLaunchKernelGGL(k_align_final, dim3(S), dim3(256), 0, stream, (const double*)partial, L.n_chunks, S,
                           surf->align, grad->align);
        if (hipGetLastError() != hipSuccess) return KF_E_HIP;
    }
    return KF_OK;
}

}  // extern "C"
