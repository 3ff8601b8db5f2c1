// Measuring surfaces of every type in one transport routine (Sect. 4.2.1:
// the propagator serves every surface type; Sect. 4.3: the surface data):
// planes, discs, cylinders and lines (straws).  Used by the fit kernels
// built for detectors with cylinders or lines; the plane/disc kernels keep
// transport() of kf_device.hpp.
//
// Surface-table entry (14 doubles, as for planes and discs): centre c,
// rotation R (row-major, columns u v w), x/X0, and in slot 13 the type: 0
// plane, 1 disc, 3 line (wire through c along w), or, for a cylinder (axis
// through c along w), minus its radius.
//
// Local coordinates and their frames:
//   cylinder  l0 = w.d (along the axis), l1 = atan2(v.d, u.d) (azimuth),
//             d = r - c; r = c + rho (cos l1 u + sin l1 v) + l0 w
//   line      l0 = e.d (signed distance of closest approach), l1 = w.d,
//             e = (w x T)/|w x T|; r = c + l0 e + l1 w (e turns with T)
// Landing on a cylinder takes the straight-line path to the crossing where
// the track moves outward (the larger root); on a line the Newton step
// -g/g' of g = d_perp . T (zero at the closest approach), g' = |T_perp|^2 +
// d_perp . T' > 1e-6.  The path correction moves a variation back onto the
// constraint along dF/ds: cylinder grad g = (d_perp, 0), line (T_perp,
// d_perp) in (r, T).
#pragma once
#include "kf_device.hpp"

namespace kfm {

__device__ inline bool is_cyl(const double* __restrict__ s) { return s[13] < 0.0; }
__device__ inline bool is_line(const double* __restrict__ s) { return s[13] == 3.0; }
__device__ inline bool is_curved(const double* __restrict__ s) { return s[13] < 0.0 || s[13] == 3.0; }
// loc1 is an azimuth (disc, cylinder): its residuals wrap
__device__ inline bool azimuth_loc1(const double* __restrict__ s) { return s[13] < 0.0 || s[13] == 1.0; }

__device__ inline double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Bound -> free position on surface s: r of the local coordinates x[0],
// x[1] (with the direction T for a line), the columns e0 = dr/dl0, e1 =
// dr/dl1 and dr/dphi, dr/dtheta in ep, et (a line's frame turns with T;
// zero for the other types).  Tp, Tt: dT/dphi, dT/dtheta.
__device__ inline void surf_point(const double* __restrict__ s, const double x[6], const double T[3],
                                  const double Tp[3], const double Tt[3], double r[3], double e0[3], double e1[3],
                                  double ep[3], double et[3]) {
    const double u[3] = {s[3], s[6], s[9]}, v[3] = {s[4], s[7], s[10]}, w[3] = {s[5], s[8], s[11]};
#pragma unroll
    for (int i = 0; i < 3; ++i) { ep[i] = 0.0; et[i] = 0.0; }
    if (is_cyl(s)) {
        const double rho = -s[13];
        double sl, cl;
        angle_sincos(x[1], &sl, &cl);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            r[i] = s[i] + rho * (cl * u[i] + sl * v[i]) + x[0] * w[i];
            e0[i] = w[i];
            e1[i] = rho * (cl * v[i] - sl * u[i]);
        }
    } else if (is_line(s)) {
        double m[3], mp[3], mt[3];
        cross(w, T, m);
        cross(w, Tp, mp);
        cross(w, Tt, mt);
        const double mn = sqrt(dot3(m, m));
        const double e[3] = {m[0] / mn, m[1] / mn, m[2] / mn};
        const double epd = dot3(e, mp), etd = dot3(e, mt);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            r[i] = s[i] + x[0] * e[i] + x[1] * w[i];
            e0[i] = e[i];
            e1[i] = w[i];
            ep[i] = x[0] * (mp[i] - e[i] * epd) / mn;
            et[i] = x[0] * (mt[i] - e[i] * etd) / mn;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) r[i] = s[i] + loc_offset(s, x, i);
        loc_frame(s, x, e0, e1);
    }
}

// Free -> bound on surface s at (r, T): local coordinates l, their
// gradients in r (g0, g1) and, for a line, the gradient of l0 in T (h0;
// zero for the other types).  T is taken as given (not renormalised).
__device__ inline void surf_local(const double* __restrict__ s, const double r[3], const double T[3], double l[2],
                                  double g0[3], double g1[3], double h0[3]) {
    const double u[3] = {s[3], s[6], s[9]}, v[3] = {s[4], s[7], s[10]}, w[3] = {s[5], s[8], s[11]};
    const double d[3] = {r[0] - s[0], r[1] - s[1], r[2] - s[2]};
    const double ca = dot3(u, d), cb = dot3(v, d);
#pragma unroll
    for (int i = 0; i < 3; ++i) h0[i] = 0.0;
    if (is_cyl(s)) {
        const double q2 = ca * ca + cb * cb;
        l[0] = dot3(w, d);
        l[1] = atan2(cb, ca);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            g0[i] = w[i];
            g1[i] = (ca * v[i] - cb * u[i]) / q2;
        }
    } else if (is_line(s)) {
        double m[3];
        cross(w, T, m);
        const double mn = sqrt(dot3(m, m));
        const double e[3] = {m[0] / mn, m[1] / mn, m[2] / mn};
        const double de = dot3(e, d);
        l[0] = de;
        l[1] = dot3(w, d);
        // d(d.e)/dT = ((d - (d.e) e) x w) / |w x T|
        const double dp[3] = {d[0] - de * e[0], d[1] - de * e[1], d[2] - de * e[2]};
        double q[3];
        cross(dp, w, q);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            g0[i] = e[i];
            g1[i] = w[i];
            h0[i] = q[i] / mn;
        }
    } else if (is_disc(s)) {
        const double rr = sqrt(ca * ca + cb * cb);
        l[0] = rr;
        l[1] = atan2(cb, ca);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            g0[i] = (ca * u[i] + cb * v[i]) / rr;
            g1[i] = (ca * v[i] - cb * u[i]) / (rr * rr);
        }
    } else {
        l[0] = ca;
        l[1] = cb;
#pragma unroll
        for (int i = 0; i < 3; ++i) { g0[i] = u[i]; g1[i] = v[i]; }
    }
}

// Distance to go along the trajectory from (r, T) onto the cylinder or line
// s, and the constraint's gradient there: dp = d_perp, Tp = T_perp.  Tdot =
// dT/ds at r (used by a line only).  ST_NO_INTERSECT where there is none.
__device__ inline int curved_go(const double* __restrict__ s, const double r[3], const double T[3],
                                const double Tdot[3], double* go, double dp[3], double Tp[3]) {
    const double w[3] = {s[5], s[8], s[11]};
    const double d[3] = {r[0] - s[0], r[1] - s[1], r[2] - s[2]};
    const double dw = dot3(w, d), Tw = dot3(w, T);
#pragma unroll
    for (int i = 0; i < 3; ++i) { dp[i] = d[i] - dw * w[i]; Tp[i] = T[i] - Tw * w[i]; }
    const double dpT = dot3(dp, Tp), TpT = dot3(Tp, Tp);
    if (is_cyl(s)) {
        const double rho = -s[13];
        const double c0 = dot3(dp, dp) - rho * rho;
        const double disc = dpT * dpT - TpT * c0;
        if (!(TpT > 1e-12) || !(disc >= 0.0)) return ST_NO_INTERSECT;
        // the outward crossing, in the form without cancellation
        const double sq = sqrt(disc);
        *go = dpT <= 0.0 ? (sq - dpT) / TpT : -c0 / (dpT + sq);
        return ST_OK;
    }
    const double gp = TpT + dot3(dp, Tdot);
    if (!(gp > 1e-6)) return ST_NO_INTERSECT;
    *go = -dpT / gp;
    return ST_OK;
}

// Bound-to-bound transport between surfaces of any type: transport() of
// kf_device.hpp with the start frame, the landing rule, the final move, the
// path correction and the end frame of each type.  Same step control and
// the same FP64 anchor for the stepping precision P.
template <class P, int FK>
__device__ inline int transport_c(const Field<P, FK>& fl, const FieldDef& fd, const Cfg& cfg,
                                  const double* __restrict__ sa, const double* __restrict__ sb,
                                  const double x[6], double xp[6], double F[25], int* trials_out) {
    using R = double;
    using V = P;
    R sp, cp, st, ct;
    angle_sincos(x[2], &sp, &cp);
    angle_sincos(x[3], &st, &ct);
    const R T0[3] = {cp * st, sp * st, ct};
    R r0[3];
    P Mr[3][5], MT[3][5];
    {
        const R Tph[3] = {-(sp * st), cp * st, 0.0}, Tth[3] = {cp * ct, sp * ct, -st};
        R e0[3], e1[3], ep[3], et[3];
        surf_point(sa, x, T0, Tph, Tth, r0, e0, e1, ep, et);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int j = 0; j < 5; ++j) { Mr[i][j] = P(0); MT[i][j] = P(0); }
            if (TangentCols<FK>::J0 == 0) {
                Mr[i][0] = P(e0[i]);
                Mr[i][1] = P(e1[i]);
            }
            Mr[i][2] = P(ep[i]);
            Mr[i][3] = P(et[i]);
            MT[i][2] = P(Tph[i]);
            MT[i][3] = P(Tth[i]);
        }
    }
    const R lam_d = x[4];
    const P lam = P(lam_d);
    const R lk = lam_d * kKappa;
    const R gd = sqrt(1.0 + cfg.mass * cfg.mass * lam_d * lam_d) / kC;     // dt/ds
    const R gpd = cfg.mass * cfg.mass * lam_d / (kC * kC * gd);            // d(dt/ds)/d(q/p)
    R Mtl = 0.0;

    const bool cb = is_curved(sb);
    const bool lb = is_line(sb);
    const R nb[3] = {sb[5], sb[8], sb[11]};
    const R d0 = nb[0] * (sb[0] - r0[0]) + nb[1] * (sb[1] - r0[1]) + nb[2] * (sb[2] - r0[2]);
    const V tol = V(cfg.tol);
    const bool mixed = sizeof(V) < sizeof(double);
    const double ltol = mixed ? 1e-5 : cfg.land_tol;
    Field<R, FK> f64;
    f64.init(fd);
    R rl[3] = {R(0.0), R(0.0), R(0.0)};
    P dr[3] = {P(0), P(0), P(0)}, dT[3] = {P(0), P(0), P(0)};
    R dt = 0.0;
    V hmag = V(-1);
    int trials = 0;
    int status = ST_OK;
    Stages<P, FK> S;
    for (;;) {
        P T[3], rabs[3];
        R Td[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Td[i] = T0[i] + R(dT[i]);
            T[i] = P(Td[i]);
            rabs[i] = P(r0[i] + rl[i]) + dr[i];
        }
        R go;
        if (cb) {
            R rr[3], Tdot[3] = {0.0, 0.0, 0.0}, dp[3], Tp[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) rr[i] = r0[i] + rl[i] + R(dr[i]);
            if (lb) {
                R B[3], TB[3];
                f64.eval(rr, B);
                cross(Td, B, TB);
#pragma unroll
                for (int i = 0; i < 3; ++i) Tdot[i] = lk * TB[i];
            }
            status = curved_go(sb, rr, Td, Tdot, &go, dp, Tp);
            if (status != ST_OK) break;
            if (::fabs(go) < ltol) break;
        } else {
            const R nTd = nb[0] * Td[0] + nb[1] * Td[1] + nb[2] * Td[2];
            const R distd = d0 - (nb[0] * rl[0] + nb[1] * rl[1] + nb[2] * rl[2])
                                - (nb[0] * R(dr[0]) + nb[1] * R(dr[1]) + nb[2] * R(dr[2]));
            if (::fabs(nTd) < 1e-6) { status = ST_NO_INTERSECT; break; }
            if (::fabs(distd) < ltol) break;
            go = distd / nTd;
        }
        if (trials >= cfg.max_steps) { status = ST_STEP_CAP; break; }
        const P d = P(go);
        const V dv = d;
        if (hmag < V(0)) hmag = dv < V(0) ? -dv : dv;
        const P h = ((dv < V(0) ? -dv : dv) <= hmag) ? d : P(dv < V(0) ? -hmag : hmag);
        P k[4][3];
        const V err = rkn_trial<P, FK>(fl, rabs, T, lam, h, S, k);
        ++trials;
        phase_boundary();
        const V tiny = V(mixed ? 1e-30 : 1e-300);
        V fac = V(0.9) * sqrt(sqrt(tol / (err > tiny ? err : tiny)));
        fac = fac < V(0.25) ? V(0.25) : (fac > V(4) ? V(4) : fac);
        if (err <= tol) {
            rkn_tangent<P, FK>(fl, S, k, lam, h, T, Mr, MT);
            phase_boundary();
            const R hd = R(h);
            Mtl = Mtl + hd * gpd;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                rl[i] = rl[i] + hd * Td[i];
                dr[i] = dr[i] + h * h * (P(1) / P(6)) * (k[0][i] + k[1][i] + k[2][i]);
                dT[i] = dT[i] + h * (P(1) / P(6)) * (k[0][i] + P(2) * k[1][i] + P(2) * k[2][i] + k[3][i]);
            }
            dt = dt + hd * gd;
        }
        const V hv = h;
        hmag = (hv < V(0) ? -hv : hv) * fac;
    }
    *trials_out = trials;
    if (status != ST_OK) return status;

    // final free state in FP64, then the remaining distance onto the surface
    // to second order: r += d T + d^2/2 T', T += d T', t += d dt/ds
    R r[3], T[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) { r[i] = r0[i] + rl[i] + R(dr[i]); T[i] = T0[i] + R(dT[i]); }
    R t = x[5] + dt;
    {
        R B0[3], TB0[3];
        f64.eval(r, B0);
        cross(T, B0, TB0);
        R rem;
        if (cb) {
            R Tdot[3], dp[3], Tp[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) Tdot[i] = lk * TB0[i];
            // the state the loop last accepted the landing on: same result
            curved_go(sb, r, T, Tdot, &rem, dp, Tp);
        } else {
            const R nT0 = nb[0] * T[0] + nb[1] * T[1] + nb[2] * T[2];
            rem = (nb[0] * (sb[0] - r[0]) + nb[1] * (sb[1] - r[1]) + nb[2] * (sb[2] - r[2])) / nT0;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            r[i] = r[i] + rem * T[i] + 0.5 * rem * rem * lk * TB0[i];
            T[i] = T[i] + rem * lk * TB0[i];
        }
        t = t + rem * gd;
    }
    // free -> bound on surface b
    R g0[3], g1[3], h0[3];
    {
        R l[2];
        surf_local(sb, r, T, l, g0, g1, h0);
        xp[0] = l[0];
        xp[1] = l[1];
    }
    const R rho2 = T[0] * T[0] + T[1] * T[1];
    const R rho = sqrt(rho2);
    const R n2 = rho2 + T[2] * T[2];
    xp[2] = atan2(T[1], T[0]);
    xp[3] = atan2(rho, T[2]);
    xp[4] = lam_d;
    xp[5] = t;
    // F = J_fb * P_corr * (D J_bf): the path correction moves each variation
    // back onto the surface's constraint along dF/ds (gradient gr in r, gT in
    // T, rate = gradient . dF/ds), then J_fb maps it to the bound parameters
    R B[3], TxB[3];
    f64.eval(r, B);
    cross(T, B, TxB);
    R gr[3], gT[3] = {0.0, 0.0, 0.0}, irate;
    if (cb) {
        R Tdot[3], dp[3], Tp[3], go;
#pragma unroll
        for (int i = 0; i < 3; ++i) Tdot[i] = lk * TxB[i];
        curved_go(sb, r, T, Tdot, &go, dp, Tp);
        if (lb) {
#pragma unroll
            for (int i = 0; i < 3; ++i) { gr[i] = Tp[i]; gT[i] = dp[i]; }
            irate = 1.0 / (dot3(Tp, T) + dot3(dp, Tdot));
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) gr[i] = dp[i];
            irate = 1.0 / dot3(dp, T);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) gr[i] = nb[i];
        irate = 1.0 / (nb[0] * T[0] + nb[1] * T[1] + nb[2] * T[2]);
    }
    const R ip = 1.0 / rho2, ith = 1.0 / (rho * n2), in2 = 1.0 / n2;
    // the loc0/loc1 columns of a uniform field were never propagated: dr/dloc on surface a
    R e0[3], e1[3];
    if (TangentCols<FK>::J0 != 0) {
        const R Tph[3] = {-(sp * st), cp * st, 0.0}, Tth[3] = {cp * ct, sp * ct, -st};
        R ra[3], ep[3], et[3];
        surf_point(sa, x, T0, Tph, Tth, ra, e0, e1, ep, et);
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const bool fixed = j < TangentCols<FK>::J0;
        R mr[3], mt[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mr[i] = fixed ? (j == 0 ? e0[i] : e1[i]) : R(Mr[i][j]);
            mt[i] = fixed ? R(0.0) : R(MT[i][j]);
        }
        const R sc = (dot3(gr, mr) + dot3(gT, mt)) * irate;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mr[i] = mr[i] - T[i] * sc;
            mt[i] = mt[i] - lk * TxB[i] * sc;
        }
        F[0 * 5 + j] = dot3(g0, mr) + dot3(h0, mt);
        F[1 * 5 + j] = dot3(g1, mr);
        F[2 * 5 + j] = (T[0] * mt[1] - T[1] * mt[0]) * ip;
        F[3 * 5 + j] = T[2] * (T[0] * mt[0] + T[1] * mt[1]) * ith - rho * mt[2] * in2;
        F[4 * 5 + j] = (j == 4 ? Mtl : R(0.0)) - gd * sc;
    }
    return ST_OK;
}

// Thin-scatterer noise on surface s (any type) for the filtered state x:
// x/X0 over the cosine of the incidence on the surface normal (plane, disc:
// w; cylinder: the radial direction at the state's azimuth); a line is
// crossed across its wire, x/X0 over |w x T|.
__device__ inline void highland_c(const double* __restrict__ s, const double x[6], double mass, double* q22,
                                  double* q33) {
    const double x0 = s[12];
    if (!(x0 > 0.0)) { *q22 = 0.0; *q33 = 0.0; return; }
    double sp, cp, st, ct;
    angle_sincos(x[2], &sp, &cp);
    angle_sincos(x[3], &st, &ct);
    const double T[3] = {cp * st, sp * st, ct};
    double nT;
    if (is_cyl(s)) {
        double sl, cl;
        angle_sincos(x[1], &sl, &cl);
        nT = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) nT = nT + (cl * s[3 + 3 * i + 0] + sl * s[3 + 3 * i + 1]) * T[i];
    } else if (is_line(s)) {
        const double w[3] = {s[5], s[8], s[11]};
        double m[3];
        cross(w, T, m);
        nT = sqrt(dot3(m, m));
    } else {
        nT = s[3 + 2] * T[0] + s[3 + 5] * T[1] + s[3 + 8] * T[2];
    }
    const double path = x0 / fabs(nT);
    const double p = 1.0 / fabs(x[4]);
    const double beta = p / sqrt(p * p + mass * mass);
    const double th0 = 0.0136 / (beta * p) * sqrt(path) * (1.0 + 0.038 * log(path / (beta * beta)));
    *q33 = th0 * th0;
    *q22 = th0 * th0 / (st * st);
}

// One-dimensional gain-matrix update (a straw measures loc0 only: H = e0^T),
// Joseph form with the scalar residual covariance S = V00 + Cp00:
//   Cf = Cp - K P - P^T K^T + K S K^T,  P = H Cp,  K = Cp H^T / S
__device__ inline int kalman_update1(const double xp[6], const double Cp[21], double m0, double V0, double xf[6],
                                     double Cf[21], double* chi2) {
    const double r = m0 - xp[0];
    const double S = V0 + Cp[sy(0, 0)];
    if (!(S > 0.0)) return ST_NOT_SPD;
    const double iS = 1.0 / S;
    double K[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) K[i] = Cp[sy(0, i)] * iS;
#pragma unroll
    for (int i = 0; i < 6; ++i) xf[i] = xp[i] + K[i] * r;
    xf[2] = wrap_phi(xf[2]);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j)
            Cf[sy(i, j)] = Cp[sy(i, j)] - K[i] * Cp[sy(0, j)] - Cp[sy(0, i)] * K[j] + K[i] * S * K[j];
    *chi2 = r * r * iS;
    return ST_OK;
}

// The update of a hit on surface type `type` (0 plane, 1 disc, 2 cylinder,
// 3 line): one-dimensional on a line, the azimuth residual wrapped on discs
// and cylinders.
__device__ inline int update_typed(int type, const double xp[6], const double Cp[21], const double m[2],
                                   const double V[3], double xf[6], double Cf[21], double* chi2) {
    if (type == 3) return kalman_update1(xp, Cp, m[0], V[0], xf, Cf, chi2);
    return kalman_update(xp, Cp, m, V, xf, Cf, chi2, type == 1 || type == 2);
}

// Table type slot -> surface type number
__device__ inline int table_type(const double* __restrict__ s) {
    return s[13] < 0.0 ? 2 : (s[13] == 1.0 ? 1 : (s[13] == 3.0 ? 3 : 0));
}

}  // namespace kfm
