// kf_gap_reverse.hpp -- reverse mode through one propagation gap.
//
// The gap maps the bound state x on surface a to the predicted state xp on
// surface b and the transport Jacobian F (Sect. 4.1: adaptive RKN stepping,
// forward tangents of the step map, final move onto the plane, path
// correction, local<->global conversions).  Given the adjoints of xp and F,
// gap_reverse returns the adjoints of x and of the 12 placement values
// (c, R) of each surface.
//
// The step sequence is the forward pass's: gap_run replays the adaptive loop
// with the same routines (rkn_trial, rkn_tangent) and the same expressions as
// transport, in the same stepping precision P (double, or float for the mixed
// fit: FP32 increments on the FP64 anchor), so it takes the same decisions.
// Everything after the replay is FP64: each replayed state is widened and the
// reverse sweep evaluates the derivatives there, accumulating in FP64.  Reverse order: the final part
// (free -> bound, F, final move) at the landed state, then the accepted steps
// from last to first, the state at the start of each recovered by replaying
// the gap from its start (a few steps per gap, so the quadratic replay cost
// stays small and nothing is stored), then the bound -> free start.
//
// Per accepted step (state r, T, tangents Mr, MT, step h):
//   stages  k1 = lk T x B(r), r2 = r + h/2 T + h^2/8 k1, T2 = T + h/2 k1,
//           k2 = lk T2 x B(r2), T3 = T + h/2 k2, k3 = lk T3 x B(r2),
//           r4 = r + h T + h^2/2 k3, T4 = T + h k3, k4 = lk T4 x B(r4)
//   update  r' = r + h T + h^2/6 (k1+k2+k3), T' = T + h/6 (k1+2k2+2k3+k4),
//           t' = t + h gd, Mtl' = Mtl + h gpd, (Mr, MT)' = the same stage
//           equations linearised column by column (lk = (q/p) kappa)
// A step capped by the distance to plane b has h = n.(c_b - r)/(n.T), which is
// differentiated; controller-set sizes are constants.
#pragma once
#include "kf_device.hpp"

namespace kfm {

// running state of a gap replay: the FP64 anchor (start state, straight-line
// part rl of the position, time, d t / d(q/p)) and the increments and tangent
// columns in the stepping precision P, as transport keeps them
template <class P, int FK>
struct GapRun {
    double r0[3], T0[3], nb[3];
    double lam, gd, gpd, d0;
    double rl[3];
    P dr[3], dT[3];
    double dt, Mtl;
    P hmag;
    P Mr[3][5], MT[3][5];
    int trials, accepted;
};

// Start of the gap: bound -> free on surface a (a plane), initial tangents.
template <class P, int FK>
__device__ inline void gap_start(const Cfg& cfg, const double* sa, const double* sb, const double x[6],
                                 GapRun<P, FK>& g) {
    double sp, cp, st, ct;
    angle_sincos(x[2], &sp, &cp);
    angle_sincos(x[3], &st, &ct);
#pragma unroll
    for (int i = 0; i < 3; ++i) g.r0[i] = sa[i] + (x[0] * sa[3 + 3 * i + 0] + x[1] * sa[3 + 3 * i + 1]);
    g.T0[0] = cp * st; g.T0[1] = sp * st; g.T0[2] = ct;
    g.lam = x[4];
    g.gd = sqrt(1.0 + cfg.mass * cfg.mass * g.lam * g.lam) / kC;
    g.gpd = cfg.mass * cfg.mass * g.lam / (kC * kC * g.gd);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 5; ++j) { g.Mr[i][j] = P(0); g.MT[i][j] = P(0); }
        if (TangentCols<FK>::J0 == 0) {
            g.Mr[i][0] = P(sa[3 + 3 * i + 0]);
            g.Mr[i][1] = P(sa[3 + 3 * i + 1]);
        }
    }
    g.MT[0][2] = P(-(sp * st)); g.MT[1][2] = P(cp * st); g.MT[2][2] = P(0);
    g.MT[0][3] = P(cp * ct);    g.MT[1][3] = P(sp * ct); g.MT[2][3] = P(-st);
    g.Mtl = 0.0;
    g.nb[0] = sb[3 + 2]; g.nb[1] = sb[3 + 5]; g.nb[2] = sb[3 + 8];
    g.d0 = g.nb[0] * (sb[0] - g.r0[0]) + g.nb[1] * (sb[1] - g.r0[1]) + g.nb[2] * (sb[2] - g.r0[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) { g.rl[i] = 0.0; g.dr[i] = P(0); g.dT[i] = P(0); }
    g.dt = 0.0;
    g.hmag = P(-1);
    g.trials = 0;
    g.accepted = 0;
}

// Replay the adaptive loop: the expressions of transport<P>, term for term.
// Returns 1 when the accepted step number `stop` is reached, with the state
// at its start and its h, capped flag, stages and k; 0 when the gap has
// landed (state before the final move); -1 if the replay fails.
template <class P, int FK>
__device__ inline int gap_run(const Field<P, FK>& fl, const Cfg& cfg, int stop, GapRun<P, FK>& g,
                              P& h_out, bool& capped_out, Stages<P, FK>& S, P k[4][3]) {
    using R = double;
    using V = P;
    const V tol = V(cfg.tol);
    const bool mixed = sizeof(V) < sizeof(double);
    const P lam = P(g.lam);
    for (;;) {
        P T[3], rabs[3];
        R Td[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Td[i] = g.T0[i] + R(g.dT[i]);
            T[i] = P(Td[i]);
            rabs[i] = P(g.r0[i] + g.rl[i]) + g.dr[i];
        }
        const R nTd = g.nb[0] * Td[0] + g.nb[1] * Td[1] + g.nb[2] * Td[2];
        const R distd = g.d0 - (g.nb[0] * g.rl[0] + g.nb[1] * g.rl[1] + g.nb[2] * g.rl[2])
                             - (g.nb[0] * R(g.dr[0]) + g.nb[1] * R(g.dr[1]) + g.nb[2] * R(g.dr[2]));
        if (::fabs(nTd) < 1e-6) return -1;
        const double ltol = mixed ? 1e-5 : cfg.land_tol;
        if (::fabs(distd) < ltol) return 0;
        if (g.trials >= cfg.max_steps) return -1;
        const P d = P(distd / nTd);
        const V dv = d;
        if (g.hmag < V(0)) g.hmag = dv < V(0) ? -dv : dv;
        const bool capped = (dv < V(0) ? -dv : dv) <= g.hmag;
        const P h = capped ? d : P(dv < V(0) ? -g.hmag : g.hmag);
        const V err = rkn_trial<P, FK>(fl, rabs, T, lam, h, S, k);
        ++g.trials;
        const V tiny = V(mixed ? 1e-30 : 1e-300);
        V fac = V(0.9) * sqrt(sqrt(tol / (err > tiny ? err : tiny)));
        fac = fac < V(0.25) ? V(0.25) : (fac > V(4) ? V(4) : fac);
        if (err <= tol) {
            if (g.accepted == stop) {
                h_out = h;
                capped_out = capped;
                return 1;
            }
            rkn_tangent<P, FK>(fl, S, k, lam, h, T, g.Mr, g.MT);
            const R hd = R(h);
            g.Mtl = g.Mtl + hd * g.gpd;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                g.rl[i] = g.rl[i] + hd * Td[i];
                g.dr[i] = g.dr[i] + h * h * (P(1) / P(6)) * (k[0][i] + k[1][i] + k[2][i]);
                g.dT[i] = g.dT[i] + h * (P(1) / P(6)) * (k[0][i] + P(2) * k[1][i] + P(2) * k[2][i] + k[3][i]);
            }
            g.dt = g.dt + hd * g.gd;
            ++g.accepted;
        }
        const V hv = h;
        g.hmag = (hv < V(0) ? -hv : hv) * fac;
    }
}

// The replayed state in FP64 for the reverse sweep (the FP64 replay is
// already that state).
template <int FK>
__device__ inline const GapRun<double, FK>& widen(const GapRun<double, FK>& g, GapRun<double, FK>&) { return g; }
template <int FK>
__device__ inline const GapRun<double, FK>& widen(const GapRun<float, FK>& g, GapRun<double, FK>& w) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        w.r0[i] = g.r0[i];
        w.T0[i] = g.T0[i];
        w.nb[i] = g.nb[i];
        w.rl[i] = g.rl[i];
        w.dr[i] = double(g.dr[i]);
        w.dT[i] = double(g.dT[i]);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            w.Mr[i][j] = double(g.Mr[i][j]);
            w.MT[i][j] = double(g.MT[i][j]);
        }
    }
    w.lam = g.lam;
    w.gd = g.gd;
    w.gpd = g.gpd;
    w.d0 = g.d0;
    w.dt = g.dt;
    w.Mtl = g.Mtl;
    w.hmag = double(g.hmag);
    w.trials = g.trials;
    w.accepted = g.accepted;
    return w;
}

// grad B at r applied to v is Field::grad_apply; its transpose:
//   (grad B)^T w = (g z w0, g z w1, g x w0 + g y w1 - 2 g z w2)
template <int FK>
__device__ inline void gradT_apply(const Field<double, FK>& fl, const double r[3], const double w[3], double o[3]) {
    if (FK == FIELD_UNIFORM) {
        o[0] = 0.0; o[1] = 0.0; o[2] = 0.0;
        return;
    }
    const double g = fl.g;
    o[0] = g * r[2] * w[0];
    o[1] = g * r[2] * w[1];
    o[2] = g * (r[0] * w[0] + r[1] * w[1] - 2.0 * r[2] * w[2]);
}

// d/dr of w . ((grad B)(r) v) for fixed v and w (the field is quadratic, so
// this is a constant bilinear form):  w0 g (z v0 + x v2) + w1 g (z v1 + y v2)
// - 2 w2 g z v2
template <int FK>
__device__ inline void grad2_apply(const Field<double, FK>& fl, const double v[3], const double w[3], double o[3]) {
    if (FK == FIELD_UNIFORM) {
        o[0] = 0.0; o[1] = 0.0; o[2] = 0.0;
        return;
    }
    const double g = fl.g;
    o[0] = g * w[0] * v[2];
    o[1] = g * w[1] * v[2];
    o[2] = g * (w[0] * v[0] + w[1] * v[1] - 2.0 * w[2] * v[2]);
}

__device__ inline double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// adjoint of c = a x b: abar += b x cbar, bbar += cbar x a
__device__ inline void cross_vjp(const double a[3], const double b[3], const double cb[3], double ab[3], double bb[3]) {
    double t[3];
    cross(b, cb, t);
#pragma unroll
    for (int i = 0; i < 3; ++i) ab[i] += t[i];
    cross(cb, a, t);
#pragma unroll
    for (int i = 0; i < 3; ++i) bb[i] += t[i];
}

// adjoints carried backwards through a gap
struct GapBar {
    double r[3], T[3];        // position and direction
    double t;                 // time
    double Mr[3][5], MT[3][5];
    double Mtl;
    double lam, gd, gpd;
};

// Adjoints of the two surfaces' placements.  Between the gap's end and its
// start they wait in memory (in gap_reverse: the slots of F's adjoint, read
// by then), which takes 42 registers off the reverse of the steps; only a
// capped step adds to them (PK_NB, PK_CB).
struct PlaceBar {
    double cb[3], ub[3], vb[3], nb[3];   // surface b placement
    double ca[3], ua[3], va[3];          // surface a placement (n_a enters only the noise)
};
constexpr int PK_CB = 0, PK_NB = 3, PK_UB = 6, PK_VB = 9, PK_CA = 12, PK_UA = 15, PK_VA = 18, PK_N = 21;

template <class MP>
__device__ inline void park_store(MP m, int64_t fs, const PlaceBar& pb) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        m[(PK_CB + i) * fs] = pb.cb[i]; m[(PK_NB + i) * fs] = pb.nb[i];
        m[(PK_UB + i) * fs] = pb.ub[i]; m[(PK_VB + i) * fs] = pb.vb[i];
        m[(PK_CA + i) * fs] = pb.ca[i]; m[(PK_UA + i) * fs] = pb.ua[i];
        m[(PK_VA + i) * fs] = pb.va[i];
    }
}

template <class MP>
__device__ inline void park_load(MP m, int64_t fs, PlaceBar& pb) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        pb.cb[i] = m[(PK_CB + i) * fs]; pb.nb[i] = m[(PK_NB + i) * fs];
        pb.ub[i] = m[(PK_UB + i) * fs]; pb.vb[i] = m[(PK_VB + i) * fs];
        pb.ca[i] = m[(PK_CA + i) * fs]; pb.ua[i] = m[(PK_UA + i) * fs];
        pb.va[i] = m[(PK_VA + i) * fs];
    }
}

// Reverse of one accepted step.  Inputs: the state at the step start (g), its
// h, capped flag and stage accelerations k; gb holds the adjoints of the step's outputs
// on entry and of its inputs on return; a capped step also adds to the parked
// placement adjoints (PlaceBar layout, entry q at pk[q * fs]).
template <int FK, class MP>
__device__ inline void step_reverse(const Field<double, FK>& fl, const double* sb, const GapRun<double, FK>& g,
                                    double h, bool capped, const double k[4][3], GapBar& gb, MP pk, int64_t fs) {
    // explicit q/p dependence of stage k_i = (q/p) kappa T_i x B_i: kappa T_i x B_i
    // (one form for every q/p, q/p = 0 included; reversed through T_i and B_i)
    const double lam = g.lam, lk = lam * kKappa;
    double r[3], T[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        r[i] = (g.r0[i] + g.rl[i]) + g.dr[i];
        T[i] = g.T0[i] + g.dT[i];
    }
    // stage positions, directions and fields
    double rs[4][3], Ts[4][3], Bs[4][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        rs[0][i] = r[i];
        Ts[0][i] = T[i];
        rs[1][i] = r[i] + 0.5 * h * T[i] + h * h * 0.125 * k[0][i];
        Ts[1][i] = T[i] + 0.5 * h * k[0][i];
        rs[2][i] = rs[1][i];
        Ts[2][i] = T[i] + 0.5 * h * k[1][i];
        rs[3][i] = r[i] + h * T[i] + h * h * 0.5 * k[2][i];
        Ts[3][i] = T[i] + h * k[2][i];
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) fl.eval(rs[st], Bs[st]);
    double hb = 0.0, lkb = 0.0;
    double kb[4][3], Tsb[4][3], rsb[4][3], Bsb[4][3];
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int i = 0; i < 3; ++i) { kb[st][i] = 0.0; Tsb[st][i] = 0.0; rsb[st][i] = 0.0; Bsb[st][i] = 0.0; }
    // (a) t' = t + h gd; Mtl' = Mtl + h gpd
    hb += gb.t * g.gd + gb.Mtl * g.gpd;
    gb.gd += gb.t * h;
    gb.gpd += gb.Mtl * h;
    // (b) r' = r + h T + h^2/6 (k1+k2+k3); T' = T + h/6 (k1+2k2+2k3+k4)
    {
        double rb[3], Tb[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) { rb[i] = gb.r[i]; Tb[i] = gb.T[i]; }
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            s1 += rb[i] * (k[0][i] + k[1][i] + k[2][i]);
            s2 += Tb[i] * (k[0][i] + 2.0 * k[1][i] + 2.0 * k[2][i] + k[3][i]);
        }
        hb += dot3(rb, T) + (h / 3.0) * s1 + s2 / 6.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            gb.T[i] += h * rb[i];
            kb[0][i] += h * h / 6.0 * rb[i] + h / 6.0 * Tb[i];
            kb[1][i] += h * h / 6.0 * rb[i] + h / 3.0 * Tb[i];
            kb[2][i] += h * h / 6.0 * rb[i] + h / 3.0 * Tb[i];
            kb[3][i] += h / 6.0 * Tb[i];
        }
    }
    // (c) tangent columns: forward intermediates recomputed, then reversed
#pragma unroll
    for (int j = TangentCols<FK>::J0; j < 5; ++j) {
        double dTs[4][3], drs[4][3], dk[4][3], gs[4][3];
        {
            double MTj[3], Mrj[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) { MTj[i] = g.MT[i][j]; Mrj[i] = g.Mr[i][j]; }
#pragma unroll
            for (int st = 0; st < 4; ++st) {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    if (st == 0) { dTs[0][i] = MTj[i]; drs[0][i] = Mrj[i]; }
                    else if (st == 1) { dTs[1][i] = MTj[i] + 0.5 * h * dk[0][i];
                                        drs[1][i] = Mrj[i] + 0.5 * h * MTj[i] + h * h * 0.125 * dk[0][i]; }
                    else if (st == 2) { dTs[2][i] = MTj[i] + 0.5 * h * dk[1][i]; drs[2][i] = drs[1][i]; }
                    else { dTs[3][i] = MTj[i] + h * dk[2][i];
                           drs[3][i] = Mrj[i] + h * MTj[i] + h * h * 0.5 * dk[2][i]; }
                }
                double c1[3], c2[3];
                if (FK == FIELD_UNIFORM) {
                    gs[st][0] = 0.0; gs[st][1] = 0.0; gs[st][2] = 0.0;
                } else {
                    fl.grad_apply(rs[st], drs[st], gs[st]);
                }
                cross(dTs[st], Bs[st], c1);
                cross(Ts[st], gs[st], c2);
#pragma unroll
                for (int i = 0; i < 3; ++i) dk[st][i] = lk * (c1[i] + c2[i]);
                if (j == 4) {
                    double q[3];
                    cross(Ts[st], Bs[st], q);
#pragma unroll
                    for (int i = 0; i < 3; ++i) dk[st][i] += kKappa * q[i];
                }
            }
        }
        double Mrb[3], MTb[3], dkb[4][3], dTb[4][3], drb[4][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double mrb = gb.Mr[i][j], mtb = gb.MT[i][j];
            Mrb[i] = mrb;
            MTb[i] = mtb + h * mrb;
            hb += mrb * (g.MT[i][j] + (h / 3.0) * (dk[0][i] + dk[1][i] + dk[2][i])) +
                  mtb * (dk[0][i] + 2.0 * dk[1][i] + 2.0 * dk[2][i] + dk[3][i]) / 6.0;
            dkb[0][i] = h * h / 6.0 * mrb + h / 6.0 * mtb;
            dkb[1][i] = h * h / 6.0 * mrb + h / 3.0 * mtb;
            dkb[2][i] = h * h / 6.0 * mrb + h / 3.0 * mtb;
            dkb[3][i] = h / 6.0 * mtb;
        }
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int i = 0; i < 3; ++i) { dTb[st][i] = 0.0; drb[st][i] = 0.0; }
#pragma unroll
        for (int st = 3; st >= 0; --st) {
            // dk = lk (dT x B + T x g) + [j = 4] k / lam,  g = (grad B)(r_st) dr
            double c1[3], c2[3], e[3], gbar[3];
            cross(dTs[st], Bs[st], c1);
            cross(Ts[st], gs[st], c2);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                lkb += dkb[st][i] * (c1[i] + c2[i]);
                e[i] = lk * dkb[st][i];
                gbar[i] = 0.0;
            }
            if (j == 4) {
                double eq[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) eq[i] = kKappa * dkb[st][i];
                cross_vjp(Ts[st], Bs[st], eq, Tsb[st], Bsb[st]);
            }
            cross_vjp(dTs[st], Bs[st], e, dTb[st], Bsb[st]);
            cross_vjp(Ts[st], gs[st], e, Tsb[st], gbar);
            if (FK != FIELD_UNIFORM) {
                double t1[3], t2[3];
                gradT_apply(fl, rs[st], gbar, t1);
                grad2_apply(fl, drs[st], gbar, t2);
#pragma unroll
                for (int i = 0; i < 3; ++i) { drb[st][i] += t1[i]; rsb[st][i] += t2[i]; }
            }
            // stage inputs
            if (st == 3) {
                // dT4 = MT + h dk3; dr4 = Mr + h MT + h^2/2 dk3
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    MTb[i] += dTb[3][i] + h * drb[3][i];
                    Mrb[i] += drb[3][i];
                    hb += dTb[3][i] * dk[2][i] + drb[3][i] * (g.MT[i][j] + h * dk[2][i]);
                    dkb[2][i] += h * dTb[3][i] + h * h * 0.5 * drb[3][i];
                }
            } else if (st == 2) {
                // dT3 = MT + h/2 dk2; dr3 = dr2
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    MTb[i] += dTb[2][i];
                    hb += 0.5 * dTb[2][i] * dk[1][i];
                    dkb[1][i] += 0.5 * h * dTb[2][i];
                    drb[1][i] += drb[2][i];                 // dr3 = dr2
                }
            } else if (st == 1) {
                // dT2 = MT + h/2 dk1; dr2 = Mr + h/2 MT + h^2/8 dk1 (drb[1] includes dr3's adjoint)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double d2 = drb[1][i];
                    MTb[i] += dTb[1][i] + 0.5 * h * d2;
                    Mrb[i] += d2;
                    hb += 0.5 * dTb[1][i] * dk[0][i] + d2 * (0.5 * g.MT[i][j] + 0.25 * h * dk[0][i]);
                    dkb[0][i] += 0.5 * h * dTb[1][i] + h * h * 0.125 * d2;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    MTb[i] += dTb[0][i];
                    Mrb[i] += drb[0][i];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) { gb.Mr[i][j] = Mrb[i]; gb.MT[i][j] = MTb[i]; }
        phase_boundary();   // one column's temporaries at a time
    }
    // (d) primal stages, 4 -> 1: k_st = lk T_st x B(r_st)
#pragma unroll
    for (int st = 3; st >= 0; --st) {
        double TxB[3], e[3];
        cross(Ts[st], Bs[st], TxB);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lkb += kb[st][i] * TxB[i];
            e[i] = lk * kb[st][i];
        }
        cross_vjp(Ts[st], Bs[st], e, Tsb[st], Bsb[st]);
        if (FK != FIELD_UNIFORM) {
            double t1[3];
            gradT_apply(fl, rs[st], Bsb[st], t1);
#pragma unroll
            for (int i = 0; i < 3; ++i) rsb[st][i] += t1[i];
        }
        if (st == 3) {
            // T4 = T + h k3; r4 = r + h T + h^2/2 k3
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                gb.T[i] += Tsb[3][i] + h * rsb[3][i];
                gb.r[i] += rsb[3][i];
                hb += Tsb[3][i] * k[2][i] + rsb[3][i] * (T[i] + h * k[2][i]);
                kb[2][i] += h * Tsb[3][i] + h * h * 0.5 * rsb[3][i];
            }
        } else if (st == 2) {
            // T3 = T + h/2 k2; r3 = r2
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                gb.T[i] += Tsb[2][i];
                hb += 0.5 * Tsb[2][i] * k[1][i];
                kb[1][i] += 0.5 * h * Tsb[2][i];
                rsb[1][i] += rsb[2][i];
            }
        } else if (st == 1) {
            // T2 = T + h/2 k1; r2 = r + h/2 T + h^2/8 k1
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                gb.T[i] += Tsb[1][i] + 0.5 * h * rsb[1][i];
                gb.r[i] += rsb[1][i];
                hb += 0.5 * Tsb[1][i] * k[0][i] + rsb[1][i] * (0.5 * T[i] + 0.25 * h * k[0][i]);
                kb[0][i] += 0.5 * h * Tsb[1][i] + h * h * 0.125 * rsb[1][i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                gb.T[i] += Tsb[0][i];
                gb.r[i] += rsb[0][i];
            }
        }
    }
    gb.lam += lkb * kKappa;
    // (e) a step capped by the distance to plane b: h = n.(c_b - r) / (n.T)
    if (capped) {
        const double nT = dot3(g.nb, T);
        const double dist = g.nb[0] * (sb[0] - r[0]) + g.nb[1] * (sb[1] - r[1]) + g.nb[2] * (sb[2] - r[2]);
        const double db = hb / nT, nTb = -hb * dist / (nT * nT);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            pk[(PK_NB + i) * fs] += db * (sb[i] - r[i]) + nTb * T[i];
            pk[(PK_CB + i) * fs] += db * g.nb[i];
            gb.r[i] -= db * g.nb[i];
            gb.T[i] += nTb * g.nb[i];
        }
    }
}

// Reverse of the gap's end: final second-order move onto plane b, free ->
// bound on b, and the transport Jacobian (path correction, J_fb) built from
// the tangent columns.  g holds the landed state (before the final move); the
// adjoints of xp and F are read through xpb[6] and Fb (entry q of F at
// Fb[q * fs], read one column at a time; FbP is the pointer type, so the
// caller decides the memory it lives in).  Sets gb and the placement
// adjoints pb.
template <int FK, class FbP>
__device__ inline void end_reverse(const Field<double, FK>& fl, const double* sa, const double* sb,
                                   const GapRun<double, FK>& g, double t0, const double xpb[6], FbP Fb, int64_t fs,
                                   GapBar& gb, PlaceBar& pb) {
    const double lam = g.lam, lk = lam * kKappa;
    // landed state and the final move
    double rp[3], Tp[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        rp[i] = g.r0[i] + g.rl[i] + g.dr[i];
        Tp[i] = g.T0[i] + g.dT[i];
    }
    const double nb[3] = {sb[3 + 2], sb[3 + 5], sb[3 + 8]};
    const double u[3] = {sb[3 + 0], sb[3 + 3], sb[3 + 6]};
    const double v[3] = {sb[3 + 1], sb[3 + 4], sb[3 + 7]};
    const double nT0 = dot3(nb, Tp);
    const double dist0 = nb[0] * (sb[0] - rp[0]) + nb[1] * (sb[1] - rp[1]) + nb[2] * (sb[2] - rp[2]);
    const double rem = dist0 / nT0;
    double B0[3], TB0[3];
    fl.eval(rp, B0);
    cross(Tp, B0, TB0);
    double r[3], T[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        r[i] = rp[i] + rem * Tp[i] + 0.5 * rem * rem * lk * TB0[i];
        T[i] = Tp[i] + rem * lk * TB0[i];
    }
    const double t = t0 + g.dt + rem * g.gd;
    (void)t;
    // clear adjoints
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gb.r[i] = 0.0; gb.T[i] = 0.0;
        pb.cb[i] = 0.0; pb.ub[i] = 0.0; pb.vb[i] = 0.0; pb.nb[i] = 0.0;
        pb.ca[i] = 0.0; pb.ua[i] = 0.0; pb.va[i] = 0.0;
#pragma unroll
        for (int j = 0; j < 5; ++j) { gb.Mr[i][j] = 0.0; gb.MT[i][j] = 0.0; }
    }
    gb.t = xpb[5];
    gb.Mtl = 0.0;
    gb.lam = xpb[4];
    gb.gd = 0.0;
    gb.gpd = 0.0;
    // ---- free -> bound on surface b ----
    const double dd[3] = {r[0] - sb[0], r[1] - sb[1], r[2] - sb[2]};
    double rb[3], Tb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        pb.ub[i] += xpb[0] * dd[i];
        pb.vb[i] += xpb[1] * dd[i];
        rb[i] = xpb[0] * u[i] + xpb[1] * v[i];
        pb.cb[i] -= rb[i];
        Tb[i] = 0.0;
    }
    const double rho2 = T[0] * T[0] + T[1] * T[1];
    const double rho = sqrt(rho2);
    const double n2 = rho2 + T[2] * T[2];
    const double ip = 1.0 / rho2, ith = 1.0 / (rho * n2), in2 = 1.0 / n2;
    Tb[0] += xpb[2] * (-T[1] * ip) + xpb[3] * T[2] * T[0] * ith;
    Tb[1] += xpb[2] * (T[0] * ip) + xpb[3] * T[2] * T[1] * ith;
    Tb[2] += xpb[3] * (-rho * in2);
    // ---- F from the tangent columns ----
    double B[3], TxB[3];
    fl.eval(r, B);
    cross(T, B, TxB);
    const double nTd = dot3(nb, T);
    const double inT = 1.0 / nTd;
    double ipb = 0.0, ithb = 0.0, in2b = 0.0, rhob = 0.0, inTb = 0.0, lkb = 0.0;
    double TxBb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const bool fixed = j < TangentCols<FK>::J0;
        double mr[3], mt[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mr[i] = fixed ? sa[3 + 3 * i + j] : g.Mr[i][j];
            mt[i] = fixed ? 0.0 : g.MT[i][j];
        }
        const double q = dot3(nb, mr);
        const double sc = q * inT;
        double mrp[3], mtp[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mrp[i] = mr[i] - T[i] * sc;
            mtp[i] = mt[i] - lk * TxB[i] * sc;
        }
        const double F0b = Fb[(0 * 5 + j) * fs], F1b = Fb[(1 * 5 + j) * fs], F2b = Fb[(2 * 5 + j) * fs],
                     F3b = Fb[(3 * 5 + j) * fs], F4b = Fb[(4 * 5 + j) * fs];
        double mrpb[3], mtpb[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            pb.ub[i] += F0b * mrp[i];
            pb.vb[i] += F1b * mrp[i];
            mrpb[i] = F0b * u[i] + F1b * v[i];
        }
        // F2 = (T0 mt1 - T1 mt0) ip
        mtpb[0] = -F2b * T[1] * ip;
        mtpb[1] = F2b * T[0] * ip;
        mtpb[2] = 0.0;
        Tb[0] += F2b * mtp[1] * ip;
        Tb[1] -= F2b * mtp[0] * ip;
        ipb += F2b * (T[0] * mtp[1] - T[1] * mtp[0]);
        // F3 = T2 (T0 mt0 + T1 mt1) ith - rho mt2 in2
        const double w3 = T[0] * mtp[0] + T[1] * mtp[1];
        mtpb[0] += F3b * T[2] * T[0] * ith;
        mtpb[1] += F3b * T[2] * T[1] * ith;
        mtpb[2] += -F3b * rho * in2;
        Tb[2] += F3b * w3 * ith;
        Tb[0] += F3b * T[2] * mtp[0] * ith;
        Tb[1] += F3b * T[2] * mtp[1] * ith;
        ithb += F3b * T[2] * w3;
        rhob += -F3b * mtp[2] * in2;
        in2b += -F3b * rho * mtp[2];
        // F4 = [j = 4] Mtl - gd sc
        double scb = -F4b * g.gd;
        gb.gd += -F4b * sc;
        if (j == 4) gb.Mtl += F4b;
        // mr' = mr - T sc; mt' = mt - lk TxB sc
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Tb[i] -= mrpb[i] * sc;
            TxBb[i] -= lk * sc * mtpb[i];
        }
        scb -= dot3(mrpb, T) + lk * dot3(mtpb, TxB);
        lkb -= dot3(mtpb, TxB) * sc;
        // sc = (n . mr) / (n . T)
        const double qb = scb * inT;
        inTb += scb * q;
        double mrb[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            pb.nb[i] += qb * mr[i];
            mrb[i] = mrpb[i] + qb * nb[i];
        }
        if (fixed) {
            // the loc0 / loc1 columns are (u_a, v_a) of surface a
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (j == 0) pb.ua[i] += mrb[i];
                else pb.va[i] += mrb[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                gb.Mr[i][j] += mrb[i];
                gb.MT[i][j] += mtpb[i];
            }
        }
    }
    // scalars built from T: ip = 1/rho^2, ith = 1/(rho n2), in2 = 1/n2, inT = 1/(n.T)
    rhob += ipb * (-2.0 / (rho2 * rho)) + ithb * (-1.0 / (rho2 * n2));
    double n2b = ithb * (-1.0 / (rho * n2 * n2)) + in2b * (-1.0 / (n2 * n2));
    const double nTb = inTb * (-1.0 / (nTd * nTd));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        pb.nb[i] += nTb * T[i];
        Tb[i] += nTb * nb[i] + 2.0 * n2b * T[i];
    }
    Tb[0] += rhob * T[0] / rho;
    Tb[1] += rhob * T[1] / rho;
    // TxB = T x B(r)
    {
        double Bb[3] = {0.0, 0.0, 0.0};
        cross_vjp(T, B, TxBb, Tb, Bb);
        double t1[3];
        gradT_apply(fl, r, Bb, t1);
#pragma unroll
        for (int i = 0; i < 3; ++i) rb[i] += t1[i];
    }
    // ---- final move: r = rp + rem Tp + rem^2/2 lk TB0, T = Tp + rem lk TB0, t += rem gd ----
    double remb = dot3(rb, Tp) + rem * lk * dot3(rb, TB0) + lk * dot3(Tb, TB0) + gb.t * g.gd;
    gb.gd += gb.t * rem;
    lkb += 0.5 * rem * rem * dot3(rb, TB0) + rem * dot3(Tb, TB0);
    double TB0b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        TB0b[i] = 0.5 * rem * rem * lk * rb[i] + rem * lk * Tb[i];
        gb.r[i] = rb[i];
        gb.T[i] = Tb[i] + rem * rb[i];
    }
    {
        double B0b[3] = {0.0, 0.0, 0.0};
        cross_vjp(Tp, B0, TB0b, gb.T, B0b);
        double t1[3];
        gradT_apply(fl, rp, B0b, t1);
#pragma unroll
        for (int i = 0; i < 3; ++i) gb.r[i] += t1[i];
    }
    // rem = n.(c_b - rp) / (n.Tp)
    {
        const double distb = remb / nT0, nT0b = -remb * rem / nT0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            pb.nb[i] += distb * (sb[i] - rp[i]) + nT0b * Tp[i];
            pb.cb[i] += distb * nb[i];
            gb.r[i] -= distb * nb[i];
            gb.T[i] += nT0b * nb[i];
        }
    }
    gb.lam += lkb * kKappa;
}

// Reverse of the gap's start: bound -> free on surface a and the initial
// tangent columns; adds to xb[0..4] and the surface-a adjoints.
template <int FK>
__device__ inline void start_reverse(const Cfg& cfg, const double* sa, const double x[6], const GapRun<double, FK>& g,
                                     const GapBar& gb, PlaceBar& pb, double xb[6]) {
    double sp, cp, st, ct;
    angle_sincos(x[2], &sp, &cp);
    angle_sincos(x[3], &st, &ct);
    const double ua[3] = {sa[3 + 0], sa[3 + 3], sa[3 + 6]};
    const double va[3] = {sa[3 + 1], sa[3 + 4], sa[3 + 7]};
    // r0 = c_a + x0 u_a + x1 v_a
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        pb.ca[i] += gb.r[i];
        pb.ua[i] += x[0] * gb.r[i];
        pb.va[i] += x[1] * gb.r[i];
    }
    xb[0] += dot3(gb.r, ua);
    xb[1] += dot3(gb.r, va);
    if (TangentCols<FK>::J0 == 0) {
        // the propagated loc0 / loc1 columns start as u_a, v_a
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            pb.ua[i] += gb.Mr[i][0];
            pb.va[i] += gb.Mr[i][1];
        }
    }
    // T0 = (cp st, sp st, ct); MT col 2 = dT0/dphi, col 3 = dT0/dtheta
    const double dTdp[3] = {-sp * st, cp * st, 0.0};
    const double dTdt[3] = {cp * ct, sp * ct, -st};
    const double d2pp[3] = {-cp * st, -sp * st, 0.0};
    const double d2pt[3] = {-sp * ct, cp * ct, 0.0};
    const double d2tt[3] = {-cp * st, -sp * st, -ct};
    double MT2b[3], MT3b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) { MT2b[i] = gb.MT[i][2]; MT3b[i] = gb.MT[i][3]; }
    xb[2] += dot3(gb.T, dTdp) + dot3(MT2b, d2pp) + dot3(MT3b, d2pt);
    xb[3] += dot3(gb.T, dTdt) + dot3(MT2b, d2pt) + dot3(MT3b, d2tt);
    // gd = sqrt(1 + m^2 lam^2)/c, gpd = m^2 lam / (c^2 gd)
    const double m2 = cfg.mass * cfg.mass;
    double lamb = gb.lam + gb.gd * g.gpd;
    lamb += gb.gpd * (m2 / (kC * kC * g.gd)) * (1.0 - g.lam * g.gpd / g.gd);
    xb[4] += lamb;
    xb[5] += gb.t;
}

// The gap's start state x, entry i at xs[i * fs], read afresh at each use (a
// volatile read, which the compiler may neither merge nor hoist), so that the
// six values are not held in registers through the reverse of the steps.
template <class MP>
__device__ inline void reload_x(MP xs, int64_t fs, double x[6]) {
    using E = typename std::remove_pointer<MP>::type;
#pragma unroll
    for (int i = 0; i < 6; ++i) x[i] = *(volatile E*)(xs + i * fs);
}

// Reverse of one gap: xb += dL/dx, sab/sbb (13 each: c, R row-major; x/X0
// unused) += dL/d(surface placement), for the start state x (memory: entry i
// at xs[i * fs], as Fb), the adjoints xpb of the predicted
// state and Fb of the stored transport Jacobian (entry q at Fb[q * fs]; FbP
// as in end_reverse, writable: once read, its first PK_N slots hold the
// placement adjoints, so the caller's Fb is overwritten).  P: the forward
// pass's stepping precision, which the replay uses.  Returns false if the
// replay did not reproduce a successful gap.
template <class P, int FK, class FbP>
__device__ inline bool gap_reverse(const FieldDef& fd, const Cfg& cfg_in, const double* sa, const double* sb,
                                   FbP xs, const double xpb[6], FbP Fb, int64_t fs, double xb[6],
                                   double sab[13], double sbb[13]) {
    // a private copy: the replay loops read these settings from registers
    // instead of reloading them through the reference after every store
    const Cfg cfg = cfg_in;
    Field<double, FK> fl;
    fl.init(fd);
    Field<P, FK> flp;
    flp.init(fd);
    GapRun<P, FK> g;
    GapRun<double, FK> gw;
    Stages<P, FK> S;
    P k[4][3], h;
    bool capped;
    {
        double x[6];
        reload_x(xs, fs, x);
        gap_start<P, FK>(cfg, sa, sb, x, g);
    }
    if (gap_run<P, FK>(flp, cfg, 1 << 30, g, h, capped, S, k) != 0) return false;
    const int n_acc = g.accepted;
    GapBar gb;
    {
        PlaceBar pe;
        double x[6];
        reload_x(xs, fs, x);
        end_reverse<FK>(fl, sa, sb, widen<FK>(g, gw), x[5], xpb, Fb, fs, gb, pe);
        park_store(Fb, fs, pe);     // F's adjoint has been read: its slots take the placement adjoints
    }
    for (int s = n_acc - 1; s >= 0; --s) {
        {
            double x[6];
            reload_x(xs, fs, x);
            gap_start<P, FK>(cfg, sa, sb, x, g);
        }
        if (gap_run<P, FK>(flp, cfg, s, g, h, capped, S, k) != 1) return false;
        double kd[4][3];
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int i = 0; i < 3; ++i) kd[st][i] = double(k[st][i]);
        step_reverse<FK>(fl, sb, widen<FK>(g, gw), double(h), capped, kd, gb, Fb, fs);
    }
    PlaceBar pb;
    park_load(Fb, fs, pb);
    double x[6];
    reload_x(xs, fs, x);
    gap_start<P, FK>(cfg, sa, sb, x, g);
    start_reverse<FK>(cfg, sa, x, widen<FK>(g, gw), gb, pb, xb);
    // surface placement adjoints in the 13-value layout: c, then R row-major
    // (columns u, v, n)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        sab[i] += pb.ca[i];
        sab[3 + 3 * i + 0] += pb.ua[i];
        sab[3 + 3 * i + 1] += pb.va[i];
        sbb[i] += pb.cb[i];
        sbb[3 + 3 * i + 0] += pb.ub[i];
        sbb[3 + 3 * i + 1] += pb.vb[i];
        sbb[3 + 3 * i + 2] += pb.nb[i];
    }
    // the initial distance d0 = n_b.(c_b - r0) enters only through the
    // capped steps and the final move, whose reverses above use the current
    // position directly
    return true;
}

// Alignment gradient (dx, dy, dz, alpha, beta, gamma) about a surface's
// current placement from the adjoints of its 13 values: translations are the
// centre's adjoint; a rotation about local axis a moves column j of R by
// R (e_a x e_j).
__device__ inline void placement_to_alignment(const double* s, const double sbar[13], double g[6]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = sbar[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // e_a x e_j
            const double c0 = (a == 1 && j == 2) ? 1.0 : ((a == 2 && j == 1) ? -1.0 : 0.0);
            const double c1 = (a == 2 && j == 0) ? 1.0 : ((a == 0 && j == 2) ? -1.0 : 0.0);
            const double c2 = (a == 0 && j == 1) ? 1.0 : ((a == 1 && j == 0) ? -1.0 : 0.0);
#pragma unroll
            for (int i = 0; i < 3; ++i)
                acc += sbar[3 + 3 * i + j] * (s[3 + 3 * i + 0] * c0 + s[3 + 3 * i + 1] * c1 + s[3 + 3 * i + 2] * c2);
        }
        g[3 + a] = acc;
    }
}

}  // namespace kfm
