// kf_device.hpp -- device-side arithmetic of the batched Kalman-filter track fit.
//
// One lane fits one track.  Every small matrix lives in registers: loops over
// matrix indices have compile-time bounds and are fully unrolled, so the
// structural zeros and ones of the Jacobians fold away and nothing is indexed
// dynamically (which would push arrays to scratch memory).
//
// Paper: Sect. 2 (Kalman step, gain-matrix update, RTS smoother with stored
// Jacobians, chi2 from residuals, the six bound parameters), Sect. 4.1
// (adaptive Runge-Kutta-Nystrom transport with transport Jacobian and
// local<->global Jacobians; 8-component global representation), Sect. 4.2.4
// (the smoother's inverse in FP64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kfm {

constexpr double kC = 299.792458;         // speed of light, mm/ns
constexpr double kKappa = 0.299792458e-3; // curvature per (q/p) per tesla, 1/mm per (GeV^-1 T)
constexpr double kPi = 3.141592653589793238462643383279502884;

enum : int { ST_OK = 0, ST_NO_INTERSECT = 1, ST_STEP_CAP = 2, ST_NOT_SPD = 3, ST_BAD_INPUT = 4, ST_TOO_FEW = 5 };
enum : int { FIELD_UNIFORM = 0, FIELD_SOLENOID = 1, FIELD_MAP = 2 };

// packed index of symmetric 6x6 element (i, j): upper triangle, row-major
__host__ __device__ constexpr int sy(int i, int j) {
    return i <= j ? (i * (11 - i)) / 2 + j : (j * (11 - j)) / 2 + i;
}
// stored rows of the bound transport Jacobian F: rows l0, l1, phi, theta, t
// (the q/p row is e4 and the t column is e5, both implied); 5 x 5 = 25 entries
__host__ __device__ constexpr int frow(int i) { return i < 4 ? i : 4; }

// surface table entry in LDS: c[3], R[9] (row-major, columns u v n), x/X0,
// type (0 plane, 1 disc; the kernels built for cylinders and lines also hold
// 3 for a line and minus the radius for a cylinder there)
constexpr int SURF_STRIDE = 14;
__device__ inline bool is_disc(const double* __restrict__ s) { return s[13] == 1.0; }

struct FieldDef {
    int kind;
    double b0[3];
    double a;
    // FIELD_MAP: grid points mo + (i, j, k) / mih, mn per axis, values [k][j][i][3]
    const double* map;
    double mo[3];
    double mih[3];    // 1 / spacing
    int mn[3];
};

struct Cfg {
    int ms;
    double mass;
    double tol;
    double land_tol;
    int max_steps;
};

template <class P> __device__ inline P pabs(P x) { return x < P(0) ? -x : x; }

// Phase boundary for the instruction scheduler: nothing is moved across it.
// The fit is a chain of register-heavy phases (propagation, covariance
// transport, gain solve, update, smoother); letting the scheduler interleave
// neighbouring phases for ILP would add their live sets together.
__device__ inline void phase_boundary() { __builtin_amdgcn_sched_barrier(0); }

// Device-memory pointers in the global address space.  Kernel arguments and
// pointers passed through structs are generic (flat) to the compiler; a flat
// access also counts against the LDS/scalar wait counter, so every LDS wait
// behind it would wait for the memory access as well.  Casting to address
// space 1 makes the compiler emit global_load / global_store.
template <class T>
__device__ inline __attribute__((address_space(1))) T* gbl(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// sin and cos of an angle of the track model.  The library routine carries a
// large-argument reduction (Payne-Hanek) whose registers make the compiler
// spill in the hot loops although it never runs for these angles.  Here:
// k = nearest integer to x / (pi/2); r = x - k pi/2 with pi/2 split into three
// doubles (A + B + C, each the rounded remainder of the previous) and fused
// multiply-adds, so every product k A, k B, k C enters exactly and r carries
// an absolute error of ~2e-16 up to |x| ~ 2^50 (beyond that only the
// reduction's accuracy degrades; inf and NaN give NaN); then the Taylor series
// of sin and cos on |r| <= pi/4, cut after the r^17 and r^18 terms (remainder
// below 1e-19), and the quadrant k mod 4.
__device__ inline void angle_sincos(double x, double* s, double* c) {
    constexpr double TWO_OVER_PI = 0x1.45f306dc9c883p-1;
    constexpr double PIO2_A = 0x1.921fb54442d18p+0, PIO2_B = 0x1.1a62633145c07p-54,
                     PIO2_C = -0x1.f1976b7ed8fbcp-110;
    const double k = rint(x * TWO_OVER_PI);
    double r = fma(-k, PIO2_A, x);
    r = fma(-k, PIO2_B, r);
    r = fma(-k, PIO2_C, r);
    const double z = r * r;
    // sin r = r (1 - z/3! + z^2/5! - ... + z^8/17!)
    double ps = 1.0 / 355687428096000.0;
    ps = fma(ps, z, -1.0 / 1307674368000.0);
    ps = fma(ps, z, 1.0 / 6227020800.0);
    ps = fma(ps, z, -1.0 / 39916800.0);
    ps = fma(ps, z, 1.0 / 362880.0);
    ps = fma(ps, z, -1.0 / 5040.0);
    ps = fma(ps, z, 1.0 / 120.0);
    ps = fma(ps, z, -1.0 / 6.0);
    const double sr = fma(r * z, ps, r);
    // cos r = 1 - z/2! + z^2/4! - ... - z^9/18!
    double pc = -1.0 / 6402373705728000.0;
    pc = fma(pc, z, 1.0 / 20922789888000.0);
    pc = fma(pc, z, -1.0 / 87178291200.0);
    pc = fma(pc, z, 1.0 / 479001600.0);
    pc = fma(pc, z, -1.0 / 3628800.0);
    pc = fma(pc, z, 1.0 / 40320.0);
    pc = fma(pc, z, -1.0 / 720.0);
    pc = fma(pc, z, 1.0 / 24.0);
    pc = fma(pc, z, -0.5);
    const double cr = fma(pc, z, 1.0);
    const int n = (int)(k - 4.0 * floor(k * 0.25));      // k mod 4, exact for |k| < 2^53
    const double sa = (n & 1) ? cr : sr;
    const double ca = (n & 1) ? sr : cr;
    *s = (n & 2) ? -sa : sa;
    *c = ((n + 1) & 2) ? -ca : ca;
}

template <class P>
__device__ inline void cross(const P a[3], const P b[3], P o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Angle into (-pi, pi].  Every angle a fit of inputs at the detector's scale
// produces lies within a few turns; one of 64 rad or more (ten turns; only
// absurd hit or seed values lead there) becomes NaN, which ends both loops at
// once, so no input can keep a lane looping (the track then fails).
__device__ inline double wrap_phi(double p) {
    p = ::fabs(p) < 64.0 ? p : __longlong_as_double(0x7ff8000000000000LL);
    while (p > kPi) p -= 2.0 * kPi;
    while (p <= -kPi) p += 2.0 * kPi;
    return p;
}

// ---------------------------------------------------------------------------
// magnetic field in the propagation precision
// ---------------------------------------------------------------------------
template <class P, int FK>
struct Field {
    P b[3];   // uniform value, or (0, 0, b0z) for the solenoid
    P g;      // a * b0z
    P a;
    __device__ void init(const FieldDef& f) {
        for (int i = 0; i < 3; ++i) b[i] = P(f.b0[i]);
        a = P(f.a);
        g = P(f.a * f.b0[2]);
    }
    __device__ inline void eval(const P r[3], P B[3]) const {
        if (FK == FIELD_UNIFORM) {
            B[0] = b[0]; B[1] = b[1]; B[2] = b[2];
        } else {
            B[0] = g * r[0] * r[2];
            B[1] = g * r[1] * r[2];
            B[2] = b[2] - g * r[2] * r[2];
        }
    }
    // dB_a/dr_b applied to v: (grad B) v
    __device__ inline void grad_apply(const P r[3], const P v[3], P o[3]) const {
        o[0] = g * (r[2] * v[0] + r[0] * v[2]);
        o[1] = g * (r[2] * v[1] + r[1] * v[2]);
        o[2] = P(-2) * g * r[2] * v[2];
    }
};

// Tabulated field: trilinear interpolation in the grid cell holding r; a
// coordinate outside the grid is clamped to the boundary (no gradient along
// that axis).  The cell index and weights are formed in FP64 from the
// position, the corner values are read from global memory (the map is shared
// by every lane and stays in the caches).
template <class P>
struct Field<P, FIELD_MAP> {
    const double* m;
    double mo[3], mih[3];
    int mn[3];
    __device__ void init(const FieldDef& f) {
        m = f.map;
        for (int i = 0; i < 3; ++i) { mo[i] = f.mo[i]; mih[i] = f.mih[i]; mn[i] = f.mn[i]; }
    }
    // the cell (base index of its low corner) and the weights w1 (fraction
    // across the cell) and dw (d w1 / dr, zero where clamped) along each axis
    __device__ inline int64_t cell(const P r[3], P w1[3], P dw[3]) const {
        int idx[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double u = (double(r[a]) - mo[a]) * mih[a];
            double du = mih[a];
            const double top = double(mn[a] - 1);
            if (u <= 0.0) { u = 0.0; du = 0.0; }
            if (u >= top) { u = top; du = 0.0; }
            int i = u >= 0.0 ? (int)floor(u) : 0;     // a NaN position reads cell 0 (in bounds)
            i = i > mn[a] - 2 ? mn[a] - 2 : i;
            idx[a] = i;
            w1[a] = P(u - double(i));
            dw[a] = P(du);
        }
        return 3 * (((int64_t)idx[2] * mn[1] + idx[1]) * mn[0] + idx[0]);
    }
    __device__ inline void eval(const P r[3], P B[3]) const {
        P w1[3], dw[3];
        const auto c = gbl(m) + cell(r, w1, dw);
        const int64_t sy = 3 * (int64_t)mn[0], sz = sy * mn[1];
        B[0] = B[1] = B[2] = P(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int di = k & 1, dj = (k >> 1) & 1, dk = k >> 2;
            const P w = (di ? w1[0] : P(1) - w1[0]) * (dj ? w1[1] : P(1) - w1[1]) * (dk ? w1[2] : P(1) - w1[2]);
            const auto v = c + dk * sz + dj * sy + 3 * di;
#pragma unroll
            for (int q = 0; q < 3; ++q) B[q] += w * P(v[q]);
        }
    }
    // the field and its gradient G[3 q + a] = dB_q/dr_a in one pass over the corners
    __device__ inline void eval_grad(const P r[3], P B[3], P G[9]) const {
        P w1[3], dw[3];
        const auto c = gbl(m) + cell(r, w1, dw);
        const int64_t sy = 3 * (int64_t)mn[0], sz = sy * mn[1];
#pragma unroll
        for (int q = 0; q < 3; ++q) B[q] = P(0);
#pragma unroll
        for (int q = 0; q < 9; ++q) G[q] = P(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int di = k & 1, dj = (k >> 1) & 1, dk = k >> 2;
            const P wx = di ? w1[0] : P(1) - w1[0], wy = dj ? w1[1] : P(1) - w1[1], wz = dk ? w1[2] : P(1) - w1[2];
            const P sx = di ? dw[0] : -dw[0], sy_ = dj ? dw[1] : -dw[1], sz_ = dk ? dw[2] : -dw[2];
            const auto v = c + dk * sz + dj * sy + 3 * di;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const P vq = P(v[q]);
                B[q] += wx * wy * wz * vq;
                G[3 * q + 0] += sx * wy * wz * vq;
                G[3 * q + 1] += wx * sy_ * wz * vq;
                G[3 * q + 2] += wx * wy * sz_ * vq;
            }
        }
    }
    __device__ inline void grad_apply(const P r[3], const P v3[3], P o[3]) const {
        P w1[3], dw[3];
        const auto c = gbl(m) + cell(r, w1, dw);
        const int64_t sy = 3 * (int64_t)mn[0], sz = sy * mn[1];
        o[0] = o[1] = o[2] = P(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int di = k & 1, dj = (k >> 1) & 1, dk = k >> 2;
            const P wx = di ? w1[0] : P(1) - w1[0], wy = dj ? w1[1] : P(1) - w1[1], wz = dk ? w1[2] : P(1) - w1[2];
            const P sx = di ? dw[0] : -dw[0], sy_ = dj ? dw[1] : -dw[1], sz_ = dk ? dw[2] : -dw[2];
            // d(weight)/dr . v
            const P dwv = sx * wy * wz * v3[0] + wx * sy_ * wz * v3[1] + wx * wy * sz_ * v3[2];
            const auto v = c + dk * sz + dj * sy + 3 * di;
#pragma unroll
            for (int q = 0; q < 3; ++q) o[q] += dwv * P(v[q]);
        }
    }
};

// ---------------------------------------------------------------------------
// one Runge-Kutta-Nystrom trial step (Sect. 4.1), state on an FP64 anchor:
//   position r = r0 + dr, direction T = T0 + dT, time t = t0 + dt
//   r' = T, T' = (q/p) kappa T x B(r), t' = sqrt(1 + m^2 (q/p)^2)/c
// ---------------------------------------------------------------------------
template <class P, int FK>
struct Stages {
    P T[4][3];    // solenoid: stage directions
    P B[4][3];    // solenoid: field at the stage points
    P r[4][3];    // solenoid: absolute stage positions
    P r2[3];      // uniform: midpoint position (unused by the field)
};

// Map: the field gradient is kept per stage point instead of the position
// (stages 2 and 3 share the midpoint, so three gradients), so the tangent
// update does not read the map again.
template <class P>
struct Stages<P, FIELD_MAP> {
    P T[4][3];
    P B[4][3];
    P G[3][9];    // dB_q/dr_a at the start, the midpoint and the end point
    P r2[3];      // midpoint position
};
__host__ __device__ constexpr int stage_point(int st) { return st == 0 ? 0 : (st == 3 ? 2 : 1); }

// Returns the error estimate h^2 |k1 - k2 - k3 + k4|_1; k receives the stage
// accelerations k_i = (q/p) kappa T_i x B(r_i).
template <class P, int FK>
__device__ inline P rkn_trial(const Field<P, FK>& fl, const P rabs[3], const P T[3], P lam, P h,
                              Stages<P, FK>& S, P k[4][3]) {
    const P h2 = h * P(0.5), hh = h * h, lk = lam * P(kKappa);
    P B[3];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        P rs[3], Ts[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (st == 0) { rs[i] = rabs[i]; Ts[i] = T[i]; }
            else if (st == 1) { rs[i] = rabs[i] + h2 * T[i] + hh * P(0.125) * k[0][i]; Ts[i] = T[i] + h2 * k[0][i]; }
            else if (st == 2) {
                if constexpr (FK == FIELD_SOLENOID) rs[i] = S.r[1][i]; else rs[i] = S.r2[i];
                Ts[i] = T[i] + h2 * k[1][i];
            }
            else { rs[i] = rabs[i] + h * T[i] + hh * P(0.5) * k[2][i]; Ts[i] = T[i] + h * k[2][i]; }
        }
        if constexpr (FK == FIELD_UNIFORM) {
            if (st == 0) fl.eval(rs, B);
        } else if constexpr (FK == FIELD_MAP) {
            // the third stage sits at the second one's point: same field and gradient
            if (st != 2) fl.eval_grad(rs, B, S.G[stage_point(st)]);
        } else {
            fl.eval(rs, B);
        }
        P c[3];
        cross(Ts, B, c);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            k[st][i] = lk * c[i];
            if constexpr (FK == FIELD_SOLENOID) { S.T[st][i] = Ts[i]; S.B[st][i] = B[i]; S.r[st][i] = rs[i]; }
            else if constexpr (FK == FIELD_MAP) { S.T[st][i] = Ts[i]; S.B[st][i] = B[i]; if (st == 1) S.r2[i] = rs[i]; }
            else if (st == 1) S.r2[i] = rs[i];
        }
    }
    P e = P(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) e += pabs(k[0][i] - k[1][i] - k[2][i] + k[3][i]);
    return hh * e;
}

// Transport-Jacobian update for an accepted step: the columns (l0, l1, phi,
// theta, q/p) of d(free state)/d(bound start) are pushed through the stage
// equations at fixed h (forward tangents).  The explicit q/p dependence of a
// stage is d k_i/d(q/p) = kappa T_i x B_i, formed as k_i / (q/p); for q/p = 0
// exactly (no curvature: every stage direction is the step's start direction
// T0) it is kappa T0 x B_i itself.
// In a uniform field dk/dr = 0, so the l0 and l1 columns stay (u, v; 0, 0)
// exactly and are neither stored nor propagated: columns start at JT0.
template <int FK> struct TangentCols { static constexpr int J0 = (FK == FIELD_UNIFORM) ? 2 : 0; };
template <class P, int FK>
__device__ inline void rkn_tangent(const Field<P, FK>& fl, const Stages<P, FK>& S, const P k[4][3], P lam, P h,
                                   const P T0[3], P Mr[3][5], P MT[3][5]) {
    const bool straight = lam == P(0);
    const P h2 = h * P(0.5), hh = h * h, lk = lam * P(kKappa), ilam = straight ? P(0) : P(1) / lam;
    P LB[3], kq0[3];
    if constexpr (FK == FIELD_UNIFORM) {
#pragma unroll
        for (int i = 0; i < 3; ++i) LB[i] = lk * fl.b[i];
        cross(T0, fl.b, kq0);
#pragma unroll
        for (int i = 0; i < 3; ++i) kq0[i] *= P(kKappa);
    }
#pragma unroll
    for (int j = TangentCols<FK>::J0; j < 5; ++j) {
        P dk[3], sR[3], sT[3], dr2[3];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            P dT[3], dr[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (st == 0) { dT[i] = MT[i][j]; dr[i] = Mr[i][j]; }
                else if (st == 1) { dT[i] = MT[i][j] + h2 * dk[i]; dr2[i] = Mr[i][j] + h2 * MT[i][j] + hh * P(0.125) * dk[i]; dr[i] = dr2[i]; }
                else if (st == 2) { dT[i] = MT[i][j] + h2 * dk[i]; dr[i] = dr2[i]; }
                else { dT[i] = MT[i][j] + h * dk[i]; dr[i] = Mr[i][j] + h * MT[i][j] + hh * P(0.5) * dk[i]; }
            }
            P c[3];
            if (FK == FIELD_UNIFORM) {
                cross(dT, LB, c);
            } else {
                P g[3], c2[3];
                cross(dT, S.B[st], c);
                if constexpr (FK == FIELD_MAP) {
                    const P* G = S.G[stage_point(st)];
#pragma unroll
                    for (int q = 0; q < 3; ++q) g[q] = G[3 * q] * dr[0] + G[3 * q + 1] * dr[1] + G[3 * q + 2] * dr[2];
                } else {
                    fl.grad_apply(S.r[st], dr, g);
                }
                cross(S.T[st], g, c2);
#pragma unroll
                for (int i = 0; i < 3; ++i) c[i] = lk * (c[i] + c2[i]);
            }
            P kq[3] = {P(0), P(0), P(0)};
            if (j == 4) {
                if constexpr (FK == FIELD_UNIFORM) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) kq[i] = straight ? kq0[i] : k[st][i] * ilam;
                } else {
#pragma unroll
                    for (int i = 0; i < 3; ++i) kq[i] = k[st][i] * ilam;
                    if (straight) {
                        cross(T0, S.B[st], kq);
#pragma unroll
                        for (int i = 0; i < 3; ++i) kq[i] *= P(kKappa);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                dk[i] = (j == 4) ? c[i] + kq[i] : c[i];
                if (st == 0) { sR[i] = dk[i]; sT[i] = dk[i]; }
                else if (st < 3) { sR[i] += dk[i]; sT[i] += P(2) * dk[i]; }
                else sT[i] += dk[i];
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const P dT1 = MT[i][j];
            Mr[i][j] = Mr[i][j] + h * dT1 + hh * (P(1) / P(6)) * sR[i];
            MT[i][j] = dT1 + h * (P(1) / P(6)) * sT[i];
        }
        phase_boundary();   // one column's temporaries at a time
    }
}

// ---------------------------------------------------------------------------
// bound -> free at surface a, adaptive propagation to plane b, path
// correction, free -> bound.  Outputs the predicted bound state and the
// 6x6 transport Jacobian F (25 stored entries).  Returns a status.
// Step control (same decisions as the FP64 reference fit):
//   first trial = signed straight-line distance d = n.(c - r)/(n.T);
//   every trial is capped by |d| (then h = d);
//   accept if err <= tol; next trial |h| * clamp(0.9 (tol/err)^(1/4), 1/4, 4);
//   land when |n.(c - r)| < land_tol, then move the remaining distance onto
//   the plane in FP64, to second order in that distance.
// MIXED (P = float): stepping and tangents in FP32 on increments from the
// FP64 anchor; the landing loop stops at an FP32-resolvable distance and the
// same FP64 second-order move finishes it.
// ---------------------------------------------------------------------------
// P is the stepping type (double, or float for MIXED); everything else is
// FP64.  Surfaces a and b are 14 values each (c, R, x/X0, type).
// Local -> global on a surface: position r = c + offset(loc), and the
// columns e0 = dr/dloc0, e1 = dr/dloc1.  Plane: offset l0 u + l1 v; disc:
// l0 (cos l1 u + sin l1 v).
__device__ inline void loc_frame(const double* __restrict__ s, const double x[6], double e0[3], double e1[3]) {
    if (is_disc(s)) {
        double sl, cl;
        angle_sincos(x[1], &sl, &cl);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            e0[i] = cl * s[3 + 3 * i + 0] + sl * s[3 + 3 * i + 1];
            e1[i] = x[0] * (cl * s[3 + 3 * i + 1] - sl * s[3 + 3 * i + 0]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) { e0[i] = s[3 + 3 * i + 0]; e1[i] = s[3 + 3 * i + 1]; }
    }
}
__device__ inline double loc_offset(const double* __restrict__ s, const double x[6], int i) {
    if (is_disc(s)) {
        double sl, cl;
        angle_sincos(x[1], &sl, &cl);
        return x[0] * (cl * s[3 + 3 * i + 0] + sl * s[3 + 3 * i + 1]);
    }
    return x[0] * s[3 + 3 * i + 0] + x[1] * s[3 + 3 * i + 1];
}

template <class P, int FK>
__device__ inline int transport(const Field<P, FK>& fl, const FieldDef& fd, const Cfg& cfg,
                                const double* __restrict__ sa, const double* __restrict__ sb,
                                const double x[6], double xp[6], double F[25], int* trials_out) {
    using R = double;
    using V = P;    // step-control bookkeeping
    // bound -> free on surface a
    R sp, cp, st, ct;
    angle_sincos(x[2], &sp, &cp);
    angle_sincos(x[3], &st, &ct);
    R r0[3], T0[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) r0[i] = sa[i] + loc_offset(sa, x, i);
    T0[0] = cp * st; T0[1] = sp * st; T0[2] = ct;
    const R lam_d = x[4];
    const P lam = P(lam_d);
    const R gd = sqrt(1.0 + cfg.mass * cfg.mass * lam_d * lam_d) / kC;     // dt/ds
    const R gpd = cfg.mass * cfg.mass * lam_d / (kC * kC * gd);            // d(dt/ds)/d(q/p)
    P Mr[3][5], MT[3][5];
    {
        R e0[3], e1[3];
        if (TangentCols<FK>::J0 == 0) loc_frame(sa, x, e0, e1);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int j = 0; j < 5; ++j) { Mr[i][j] = P(0); MT[i][j] = P(0); }
            if (TangentCols<FK>::J0 == 0) {
                Mr[i][0] = P(e0[i]);
                Mr[i][1] = P(e1[i]);
            }
        }
    }
    MT[0][2] = P(-(sp * st)); MT[1][2] = P(cp * st); MT[2][2] = P(0);
    MT[0][3] = P(cp * ct);    MT[1][3] = P(sp * ct); MT[2][3] = P(-st);
    R Mtl = 0.0;     // d t / d(q/p) accumulated over accepted steps

    const R nb[3] = {sb[3 + 2], sb[3 + 5], sb[3 + 8]};
    const R d0 = nb[0] * (sb[0] - r0[0]) + nb[1] * (sb[1] - r0[1]) + nb[2] * (sb[2] - r0[2]);
    const V tol = V(cfg.tol);
    const bool mixed = sizeof(V) < sizeof(double);
    // position = r0 + rl + dr: rl (FP64) collects the straight-line part h T of
    // every step, dr the curvature part h^2/6 (k1 + k2 + k3) in precision P;
    // direction = T0 + dT.  In FP32 the big h T term would cost ~1e-7 relative
    // over a long step, so only the small curvature increments are FP32.
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
        const R nTd = nb[0] * Td[0] + nb[1] * Td[1] + nb[2] * Td[2];
        const R distd = d0 - (nb[0] * rl[0] + nb[1] * rl[1] + nb[2] * rl[2])
                            - (nb[0] * R(dr[0]) + nb[1] * R(dr[1]) + nb[2] * R(dr[2]));
        if (::fabs(nTd) < 1e-6) { status = ST_NO_INTERSECT; break; }
        // FP32 curvature increments resolve ~1e-7 mm; the FP64 move below finishes the landing
        const double ltol = mixed ? 1e-5 : cfg.land_tol;
        if (::fabs(distd) < ltol) break;
        if (trials >= cfg.max_steps) { status = ST_STEP_CAP; break; }
        const P d = P(distd / nTd);
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

    // final free state in FP64, then the remaining distance d onto the plane,
    // second order in d: r += d T + d^2/2 T', T += d T', t += d dt/ds
    R r[3], T[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) { r[i] = r0[i] + rl[i] + R(dr[i]); T[i] = T0[i] + R(dT[i]); }
    R t = x[5] + dt;
    Field<R, FK> f64;
    f64.init(fd);
    {
        const R nT0 = nb[0] * T[0] + nb[1] * T[1] + nb[2] * T[2];
        const R rem = (nb[0] * (sb[0] - r[0]) + nb[1] * (sb[1] - r[1]) + nb[2] * (sb[2] - r[2])) / nT0;
        R B0[3], TB0[3];
        f64.eval(r, B0);
        cross(T, B0, TB0);
        const R lk = lam_d * kKappa;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            r[i] = r[i] + rem * T[i] + 0.5 * rem * rem * lk * TB0[i];
            T[i] = T[i] + rem * lk * TB0[i];
        }
        t = t + rem * gd;
    }
    const R nTd = nb[0] * T[0] + nb[1] * T[1] + nb[2] * T[2];
    // free -> bound on surface b: the local rows g0, g1 are d loc / d r
    const R u[3] = {sb[3 + 0], sb[3 + 3], sb[3 + 6]};
    const R v[3] = {sb[3 + 1], sb[3 + 4], sb[3 + 7]};
    const R dd[3] = {r[0] - sb[0], r[1] - sb[1], r[2] - sb[2]};
    R g0[3], g1[3];
    {
        const R ca = u[0] * dd[0] + u[1] * dd[1] + u[2] * dd[2];
        const R cb = v[0] * dd[0] + v[1] * dd[1] + v[2] * dd[2];
        if (is_disc(sb)) {
            const R rr = sqrt(ca * ca + cb * cb);
            xp[0] = rr;
            xp[1] = atan2(cb, ca);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                g0[i] = (ca * u[i] + cb * v[i]) / rr;
                g1[i] = (ca * v[i] - cb * u[i]) / (rr * rr);
            }
        } else {
            xp[0] = ca;
            xp[1] = cb;
#pragma unroll
            for (int i = 0; i < 3; ++i) { g0[i] = u[i]; g1[i] = v[i]; }
        }
    }
    const R rho2 = T[0] * T[0] + T[1] * T[1];
    const R rho = sqrt(rho2);
    const R n2 = rho2 + T[2] * T[2];
    xp[2] = atan2(T[1], T[0]);
    xp[3] = atan2(rho, T[2]);
    xp[4] = lam_d;
    xp[5] = t;
    // F = J_fb * P_corr * (D J_bf), one column at a time: the path correction
    // moves each variation back onto the plane along dF/ds, then J_fb maps it
    // to the bound parameters of surface b
    R B[3], TxB[3];
    f64.eval(r, B);
    cross(T, B, TxB);
    const R lk = lam_d * kKappa;
    const R inT = 1.0 / nTd, ip = 1.0 / rho2, ith = 1.0 / (rho * n2), in2 = 1.0 / n2;
    // the loc0/loc1 columns of a uniform field were never propagated: dr/dloc on surface a
    R e0[3], e1[3];
    if (TangentCols<FK>::J0 != 0) loc_frame(sa, x, e0, e1);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        // columns below J0 were never propagated: (u, v) of surface a, no direction part
        const bool fixed = j < TangentCols<FK>::J0;
        R mr[3], mt[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mr[i] = fixed ? (j == 0 ? e0[i] : e1[i]) : R(Mr[i][j]);
            mt[i] = fixed ? R(0.0) : R(MT[i][j]);
        }
        const R sc = (nb[0] * mr[0] + nb[1] * mr[1] + nb[2] * mr[2]) * inT;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mr[i] = mr[i] - T[i] * sc;
            mt[i] = mt[i] - lk * TxB[i] * sc;
        }
        F[0 * 5 + j] = g0[0] * mr[0] + g0[1] * mr[1] + g0[2] * mr[2];
        F[1 * 5 + j] = g1[0] * mr[0] + g1[1] * mr[1] + g1[2] * mr[2];
        F[2 * 5 + j] = (T[0] * mt[1] - T[1] * mt[0]) * ip;
        F[3 * 5 + j] = T[2] * (T[0] * mt[0] + T[1] * mt[1]) * ith - rho * mt[2] * in2;
        F[4 * 5 + j] = (j == 4 ? Mtl : R(0.0)) - gd * sc;
    }
    return ST_OK;
}

// ---------------------------------------------------------------------------
// bound state on plane a -> perigee of the line through c parallel to z
// (Sect. 2; Sect. 5.2 quotes the fitted parameters there), in FP64.  The
// distance to go is the Newton step d = -g/g' of the constraint
// g = (r - c)_perp . T_perp, g' = |T_perp|^2 + (r - c)_perp . T'_perp (a
// closest approach needs g' > 0), with the plane transport's step control;
// land when |d| < land_tol, then move d to second order.  Bound parameters
// (d0, z0, phi, theta, q/p, t): d0 = (r - c) . u, u = (-T_y, T_x, 0)/|T_perp|,
// z0 = r_z - c_z.  F (25 stored entries) carries the path correction that
// moves a variation back onto g = 0 along dF/ds.
// ---------------------------------------------------------------------------
template <int FK>
__device__ inline int transport_perigee(const FieldDef& fd, const Cfg& cfg, const double* __restrict__ sa,
                                        const double c[3], const double x[6], double xp[6], double F[25],
                                        int* trials_out) {
    using R = double;
    Field<R, FK> fl;
    fl.init(fd);
    R sp, cp, st, ct;
    angle_sincos(x[2], &sp, &cp);
    angle_sincos(x[3], &st, &ct);
    R r[3], T[3], e0[3], e1[3];
    loc_frame(sa, x, e0, e1);       // dr/dloc on surface a (also the fixed columns of a uniform field)
#pragma unroll
    for (int i = 0; i < 3; ++i) r[i] = sa[i] + loc_offset(sa, x, i);
    T[0] = cp * st; T[1] = sp * st; T[2] = ct;
    const R lam = x[4];
    const R lk = lam * kKappa;
    const R gd = sqrt(1.0 + cfg.mass * cfg.mass * lam * lam) / kC;
    const R gpd = cfg.mass * cfg.mass * lam / (kC * kC * gd);
    R Mr[3][5], MT[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 5; ++j) { Mr[i][j] = 0.0; MT[i][j] = 0.0; }
        if (TangentCols<FK>::J0 == 0) {
            Mr[i][0] = e0[i];
            Mr[i][1] = e1[i];
        }
    }
    MT[0][2] = -(sp * st); MT[1][2] = cp * st; MT[2][2] = 0.0;
    MT[0][3] = cp * ct;    MT[1][3] = sp * ct; MT[2][3] = -st;
    R Mtl = 0.0, t = x[5], hmag = -1.0;
    int trials = 0, status = ST_OK;
    Stages<R, FK> S;
    for (;;) {
        R B[3], TB[3];
        fl.eval(r, B);
        cross(T, B, TB);
        const R dx = r[0] - c[0], dy = r[1] - c[1];
        const R g = dx * T[0] + dy * T[1];
        const R gp = T[0] * T[0] + T[1] * T[1] + lk * (dx * TB[0] + dy * TB[1]);
        if (!(gp > 1e-6)) { status = ST_NO_INTERSECT; break; }
        const R d = -g / gp;
        if (::fabs(d) < cfg.land_tol) break;
        if (trials >= cfg.max_steps) { status = ST_STEP_CAP; break; }
        if (hmag < 0.0) hmag = ::fabs(d);
        const R h = (::fabs(d) <= hmag) ? d : ::copysign(hmag, d);
        R k[4][3];
        const R err = rkn_trial<R, FK>(fl, r, T, lam, h, S, k);
        ++trials;
        phase_boundary();
        R fac = 0.9 * sqrt(sqrt(cfg.tol / (err > 1e-300 ? err : 1e-300)));
        fac = fac < 0.25 ? 0.25 : (fac > 4.0 ? 4.0 : fac);
        if (err <= cfg.tol) {
            rkn_tangent<R, FK>(fl, S, k, lam, h, T, Mr, MT);
            phase_boundary();
            Mtl = Mtl + h * gpd;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                r[i] = r[i] + h * T[i] + h * h * (1.0 / 6.0) * (k[0][i] + k[1][i] + k[2][i]);
                T[i] = T[i] + h * (1.0 / 6.0) * (k[0][i] + 2.0 * k[1][i] + 2.0 * k[2][i] + k[3][i]);
            }
            t = t + h * gd;
        }
        hmag = ::fabs(h) * fac;
    }
    *trials_out = trials;
    if (status != ST_OK) return status;
    {
        R B[3], TB[3];
        fl.eval(r, B);
        cross(T, B, TB);
        const R dx = r[0] - c[0], dy = r[1] - c[1];
        const R gp = T[0] * T[0] + T[1] * T[1] + lk * (dx * TB[0] + dy * TB[1]);
        const R d = -(dx * T[0] + dy * T[1]) / gp;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            r[i] = r[i] + d * T[i] + 0.5 * d * d * lk * TB[i];
            T[i] = T[i] + d * lk * TB[i];
        }
        t = t + d * gd;
    }
    R B[3], TB[3];
    fl.eval(r, B);
    cross(T, B, TB);
    const R Tp[3] = {lk * TB[0], lk * TB[1], lk * TB[2]};
    const R dx = r[0] - c[0], dy = r[1] - c[1];
    const R gp = T[0] * T[0] + T[1] * T[1] + dx * Tp[0] + dy * Tp[1];
    const R rho2 = T[0] * T[0] + T[1] * T[1];
    const R rho = sqrt(rho2);
    const R n2 = rho2 + T[2] * T[2];
    const R ux = -T[1] / rho, uy = T[0] / rho;
    const R gperp = dx * T[0] + dy * T[1];
    xp[0] = dx * ux + dy * uy;
    xp[1] = r[2] - c[2];
    xp[2] = atan2(T[1], T[0]);
    xp[3] = atan2(rho, T[2]);
    xp[4] = lam;
    xp[5] = t;
    const R igp = 1.0 / gp, ip = 1.0 / rho2, ith = 1.0 / (rho * n2), in2 = 1.0 / n2, ir3 = gperp / (rho2 * rho);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const bool fixed = j < TangentCols<FK>::J0;
        R mr[3], mt[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mr[i] = fixed ? (j == 0 ? e0[i] : e1[i]) : Mr[i][j];
            mt[i] = fixed ? R(0.0) : MT[i][j];
        }
        const R sc = (T[0] * mr[0] + T[1] * mr[1] + dx * mt[0] + dy * mt[1]) * igp;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mr[i] = mr[i] - T[i] * sc;
            mt[i] = mt[i] - Tp[i] * sc;
        }
        F[0 * 5 + j] = ux * mr[0] + uy * mr[1] + (T[1] * mt[0] - T[0] * mt[1]) * ir3;
        F[1 * 5 + j] = mr[2];
        F[2 * 5 + j] = (T[0] * mt[1] - T[1] * mt[0]) * ip;
        F[3 * 5 + j] = T[2] * (T[0] * mt[0] + T[1] * mt[1]) * ith - rho * mt[2] * in2;
        F[4 * 5 + j] = (j == 4 ? Mtl : R(0.0)) - gd * sc;
    }
    return ST_OK;
}

// ---------------------------------------------------------------------------
// thin-scatterer noise on surface s for the filtered state x (PDG Highland)
// Q = diag(0, 0, theta0^2 / sin^2(theta), theta0^2, 0, 0)
// ---------------------------------------------------------------------------
__device__ inline void highland(const double* __restrict__ s, const double x[6], double mass, double* q22, double* q33) {
    const double x0 = s[12];
    if (!(x0 > 0.0)) { *q22 = 0.0; *q33 = 0.0; return; }
    double sp, cp, st, ct;
    angle_sincos(x[2], &sp, &cp);
    angle_sincos(x[3], &st, &ct);
    const double nT = s[3 + 2] * cp * st + s[3 + 5] * sp * st + s[3 + 8] * ct;
    const double path = x0 / fabs(nT);
    const double p = 1.0 / fabs(x[4]);
    const double beta = p / sqrt(p * p + mass * mass);
    const double th0 = 0.0136 / (beta * p) * sqrt(path) * (1.0 + 0.038 * log(path / (beta * beta)));
    *q33 = th0 * th0;
    *q22 = th0 * th0 / (st * st);
}

// ---------------------------------------------------------------------------
// covariance transport Cp = F C F^T (C symmetric packed, F with implied
// q/p row e4 and t column e5)
// ---------------------------------------------------------------------------
__device__ inline double fget(const double F[25], int i, int j) {
    // valid for compile-time i, j after unrolling
    return (i == 4) ? (j == 4 ? 1.0 : 0.0) : (j == 5 ? (i == 5 ? 1.0 : 0.0) : F[frow(i) * 5 + j]);
}

__device__ inline void transport_cov(const double F[25], const double C[21], double Cp[21]) {
    // one row g = (F C)[i, :] at a time, then Cp[i][l] = g . F[l, :] for l >= i
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double g[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            if (i == 4) { g[m] = C[sy(4, m)]; continue; }
            double acc = (i == 5) ? C[sy(5, m)] : 0.0;
#pragma unroll
            for (int j = 0; j < 5; ++j) acc += F[frow(i) * 5 + j] * C[sy(j, m)];
            g[m] = acc;
        }
#pragma unroll
        for (int l = i; l < 6; ++l) {
            double acc;
            if (l == 4) acc = g[4];
            else {
                acc = (l == 5) ? g[5] : 0.0;
#pragma unroll
                for (int m = 0; m < 5; ++m) acc += g[m] * F[frow(l) * 5 + m];
            }
            Cp[sy(i, l)] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// gain-matrix update with H = [I2 0] (Sect. 2), Joseph covariance form:
//   Cf = (I - K H) Cp (I - K H)^T + K V K^T
//      = Cp - K P - P^T K^T + K S K^T,  P = H Cp, S = V + H Cp H^T
// ---------------------------------------------------------------------------
__device__ inline int kalman_update(const double xp[6], const double Cp[21], const double m[2],
                                    const double V[3], double xf[6], double Cf[21], double* chi2,
                                    bool ang1 = false) {
    // ang1: the second local coordinate is an azimuth (disc), residual and value in (-pi, pi]
    const double r0 = m[0] - xp[0], r1 = ang1 ? wrap_phi(m[1] - xp[1]) : m[1] - xp[1];
    const double S00 = V[0] + Cp[sy(0, 0)], S01 = V[1] + Cp[sy(0, 1)], S11 = V[2] + Cp[sy(1, 1)];
    const double det = S00 * S11 - S01 * S01;
    if (!(S00 > 0.0 && det > 0.0)) return ST_NOT_SPD;
    const double idet = 1.0 / det;
    const double I00 = S11 * idet, I01 = -S01 * idet, I11 = S00 * idet;
    double K[6][2];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const double p0 = Cp[sy(0, i)], p1 = Cp[sy(1, i)];
        K[i][0] = p0 * I00 + p1 * I01;
        K[i][1] = p0 * I01 + p1 * I11;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) xf[i] = xp[i] + K[i][0] * r0 + K[i][1] * r1;
    xf[2] = wrap_phi(xf[2]);
    if (ang1) xf[1] = wrap_phi(xf[1]);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        // (K S)_i
        const double ks0 = K[i][0] * S00 + K[i][1] * S01;
        const double ks1 = K[i][0] * S01 + K[i][1] * S11;
#pragma unroll
        for (int j = i; j < 6; ++j) {
            const double kp = K[i][0] * Cp[sy(0, j)] + K[i][1] * Cp[sy(1, j)];
            const double pk = Cp[sy(0, i)] * K[j][0] + Cp[sy(1, i)] * K[j][1];
            const double ksk = ks0 * K[j][0] + ks1 * K[j][1];
            Cf[sy(i, j)] = Cp[sy(i, j)] - kp - pk + ksk;
        }
    }
    *chi2 = r0 * (I00 * r0 + I01 * r1) + r1 * (I01 * r0 + I11 * r1);
    return ST_OK;
}

// ---------------------------------------------------------------------------
// FP64 Cholesky factor of an SPD 6x6 (Sect. 4.2.4: the smoother's inverse is
// done in FP64): L packed with sy(i, j), i >= j; id[j] = 1 / L[j][j].
// ---------------------------------------------------------------------------
__device__ inline bool chol6(const double A[21], double L[21], double id[6]) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double s = A[sy(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= L[sy(j, k)] * L[sy(j, k)];
        ok = ok && (s > 0.0);
        const double l = sqrt(s > 0.0 ? s : 1.0);
        L[sy(j, j)] = l;
        id[j] = 1.0 / l;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double t = A[sy(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= L[sy(i, k)] * L[sy(j, k)];
            L[sy(i, j)] = t * id[j];
        }
    }
    return ok;
}

// solve (L L^T) v = b in place
__device__ inline void chol_solve6(const double L[21], const double id[6], double v[6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = v[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[sy(i, k)] * v[k];
        v[i] = s * id[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = v[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[sy(k, i)] * v[k];
        v[i] = s * id[i];
    }
}

// Row c of the RTS smoother gain A = C F^T Cp^{-1} (Sect. 2): with
// Cp = L L^T, column c of A^T = Cp^{-1} (F C)[:, c].
__device__ inline void smoother_gain_row(const double F[25], const double C[21], const double L[21],
                                         const double id[6], int c, double g[6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        if (i == 4) { g[i] = C[sy(4, c)]; continue; }
        double acc = (i == 5) ? C[sy(5, c)] : 0.0;
#pragma unroll
        for (int j = 0; j < 5; ++j) acc += F[frow(i) * 5 + j] * C[sy(j, c)];
        g[i] = acc;
    }
    chol_solve6(L, id, g);
}

// ---------------------------------------------------------------------------
// RTS smoother step (Sect. 2) with the stored gain A of the step k -> k+1:
//   xs = xf + A (xs1 - xp1),  Cs = Cf + A (Cs1 - Cp1) A^T
// split in three phases so each loads only what it needs:
//   rts_diff: dx = xs1 - xp1 (phi wrapped), Cs1 -> D = Cs1 - Cp1 in place
//   rts_mean: xs = xf + A dx
//   rts_cov:  Cs = Cf + A D A^T  (R holds Cf on entry, the result on exit)
// ---------------------------------------------------------------------------
__device__ inline void rts_diff(const double xs1[6], double CsD[21], const double xp1[6], const double Cp1[21],
                                double dx[6], bool ang1 = false) {
#pragma unroll
    for (int i = 0; i < 6; ++i) dx[i] = xs1[i] - xp1[i];
    dx[2] = wrap_phi(dx[2]);
    if (ang1) dx[1] = wrap_phi(dx[1]);
#pragma unroll
    for (int q = 0; q < 21; ++q) CsD[q] -= Cp1[q];
}

__device__ inline void rts_mean(const double xf[6], const double A[36], const double dx[6], double xs[6],
                                bool ang1 = false) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double acc = xf[i];
#pragma unroll
        for (int k = 0; k < 6; ++k) acc += A[6 * i + k] * dx[k];
        xs[i] = acc;
    }
    xs[2] = wrap_phi(xs[2]);
    if (ang1) xs[1] = wrap_phi(xs[1]);
}

__device__ inline void rts_cov(const double A[36], const double D[21], double R[21]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double e[6];                                     // row i of A D
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) acc += A[6 * i + k] * D[sy(k, m)];
            e[m] = acc;
        }
#pragma unroll
        for (int j = i; j < 6; ++j) {
            double acc = R[sy(i, j)];
#pragma unroll
            for (int m = 0; m < 6; ++m) acc += e[m] * A[6 * j + m];
            R[sy(i, j)] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Two-filter smoother step (Sect. 2, Fig. 2): the forward estimate (xf, Cf)
// and the backward filter's prediction (xb, Cb) of the same state are
// independent; their combination with K = Cf (Cf + Cb)^{-1} is
//   xs = xf + K (xb - xf)                          (phi difference wrapped)
//   Cs = (I - K) Cf (I - K)^T + K Cb K^T           (covariance of that sum)
// Column c of K^T is (Cf + Cb)^{-1} Cf[:, c] (FP64 Cholesky).  Returns false
// if Cf + Cb is not positive definite.
// ---------------------------------------------------------------------------
__device__ inline bool two_filter_combine(const double xf[6], const double Cf[21], const double xb[6],
                                          const double Cb[21], double xs[6], double Cs[21], bool ang1 = false) {
    double L[21], id[6], S[21];
#pragma unroll
    for (int q = 0; q < 21; ++q) S[q] = Cf[q] + Cb[q];
    const bool ok = chol6(S, L, id);
    double K[36];                                    // K[6 * i + c]
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double g[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) g[i] = Cf[sy(i, c)];
        chol_solve6(L, id, g);                       // column c of K^T = row c of K
#pragma unroll
        for (int i = 0; i < 6; ++i) K[6 * c + i] = g[i];
    }
    double dx[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) dx[i] = xb[i] - xf[i];
    dx[2] = wrap_phi(dx[2]);
    if (ang1) dx[1] = wrap_phi(dx[1]);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double acc = xf[i];
#pragma unroll
        for (int k = 0; k < 6; ++k) acc += K[6 * i + k] * dx[k];
        xs[i] = acc;
    }
    xs[2] = wrap_phi(xs[2]);
    if (ang1) xs[1] = wrap_phi(xs[1]);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double e[6], f[6];                           // row i of (I - K) Cf and of K Cb
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            double a = Cf[sy(i, m)], b = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                a -= K[6 * i + k] * Cf[sy(k, m)];
                b += K[6 * i + k] * Cb[sy(k, m)];
            }
            e[m] = a;
            f[m] = b;
        }
#pragma unroll
        for (int j = i; j < 6; ++j) {
            double acc = e[j];
#pragma unroll
            for (int m = 0; m < 6; ++m) acc += f[m] * K[6 * j + m] - e[m] * K[6 * j + m];
            Cs[sy(i, j)] = acc;
        }
    }
    return ok;
}

}  // namespace kfm
