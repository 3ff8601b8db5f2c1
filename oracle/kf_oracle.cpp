// kf_oracle.cpp -- plain FP64 CPU oracle for batched Kalman-filter track fitting.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may load or call
// this file: it exists so that tests, the smoke check and the benchmark's
// CPU-baseline leg can compare the HIP library with a slow, obviously correct
// implementation.  It shares no code, header, table or constant with the HIP
// library.
//
// What it computes (paper: Sect. 2 "The Kalman Filter and ACTS", Fig. 1 and
// Fig. 2; Sect. 4.1 "Parallelization Strategy"; Sect. 4.2.4 "Precision and
// Rounding"):
//   * a track is a 6-vector of bound parameters (loc0, loc1, phi, theta, q/p, t)
//     on a surface with its 6x6 covariance (Sect. 2, parameter list);
//   * each Kalman step propagates the state to the next measurement surface
//     with an adaptive Runge-Kutta-Nystrom integrator, transports the
//     covariance with the transport Jacobian, including the local->global and
//     global->local Jacobians (Sect. 4.1), then combines prediction and
//     measurement with the gain-matrix formalism (Sect. 2, step 3);
//   * after the last surface a Rauch-Tung-Striebel smoother runs backwards
//     with the Jacobians stored during the forward pass (Sect. 2, smoother
//     paragraph); the inverse it needs is done in FP64 (Sect. 4.2.4);
//   * as the alternative smoother of Sect. 2 (Fig. 2), a second Kalman filter
//     runs from the last hit back to the seed surface, propagating against the
//     direction of flight, and its predictions are combined with the forward
//     filtered states;
//   * the chi2 is built from measurement residuals (Sect. 2);
//   * optionally the fitted state is carried to the perigee of a line
//     parallel to z (the parameters Sect. 5.2 quotes), the field is read
//     from a tabulated map with trilinear interpolation (the stored field
//     information of Sect. 4.1), and measuring surfaces are discs with polar
//     local coordinates (a second surface type).
// The paper defers the formulas to the works it cites (Kalman filter for
// track fitting, RTS smoother, Runge-Kutta-Nystrom of Myrheim and Bugge);
// the textbook forms are written out below.  Where the paper is silent the
// reading used here is stated next to the code (units, frames, step control,
// Joseph covariance update, noise placement, alignment parametrisation).
//
// Scalar template: every arithmetic routine is written once for a scalar S.
//   double        -- the oracle proper;
//   Dual<N>       -- forward-mode derivatives (exact JVPs of this algorithm);
//   Cnt           -- counts non-trivial floating-point operations.
// Discrete decisions (step accept/reject, landing, status) always look at the
// value part only.
//
// Pins (tests/test_oracle_*.py): joint-Gaussian conditioning for the linear
// filter+smoother core (and, with a weak prior as one more observation, for
// the two-filter smoother), straight-line closed forms for B = 0, the exact
// helix for uniform B, DOP853 for the solenoid (also to the perigee), scipy's
// grid interpolator for the map, finite differences for every Jacobian,
// Gauss-Newton least squares for a field-free fit, pull and chi2 statistics
// (planes, discs, perigee), envelope theorem and finite differences for the
// gradients.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace kfo {

// ---------------------------------------------------------------------------
// constants (units: mm, GeV, T, ns, rad)
// ---------------------------------------------------------------------------
static const double kC = 299.792458;        // speed of light [mm/ns]
static const double kB = 0.299792458e-3;    // q/p * kB * B = curvature [1/mm] for p in GeV, B in T
static const double kPi = 3.14159265358979323846;

enum Status { ST_OK = 0, ST_NO_INTERSECT = 1, ST_STEP_CAP = 2, ST_NOT_SPD = 3, ST_BAD_INPUT = 4, ST_TOO_FEW = 5 };

// ---------------------------------------------------------------------------
// scalar types
// ---------------------------------------------------------------------------
inline double val(double x) { return x; }

template <int N>
struct Dual {
    double v;
    double d[N];
    Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
    Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
};
template <int N> inline double val(const Dual<N>& x) { return x.v; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v + b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v - b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v * b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v / b.v); for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a) { Dual<N> r(-a.v); for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) { Dual<N> r(a.v * b); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r; }
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> inline Dual<N> chain(const Dual<N>& a, double f, double df) { Dual<N> r(f); for (int i = 0; i < N; ++i) r.d[i] = df * a.d[i]; return r; }
template <int N> inline Dual<N> sin(const Dual<N>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int N> inline Dual<N> cos(const Dual<N>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int N> inline Dual<N> sqrt(const Dual<N>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int N> inline Dual<N> log(const Dual<N>& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
template <int N> inline Dual<N> fabs(const Dual<N>& a) { return a.v < 0 ? -a : a; }
template <int N> inline Dual<N> atan2(const Dual<N>& y, const Dual<N>& x) {
    double q = x.v * x.v + y.v * y.v;
    Dual<N> r(std::atan2(y.v, x.v));
    for (int i = 0; i < N; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) / q;
    return r;
}

// operation counter: an operation is counted unless it is trivial
// (a product with an exact 0 or +-1, a sum with an exact 0).
struct Counts { long long add = 0, mul = 0, div = 0, sqrt = 0, trans = 0; };
static thread_local Counts g_cnt;
struct Cnt {
    double v;
    Cnt() : v(0.0) {}
    Cnt(double x) : v(x) {}
};
inline double val(const Cnt& x) { return x.v; }
inline bool triv_mul(double a) { return a == 0.0 || a == 1.0 || a == -1.0; }
inline Cnt operator+(Cnt a, Cnt b) { if (a.v != 0.0 && b.v != 0.0) ++g_cnt.add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { if (a.v != 0.0 && b.v != 0.0) ++g_cnt.add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { if (!triv_mul(a.v) && !triv_mul(b.v)) ++g_cnt.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { if (!(b.v == 1.0 || b.v == -1.0) && a.v != 0.0) ++g_cnt.div; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator+(Cnt a, double b) { return a + Cnt(b); }
inline Cnt operator+(double a, Cnt b) { return Cnt(a) + b; }
inline Cnt operator-(Cnt a, double b) { return a - Cnt(b); }
inline Cnt operator-(double a, Cnt b) { return Cnt(a) - b; }
inline Cnt operator*(Cnt a, double b) { return a * Cnt(b); }
inline Cnt operator*(double a, Cnt b) { return Cnt(a) * b; }
inline Cnt operator/(Cnt a, double b) { return a / Cnt(b); }
inline Cnt operator/(double a, Cnt b) { return Cnt(a) / b; }
inline Cnt sin(Cnt a) { ++g_cnt.trans; return Cnt(std::sin(a.v)); }
inline Cnt cos(Cnt a) { ++g_cnt.trans; return Cnt(std::cos(a.v)); }
inline Cnt sqrt(Cnt a) { ++g_cnt.sqrt; return Cnt(std::sqrt(a.v)); }
inline Cnt log(Cnt a) { ++g_cnt.trans; return Cnt(std::log(a.v)); }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v)); }
inline Cnt atan2(Cnt y, Cnt x) { ++g_cnt.trans; return Cnt(std::atan2(y.v, x.v)); }

using std::sin; using std::cos; using std::sqrt; using std::log; using std::fabs; using std::atan2;

// ---------------------------------------------------------------------------
// problem description
// ---------------------------------------------------------------------------
// tabulated field: values at origin + (i, j, k) * spacing, stored [k][j][i][3]
struct FieldMap { int n[3]; double origin[3]; double spacing[3]; const double* values; };
// kind 0 uniform b0; 1: Bz=b0z(1-a z^2), Bx=a b0z x z, By=a b0z y z; 2: the tabulated map
struct FieldDef { int kind; double b0[3]; double a; const FieldMap* map = nullptr; };

struct Cfg {
    int ms;            // apply multiple-scattering process noise
    double mass;       // particle mass [GeV]
    double tol;        // RKN local error tolerance on h^2 |k1-k2-k3+k4|_1 [mm]
    double land_tol;   // landing tolerance on the distance to the plane [mm]
    int max_steps;     // maximum RKN trials per surface-to-surface gap
    int smoother = 0;          // 0: RTS with the stored Jacobians; 1: forward + backward filter combined
    double bwd_scale = 1e3;    // two-filter: the backward filter starts from the last filtered
                               // covariance multiplied by this factor
    int target = 0;            // 0: the fitted state on the seed surface; 1: at the perigee
    double perigee[3] = {0.0, 0.0, 0.0};   // perigee line: through this point, parallel to z
};

// Surface types (d = r - c; R columns u, v, w with w = n for the flat ones):
//   0 plane     local (u.d, v.d)
//   1 disc      the plane's polar coordinates (|(u.d, v.d)|, atan2(v.d, u.d))
//   2 cylinder  axis through c along w, radius rho: local (w.d, atan2(v.d, u.d)),
//               the position along the axis and the azimuth about it
//   3 line      a wire through c along w (a straw): local (signed distance of
//               closest approach d.e with e = (w x T)/|w x T|, position w.d
//               along the wire); only loc0 is measured
template <class S>
struct Surf {                 // R columns: u, v, n; x0 = thickness in X0
    S c[3]; S R[3][3]; double x0;
    int type = 0;             // as above
    double radius = 0.0;      // cylinder radius (type 2)
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// Angle into (-pi, pi].  An angle of 64 rad or more (ten turns) is no angle
// a fit of inputs at the detector's scale produces (only absurd hit or seed
// values lead there): it becomes NaN, the track then fails, and no input keeps
// the loops going (reading r28).
template <class S> inline S wrap_phi(S phi) {
    if (!(std::fabs(val(phi)) < 64.0)) return S(NAN);
    while (val(phi) > kPi) phi = phi - 2.0 * kPi;
    while (val(phi) <= -kPi) phi = phi + 2.0 * kPi;
    return phi;
}

template <class S, int R, int K, int C>
void matmul(const S (&a)[R][K], const S (&b)[K][C], S (&out)[R][C]) {
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < C; ++j) {
            S acc = 0.0;
            for (int k = 0; k < K; ++k) acc = acc + a[i][k] * b[k][j];
            out[i][j] = acc;
        }
}

template <class S, int R, int C>
void transpose(const S (&a)[R][C], S (&out)[C][R]) {
    for (int i = 0; i < R; ++i) for (int j = 0; j < C; ++j) out[j][i] = a[i][j];
}

template <class S>
void cross(const S a[3], const S b[3], S out[3]) {
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

// Cholesky factor L (lower) of an SPD matrix; false if a pivot is not positive.
template <class S>
bool cholesky6(const S (&A)[6][6], S (&L)[6][6]) {
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) L[i][j] = 0.0;
    for (int j = 0; j < 6; ++j) {
        S s = A[j][j];
        for (int k = 0; k < j; ++k) s = s - L[j][k] * L[j][k];
        if (!(val(s) > 0.0)) return false;
        L[j][j] = sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            S t = A[i][j];
            for (int k = 0; k < j; ++k) t = t - L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    return true;
}

// Solve (L L^T) X = B for X (6 x 6 right-hand sides).
template <class S>
void chol_solve6(const S (&L)[6][6], const S (&B)[6][6], S (&X)[6][6]) {
    for (int c = 0; c < 6; ++c) {
        S y[6];
        for (int i = 0; i < 6; ++i) {
            S s = B[i][c];
            for (int k = 0; k < i; ++k) s = s - L[i][k] * y[k];
            y[i] = s / L[i][i];
        }
        for (int i = 5; i >= 0; --i) {
            S s = y[i];
            for (int k = i + 1; k < 6; ++k) s = s - L[k][i] * X[k][c];
            X[i][c] = s / L[i][i];
        }
    }
}

// ---------------------------------------------------------------------------
// magnetic field and its gradient dB[a][b] = dB_a / dr_b
// ---------------------------------------------------------------------------
// Tabulated field (kind 2, the position-dependent field information of
// Sect. 4.1 stored as a map): trilinear interpolation in the grid cell that
// holds the point.  A coordinate outside the grid is clamped to the grid's
// boundary, where the field is the boundary's and its derivative along that
// axis is zero.
template <class S>
void map_field(const FieldMap& m, const S r[3], S B[3], S dB[3][3]) {
    int idx[3];
    S w1[3];
    double dudx[3];
    for (int a = 0; a < 3; ++a) {
        S u = (r[a] - m.origin[a]) / m.spacing[a];
        dudx[a] = 1.0 / m.spacing[a];
        if (val(u) <= 0.0) { u = S(0.0); dudx[a] = 0.0; }
        if (val(u) >= double(m.n[a] - 1)) { u = S(double(m.n[a] - 1)); dudx[a] = 0.0; }
        int i = val(u) >= 0.0 ? (int)std::floor(val(u)) : 0;     // a NaN position reads cell 0
        if (i > m.n[a] - 2) i = m.n[a] - 2;
        idx[a] = i;
        w1[a] = u - double(i);
    }
    for (int c = 0; c < 3; ++c) { B[c] = 0.0; for (int a = 0; a < 3; ++a) dB[c][a] = 0.0; }
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                const double* v = m.values + 3 * (((size_t)(idx[2] + dk) * m.n[1] + (idx[1] + dj)) * m.n[0]
                                                   + (idx[0] + di));
                S wx = di ? w1[0] : S(1.0) - w1[0];
                S wy = dj ? w1[1] : S(1.0) - w1[1];
                S wz = dk ? w1[2] : S(1.0) - w1[2];
                double sx = di ? dudx[0] : -dudx[0];
                double sy = dj ? dudx[1] : -dudx[1];
                double sz = dk ? dudx[2] : -dudx[2];
                for (int c = 0; c < 3; ++c) {
                    B[c] = B[c] + wx * wy * wz * v[c];
                    dB[c][0] = dB[c][0] + sx * wy * wz * v[c];
                    dB[c][1] = dB[c][1] + wx * sy * wz * v[c];
                    dB[c][2] = dB[c][2] + wx * wy * sz * v[c];
                }
            }
}

template <class S>
void field_at(const FieldDef& f, const S r[3], S B[3], S dB[3][3]) {
    if (f.kind == 2) { map_field(*f.map, r, B, dB); return; }
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) dB[i][j] = 0.0;
    if (f.kind == 0) {
        for (int i = 0; i < 3; ++i) B[i] = f.b0[i];
        return;
    }
    // solenoid-like: divergence free, Bz = B0 (1 - a z^2), B_rho = a B0 rho z
    const double g = f.a * f.b0[2];
    B[0] = g * r[0] * r[2];
    B[1] = g * r[1] * r[2];
    B[2] = f.b0[2] * (1.0 - f.a * r[2] * r[2]);
    dB[0][0] = g * r[2]; dB[0][2] = g * r[0];
    dB[1][1] = g * r[2]; dB[1][2] = g * r[1];
    dB[2][2] = -2.0 * g * r[2];
}

// ---------------------------------------------------------------------------
// local (bound) <-> global (free) parameters  (Sect. 4.1: transform Jacobians)
// free vector: (x, y, z, t, Tx, Ty, Tz, q/p); bound: (l0, l1, phi, theta, q/p, t)
// ---------------------------------------------------------------------------
template <class S>
void bound_to_free(const Surf<S>& s, const S P[6], S F[8], S J[8][6]) {
    S sp = sin(P[2]), cp = cos(P[2]), st = sin(P[3]), ct = cos(P[3]);
    for (int i = 0; i < 8; ++i) for (int j = 0; j < 6; ++j) J[i][j] = 0.0;
    if (s.type == 2) {
        // cylinder: r = c + rho (cos l1 u + sin l1 v) + l0 w
        S cl = cos(P[1]), sl = sin(P[1]);
        for (int i = 0; i < 3; ++i) {
            F[i] = s.c[i] + s.radius * (cl * s.R[i][0] + sl * s.R[i][1]) + P[0] * s.R[i][2];
            J[i][0] = s.R[i][2];
            J[i][1] = s.radius * (cl * s.R[i][1] - sl * s.R[i][0]);
        }
    } else if (s.type == 3) {
        // line: r = c + l0 e + l1 w, e = (w x T)/|w x T| with T from (phi, theta)
        S T[3] = {cp * st, sp * st, ct};
        S dTp[3] = {-(sp * st), cp * st, S(0.0)};
        S dTt[3] = {cp * ct, sp * ct, -st};
        S w[3] = {s.R[0][2], s.R[1][2], s.R[2][2]};
        S m[3], mp[3], mt[3];
        cross(w, T, m);
        cross(w, dTp, mp);
        cross(w, dTt, mt);
        S mn = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        S e[3] = {m[0] / mn, m[1] / mn, m[2] / mn};
        // de = (I - e e^T) dm / |m|
        S ep = (e[0] * mp[0] + e[1] * mp[1] + e[2] * mp[2]);
        S et = (e[0] * mt[0] + e[1] * mt[1] + e[2] * mt[2]);
        for (int i = 0; i < 3; ++i) {
            F[i] = s.c[i] + P[0] * e[i] + P[1] * w[i];
            J[i][0] = e[i];
            J[i][1] = w[i];
            J[i][2] = P[0] * (mp[i] - e[i] * ep) / mn;
            J[i][3] = P[0] * (mt[i] - e[i] * et) / mn;
        }
    } else if (s.type == 1) {
        // disc: r = c + l0 (cos l1 u + sin l1 v)
        S cl = cos(P[1]), sl = sin(P[1]);
        for (int i = 0; i < 3; ++i) {
            S e = cl * s.R[i][0] + sl * s.R[i][1];
            F[i] = s.c[i] + P[0] * e;
            J[i][0] = e;
            J[i][1] = P[0] * (cl * s.R[i][1] - sl * s.R[i][0]);
        }
    } else {
        for (int i = 0; i < 3; ++i) F[i] = s.c[i] + P[0] * s.R[i][0] + P[1] * s.R[i][1];
        for (int i = 0; i < 3; ++i) { J[i][0] = s.R[i][0]; J[i][1] = s.R[i][1]; }
    }
    F[3] = P[5];
    F[4] = cp * st; F[5] = sp * st; F[6] = ct;
    F[7] = P[4];
    J[3][5] = 1.0;
    J[4][2] = -(sp * st); J[5][2] = cp * st;
    J[4][3] = cp * ct;    J[5][3] = sp * ct;  J[6][3] = -st;
    J[7][4] = 1.0;
}

// The exact expressions are differentiated; T is not renormalised.
template <class S>
void free_to_bound(const Surf<S>& s, const S F[8], S P[6], S J[6][8]) {
    S d[3];
    for (int i = 0; i < 3; ++i) d[i] = F[i] - s.c[i];
    S a = s.R[0][0] * d[0] + s.R[1][0] * d[1] + s.R[2][0] * d[2];
    S b = s.R[0][1] * d[0] + s.R[1][1] * d[1] + s.R[2][1] * d[2];
    S rr = 0.0;
    S e[3] = {S(0.0), S(0.0), S(0.0)}, dl0dT[3] = {S(0.0), S(0.0), S(0.0)};
    if (s.type == 1) {
        rr = sqrt(a * a + b * b);
        P[0] = rr;
        P[1] = atan2(b, a);
    } else if (s.type == 2) {
        P[0] = s.R[0][2] * d[0] + s.R[1][2] * d[1] + s.R[2][2] * d[2];
        P[1] = atan2(b, a);
    } else if (s.type == 3) {
        // signed distance along e = (w x T)/|w x T| (T as given, not renormalised)
        S w[3] = {s.R[0][2], s.R[1][2], s.R[2][2]};
        S T[3] = {F[4], F[5], F[6]};
        S m[3];
        cross(w, T, m);
        S mn = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        for (int i = 0; i < 3; ++i) e[i] = m[i] / mn;
        S de = e[0] * d[0] + e[1] * d[1] + e[2] * d[2];
        P[0] = de;
        P[1] = w[0] * d[0] + w[1] * d[1] + w[2] * d[2];
        // d(d.e)/dT = ((d - (d.e) e) x w) / |m|
        S dp[3] = {d[0] - de * e[0], d[1] - de * e[1], d[2] - de * e[2]};
        S q[3];
        cross(dp, w, q);
        for (int i = 0; i < 3; ++i) dl0dT[i] = q[i] / mn;
    } else {
        P[0] = a;
        P[1] = b;
    }
    S tx = F[4], ty = F[5], tz = F[6];
    S rho2 = tx * tx + ty * ty;
    S rho = sqrt(rho2);
    S n2 = rho2 + tz * tz;
    P[2] = atan2(ty, tx);
    P[3] = atan2(rho, tz);
    P[4] = F[7];
    P[5] = F[3];
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 8; ++j) J[i][j] = 0.0;
    if (s.type == 1) {
        for (int i = 0; i < 3; ++i) {
            J[0][i] = (a * s.R[i][0] + b * s.R[i][1]) / rr;
            J[1][i] = (a * s.R[i][1] - b * s.R[i][0]) / (rr * rr);
        }
    } else if (s.type == 2) {
        S q2 = a * a + b * b;
        for (int i = 0; i < 3; ++i) {
            J[0][i] = s.R[i][2];
            J[1][i] = (a * s.R[i][1] - b * s.R[i][0]) / q2;
        }
    } else if (s.type == 3) {
        for (int i = 0; i < 3; ++i) {
            J[0][i] = e[i];
            J[0][4 + i] = dl0dT[i];
            J[1][i] = s.R[i][2];
        }
    } else {
        for (int i = 0; i < 3; ++i) { J[0][i] = s.R[i][0]; J[1][i] = s.R[i][1]; }
    }
    J[2][4] = -ty / rho2;  J[2][5] = tx / rho2;
    J[3][4] = tx * tz / (rho * n2); J[3][5] = ty * tz / (rho * n2); J[3][6] = -rho / n2;
    J[4][7] = 1.0;
    J[5][3] = 1.0;
}

// ---------------------------------------------------------------------------
// Runge-Kutta-Nystrom step (Sect. 4.1; Myrheim-Bugge form)
//   r' = T,  T' = (q/p) kB T x B(r),  t' = sqrt(1 + m^2 (q/p)^2) / c,  (q/p)' = 0
// with the derivative of the step map at fixed h (transport Jacobian).
// ---------------------------------------------------------------------------
template <class S>
void stage(const FieldDef& f, const S r[3], const S T[3], const S (&dr)[3][8], const S (&dT)[3][8],
           S lam, S k[3], S (&dk)[3][8]) {
    S B[3], dB[3][3], TxB[3];
    field_at(f, r, B, dB);
    cross(T, B, TxB);
    for (int i = 0; i < 3; ++i) k[i] = lam * kB * TxB[i];
    for (int j = 0; j < 8; ++j) {
        S dTj[3] = {dT[0][j], dT[1][j], dT[2][j]};
        S dBj[3];
        for (int a = 0; a < 3; ++a) dBj[a] = dB[a][0] * dr[0][j] + dB[a][1] * dr[1][j] + dB[a][2] * dr[2][j];
        S c1[3], c2[3];
        cross(dTj, B, c1);
        cross(T, dBj, c2);
        for (int i = 0; i < 3; ++i) {
            dk[i][j] = lam * kB * (c1[i] + c2[i]);
            if (j == 7) dk[i][j] = dk[i][j] + kB * TxB[i];
        }
    }
}

template <class S>
double rkn_step(const FieldDef& f, double mass, const S F[8], S h, S Fn[8], S (&D)[8][8]) {
    const S lam = F[7];
    S r[3] = {F[0], F[1], F[2]}, T[3] = {F[4], F[5], F[6]};
    S dr1[3][8], dT1[3][8];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 8; ++j) { dr1[i][j] = (j == i) ? 1.0 : 0.0; dT1[i][j] = (j == 4 + i) ? 1.0 : 0.0; }
    S k1[3], k2[3], k3[3], k4[3], dk1[3][8], dk2[3][8], dk3[3][8], dk4[3][8];
    S h2 = h * 0.5, hh = h * h;
    stage(f, r, T, dr1, dT1, lam, k1, dk1);
    // stage 2 and 3 at the midpoint position
    S r2[3], T2[3], dr2[3][8], dT2[3][8];
    for (int i = 0; i < 3; ++i) {
        r2[i] = r[i] + h2 * T[i] + hh * 0.125 * k1[i];
        T2[i] = T[i] + h2 * k1[i];
        for (int j = 0; j < 8; ++j) {
            dr2[i][j] = dr1[i][j] + h2 * dT1[i][j] + hh * 0.125 * dk1[i][j];
            dT2[i][j] = dT1[i][j] + h2 * dk1[i][j];
        }
    }
    stage(f, r2, T2, dr2, dT2, lam, k2, dk2);
    S T3[3], dT3[3][8];
    for (int i = 0; i < 3; ++i) {
        T3[i] = T[i] + h2 * k2[i];
        for (int j = 0; j < 8; ++j) dT3[i][j] = dT1[i][j] + h2 * dk2[i][j];
    }
    stage(f, r2, T3, dr2, dT3, lam, k3, dk3);
    // stage 4 at the end point
    S r4[3], T4[3], dr4[3][8], dT4[3][8];
    for (int i = 0; i < 3; ++i) {
        r4[i] = r[i] + h * T[i] + hh * 0.5 * k3[i];
        T4[i] = T[i] + h * k3[i];
        for (int j = 0; j < 8; ++j) {
            dr4[i][j] = dr1[i][j] + h * dT1[i][j] + hh * 0.5 * dk3[i][j];
            dT4[i][j] = dT1[i][j] + h * dk3[i][j];
        }
    }
    stage(f, r4, T4, dr4, dT4, lam, k4, dk4);
    // combine
    for (int i = 0; i < 3; ++i) {
        Fn[i] = r[i] + h * T[i] + hh / 6.0 * (k1[i] + k2[i] + k3[i]);
        Fn[4 + i] = T[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    S g = sqrt(1.0 + mass * mass * lam * lam);
    Fn[3] = F[3] + h * g / kC;
    Fn[7] = lam;
    for (int i = 0; i < 8; ++i) for (int j = 0; j < 8; ++j) D[i][j] = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 8; ++j) {
            D[i][j] = dr1[i][j] + h * dT1[i][j] + hh / 6.0 * (dk1[i][j] + dk2[i][j] + dk3[i][j]);
            D[4 + i][j] = dT1[i][j] + h / 6.0 * (dk1[i][j] + 2.0 * dk2[i][j] + 2.0 * dk3[i][j] + dk4[i][j]);
        }
    D[3][3] = 1.0;
    D[3][7] = h * mass * mass * lam / (kC * g);
    D[7][7] = 1.0;
    // local error estimate (values only: the controller is not differentiated)
    double e = 0.0;
    for (int i = 0; i < 3; ++i) e += std::fabs(val(k1[i]) - val(k2[i]) - val(k3[i]) + val(k4[i]));
    return val(h) * val(h) * e;
}

// Adaptive propagation of the free state F onto the plane of surface `s`.
// Step control (reading; the paper only says "adaptive"):
//   first trial = the signed straight-line distance d = n.(c - r)/(n.T);
//   every trial is capped by |d| (then h = d exactly);
//   accept if err <= tol; next trial magnitude |h| * clamp(0.9 (tol/err)^(1/4), 0.25, 4);
//   stop when |n.(c - r)| < land_tol, then move the remaining distance d onto
//   the plane to second order in d.
// D receives the product of the accepted steps' Jacobians.
// Curved measuring surfaces (cylinder, line): the distance to go and, at the
// landed point, the constraint g = 0 that defines the surface, its rate
// g' = dg/ds along the trajectory and its gradient in the free state.
//   cylinder: g = (|d_perp|^2 - rho^2)/2, d_perp = d - (w.d) w; the distance to
//             go is the straight-line path length to the crossing of
//             |d_perp + s T_perp| = rho where the track moves outward (the
//             larger root; none: no intersection), so a cylinder is reached
//             from inside going forward and from outside going backward;
//             grad g = (d_perp, 0, 0, 0, 0)
//   line:     g = d_perp . T (zero at the closest approach to the wire); the
//             distance to go is the Newton step -g/g', g' = |T_perp|^2 +
//             d_perp . T' (must exceed 1e-6: a closest, not a farthest,
//             approach); grad g = (T_perp, 0, d_perp, 0)
template <class S>
int curved_step(const FieldDef& f, double mass, const Surf<S>& s, const S F[8], S* step, S* g, S* gp, S dg[8],
                S dFds[8]) {
    S r[3] = {F[0], F[1], F[2]}, T[3] = {F[4], F[5], F[6]};
    S B[3], dB[3][3], TxB[3];
    field_at(f, r, B, dB);
    cross(T, B, TxB);
    S lam = F[7];
    for (int i = 0; i < 3; ++i) { dFds[i] = T[i]; dFds[4 + i] = lam * kB * TxB[i]; }
    dFds[3] = sqrt(1.0 + mass * mass * lam * lam) / kC;
    dFds[7] = 0.0;
    S w[3] = {s.R[0][2], s.R[1][2], s.R[2][2]};
    S d[3] = {r[0] - s.c[0], r[1] - s.c[1], r[2] - s.c[2]};
    S dw = w[0] * d[0] + w[1] * d[1] + w[2] * d[2];
    S Tw = w[0] * T[0] + w[1] * T[1] + w[2] * T[2];
    S dp[3], Tp[3];
    for (int i = 0; i < 3; ++i) { dp[i] = d[i] - dw * w[i]; Tp[i] = T[i] - Tw * w[i]; }
    for (int i = 0; i < 8; ++i) dg[i] = 0.0;
    S dpT = dp[0] * Tp[0] + dp[1] * Tp[1] + dp[2] * Tp[2];
    S TpT = Tp[0] * Tp[0] + Tp[1] * Tp[1] + Tp[2] * Tp[2];
    if (s.type == 2) {
        S dpd = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
        S c0 = dpd - s.radius * s.radius;
        *g = 0.5 * c0;
        *gp = dpT;
        for (int i = 0; i < 3; ++i) dg[i] = dp[i];
        S disc = dpT * dpT - TpT * c0;
        if (!(val(TpT) > 1e-12) || !(val(disc) >= 0.0)) return ST_NO_INTERSECT;
        // the crossing where the track moves outward (d_perp . T_perp = +sqrt(disc)
        // there), the larger root, in the form without cancellation
        S sq = sqrt(disc);
        if (val(dpT) <= 0.0) *step = (sq - dpT) / TpT;
        else *step = -c0 / (dpT + sq);
        return ST_OK;
    }
    // line
    *g = dpT;
    *gp = TpT + dp[0] * dFds[4] + dp[1] * dFds[5] + dp[2] * dFds[6];
    for (int i = 0; i < 3; ++i) { dg[i] = Tp[i]; dg[4 + i] = dp[i]; }
    if (!(val(*gp) > 1e-6)) return ST_NO_INTERSECT;
    *step = -(*g) / (*gp);
    return ST_OK;
}

// Adaptive propagation onto a curved surface, with the plane propagation's
// step control on the distance to go of curved_step; land when that
// distance is below land_tol, then move it to second order.
template <class S>
int propagate_curved(const FieldDef& f, const Cfg& cfg, const Surf<S>& s, S F[8], S (&D)[8][8], int* n_trials) {
    for (int i = 0; i < 8; ++i) for (int j = 0; j < 8; ++j) D[i][j] = (i == j) ? 1.0 : 0.0;
    double hmag = -1.0;
    int trials = 0;
    for (;;) {
        S d, g, gp, dg[8], dFds[8];
        int st = curved_step(f, cfg.mass, s, F, &d, &g, &gp, dg, dFds);
        if (st != ST_OK) { *n_trials = trials; return st; }
        if (std::fabs(val(d)) < cfg.land_tol) break;
        if (trials >= cfg.max_steps) { *n_trials = trials; return ST_STEP_CAP; }
        if (hmag < 0.0) hmag = std::fabs(val(d));
        S h = (std::fabs(val(d)) <= hmag) ? d : S(std::copysign(hmag, val(d)));
        S Fn[8], Ds[8][8];
        double err = rkn_step(f, cfg.mass, F, h, Fn, Ds);
        ++trials;
        double fac = 0.9 * std::pow(cfg.tol / std::max(err, 1e-300), 0.25);
        fac = std::min(4.0, std::max(0.25, fac));
        if (err <= cfg.tol) {
            for (int i = 0; i < 8; ++i) F[i] = Fn[i];
            S Dn[8][8];
            matmul(Ds, D, Dn);
            for (int i = 0; i < 8; ++i) for (int j = 0; j < 8; ++j) D[i][j] = Dn[i][j];
        }
        hmag = std::fabs(val(h)) * fac;
    }
    {
        S d, g, gp, dg[8], dFds[8];
        curved_step(f, cfg.mass, s, F, &d, &g, &gp, dg, dFds);
        for (int i = 0; i < 3; ++i) {
            F[i] = F[i] + d * dFds[i] + 0.5 * d * d * dFds[4 + i];
            F[4 + i] = F[4 + i] + d * dFds[4 + i];
        }
        F[3] = F[3] + d * dFds[3];
    }
    *n_trials = trials;
    return ST_OK;
}

template <class S>
int propagate(const FieldDef& f, const Cfg& cfg, const Surf<S>& s, S F[8], S (&D)[8][8], int* n_trials) {
    if (s.type == 2 || s.type == 3) return propagate_curved(f, cfg, s, F, D, n_trials);
    for (int i = 0; i < 8; ++i) for (int j = 0; j < 8; ++j) D[i][j] = (i == j) ? 1.0 : 0.0;
    const S* n3[3] = {&s.R[0][2], &s.R[1][2], &s.R[2][2]};
    double hmag = -1.0;
    int trials = 0;
    for (;;) {
        S nT = *n3[0] * F[4] + *n3[1] * F[5] + *n3[2] * F[6];
        S dist = *n3[0] * (s.c[0] - F[0]) + *n3[1] * (s.c[1] - F[1]) + *n3[2] * (s.c[2] - F[2]);
        if (std::fabs(val(nT)) < 1e-6) { *n_trials = trials; return ST_NO_INTERSECT; }
        if (std::fabs(val(dist)) < cfg.land_tol) break;
        if (trials >= cfg.max_steps) { *n_trials = trials; return ST_STEP_CAP; }
        S d = dist / nT;
        if (hmag < 0.0) hmag = std::fabs(val(d));
        S h = (std::fabs(val(d)) <= hmag) ? d : S(std::copysign(hmag, val(d)));
        S Fn[8], Ds[8][8];
        double err = rkn_step(f, cfg.mass, F, h, Fn, Ds);
        ++trials;
        double fac = 0.9 * std::pow(cfg.tol / std::max(err, 1e-300), 0.25);
        fac = std::min(4.0, std::max(0.25, fac));
        if (err <= cfg.tol) {
            for (int i = 0; i < 8; ++i) F[i] = Fn[i];
            S Dn[8][8];
            matmul(Ds, D, Dn);
            for (int i = 0; i < 8; ++i) for (int j = 0; j < 8; ++j) D[i][j] = Dn[i][j];
        }
        hmag = std::fabs(val(h)) * fac;
    }
    // Final move onto the plane, second order in the remaining distance d
    // (|d| < land_tol): r += d T + d^2/2 T', T += d T', t += d dt/ds.  The
    // result then lies on the plane to rounding whether or not one more
    // landing iteration was taken.
    {
        S nT = *n3[0] * F[4] + *n3[1] * F[5] + *n3[2] * F[6];
        S dist = *n3[0] * (s.c[0] - F[0]) + *n3[1] * (s.c[1] - F[1]) + *n3[2] * (s.c[2] - F[2]);
        S d = dist / nT;
        S r[3] = {F[0], F[1], F[2]}, T[3] = {F[4], F[5], F[6]};
        S B[3], dB[3][3], TxB[3];
        field_at(f, r, B, dB);
        cross(T, B, TxB);
        S lam = F[7];
        for (int i = 0; i < 3; ++i) {
            F[i] = F[i] + d * T[i] + 0.5 * d * d * lam * kB * TxB[i];
            F[4 + i] = F[4 + i] + d * lam * kB * TxB[i];
        }
        F[3] = F[3] + d * sqrt(1.0 + cfg.mass * cfg.mass * lam * lam) / kC;
    }
    *n_trials = trials;
    return ST_OK;
}

// Path correction at the target plane: a variation of the free state is moved
// along the trajectory back onto the plane (first order).
template <class S>
void path_correction(const FieldDef& f, double mass, const Surf<S>& s, const S F[8], S (&Pc)[8][8]) {
    if (s.type == 2 || s.type == 3) {
        // onto the constraint g = 0 along dF/ds: P = I - dF/ds grad(g)^T / g'
        // (g' = grad(g) . dF/ds)
        S d, g, gp, dg[8], dFds[8];
        curved_step(f, mass, s, F, &d, &g, &gp, dg, dFds);
        S rate = 0.0;
        for (int j = 0; j < 8; ++j) rate = rate + dg[j] * dFds[j];
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) Pc[i][j] = ((i == j) ? S(1.0) : S(0.0)) - dFds[i] * dg[j] / rate;
        return;
    }
    S r[3] = {F[0], F[1], F[2]}, T[3] = {F[4], F[5], F[6]};
    S B[3], dB[3][3], TxB[3];
    field_at(f, r, B, dB);
    cross(T, B, TxB);
    S lam = F[7];
    S dFds[8];
    for (int i = 0; i < 3; ++i) { dFds[i] = T[i]; dFds[4 + i] = lam * kB * TxB[i]; }
    dFds[3] = sqrt(1.0 + mass * mass * lam * lam) / kC;
    dFds[7] = 0.0;
    S n[3] = {s.R[0][2], s.R[1][2], s.R[2][2]};
    S nT = n[0] * T[0] + n[1] * T[1] + n[2] * T[2];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            S nj = (j < 3) ? n[j] : S(0.0);
            Pc[i][j] = ((i == j) ? S(1.0) : S(0.0)) - dFds[i] * nj / nT;
        }
}

// Bound-to-bound transport: x on surface a -> x' on surface b, with F = dx'/dx.
template <class S>
int transport(const FieldDef& f, const Cfg& cfg, const Surf<S>& sa, const Surf<S>& sb, const S x[6],
              S xo[6], S (&Fk)[6][6], int* n_trials) {
    S F[8], Jbf[8][6], D[8][8], Pc[8][8], Jfb[6][8];
    bound_to_free(sa, x, F, Jbf);
    int st = propagate(f, cfg, sb, F, D, n_trials);
    if (st != ST_OK) return st;
    path_correction(f, cfg.mass, sb, F, Pc);
    free_to_bound(sb, F, xo, Jfb);
    S A[6][8], Bm[6][8], Cm[6][8];
    matmul(Jfb, Pc, A);
    matmul(A, D, Bm);
    (void)Cm;
    matmul(Bm, Jbf, Fk);
    return ST_OK;
}

// ---------------------------------------------------------------------------
// Perigee (Sect. 2; Sect. 5.2 quotes the fitted parameters there): the line
// through the reference point c parallel to z.  At the point of closest
// approach (r - c)_perp is orthogonal to T_perp; the bound parameters are
// (d0, z0, phi, theta, q/p, t) with d0 = (r - c) . u, u = (-T_y, T_x, 0)/|T_perp|
// (z cross the transverse direction), and z0 = r_z - c_z.
// ---------------------------------------------------------------------------
// constraint g = (r - c)_perp . T_perp, zero at the closest approach; its rate
// along the trajectory g' = |T_perp|^2 + (r - c)_perp . T'_perp; its gradient
// in the free state; dF/ds.
template <class S>
void perigee_g(const FieldDef& f, double mass, const double c[3], const S F[8], S* g, S* gp, S dg[8],
               S dFds[8]) {
    S r[3] = {F[0], F[1], F[2]}, T[3] = {F[4], F[5], F[6]};
    S B[3], dB[3][3], TxB[3];
    field_at(f, r, B, dB);
    cross(T, B, TxB);
    S lam = F[7];
    for (int i = 0; i < 3; ++i) { dFds[i] = T[i]; dFds[4 + i] = lam * kB * TxB[i]; }
    dFds[3] = sqrt(1.0 + mass * mass * lam * lam) / kC;
    dFds[7] = 0.0;
    S dx = r[0] - c[0], dy = r[1] - c[1];
    *g = dx * T[0] + dy * T[1];
    *gp = T[0] * T[0] + T[1] * T[1] + dx * dFds[4] + dy * dFds[5];
    for (int i = 0; i < 8; ++i) dg[i] = 0.0;
    dg[0] = T[0]; dg[1] = T[1]; dg[4] = dx; dg[5] = dy;
}

// Adaptive propagation of the free state F to the perigee, with the plane
// propagation's step control; the distance to go is the Newton step
// d = -g/g'; land when |d| < land_tol, then move d to second order.  g' must
// stay positive (a closest approach, not a farthest point).
template <class S>
int propagate_perigee(const FieldDef& f, const Cfg& cfg, const double c[3], S F[8], S (&D)[8][8], int* n_trials) {
    for (int i = 0; i < 8; ++i) for (int j = 0; j < 8; ++j) D[i][j] = (i == j) ? 1.0 : 0.0;
    double hmag = -1.0;
    int trials = 0;
    for (;;) {
        S g, gp, dg[8], dFds[8];
        perigee_g(f, cfg.mass, c, F, &g, &gp, dg, dFds);
        if (!(val(gp) > 1e-6)) { *n_trials = trials; return ST_NO_INTERSECT; }
        S d = -g / gp;
        if (std::fabs(val(d)) < cfg.land_tol) break;
        if (trials >= cfg.max_steps) { *n_trials = trials; return ST_STEP_CAP; }
        if (hmag < 0.0) hmag = std::fabs(val(d));
        S h = (std::fabs(val(d)) <= hmag) ? d : S(std::copysign(hmag, val(d)));
        S Fn[8], Ds[8][8];
        double err = rkn_step(f, cfg.mass, F, h, Fn, Ds);
        ++trials;
        double fac = 0.9 * std::pow(cfg.tol / std::max(err, 1e-300), 0.25);
        fac = std::min(4.0, std::max(0.25, fac));
        if (err <= cfg.tol) {
            for (int i = 0; i < 8; ++i) F[i] = Fn[i];
            S Dn[8][8];
            matmul(Ds, D, Dn);
            for (int i = 0; i < 8; ++i) for (int j = 0; j < 8; ++j) D[i][j] = Dn[i][j];
        }
        hmag = std::fabs(val(h)) * fac;
    }
    {
        S g, gp, dg[8], dFds[8];
        perigee_g(f, cfg.mass, c, F, &g, &gp, dg, dFds);
        S d = -g / gp;
        for (int i = 0; i < 3; ++i) {
            F[i] = F[i] + d * dFds[i] + 0.5 * d * d * dFds[4 + i];
            F[4 + i] = F[4 + i] + d * dFds[4 + i];
        }
        F[3] = F[3] + d * dFds[3];
    }
    *n_trials = trials;
    return ST_OK;
}

template <class S>
void free_to_perigee(const double c[3], const S F[8], S P[6], S J[6][8]) {
    S tx = F[4], ty = F[5], tz = F[6];
    S rho2 = tx * tx + ty * ty;
    S rho = sqrt(rho2);
    S n2 = rho2 + tz * tz;
    S ux = -ty / rho, uy = tx / rho;
    S dx = F[0] - c[0], dy = F[1] - c[1];
    P[0] = dx * ux + dy * uy;
    P[1] = F[2] - c[2];
    P[2] = atan2(ty, tx);
    P[3] = atan2(rho, tz);
    P[4] = F[7];
    P[5] = F[3];
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 8; ++j) J[i][j] = 0.0;
    S rho3 = rho2 * rho;
    S gperp = dx * tx + dy * ty;
    J[0][0] = ux; J[0][1] = uy;
    J[0][4] = ty * gperp / rho3;
    J[0][5] = -(tx * gperp) / rho3;
    J[1][2] = 1.0;
    J[2][4] = -ty / rho2;  J[2][5] = tx / rho2;
    J[3][4] = tx * tz / (rho * n2); J[3][5] = ty * tz / (rho * n2); J[3][6] = -rho / n2;
    J[4][7] = 1.0;
    J[5][3] = 1.0;
}

// x on plane surface a -> perigee parameters, with F = dx'/dx.  The path
// correction moves a variation back onto the constraint g = 0 along dF/ds.
template <class S>
int transport_perigee(const FieldDef& f, const Cfg& cfg, const Surf<S>& sa, const double c[3], const S x[6],
                      S xo[6], S (&Fk)[6][6], int* n_trials) {
    S F[8], Jbf[8][6], D[8][8], Pc[8][8], Jfb[6][8];
    bound_to_free(sa, x, F, Jbf);
    int st = propagate_perigee(f, cfg, c, F, D, n_trials);
    if (st != ST_OK) return st;
    S g, gp, dg[8], dFds[8];
    perigee_g(f, cfg.mass, c, F, &g, &gp, dg, dFds);
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) Pc[i][j] = ((i == j) ? S(1.0) : S(0.0)) - dFds[i] * dg[j] / gp;
    free_to_perigee(c, F, xo, Jfb);
    S A[6][8], Bm[6][8];
    matmul(Jfb, Pc, A);
    matmul(A, D, Bm);
    matmul(Bm, Jbf, Fk);
    return ST_OK;
}

// ---------------------------------------------------------------------------
// multiple scattering (thin scatterer after the update, PDG Highland width)
// ---------------------------------------------------------------------------
template <class S>
void ms_noise(const Surf<S>& s, const S x[6], double mass, S (&Q)[6][6]) {
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Q[i][j] = 0.0;
    if (!(s.x0 > 0.0)) return;
    S st = sin(x[3]);
    S T[3] = {cos(x[2]) * st, sin(x[2]) * st, cos(x[3])};
    // path through the layer: x0 over the cosine of the incidence on the
    // surface normal (plane, disc: n; cylinder: the radial direction at the
    // state's azimuth); a straw (line) is crossed across its wire, x0 over
    // the sine of the angle between the track and the wire
    S nT;
    if (s.type == 2) {
        S cl = cos(x[1]), sl = sin(x[1]);
        nT = 0.0;
        for (int i = 0; i < 3; ++i) nT = nT + (cl * s.R[i][0] + sl * s.R[i][1]) * T[i];
    } else if (s.type == 3) {
        S w[3] = {s.R[0][2], s.R[1][2], s.R[2][2]}, m[3];
        cross(w, T, m);
        nT = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    } else {
        nT = s.R[0][2] * T[0] + s.R[1][2] * T[1] + s.R[2][2] * T[2];
    }
    S path = s.x0 / fabs(nT);
    S p = 1.0 / fabs(x[4]);
    S beta = p / sqrt(p * p + mass * mass);
    S th0 = 0.0136 / (beta * p) * sqrt(path) * (1.0 + 0.038 * log(path / (beta * beta)));
    Q[2][2] = th0 * th0 / (st * st);
    Q[3][3] = th0 * th0;
}

// ---------------------------------------------------------------------------
// gain-matrix update, H = [I2 0] (Sect. 2), Joseph covariance form
// ---------------------------------------------------------------------------
// ang1: the second local coordinate is an angle (disc): its residual and
// its filtered value are taken in (-pi, pi].
template <class S>
int kalman_update(const S xp[6], const S (&Cp)[6][6], const S m[2], const S (&V)[2][2],
                  S xf[6], S (&Cf)[6][6], S* chi2, bool ang1 = false) {
    S r[2] = {m[0] - xp[0], m[1] - xp[1]};
    if (ang1) r[1] = wrap_phi(r[1]);
    S Sm[2][2] = {{V[0][0] + Cp[0][0], V[0][1] + Cp[0][1]}, {V[1][0] + Cp[1][0], V[1][1] + Cp[1][1]}};
    S det = Sm[0][0] * Sm[1][1] - Sm[0][1] * Sm[1][0];
    if (!(val(Sm[0][0]) > 0.0 && val(det) > 0.0)) return ST_NOT_SPD;
    S Si[2][2] = {{Sm[1][1] / det, -Sm[0][1] / det}, {-Sm[1][0] / det, Sm[0][0] / det}};
    S K[6][2];
    for (int i = 0; i < 6; ++i)
        for (int a = 0; a < 2; ++a) K[i][a] = Cp[i][0] * Si[0][a] + Cp[i][1] * Si[1][a];
    for (int i = 0; i < 6; ++i) xf[i] = xp[i] + K[i][0] * r[0] + K[i][1] * r[1];
    xf[2] = wrap_phi(xf[2]);
    if (ang1) xf[1] = wrap_phi(xf[1]);
    S IKH[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) IKH[i][j] = ((i == j) ? S(1.0) : S(0.0)) - ((j < 2) ? K[i][j] : S(0.0));
    S T1[6][6], IKHt[6][6], T2[6][6];
    matmul(IKH, Cp, T1);
    transpose(IKH, IKHt);
    matmul(T1, IKHt, T2);
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            S kvk = 0.0;
            for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) kvk = kvk + K[i][a] * V[a][b] * K[j][b];
            Cf[i][j] = T2[i][j] + kvk;
        }
    *chi2 = r[0] * (Si[0][0] * r[0] + Si[0][1] * r[1]) + r[1] * (Si[1][0] * r[0] + Si[1][1] * r[1]);
    return ST_OK;
}

// One-dimensional update (a straw measures loc0 only): H = e0^T, the same
// gain-matrix formalism and Joseph form with a scalar residual covariance.
template <class S>
int kalman_update1(const S xp[6], const S (&Cp)[6][6], const S m0, double V00, S xf[6], S (&Cf)[6][6], S* chi2) {
    S r = m0 - xp[0];
    S Sm = V00 + Cp[0][0];
    if (!(val(Sm) > 0.0)) return ST_NOT_SPD;
    S K[6];
    for (int i = 0; i < 6; ++i) K[i] = Cp[i][0] / Sm;
    for (int i = 0; i < 6; ++i) xf[i] = xp[i] + K[i] * r;
    xf[2] = wrap_phi(xf[2]);
    S IKH[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) IKH[i][j] = ((i == j) ? S(1.0) : S(0.0)) - ((j == 0) ? K[i] : S(0.0));
    S T1[6][6], IKHt[6][6], T2[6][6];
    matmul(IKH, Cp, T1);
    transpose(IKH, IKHt);
    matmul(T1, IKHt, T2);
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) Cf[i][j] = T2[i][j] + K[i] * V00 * K[j];
    *chi2 = r * r / Sm;
    return ST_OK;
}

// Per surface type: is loc1 an azimuth (disc, cylinder), and how many local
// coordinates a hit measures (a line: loc0 only).
inline bool loc1_is_angle(int type) { return type == 1 || type == 2; }
inline int meas_dim(int type) { return type == 3 ? 1 : 2; }

template <class S>
int update_on(int type, const S xp[6], const S (&Cp)[6][6], const S m[2], const S (&V)[2][2], S xf[6],
              S (&Cf)[6][6], S* chi2) {
    if (type == 3) return kalman_update1(xp, Cp, m[0], val(V[0][0]), xf, Cf, chi2);
    return kalman_update(xp, Cp, m, V, xf, Cf, chi2, loc1_is_angle(type));
}

// ---------------------------------------------------------------------------
// Rauch-Tung-Striebel step with the stored Jacobian F (Sect. 2):
//   A = Cf F^T Cp1^{-1} (FP64 SPD solve),  xs = xf + A (xs1 - xp1),  Cs = Cf + A (Cs1 - Cp1) A^T
// ---------------------------------------------------------------------------
// ang1_next / ang1_here: the second local coordinate of state k+1 / k is an
// angle (disc) and its differences and values are taken in (-pi, pi].
template <class S>
int rts_step(const S xf[6], const S (&Cf)[6][6], const S (&F)[6][6], const S xp1[6], const S (&Cp1)[6][6],
             const S xs1[6], const S (&Cs1)[6][6], S xs[6], S (&Cs)[6][6], bool ang1_next = false,
             bool ang1_here = false) {
    S L[6][6];
    if (!cholesky6(Cp1, L)) return ST_NOT_SPD;
    S FC[6][6], At[6][6], A[6][6];
    matmul(F, Cf, FC);
    chol_solve6(L, FC, At);          // Cp1 A^T = F Cf
    transpose(At, A);
    S dx[6];
    for (int i = 0; i < 6; ++i) dx[i] = xs1[i] - xp1[i];
    dx[2] = wrap_phi(dx[2]);
    if (ang1_next) dx[1] = wrap_phi(dx[1]);
    for (int i = 0; i < 6; ++i) {
        S acc = xf[i];
        for (int k = 0; k < 6; ++k) acc = acc + A[i][k] * dx[k];
        xs[i] = acc;
    }
    xs[2] = wrap_phi(xs[2]);
    if (ang1_here) xs[1] = wrap_phi(xs[1]);
    S dC[6][6], T1[6][6], T2[6][6];
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) dC[i][j] = Cs1[i][j] - Cp1[i][j];
    matmul(A, dC, T1);
    matmul(T1, At, T2);
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Cs[i][j] = Cf[i][j] + T2[i][j];
    return ST_OK;
}

// ---------------------------------------------------------------------------
// Two-filter smoother (Sect. 2, Fig. 2: the smoother run as a second filter
// from the last hit back to the first, whose predictions are combined with
// the forward filter's estimates).  Two independent estimates (xf, Cf) and
// (xb, Cb) of one state combine with the gain K = Cf (Cf + Cb)^{-1}:
//   xs = xf + K (xb - xf)                                  (phi difference wrapped)
//   Cs = (I - K) Cf (I - K)^T + K Cb K^T                   (covariance of that sum)
// Cholesky of Cf + Cb: K^T = (Cf + Cb)^{-1} Cf.
// ---------------------------------------------------------------------------
template <class S>
int two_filter_combine(const S xf[6], const S (&Cf)[6][6], const S xb[6], const S (&Cb)[6][6],
                       S xs[6], S (&Cs)[6][6], bool ang1 = false) {
    S Sm[6][6], L[6][6], Kt[6][6], K[6][6];
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Sm[i][j] = Cf[i][j] + Cb[i][j];
    if (!cholesky6(Sm, L)) return ST_NOT_SPD;
    chol_solve6(L, Cf, Kt);
    transpose(Kt, K);
    S dx[6];
    for (int i = 0; i < 6; ++i) dx[i] = xb[i] - xf[i];
    dx[2] = wrap_phi(dx[2]);
    if (ang1) dx[1] = wrap_phi(dx[1]);
    for (int i = 0; i < 6; ++i) {
        S acc = xf[i];
        for (int k = 0; k < 6; ++k) acc = acc + K[i][k] * dx[k];
        xs[i] = acc;
    }
    xs[2] = wrap_phi(xs[2]);
    if (ang1) xs[1] = wrap_phi(xs[1]);
    S IK[6][6], IKt[6][6], T1[6][6], T2[6][6], T3[6][6], T4[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) IK[i][j] = ((i == j) ? S(1.0) : S(0.0)) - K[i][j];
    transpose(IK, IKt);
    matmul(IK, Cf, T1);
    matmul(T1, IKt, T2);
    matmul(K, Cb, T3);
    matmul(T3, Kt, T4);
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Cs[i][j] = T2[i][j] + T4[i][j];
    return ST_OK;
}

// Backward prediction: a state estimate (x, C) carried against the direction
// of flight by the transport G, then the thin scatterer of the surface it
// reaches (the forward model scatters after each measurement, so going back
// the scattering angle's variance is added after the transport):
//   C <- G C G^T + Q
template <class S>
void backward_predict(const S (&G)[6][6], const S (&Q)[6][6], const S (&C)[6][6], S (&Cq)[6][6]) {
    S T1[6][6], Gt[6][6], T2[6][6];
    matmul(G, C, T1);
    transpose(G, Gt);
    matmul(T1, Gt, T2);
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Cq[i][j] = T2[i][j] + Q[i][j];
}

// ---------------------------------------------------------------------------
// one track: filter + smoother
// ---------------------------------------------------------------------------
template <class S>
struct TrackOut {
    std::vector<S> xs, Cs, xf, Cf, xp, Cp;   // per hit: 6 / 36
    S tgt[6];
    S tgt_cov[6][6];
    S chi2;
    std::vector<int> trials;
    int status;
};

inline void unpack21(const double* c21, double (&C)[6][6]) {
    int k = 0;
    for (int i = 0; i < 6; ++i) for (int j = i; j < 6; ++j) { C[i][j] = c21[k]; C[j][i] = c21[k]; ++k; }
}

template <class S>
int fit_track_seed_surface(const FieldDef& f, const Cfg& cfg, const Surf<S>* surf, int n_surf,
                           int n, const int* sid, const S* m /*[n][2]*/, const double* V3 /*[n][3]*/,
                           const S* seed /*6*/, const double* seed_cov21, int seed_sid, TrackOut<S>& out) {
    out.xs.assign(6 * n, S(NAN)); out.Cs.assign(36 * n, S(NAN));
    out.xf.assign(6 * n, S(NAN)); out.Cf.assign(36 * n, S(NAN));
    out.xp.assign(6 * n, S(NAN)); out.Cp.assign(36 * n, S(NAN));
    out.trials.assign(n, 0);
    for (int i = 0; i < 6; ++i) { out.tgt[i] = NAN; for (int j = 0; j < 6; ++j) out.tgt_cov[i][j] = NAN; }
    out.chi2 = NAN;
    // input validation
    if (n < 3) return out.status = ST_TOO_FEW;
    // the seed surface is a plane; hit surfaces are planes, discs, cylinders
    // (radius > 0) or lines; a line hit has only loc0 and v00 (the rest unread)
    if (seed_sid < 0 || seed_sid >= n_surf || surf[seed_sid].type != 0) return out.status = ST_BAD_INPUT;
    for (int k = 0; k < n; ++k) {
        if (sid[k] < 0 || sid[k] >= n_surf) return out.status = ST_BAD_INPUT;
        const int ty = surf[sid[k]].type;
        if (ty < 0 || ty > 3) return out.status = ST_BAD_INPUT;
        if (ty == 2 && !(surf[sid[k]].radius > 0.0)) return out.status = ST_BAD_INPUT;
        const double* v = V3 + 3 * k;
        if (ty == 3) {
            if (!std::isfinite(val(m[2 * k])) || !std::isfinite(v[0]) || !(v[0] > 0.0)) return out.status = ST_BAD_INPUT;
            continue;
        }
        for (int a = 0; a < 2; ++a) if (!std::isfinite(val(m[2 * k + a]))) return out.status = ST_BAD_INPUT;
        if (!(std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]))) return out.status = ST_BAD_INPUT;
        if (!(v[0] > 0.0 && v[0] * v[2] - v[1] * v[1] > 0.0)) return out.status = ST_BAD_INPUT;
    }
    double C0d[6][6];
    unpack21(seed_cov21, C0d);
    for (int i = 0; i < 6; ++i) {
        if (!std::isfinite(val(seed[i]))) return out.status = ST_BAD_INPUT;
        for (int j = 0; j < 6; ++j) if (!std::isfinite(C0d[i][j])) return out.status = ST_BAD_INPUT;
    }
    S C0[6][6], L0[6][6];
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) C0[i][j] = C0d[i][j];
    if (!cholesky6(C0, L0)) return out.status = ST_BAD_INPUT;

    // forward filter: state 0 is the seed, states 1..n are the hits
    std::vector<S> Fst(36 * n);       // Fst[k] = Jacobian from state k to state k+1
    S x[6], C[6][6];
    for (int i = 0; i < 6; ++i) x[i] = seed[i];
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) C[i][j] = C0[i][j];
    int prev = seed_sid;
    S chi2 = 0.0;
    for (int k = 0; k < n; ++k) {
        S Q[6][6];
        if (cfg.ms) ms_noise(surf[prev], x, cfg.mass, Q);
        else for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Q[i][j] = 0.0;
        S xp[6], Fk[6][6];
        int st = transport(f, cfg, surf[prev], surf[sid[k]], x, xp, Fk, &out.trials[k]);
        if (st != ST_OK) return out.status = st;
        S CQ[6][6], T1[6][6], Ft[6][6], Cp[6][6];
        for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) CQ[i][j] = C[i][j] + Q[i][j];
        matmul(Fk, CQ, T1);
        transpose(Fk, Ft);
        matmul(T1, Ft, Cp);
        S mk[2] = {m[2 * k], m[2 * k + 1]};
        const double* v = V3 + 3 * k;
        S V[2][2] = {{v[0], v[1]}, {v[1], v[2]}};
        S ck;
        st = update_on(surf[sid[k]].type, xp, Cp, mk, V, x, C, &ck);
        if (st != ST_OK) return out.status = st;
        chi2 = chi2 + ck;
        for (int i = 0; i < 6; ++i) {
            out.xp[6 * k + i] = xp[i];
            out.xf[6 * k + i] = x[i];
            for (int j = 0; j < 6; ++j) {
                out.Cp[36 * k + 6 * i + j] = Cp[i][j];
                out.Cf[36 * k + 6 * i + j] = C[i][j];
                Fst[36 * k + 6 * i + j] = Fk[i][j];
            }
        }
        prev = sid[k];
    }
    // the last hit's smoothed state is its filtered state (both smoothers)
    for (int i = 0; i < 6; ++i) out.xs[6 * (n - 1) + i] = out.xf[6 * (n - 1) + i];
    for (int i = 0; i < 36; ++i) out.Cs[36 * (n - 1) + i] = out.Cf[36 * (n - 1) + i];
    if (cfg.smoother == 1) {
        // Two-filter smoother.  The backward filter starts at the last hit from
        // the forward estimate there with its covariance inflated by bwd_scale
        // (a weak prior, so that the backward estimates rest on the hits behind
        // them), takes in that hit, and then for k = n-2 .. 0 and finally the
        // seed surface: propagate back to surface k, add the scatterer of
        // surface k, combine this prediction (hits k+1 .. n-1) with the forward
        // filtered state of hit k (hits 0 .. k) into the smoothed state, and
        // take in hit k.
        S xb[6], Cb[6][6];
        {
            S xl[6], Cl[6][6], ck;
            for (int i = 0; i < 6; ++i) {
                xl[i] = out.xf[6 * (n - 1) + i];
                for (int j = 0; j < 6; ++j) Cl[i][j] = cfg.bwd_scale * out.Cf[36 * (n - 1) + 6 * i + j];
            }
            S mk[2] = {m[2 * (n - 1)], m[2 * (n - 1) + 1]};
            const double* v = V3 + 3 * (n - 1);
            S V[2][2] = {{v[0], v[1]}, {v[1], v[2]}};
            int st = update_on(surf[sid[n - 1]].type, xl, Cl, mk, V, xb, Cb, &ck);
            if (st != ST_OK) return out.status = st;
        }
        for (int k = n - 2; k >= -1; --k) {
            const Surf<S>& sa = surf[sid[k + 1]];
            const Surf<S>& sb = surf[k >= 0 ? sid[k] : seed_sid];
            S xf[6], Cf[6][6], xs[6], Cs[6][6];
            for (int i = 0; i < 6; ++i) {
                xf[i] = (k >= 0) ? out.xf[6 * k + i] : seed[i];
                for (int j = 0; j < 6; ++j) Cf[i][j] = (k >= 0) ? out.Cf[36 * k + 6 * i + j] : C0[i][j];
            }
            S xq[6], G[6][6], Q[6][6], Cq[6][6];
            int trials = 0;
            int st = transport(f, cfg, sa, sb, xb, xq, G, &trials);
            if (st != ST_OK) return out.status = st;
            // the scatterer's variance as the forward filter took it: at the
            // forward filtered state of surface k (the seed on the seed surface)
            if (cfg.ms) ms_noise(sb, xf, cfg.mass, Q);
            else for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Q[i][j] = 0.0;
            backward_predict(G, Q, Cb, Cq);
            const bool ang = k >= 0 && loc1_is_angle(surf[sid[k]].type);
            st = two_filter_combine(xf, Cf, xq, Cq, xs, Cs, ang);
            if (st != ST_OK) return out.status = st;
            for (int i = 0; i < 6; ++i) {
                if (k >= 0) out.xs[6 * k + i] = xs[i]; else out.tgt[i] = xs[i];
                for (int j = 0; j < 6; ++j) {
                    if (k >= 0) out.Cs[36 * k + 6 * i + j] = Cs[i][j]; else out.tgt_cov[i][j] = Cs[i][j];
                }
            }
            if (k >= 0) {
                S mk[2] = {m[2 * k], m[2 * k + 1]};
                const double* v = V3 + 3 * k;
                S V[2][2] = {{v[0], v[1]}, {v[1], v[2]}};
                S ck;
                st = update_on(surf[sid[k]].type, xq, Cq, mk, V, xb, Cb, &ck);
                if (st != ST_OK) return out.status = st;
            }
        }
        out.chi2 = chi2;
        return out.status = ST_OK;
    }
    // RTS smoother, k = n-2 .. 0 over hits, then the seed state
    for (int k = n - 2; k >= -1; --k) {
        S xf[6], Cf[6][6], F[6][6], xp1[6], Cp1[6][6], xs1[6], Cs1[6][6], xs[6], Cs[6][6];
        for (int i = 0; i < 6; ++i) {
            xf[i] = (k >= 0) ? out.xf[6 * k + i] : seed[i];
            xp1[i] = out.xp[6 * (k + 1) + i];
            xs1[i] = out.xs[6 * (k + 1) + i];
            for (int j = 0; j < 6; ++j) {
                Cf[i][j] = (k >= 0) ? out.Cf[36 * k + 6 * i + j] : C0[i][j];
                F[i][j] = Fst[36 * (k + 1) + 6 * i + j];
                Cp1[i][j] = out.Cp[36 * (k + 1) + 6 * i + j];
                Cs1[i][j] = out.Cs[36 * (k + 1) + 6 * i + j];
            }
        }
        int st = rts_step(xf, Cf, F, xp1, Cp1, xs1, Cs1, xs, Cs, loc1_is_angle(surf[sid[k + 1]].type),
                          k >= 0 && loc1_is_angle(surf[sid[k]].type));
        if (st != ST_OK) return out.status = st;
        for (int i = 0; i < 6; ++i) {
            if (k >= 0) out.xs[6 * k + i] = xs[i]; else out.tgt[i] = xs[i];
            for (int j = 0; j < 6; ++j) {
                if (k >= 0) out.Cs[36 * k + 6 * i + j] = Cs[i][j]; else out.tgt_cov[i][j] = Cs[i][j];
            }
        }
    }
    out.chi2 = chi2;
    return out.status = ST_OK;
}

// Filter + smoother; with a perigee target the fitted state on the seed
// surface is then propagated to the perigee, its covariance with that
// transport's Jacobian.  A failure there fails the track (NaN outputs).
template <class S>
int fit_track(const FieldDef& f, const Cfg& cfg, const Surf<S>* surf, int n_surf,
              int n, const int* sid, const S* m /*[n][2]*/, const double* V3 /*[n][3]*/,
              const S* seed /*6*/, const double* seed_cov21, int seed_sid, TrackOut<S>& out) {
    int st = fit_track_seed_surface(f, cfg, surf, n_surf, n, sid, m, V3, seed, seed_cov21, seed_sid, out);
    if (st != ST_OK || cfg.target != 1) return st;
    S xo[6], Fp[6][6], T1[6][6], Ft[6][6], Cp[6][6];
    int trials = 0;
    st = transport_perigee(f, cfg, surf[seed_sid], cfg.perigee, out.tgt, xo, Fp, &trials);
    if (st != ST_OK) {
        for (auto& v : out.xs) v = S(NAN);
        for (auto& v : out.Cs) v = S(NAN);
        for (int i = 0; i < 6; ++i) { out.tgt[i] = NAN; for (int j = 0; j < 6; ++j) out.tgt_cov[i][j] = NAN; }
        out.chi2 = NAN;
        return out.status = st;
    }
    matmul(Fp, out.tgt_cov, T1);
    transpose(Fp, Ft);
    matmul(T1, Ft, Cp);
    for (int i = 0; i < 6; ++i) {
        out.tgt[i] = xo[i];
        for (int j = 0; j < 6; ++j) out.tgt_cov[i][j] = Cp[i][j];
    }
    return ST_OK;
}

// alignment a = (dx, dy, dz, alpha, beta, gamma): c <- c + d, R <- R Rx(alpha) Ry(beta) Rz(gamma)
template <class S>
void aligned_surface(const Surf<double>& s0, const S a[6], Surf<S>& o) {
    for (int i = 0; i < 3; ++i) o.c[i] = s0.c[i] + a[i];
    S ca = cos(a[3]), sa = sin(a[3]), cb = cos(a[4]), sb = sin(a[4]), cg = cos(a[5]), sg = sin(a[5]);
    S Rx[3][3] = {{1.0, 0.0, 0.0}, {0.0, ca, -sa}, {0.0, sa, ca}};
    S Ry[3][3] = {{cb, 0.0, sb}, {0.0, 1.0, 0.0}, {-sb, 0.0, cb}};
    S Rz[3][3] = {{cg, -sg, 0.0}, {sg, cg, 0.0}, {0.0, 0.0, 1.0}};
    S R0[3][3], T1[3][3], T2[3][3], R[3][3];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) R0[i][j] = s0.R[i][j];
    matmul(R0, Rx, T1);
    matmul(T1, Ry, T2);
    matmul(T2, Rz, R);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) o.R[i][j] = R[i][j];
    o.x0 = s0.x0;
    o.type = s0.type;
    o.radius = s0.radius;
}


// ---------------------------------------------------------------------------
// glue: SoA component-major arrays <-> one track
// ---------------------------------------------------------------------------
struct Inputs {
    int n_tracks; const int32_t* off; const int32_t* sid; const double* loc; const double* cov; int64_t H;
    int n_surf; const double* center; const double* rot; const double* x0;
    const double* align;   // [6][S] alignment corrections or NULL
    FieldDef field; const double* seed; const double* seed_cov; int seed_sid;
    Cfg cfg;
    const int32_t* stype = nullptr;   // [S] surface types (0 plane, 1 disc) or NULL (all planes)
};

// Cylinder radii of the surfaces (set by kfo_set_surface_radius; like the
// field map, one table for every call until it is replaced).
static const double* g_radius = nullptr;
static int g_radius_n = 0;

// nominal surface s (before any alignment correction)
inline Surf<double> surf_nominal(const Inputs& in, int s) {
    Surf<double> o;
    for (int i = 0; i < 3; ++i) o.c[i] = in.center[i * in.n_surf + s];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) o.R[i][j] = in.rot[(3 * i + j) * in.n_surf + s];
    o.x0 = in.x0[s];
    o.type = in.stype ? in.stype[s] : 0;
    o.radius = (g_radius && s < g_radius_n) ? g_radius[s] : 0.0;
    return o;
}

// alignment correction of surface s (zero without an alignment input)
inline void align_of(const Inputs& in, int s, double a[6]) {
    for (int c = 0; c < 6; ++c) a[c] = in.align ? in.align[c * in.n_surf + s] : 0.0;
}

// surface s as fitted: the nominal one with its alignment correction applied
inline Surf<double> surf_d(const Inputs& in, int s) {
    Surf<double> o = surf_nominal(in, s);
    if (!in.align) return o;
    double a[6];
    align_of(in, s, a);
    Surf<double> r;
    aligned_surface(o, a, r);
    return r;
}

inline bool field_nonzero(const FieldDef& f) {
    return f.kind != 0 || f.b0[0] != 0.0 || f.b0[1] != 0.0 || f.b0[2] != 0.0;
}

}  // namespace kfo

using namespace kfo;

// The tabulated field that field kind 2 refers to (set by kfo_set_field_map;
// the caller keeps the array alive while it is in use).
static FieldMap g_map = {{0, 0, 0}, {0.0, 0.0, 0.0}, {1.0, 1.0, 1.0}, nullptr};

static Inputs make_inputs(int n_tracks, const int32_t* off, const int32_t* sid, const double* loc,
                          const double* cov, int n_surf, const double* center, const double* rot,
                          const double* x0, const double* align, int field_kind, const double* b0,
                          double field_a, const double* seed, const double* seed_cov, int seed_sid, int ms,
                          double mass, double tol, double land_tol, int max_steps) {
    Inputs in;
    in.n_tracks = n_tracks; in.off = off; in.sid = sid; in.loc = loc; in.cov = cov;
    in.H = off ? off[n_tracks] : 0;
    in.n_surf = n_surf; in.center = center; in.rot = rot; in.x0 = x0; in.align = align;
    in.field.kind = field_kind;
    in.field.map = &g_map;
    for (int i = 0; i < 3; ++i) in.field.b0[i] = b0[i];
    in.field.a = field_a;
    in.seed = seed; in.seed_cov = seed_cov; in.seed_sid = seed_sid;
    in.cfg.ms = ms; in.cfg.mass = mass; in.cfg.tol = tol; in.cfg.land_tol = land_tol; in.cfg.max_steps = max_steps;
    return in;
}

static const int PACK_I[21] = {0,0,0,0,0,0,1,1,1,1,1,2,2,2,2,3,3,3,4,4,5};
static const int PACK_J[21] = {0,1,2,3,4,5,1,2,3,4,5,2,3,4,5,3,4,5,4,5,5};

extern "C" {

const char* kfo_version() { return "kf-oracle fp64 1"; }

// The map of field kind 2: n[3] grid points per axis (>= 2), origin[3],
// spacing[3] (mm), values [n2][n1][n0][3] (T), kept alive by the caller.
int kfo_set_field_map(const int32_t* n, const double* origin, const double* spacing, const double* values) {
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 2 || !(spacing[a] > 0.0)) return 1;
        g_map.n[a] = n[a]; g_map.origin[a] = origin[a]; g_map.spacing[a] = spacing[a];
    }
    g_map.values = values;
    return 0;
}

// Cylinder radii per surface ([n], kept alive by the caller; NULL: none).
int kfo_set_surface_radius(int n, const double* radius) {
    g_radius = radius;
    g_radius_n = radius ? n : 0;
    return 0;
}

// Full fit of every track.  Arrays are component-major ([component][item]).
// Optional outputs may be NULL.  smoother: 0 RTS, 1 two-filter (bwd_scale:
// inflation of the backward filter's starting covariance).  target: 0 seed
// surface, 1 perigee line through `perigee` (3 values) parallel to z.
// Returns 0.
int kfo_fit(int n_tracks, const int32_t* off, const int32_t* sid, const double* loc, const double* cov,
            int n_surf, const double* center, const double* rot, const double* x0, const double* align,
            int field_kind, const double* b0, double field_a,
            const double* seed, const double* seed_cov, int seed_sid,
            int ms, double mass, double tol, double land_tol, int max_steps,
            double* par, double* pcov, double* tgt_par, double* tgt_cov, double* chi2, int32_t* ndf,
            uint8_t* status, double* filt_par, double* filt_cov, double* pred_par, double* pred_cov,
            int32_t* trials, int n_threads, int smoother, double bwd_scale, int target, const double* perigee,
            const int32_t* stype) {
    Inputs in = make_inputs(n_tracks, off, sid, loc, cov, n_surf, center, rot, x0, align, field_kind, b0, field_a,
                            seed, seed_cov, seed_sid, ms, mass, tol, land_tol, max_steps);
    in.cfg.smoother = smoother;
    in.cfg.bwd_scale = bwd_scale;
    in.cfg.target = target;
    for (int i = 0; i < 3; ++i) in.cfg.perigee[i] = perigee ? perigee[i] : 0.0;
    in.stype = stype;
    std::vector<Surf<double>> surf(n_surf);
    for (int s = 0; s < n_surf; ++s) surf[s] = surf_d(in, s);
    const int64_t H = in.H;
    const int N = n_tracks;
    const bool bnz = field_nonzero(in.field);
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
    for (int t = 0; t < N; ++t) {
        const int o = off[t], n = off[t + 1] - off[t];
        std::vector<double> m(2 * std::max(n, 0)), V(3 * std::max(n, 0));
        for (int k = 0; k < n; ++k) {
            m[2 * k] = loc[o + k]; m[2 * k + 1] = loc[H + o + k];
            for (int a = 0; a < 3; ++a) V[3 * k + a] = cov[a * H + o + k];
        }
        double sd[6], sc[21];
        for (int i = 0; i < 6; ++i) sd[i] = seed[i * N + t];
        for (int i = 0; i < 21; ++i) sc[i] = seed_cov[i * N + t];
        TrackOut<double> r;
        fit_track(in.field, in.cfg, surf.data(), n_surf, n, sid + o, m.data(), V.data(), sd, sc, seed_sid, r);
        for (int k = 0; k < n; ++k) {
            for (int i = 0; i < 6; ++i) {
                par[i * H + o + k] = r.xs[6 * k + i];
                if (filt_par) filt_par[i * H + o + k] = r.xf[6 * k + i];
                if (pred_par) pred_par[i * H + o + k] = r.xp[6 * k + i];
            }
            for (int q = 0; q < 21; ++q) {
                const int e = 6 * PACK_I[q] + PACK_J[q];
                pcov[q * H + o + k] = r.Cs[36 * k + e];
                if (filt_cov) filt_cov[q * H + o + k] = r.Cf[36 * k + e];
                if (pred_cov) pred_cov[q * H + o + k] = r.Cp[36 * k + e];
            }
            if (trials) trials[o + k] = r.trials[k];
        }
        for (int i = 0; i < 6; ++i) tgt_par[i * N + t] = r.tgt[i];
        for (int q = 0; q < 21; ++q) tgt_cov[q * N + t] = r.tgt_cov[PACK_I[q]][PACK_J[q]];
        chi2[t] = r.chi2;
        int dims = 0;     // measured coordinates: two per hit, one on a line
        for (int k = 0; k < n; ++k) {
            const int sk = sid[o + k];
            dims += (sk >= 0 && sk < n_surf) ? meas_dim(surf[sk].type) : 2;
        }
        ndf[t] = dims - (bnz ? 5 : 4);
        status[t] = (uint8_t)r.status;
    }
    return 0;
}

// One bound-to-bound transport x (on surface a) -> xo (on surface b); F = dxo/dx.
// Returns the status; trials receives the number of RKN trials.
int kfo_transport(int n_surf, const double* center, const double* rot, const double* x0,
                  int field_kind, const double* b0, double field_a, double mass, double tol,
                  double land_tol, int max_steps, int sa, int sb, const double* x, double* xo,
                  double* F, int32_t* trials, const int32_t* stype) {
    Inputs in = make_inputs(0, nullptr, nullptr, nullptr, nullptr, n_surf, center, rot, x0, nullptr, field_kind, b0,
                            field_a, nullptr, nullptr, 0, 0, mass, tol, land_tol, max_steps);
    in.stype = stype;
    Surf<double> A = surf_d(in, sa), B = surf_d(in, sb);
    double xi[6], xr[6], Fk[6][6];
    for (int i = 0; i < 6; ++i) xi[i] = x[i];
    int tr = 0;
    int st = transport(in.field, in.cfg, A, B, xi, xr, Fk, &tr);
    for (int i = 0; i < 6; ++i) { xo[i] = xr[i]; for (int j = 0; j < 6; ++j) F[6 * i + j] = Fk[i][j]; }
    *trials = tr;
    return st;
}

// Plane surface sa -> perigee line through c parallel to z; F = dxo/dx.
int kfo_transport_perigee(int n_surf, const double* center, const double* rot, const double* x0,
                          int field_kind, const double* b0, double field_a, double mass, double tol,
                          double land_tol, int max_steps, int sa, const double* c, const double* x, double* xo,
                          double* F, int32_t* trials) {
    Inputs in = make_inputs(0, nullptr, nullptr, nullptr, nullptr, n_surf, center, rot, x0, nullptr, field_kind, b0,
                            field_a, nullptr, nullptr, 0, 0, mass, tol, land_tol, max_steps);
    Surf<double> A = surf_d(in, sa);
    double xi[6], xr[6], Fk[6][6], cc[3] = {c[0], c[1], c[2]};
    for (int i = 0; i < 6; ++i) xi[i] = x[i];
    int tr = 0;
    int st = transport_perigee(in.field, in.cfg, A, cc, xi, xr, Fk, &tr);
    for (int i = 0; i < 6; ++i) { xo[i] = xr[i]; for (int j = 0; j < 6; ++j) F[6 * i + j] = Fk[i][j]; }
    *trials = tr;
    return st;
}

// The field and its gradient dB[a][b] = dB_a/dr_b at r (kind 2: the map set
// by kfo_set_field_map).
void kfo_field_at(int field_kind, const double* b0, double field_a, const double* r, double* B, double* dB) {
    FieldDef f; f.kind = field_kind; for (int i = 0; i < 3; ++i) f.b0[i] = b0[i]; f.a = field_a; f.map = &g_map;
    double rr[3] = {r[0], r[1], r[2]}, Bo[3], dBo[3][3];
    field_at(f, rr, Bo, dBo);
    for (int i = 0; i < 3; ++i) { B[i] = Bo[i]; for (int j = 0; j < 3; ++j) dB[3 * i + j] = dBo[i][j]; }
}

// One RKN step of the free state at fixed h; D = d(step map)/dF.  Returns err.
double kfo_rkn_step(int field_kind, const double* b0, double field_a, double mass, const double* F,
                    double h, double* Fn, double* D) {
    FieldDef f; f.kind = field_kind; for (int i = 0; i < 3; ++i) f.b0[i] = b0[i]; f.a = field_a; f.map = &g_map;
    double Fi[8], Fo[8], Dm[8][8];
    for (int i = 0; i < 8; ++i) Fi[i] = F[i];
    double e = rkn_step(f, mass, Fi, h, Fo, Dm);
    for (int i = 0; i < 8; ++i) { Fn[i] = Fo[i]; for (int j = 0; j < 8; ++j) D[8 * i + j] = Dm[i][j]; }
    return e;
}

// Linear-Gaussian core: states 0..n, x_{k+1} = F_k (x_k + w_k), w_k ~ N(0, Q_k),
// measurements m_k = H x_k + v_k for k = 1..n, H = [I2 0].  Runs the same
// update and RTS routines as the track fit with the prediction x_{k+1|k} = F_k x_{k|k}.
// F, Q: [n][6][6]; m: [n][2]; V: [n][3]; x0: 6; C0: [6][6].
// Outputs xs: [n+1][6], Cs: [n+1][6][6], xf: [n][6], Cf: [n][6][6], chi2: [n].
int kfo_linear_smoother(int n, const double* Fin, const double* Qin, const double* m, const double* V3,
                        const double* x0, const double* C0, double* xs_out, double* Cs_out, double* xf_out,
                        double* Cf_out, double* chi2_out) {
    std::vector<double> xf(6 * (n + 1)), Cf(36 * (n + 1)), xp(6 * (n + 1)), Cp(36 * (n + 1));
    for (int i = 0; i < 6; ++i) xf[i] = x0[i];
    for (int i = 0; i < 36; ++i) Cf[i] = C0[i];
    for (int k = 0; k < n; ++k) {
        double F[6][6], Q[6][6], C[6][6], x[6];
        for (int i = 0; i < 6; ++i) { x[i] = xf[6 * k + i]; for (int j = 0; j < 6; ++j) { F[i][j] = Fin[36 * k + 6 * i + j]; Q[i][j] = Qin[36 * k + 6 * i + j]; C[i][j] = Cf[36 * k + 6 * i + j] + Q[i][j]; } }
        double xpk[6], T1[6][6], Ft[6][6], Cpk[6][6];
        for (int i = 0; i < 6; ++i) { double a = 0; for (int j = 0; j < 6; ++j) a += F[i][j] * x[j]; xpk[i] = a; }
        matmul(F, C, T1); transpose(F, Ft); matmul(T1, Ft, Cpk);
        double mk[2] = {m[2 * k], m[2 * k + 1]};
        double V[2][2] = {{V3[3 * k], V3[3 * k + 1]}, {V3[3 * k + 1], V3[3 * k + 2]}};
        double xn[6], Cn[6][6], c2;
        int st = kalman_update(xpk, Cpk, mk, V, xn, Cn, &c2);
        if (st) return st;
        chi2_out[k] = c2;
        for (int i = 0; i < 6; ++i) {
            xp[6 * (k + 1) + i] = xpk[i]; xf[6 * (k + 1) + i] = xn[i];
            for (int j = 0; j < 6; ++j) { Cp[36 * (k + 1) + 6 * i + j] = Cpk[i][j]; Cf[36 * (k + 1) + 6 * i + j] = Cn[i][j]; }
        }
    }
    std::vector<double> xs(6 * (n + 1)), Cs(36 * (n + 1));
    for (int i = 0; i < 6; ++i) xs[6 * n + i] = xf[6 * n + i];
    for (int i = 0; i < 36; ++i) Cs[36 * n + i] = Cf[36 * n + i];
    for (int k = n - 1; k >= 0; --k) {
        double a[6], A[6][6], F[6][6], b[6], B[6][6], c[6], Cc[6][6], o[6], O[6][6];
        for (int i = 0; i < 6; ++i) {
            a[i] = xf[6 * k + i]; b[i] = xp[6 * (k + 1) + i]; c[i] = xs[6 * (k + 1) + i];
            for (int j = 0; j < 6; ++j) {
                A[i][j] = Cf[36 * k + 6 * i + j]; F[i][j] = Fin[36 * k + 6 * i + j];
                B[i][j] = Cp[36 * (k + 1) + 6 * i + j]; Cc[i][j] = Cs[36 * (k + 1) + 6 * i + j];
            }
        }
        int st = rts_step(a, A, F, b, B, c, Cc, o, O);
        if (st) return st;
        for (int i = 0; i < 6; ++i) { xs[6 * k + i] = o[i]; for (int j = 0; j < 6; ++j) Cs[36 * k + 6 * i + j] = O[i][j]; }
    }
    for (int i = 0; i < 6 * (n + 1); ++i) xs_out[i] = xs[i];
    for (int i = 0; i < 36 * (n + 1); ++i) Cs_out[i] = Cs[i];
    for (int k = 0; k < n; ++k) {
        for (int i = 0; i < 6; ++i) xf_out[6 * k + i] = xf[6 * (k + 1) + i];
        for (int i = 0; i < 36; ++i) Cf_out[36 * k + i] = Cf[36 * (k + 1) + i];
    }
    return 0;
}

// The same linear model smoothed by the two-filter routines of the track fit:
// forward filter as above; backward filter started from (xf_n, scale Cf_n),
// backward prediction x_{k|k+1} = G_k x_{k+1}, C = G_k C G_k^T + Q_k (G_k is
// the inverse of F_k, given), combined with x_{k|k} by two_filter_combine.
// G: [n][6][6]; outputs xs: [n+1][6], Cs: [n+1][6][6].
int kfo_linear_two_filter(int n, const double* Fin, const double* Gin, const double* Qin, const double* m,
                          const double* V3, const double* x0, const double* C0, double scale, double* xs_out,
                          double* Cs_out) {
    std::vector<double> xs_r(6 * (n + 1)), Cs_r(36 * (n + 1)), xf(6 * n), Cf(36 * n), chi2(n);
    int st = kfo_linear_smoother(n, Fin, Qin, m, V3, x0, C0, xs_r.data(), Cs_r.data(), xf.data(), Cf.data(),
                                 chi2.data());
    if (st) return st;
    // state n: the filtered state
    for (int i = 0; i < 6; ++i) xs_out[6 * n + i] = xf[6 * (n - 1) + i];
    for (int i = 0; i < 36; ++i) Cs_out[36 * n + i] = Cf[36 * (n - 1) + i];
    double xb[6], Cb[6][6];
    {
        double xl[6], Cl[6][6], c2;
        for (int i = 0; i < 6; ++i) {
            xl[i] = xf[6 * (n - 1) + i];
            for (int j = 0; j < 6; ++j) Cl[i][j] = scale * Cf[36 * (n - 1) + 6 * i + j];
        }
        double mk[2] = {m[2 * (n - 1)], m[2 * (n - 1) + 1]};
        const double* v = V3 + 3 * (n - 1);
        double V[2][2] = {{v[0], v[1]}, {v[1], v[2]}};
        st = kalman_update(xl, Cl, mk, V, xb, Cb, &c2);
        if (st) return st;
    }
    for (int k = n - 1; k >= 0; --k) {
        double G[6][6], Q[6][6], Cq[6][6], xq[6], a[6], A[6][6], o[6], O[6][6];
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) { G[i][j] = Gin[36 * k + 6 * i + j]; Q[i][j] = Qin[36 * k + 6 * i + j]; }
        for (int i = 0; i < 6; ++i) { double acc = 0; for (int j = 0; j < 6; ++j) acc += G[i][j] * xb[j]; xq[i] = acc; }
        backward_predict(G, Q, Cb, Cq);
        for (int i = 0; i < 6; ++i) {
            a[i] = k > 0 ? xf[6 * (k - 1) + i] : x0[i];
            for (int j = 0; j < 6; ++j) A[i][j] = k > 0 ? Cf[36 * (k - 1) + 6 * i + j] : C0[6 * i + j];
        }
        st = two_filter_combine(a, A, xq, Cq, o, O);
        if (st) return st;
        for (int i = 0; i < 6; ++i) { xs_out[6 * k + i] = o[i]; for (int j = 0; j < 6; ++j) Cs_out[36 * k + 6 * i + j] = O[i][j]; }
        if (k > 0) {
            double mk[2] = {m[2 * (k - 1)], m[2 * (k - 1) + 1]};
            const double* v = V3 + 3 * (k - 1);
            double V[2][2] = {{v[0], v[1]}, {v[1], v[2]}};
            double c2;
            st = kalman_update(xq, Cq, mk, V, xb, Cb, &c2);
            if (st) return st;
        }
    }
    return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// gradients by forward-mode dual numbers
// ---------------------------------------------------------------------------
namespace kfo {

static const int ND = 8;   // directions per dual pass
using D8 = Dual<ND>;

}  // namespace kfo

extern "C" {

// Vector-Jacobian product of L = sum_t g_chi2[t] chi2_t + sum_hits g_par . smoothed
//                                + sum_t g_tgt . target
// with respect to the measurements (g_meas [2][H]), the alignment correction
// (dx, dy, dz, alpha, beta, gamma) of every surface at its given value (align,
// zero if NULL) (g_align [6][S]) and the seed parameters (g_seed [6][N]).
// Each entry is an exact directional derivative (Dual numbers) of the fit.
// g_par, g_tgt, g_seed may be NULL.  Tracks whose fit fails contribute nothing.
int kfo_fit_vjp(int n_tracks, const int32_t* off, const int32_t* sid, const double* loc, const double* cov,
                int n_surf, const double* center, const double* rot, const double* x0, const double* align,
                int field_kind, const double* b0, double field_a,
                const double* seed, const double* seed_cov, int seed_sid,
                int ms, double mass, double tol, double land_tol, int max_steps,
                const double* g_chi2, const double* g_par, const double* g_tgt,
                double* g_meas, double* g_align, double* g_seed, int n_threads, const int32_t* stype) {
    Inputs in = make_inputs(n_tracks, off, sid, loc, cov, n_surf, center, rot, x0, align, field_kind, b0, field_a,
                            seed, seed_cov, seed_sid, ms, mass, tol, land_tol, max_steps);
    in.stype = stype;
    // derivatives are taken with respect to the alignment correction itself:
    // every pass rebuilds each surface from its nominal placement
    std::vector<Surf<double>> surf(n_surf);
    std::vector<double> a0(6 * n_surf);
    for (int s = 0; s < n_surf; ++s) { surf[s] = surf_nominal(in, s); align_of(in, s, &a0[6 * s]); }
    const int64_t H = in.H;
    const int N = n_tracks;
    for (int i = 0; i < 6 * n_surf; ++i) g_align[i] = 0.0;
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
    {
        std::vector<double> ga(6 * n_surf, 0.0);
#pragma omp for schedule(dynamic, 4)
        for (int t = 0; t < N; ++t) {
            const int o = off[t], n = off[t + 1] - off[t];
            // direction list: (kind, index, component); kind 0 meas, 1 align, 2 seed
            std::vector<int> used;
            used.push_back(seed_sid);
            for (int k = 0; k < n; ++k) used.push_back(sid[o + k]);
            std::sort(used.begin(), used.end());
            used.erase(std::unique(used.begin(), used.end()), used.end());
            struct Dir { int kind, idx, comp; };
            std::vector<Dir> dirs;
            for (int k = 0; k < n; ++k) for (int a = 0; a < 2; ++a) dirs.push_back({0, k, a});
            for (int s : used) for (int c = 0; c < 6; ++c) dirs.push_back({1, s, c});
            for (int c = 0; c < 6; ++c) dirs.push_back({2, 0, c});
            std::vector<double> V(3 * n);
            for (int k = 0; k < n; ++k) for (int a = 0; a < 3; ++a) V[3 * k + a] = cov[a * H + o + k];
            double sc[21];
            for (int i = 0; i < 21; ++i) sc[i] = seed_cov[i * N + t];
            bool failed = false;
            for (size_t d0 = 0; d0 < dirs.size() && !failed; d0 += ND) {
                std::vector<D8> m(2 * n);
                for (int k = 0; k < n; ++k) { m[2 * k] = loc[o + k]; m[2 * k + 1] = loc[H + o + k]; }
                D8 sd[6];
                for (int i = 0; i < 6; ++i) sd[i] = seed[i * N + t];
                std::vector<D8> al(6 * n_surf);
                for (int i = 0; i < 6 * n_surf; ++i) al[i] = a0[i];
                for (size_t q = 0; q < ND && d0 + q < dirs.size(); ++q) {
                    const Dir& d = dirs[d0 + q];
                    if (d.kind == 0) m[2 * d.idx + d.comp].d[q] = 1.0;
                    else if (d.kind == 1) al[6 * d.idx + d.comp].d[q] = 1.0;
                    else sd[d.comp].d[q] = 1.0;
                }
                std::vector<Surf<D8>> S8(n_surf);
                for (int s = 0; s < n_surf; ++s) aligned_surface(surf[s], &al[6 * s], S8[s]);
                TrackOut<D8> r;
                int st = fit_track(in.field, in.cfg, S8.data(), n_surf, n, sid + o, m.data(), V.data(), sd, sc,
                                   seed_sid, r);
                if (st != ST_OK) { failed = true; break; }
                for (size_t q = 0; q < ND && d0 + q < dirs.size(); ++q) {
                    double L = g_chi2 ? g_chi2[t] * r.chi2.d[q] : 0.0;
                    if (g_par)
                        for (int k = 0; k < n; ++k) for (int i = 0; i < 6; ++i) L += g_par[i * H + o + k] * r.xs[6 * k + i].d[q];
                    if (g_tgt) for (int i = 0; i < 6; ++i) L += g_tgt[i * N + t] * r.tgt[i].d[q];
                    const Dir& d = dirs[d0 + q];
                    if (d.kind == 0) g_meas[d.comp * H + o + d.idx] = L;
                    else if (d.kind == 1) ga[6 * d.idx + d.comp] += L;   // local layout [s][c]
                    else if (g_seed) g_seed[d.comp * N + t] = L;
                }
            }
            if (failed) {
                for (int k = 0; k < n; ++k) { g_meas[o + k] = NAN; g_meas[H + o + k] = NAN; }
                if (g_seed) for (int c = 0; c < 6; ++c) g_seed[c * N + t] = NAN;
            }
        }
#pragma omp critical
        for (int s = 0; s < n_surf; ++s) for (int c = 0; c < 6; ++c) g_align[c * n_surf + s] += ga[6 * s + c];
    }
    return 0;
}

// Non-trivial floating-point operations of the fit of each track.
// counts: [N][5] = add/sub, mul, div, sqrt, transcendental (sin, cos, atan2, log).
int kfo_count_ops(int n_tracks, const int32_t* off, const int32_t* sid, const double* loc, const double* cov,
                  int n_surf, const double* center, const double* rot, const double* x0, const double* align,
                  int field_kind, const double* b0, double field_a,
                  const double* seed, const double* seed_cov, int seed_sid,
                  int ms, double mass, double tol, double land_tol, int max_steps, int64_t* counts,
                  const int32_t* stype) {
    Inputs in = make_inputs(n_tracks, off, sid, loc, cov, n_surf, center, rot, x0, align, field_kind, b0, field_a,
                            seed, seed_cov, seed_sid, ms, mass, tol, land_tol, max_steps);
    in.stype = stype;
    std::vector<Surf<Cnt>> surf(n_surf);
    for (int s = 0; s < n_surf; ++s) {
        Surf<double> d = surf_d(in, s);
        for (int i = 0; i < 3; ++i) surf[s].c[i] = d.c[i];
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) surf[s].R[i][j] = d.R[i][j];
        surf[s].x0 = d.x0;
        surf[s].type = d.type;
        surf[s].radius = d.radius;
    }
    const int64_t H = in.H;
    for (int t = 0; t < n_tracks; ++t) {
        const int o = off[t], n = off[t + 1] - off[t];
        std::vector<Cnt> m(2 * n);
        std::vector<double> V(3 * n);
        for (int k = 0; k < n; ++k) {
            m[2 * k] = loc[o + k]; m[2 * k + 1] = loc[H + o + k];
            for (int a = 0; a < 3; ++a) V[3 * k + a] = cov[a * H + o + k];
        }
        Cnt sd[6]; double sc[21];
        for (int i = 0; i < 6; ++i) sd[i] = seed[i * n_tracks + t];
        for (int i = 0; i < 21; ++i) sc[i] = seed_cov[i * n_tracks + t];
        g_cnt = Counts();
        TrackOut<Cnt> r;
        fit_track(in.field, in.cfg, surf.data(), n_surf, n, sid + o, m.data(), V.data(), sd, sc, seed_sid, r);
        counts[5 * t + 0] = g_cnt.add; counts[5 * t + 1] = g_cnt.mul; counts[5 * t + 2] = g_cnt.div;
        counts[5 * t + 3] = g_cnt.sqrt; counts[5 * t + 4] = g_cnt.trans;
    }
    return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// operation counts of single routines (pins of the counting scalar)
// ---------------------------------------------------------------------------
namespace kfo {
inline void put_counts(int64_t* counts) {
    counts[0] = g_cnt.add; counts[1] = g_cnt.mul; counts[2] = g_cnt.div;
    counts[3] = g_cnt.sqrt; counts[4] = g_cnt.trans;
}
}  // namespace kfo

extern "C" {

// Counts of one gain-matrix update (H = [I2 0]): xp[6], Cp[6][6], m[2], V
// (v00, v01, v11).  counts[5] as kfo_count_ops.  Returns the update's status.
int kfo_count_update(const double* xp, const double* Cp, const double* m, const double* V3, int64_t* counts) {
    Cnt x[6], C[6][6], mm[2] = {m[0], m[1]}, V[2][2] = {{V3[0], V3[1]}, {V3[1], V3[2]}}, xf[6], Cf[6][6], c2;
    for (int i = 0; i < 6; ++i) { x[i] = xp[i]; for (int j = 0; j < 6; ++j) C[i][j] = Cp[6 * i + j]; }
    g_cnt = Counts();
    int st = kalman_update(x, C, mm, V, xf, Cf, &c2);
    put_counts(counts);
    return st;
}

// Counts of one RTS step: the filtered state (xf, Cf) of k, the transport F
// from k to k+1, the prediction (xp1, Cp1) and the smoothed state (xs1, Cs1)
// of k+1 (6 / 36 values each, row-major).
int kfo_count_rts_step(const double* xf, const double* Cf, const double* F, const double* xp1, const double* Cp1,
                       const double* xs1, const double* Cs1, int64_t* counts) {
    Cnt a[6], A[6][6], Fm[6][6], b[6], B[6][6], c[6], Cc[6][6], xs[6], Cs[6][6];
    for (int i = 0; i < 6; ++i) {
        a[i] = xf[i]; b[i] = xp1[i]; c[i] = xs1[i];
        for (int j = 0; j < 6; ++j) {
            A[i][j] = Cf[6 * i + j]; Fm[i][j] = F[6 * i + j]; B[i][j] = Cp1[6 * i + j]; Cc[i][j] = Cs1[6 * i + j];
        }
    }
    g_cnt = Counts();
    int st = rts_step(a, A, Fm, b, B, c, Cc, xs, Cs);
    put_counts(counts);
    return st;
}

// Counts of one bound-to-bound transport (arguments as kfo_transport).
int kfo_count_transport(int n_surf, const double* center, const double* rot, const double* x0, int field_kind,
                        const double* b0, double field_a, double mass, double tol, double land_tol, int max_steps,
                        int sa, int sb, const double* x, int32_t* trials, const int32_t* stype, int64_t* counts) {
    Inputs in = make_inputs(0, nullptr, nullptr, nullptr, nullptr, n_surf, center, rot, x0, nullptr, field_kind, b0,
                            field_a, nullptr, nullptr, 0, 0, mass, tol, land_tol, max_steps);
    in.stype = stype;
    Surf<Cnt> A, B;
    for (int k = 0; k < 2; ++k) {
        Surf<double> d = surf_d(in, k == 0 ? sa : sb);
        Surf<Cnt>& o = k == 0 ? A : B;
        for (int i = 0; i < 3; ++i) o.c[i] = d.c[i];
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) o.R[i][j] = d.R[i][j];
        o.x0 = d.x0;
        o.type = d.type;
        o.radius = d.radius;
    }
    Cnt xi[6], xr[6], Fk[6][6];
    for (int i = 0; i < 6; ++i) xi[i] = x[i];
    int tr = 0;
    g_cnt = Counts();
    int st = transport(in.field, in.cfg, A, B, xi, xr, Fk, &tr);
    put_counts(counts);
    *trials = tr;
    return st;
}

// Counts of the thin-scatterer noise of surface s for the bound state x.
int kfo_count_ms_noise(int n_surf, const double* center, const double* rot, const double* x0, int s,
                       const double* x, double mass, int64_t* counts) {
    Inputs in = make_inputs(0, nullptr, nullptr, nullptr, nullptr, n_surf, center, rot, x0, nullptr, 0, center, 0.0,
                            nullptr, nullptr, 0, 1, mass, 0.0, 0.0, 0);
    Surf<double> d = surf_d(in, s);
    Surf<Cnt> sf;
    for (int i = 0; i < 3; ++i) sf.c[i] = d.c[i];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) sf.R[i][j] = d.R[i][j];
    sf.x0 = d.x0;
    Cnt xi[6], Q[6][6];
    for (int i = 0; i < 6; ++i) xi[i] = x[i];
    g_cnt = Counts();
    ms_noise(sf, xi, mass, Q);
    put_counts(counts);
    return 0;
}

// Counts of the covariance prediction F (C + Q) F^T as the track fit forms it
// (F, C, Q: 6x6 row-major).
int kfo_count_cov_transport(const double* F, const double* C, const double* Q, int64_t* counts) {
    Cnt Fk[6][6], CQ[6][6], T1[6][6], Ft[6][6], Cp[6][6];
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Fk[i][j] = F[6 * i + j];
    g_cnt = Counts();
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) CQ[i][j] = Cnt(C[6 * i + j]) + Cnt(Q[6 * i + j]);
    matmul(Fk, CQ, T1);
    transpose(Fk, Ft);
    matmul(T1, Ft, Cp);
    put_counts(counts);
    return 0;
}

// Per-unit counts of the fit of track t (RTS smoother, fitted state on the
// seed surface).  The FP64 fit gives the track's states; each unit of the fit
// is then counted on those very states (full, unsymmetrised matrices):
//   units[0] seed covariance check (its Cholesky factor)
//   units[1] scatterer noise        units[2] transport (RKN steps, Jacobian)
//   units[3] F (C + Q) F^T          units[4] gain-matrix update
//   units[5] chi2 sum               units[6] RTS smoother steps
// total receives the count of the whole fit (kfo_count_ops for this track).
// Returns the track's status.
int kfo_count_units(int n_tracks, const int32_t* off, const int32_t* sid, const double* loc, const double* cov,
                    int n_surf, const double* center, const double* rot, const double* x0, const double* align,
                    int field_kind, const double* b0, double field_a,
                    const double* seed, const double* seed_cov, int seed_sid,
                    int ms, double mass, double tol, double land_tol, int max_steps, const int32_t* stype, int t,
                    int64_t* units, int64_t* total) {
    Inputs in = make_inputs(n_tracks, off, sid, loc, cov, n_surf, center, rot, x0, align, field_kind, b0, field_a,
                            seed, seed_cov, seed_sid, ms, mass, tol, land_tol, max_steps);
    in.stype = stype;
    std::vector<Surf<double>> sd(n_surf);
    std::vector<Surf<Cnt>> sc(n_surf);
    for (int s = 0; s < n_surf; ++s) {
        sd[s] = surf_d(in, s);
        for (int i = 0; i < 3; ++i) sc[s].c[i] = sd[s].c[i];
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) sc[s].R[i][j] = sd[s].R[i][j];
        sc[s].x0 = sd[s].x0;
        sc[s].type = sd[s].type;
        sc[s].radius = sd[s].radius;
    }
    const int64_t H = in.H;
    const int o = off[t], n = off[t + 1] - off[t];
    std::vector<double> md(2 * n), V(3 * n);
    std::vector<Cnt> mc(2 * n);
    for (int k = 0; k < n; ++k) {
        md[2 * k] = loc[o + k]; md[2 * k + 1] = loc[H + o + k];
        mc[2 * k] = md[2 * k]; mc[2 * k + 1] = md[2 * k + 1];
        for (int a = 0; a < 3; ++a) V[3 * k + a] = cov[a * H + o + k];
    }
    double xd[6], c21[21];
    Cnt xc[6];
    for (int i = 0; i < 6; ++i) { xd[i] = seed[i * n_tracks + t]; xc[i] = xd[i]; }
    for (int i = 0; i < 21; ++i) c21[i] = seed_cov[i * n_tracks + t];
    for (int u = 0; u < 7 * 5; ++u) units[u] = 0;
    // the whole fit, counted
    g_cnt = Counts();
    TrackOut<Cnt> rc;
    fit_track(in.field, in.cfg, sc.data(), n_surf, n, sid + o, mc.data(), V.data(), xc, c21, seed_sid, rc);
    put_counts(total);
    // the fit's states in FP64
    TrackOut<double> r;
    int st = fit_track(in.field, in.cfg, sd.data(), n_surf, n, sid + o, md.data(), V.data(), xd, c21, seed_sid, r);
    if (st != ST_OK) return st;
    auto add_unit = [&](int u) {
        units[5 * u + 0] += g_cnt.add; units[5 * u + 1] += g_cnt.mul; units[5 * u + 2] += g_cnt.div;
        units[5 * u + 3] += g_cnt.sqrt; units[5 * u + 4] += g_cnt.trans;
        g_cnt = Counts();
    };
    auto to_cnt = [](const double* a36, Cnt (&M)[6][6]) {
        for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) M[i][j] = a36[6 * i + j];
    };
    double C0d[6][6];
    unpack21(c21, C0d);
    Cnt C0[6][6], L0[6][6];
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) C0[i][j] = C0d[i][j];
    g_cnt = Counts();
    cholesky6(C0, L0);
    add_unit(0);
    // forward filter, unit by unit, from the FP64 states
    std::vector<Cnt> Fst(36 * n);
    Cnt chi2 = 0.0;
    for (int k = 0; k < n; ++k) {
        const int prev = k == 0 ? seed_sid : sid[o + k - 1];
        Cnt x[6], C[6][6];
        for (int i = 0; i < 6; ++i) {
            x[i] = k == 0 ? xd[i] : r.xf[6 * (k - 1) + i];
            for (int j = 0; j < 6; ++j) C[i][j] = k == 0 ? C0d[i][j] : r.Cf[36 * (k - 1) + 6 * i + j];
        }
        Cnt Q[6][6];
        if (in.cfg.ms) ms_noise(sc[prev], x, mass, Q);
        else for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Q[i][j] = 0.0;
        add_unit(1);
        Cnt xp[6], Fk[6][6];
        int tr = 0;
        transport(in.field, in.cfg, sc[prev], sc[sid[o + k]], x, xp, Fk, &tr);
        add_unit(2);
        Cnt CQ[6][6], T1[6][6], Ft[6][6], Cp[6][6];
        for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) CQ[i][j] = C[i][j] + Q[i][j];
        matmul(Fk, CQ, T1);
        transpose(Fk, Ft);
        matmul(T1, Ft, Cp);
        add_unit(3);
        Cnt xpk[6], Cpk[6][6], mk[2] = {mc[2 * k], mc[2 * k + 1]};
        for (int i = 0; i < 6; ++i) xpk[i] = r.xp[6 * k + i];
        to_cnt(&r.Cp[36 * k], Cpk);
        const double* v = &V[3 * k];
        Cnt Vk[2][2] = {{v[0], v[1]}, {v[1], v[2]}};
        Cnt xf[6], Cf[6][6], ck;
        update_on(sc[sid[o + k]].type, xpk, Cpk, mk, Vk, xf, Cf, &ck);
        add_unit(4);
        chi2 = chi2 + ck;
        add_unit(5);
        for (int q = 0; q < 36; ++q) Fst[36 * k + q] = Fk[q / 6][q % 6];
    }
    // RTS smoother from the FP64 states
    for (int k = n - 2; k >= -1; --k) {
        Cnt xf[6], Cf[6][6], F[6][6], xp1[6], Cp1[6][6], xs1[6], Cs1[6][6], xs[6], Cs[6][6];
        for (int i = 0; i < 6; ++i) {
            xf[i] = k >= 0 ? r.xf[6 * k + i] : xd[i];
            xp1[i] = r.xp[6 * (k + 1) + i];
            xs1[i] = r.xs[6 * (k + 1) + i];
            for (int j = 0; j < 6; ++j) {
                Cf[i][j] = k >= 0 ? r.Cf[36 * k + 6 * i + j] : C0d[i][j];
                F[i][j] = Fst[36 * (k + 1) + 6 * i + j];
                Cp1[i][j] = r.Cp[36 * (k + 1) + 6 * i + j];
                Cs1[i][j] = r.Cs[36 * (k + 1) + 6 * i + j];
            }
        }
        rts_step(xf, Cf, F, xp1, Cp1, xs1, Cs1, xs, Cs, loc1_is_angle(sc[sid[o + k + 1]].type),
                 k >= 0 && loc1_is_angle(sc[sid[o + k]].type));
        add_unit(6);
    }
    return ST_OK;
}

// Counts of one RKN step of the free state F[8] at fixed h (kfo_rkn_step).
int kfo_count_rkn_step(int field_kind, const double* b0, double field_a, double mass, const double* F, double h,
                       int64_t* counts) {
    FieldDef f; f.kind = field_kind; for (int i = 0; i < 3; ++i) f.b0[i] = b0[i]; f.a = field_a; f.map = &g_map;
    Cnt Fi[8], Fo[8], Dm[8][8];
    for (int i = 0; i < 8; ++i) Fi[i] = F[i];
    g_cnt = Counts();
    rkn_step(f, mass, Fi, Cnt(h), Fo, Dm);
    put_counts(counts);
    return 0;
}

}  // extern "C"

extern "C" {
// Multiple-scattering process noise Q (6x6, row-major) for bound state x on surface s.
int kfo_ms_noise(int n_surf, const double* center, const double* rot, const double* x0, int s,
                 const double* x, double mass, double* Q) {
    Inputs in = make_inputs(0, nullptr, nullptr, nullptr, nullptr, n_surf, center, rot, x0, nullptr, 0, center, 0.0,
                            nullptr, nullptr, 0, 1, mass, 0.0, 0.0, 0);
    Surf<double> sf = surf_d(in, s);
    double xi[6], Qm[6][6];
    for (int i = 0; i < 6; ++i) xi[i] = x[i];
    ms_noise(sf, xi, mass, Qm);
    for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) Q[6 * i + j] = Qm[i][j];
    return 0;
}
}  // extern "C"
