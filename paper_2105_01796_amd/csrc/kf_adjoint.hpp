// kf_adjoint.hpp -- reverse-mode pieces of the track-fit adjoint.
//
// The loss is L = sum_t g_chi2[t] chi2_t + sum_hits g_par . x_smoothed
// + sum_t g_tgt . x_target.  Reverse mode runs back through the RTS smoother
// (Sect. 2), the gain-matrix update, the FP64 smoother-gain solve and the
// covariance transport by hand-derived matrix adjoints below.  The
// propagation (RKN stepping with its transport Jacobian, landing, local <->
// global conversions) is reversed step by step in kf_gap_reverse.hpp; it is
// recomputed, never stored.
//
// Symmetric matrices are held packed (21 entries, sy(i, j)).  The adjoint of
// a symmetric matrix X is kept as the symmetric matrix Xb with
// dL = sum_ij Xb_ij dX_ij over all i, j.
#pragma once
#include "kf_device.hpp"

namespace kfm {

// ---------------------------------------------------------------------------
// gain-matrix update (H = [I2 0]).  In exact arithmetic the Joseph form
// equals Cp - P^T S^-1 P (P = H Cp) for the optimal gain, so its derivative is
// taken from that form:
//   r = m - xp[0:2], S = V + Cp[0:2,0:2], u = S^-1 r,
//   xf = xp + P^T u, Cf = Cp - P^T S^-1 P, chi2 = r^T u.
// In: xfb (6), Cfb (sym), chi2b.  Out: xpb (+=), Cpb (sym, +=), mb (=).
// ---------------------------------------------------------------------------
__device__ inline void update_vjp(const double xp[6], const double Cp[21], const double m[2], const double V[3],
                                  const double xfb[6], const double Cfb[21], double chi2b, double xpb[6],
                                  double Cpb[21], double mb[2]) {
    const double r0 = m[0] - xp[0], r1 = m[1] - xp[1];
    const double S00 = V[0] + Cp[sy(0, 0)], S01 = V[1] + Cp[sy(0, 1)], S11 = V[2] + Cp[sy(1, 1)];
    const double idet = 1.0 / (S00 * S11 - S01 * S01);
    const double I00 = S11 * idet, I01 = -S01 * idet, I11 = S00 * idet;
    const double u0 = I00 * r0 + I01 * r1, u1 = I01 * r0 + I11 * r1;
    double Pm[2][6];
#pragma unroll
    for (int i = 0; i < 6; ++i) { Pm[0][i] = Cp[sy(0, i)]; Pm[1][i] = Cp[sy(1, i)]; }
    // xf = xp + P^T u
    double Pb[2][6];
    double ub0 = 0.0, ub1 = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        xpb[i] += xfb[i];
        Pb[0][i] = u0 * xfb[i];
        Pb[1][i] = u1 * xfb[i];
        ub0 += Pm[0][i] * xfb[i];
        ub1 += Pm[1][i] * xfb[i];
    }
    // chi2 = r^T u
    double rb0 = chi2b * u0, rb1 = chi2b * u1;
    ub0 += chi2b * r0;
    ub1 += chi2b * r1;
    // u = Si r
    rb0 += I00 * ub0 + I01 * ub1;
    rb1 += I01 * ub0 + I11 * ub1;
    double Sib00 = ub0 * r0, Sib01 = ub0 * r1, Sib10 = ub1 * r0, Sib11 = ub1 * r1;
    // Cf = Cp - P^T Si P: Cpb += Cfb; Pb -= 2 Si P Cfb; Sib -= P Cfb P^T
    double PC[2][6];          // P Cfb
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < 6; ++i) acc += Pm[a][i] * Cfb[sy(i, j)];
            PC[a][j] = acc;
        }
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        Pb[0][j] -= 2.0 * (I00 * PC[0][j] + I01 * PC[1][j]);
        Pb[1][j] -= 2.0 * (I01 * PC[0][j] + I11 * PC[1][j]);
    }
    double PCP00 = 0.0, PCP01 = 0.0, PCP11 = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        PCP00 += PC[0][j] * Pm[0][j];
        PCP01 += PC[0][j] * Pm[1][j];
        PCP11 += PC[1][j] * Pm[1][j];
    }
    Sib00 -= PCP00; Sib01 -= PCP01; Sib10 -= PCP01; Sib11 -= PCP11;
#pragma unroll
    for (int q = 0; q < 21; ++q) Cpb[q] += Cfb[q];
    // Si = S^-1: Sb = -Si Sib Si (symmetrised)
    const double T00 = I00 * Sib00 + I01 * Sib10, T01 = I00 * Sib01 + I01 * Sib11;
    const double T10 = I01 * Sib00 + I11 * Sib10, T11 = I01 * Sib01 + I11 * Sib11;
    const double Sb00 = -(T00 * I00 + T01 * I01), Sb11 = -(T10 * I01 + T11 * I11);
    const double Sb01 = -0.5 * ((T00 * I01 + T01 * I11) + (T10 * I00 + T11 * I01));
    // S = V + Cp[0:2,0:2]; P = Cp[0:2,:] (symmetric representative of the block adjoint)
    Cpb[sy(0, 0)] += Sb00 + Pb[0][0];
    Cpb[sy(1, 1)] += Sb11 + Pb[1][1];
    Cpb[sy(0, 1)] += Sb01 + 0.5 * (Pb[0][1] + Pb[1][0]);
#pragma unroll
    for (int i = 2; i < 6; ++i) {
        Cpb[sy(0, i)] += 0.5 * Pb[0][i];
        Cpb[sy(1, i)] += 0.5 * Pb[1][i];
    }
    // r = m - xp[0:2]
    mb[0] = rb0;
    mb[1] = rb1;
    xpb[0] -= rb0;
    xpb[1] -= rb1;
}

// ---------------------------------------------------------------------------
// smoother gain A = C F^T Cp^-1 (Cp = F (C + Q) F^T).  In the smoother the
// gain of the state before hit k only enters as xs = xf + A dx, so its
// adjoint is the outer product Ab = a dx^T (a = adjoint of xs).  With
// w = Cp^-1 dx, z = F^T w, y = C a and u = A^T a:
//   Cb += sym(a z^T),  Fb += w y^T,  Cpb -= sym(u w^T).
// ---------------------------------------------------------------------------
__device__ inline void gain_vjp_rank1(const double a[6], const double w[6], const double z[6], const double y[6],
                                      const double u[6], double Cb[21], double Fb[25], double Cpb[21]) {
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) {
            Cb[sy(i, j)] += (i == j) ? a[i] * z[i] : 0.5 * (a[i] * z[j] + a[j] * z[i]);
            Cpb[sy(i, j)] -= (i == j) ? u[i] * w[i] : 0.5 * (u[i] * w[j] + u[j] * w[i]);
        }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        if (i == 4) continue;
#pragma unroll
        for (int j = 0; j < 5; ++j) Fb[frow(i) * 5 + j] += w[i] * y[j];
    }
}

// z = F^T w (F with the implied q/p row e4 and t column e5)
__device__ inline void ftw(const double F[25], const double w[6], double z[6]) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) acc += fget(F, i, j) * w[i];
        z[j] = acc;
    }
}

// v = F y
__device__ inline void fy(const double F[25], const double y[6], double v[6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) acc += fget(F, i, j) * y[j];
        v[i] = acc;
    }
}

// y = C a (C packed symmetric)
__device__ inline void symv(const double C[21], const double a[6], double y[6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) acc += C[sy(i, j)] * a[j];
        y[i] = acc;
    }
}

// ---------------------------------------------------------------------------
// covariance transport Cp = F CQ F^T:  CQb = F^T Cpb F,  Fb += 2 Cpb F CQ.
// ---------------------------------------------------------------------------
__device__ inline void covtransport_vjp(const double F[25], const double CQ[21], const double Cpb[21],
                                        double Fb[25], double CQb[21]) {
    double W[6][6];           // Cpb F
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) acc += Cpb[sy(i, k)] * fget(F, k, j);
            W[i][j] = acc;
        }
    // CQb = F^T W (symmetric)
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) acc += fget(F, k, i) * W[k][j];
            CQb[sy(i, j)] = acc;
        }
    // Fb += 2 W CQ on the stored entries
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        if (i == 4) continue;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) acc += W[i][k] * CQ[sy(k, j)];
            Fb[frow(i) * 5 + j] += 2.0 * acc;
        }
    }
}

}  // namespace kfm
