// Device helpers of the two-center Slater-Koster model shared by the matrix
// build (sk.hip) and the exact gradient (adjoint.hip): minimum-image
// displacements in the orthorhombic box, the smooth radial factor, the 4x4
// two-center block and contractions of weights with its derivative.
#pragma once

#include "mag_internal.h"

namespace mag {

struct Box {
  double L[3];
};

__device__ __forceinline__ void min_image(const Box& b, double& dx, double& dy, double& dz) {
  dx -= b.L[0] * rint(dx / b.L[0]);
  dy -= b.L[1] * rint(dy / b.L[1]);
  dz -= b.L[2] * rint(dz / b.L[2]);
}

// ---------------------------------------------------------------------------
// two-center blocks and their derivatives
// ---------------------------------------------------------------------------
// quintic smooth step from 1 at r_on to 0 at r_cut, and its derivative
__device__ __forceinline__ void smooth_cutoff(const SKModelDev& m, double r, double& fc,
                                              double& dfc) {
  const double width = m.r_cut - m.r_on;
  const double t = (r - m.r_on) / width;
  if (t <= 0.0) {
    fc = 1.0;
    dfc = 0.0;
  } else if (t >= 1.0) {
    fc = 0.0;
    dfc = 0.0;
  } else {
    const double t2 = t * t, t3 = t2 * t;
    fc = 1.0 - (10.0 * t3 - 15.0 * t3 * t + 6.0 * t3 * t2);
    dfc = -(30.0 * t2 - 60.0 * t3 + 30.0 * t3 * t) / width;
  }
}

__device__ __forceinline__ void radial(const SKModelDev& m, double r, double& u, double& du) {
  double fc, dfc;
  smooth_cutoff(m, r, fc, dfc);
  const double g = (m.r0 / r) * (m.r0 / r);
  const double dg = -2.0 * m.r0 * m.r0 / (r * r * r);
  u = g * fc;
  du = dg * fc + g * dfc;
}

// B (4x4) for displacement d from the row atom to the column atom
__device__ __forceinline__ void two_center(const SKModelDev& m, const double* V, double dx,
                                           double dy, double dz, double B[4][4]) {
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double l[3] = {dx / r, dy / r, dz / r};
  double u, du;
  radial(m, r, u, du);
  B[0][0] = V[0] * u;
  for (int a = 0; a < 3; ++a) {
    B[0][1 + a] = l[a] * V[1] * u;
    B[1 + a][0] = -l[a] * V[1] * u;
    for (int b = 0; b < 3; ++b) {
      const double ll = l[a] * l[b];
      B[1 + a][1 + b] = (ll * V[2] + ((a == b ? 1.0 : 0.0) - ll) * V[3]) * u;
    }
  }
}

// sum_ab G[a][b] dB_ab/dd  (3-vector), for weights G on the block
__device__ __forceinline__ void two_center_contract(const SKModelDev& m, const double* V,
                                                    double dx, double dy, double dz,
                                                    const double G[4][4], double out[3]) {
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double l[3] = {dx / r, dy / r, dz / r};
  double u, du;
  radial(m, r, u, du);
  for (int c = 0; c < 3; ++c) {
    const double dr = l[c];
    double acc = G[0][0] * V[0] * du * dr;
    for (int a = 0; a < 3; ++a) {
      const double dla = ((a == c ? 1.0 : 0.0) - l[a] * l[c]) / r;
      const double sp = dla * V[1] * u + l[a] * V[1] * du * dr;
      acc += G[0][1 + a] * sp - G[1 + a][0] * sp;
      for (int b = 0; b < 3; ++b) {
        const double dlb = ((b == c ? 1.0 : 0.0) - l[b] * l[c]) / r;
        const double ll = l[a] * l[b];
        const double ang = ll * V[2] + ((a == b ? 1.0 : 0.0) - ll) * V[3];
        const double dang = (dla * l[b] + l[a] * dlb) * (V[2] - V[3]);
        acc += G[1 + a][1 + b] * (dang * u + ang * du * dr);
      }
    }
    out[c] = acc;
  }
}

// radial() from r and its reciprocal ri, with the reciprocal width iw of the
// cutoff window: no division (the exact gradient evaluates it once per
// cluster block, row and pass of its contraction)
__device__ __forceinline__ void radial_ri(const SKModelDev& m, double r, double ri, double iw,
                                          double& u, double& du) {
  const double t = (r - m.r_on) * iw;
  double fc = 1.0, dfc = 0.0;
  if (t >= 1.0) {
    fc = 0.0;
  } else if (t > 0.0) {
    const double t2 = t * t, t3 = t2 * t;
    fc = 1.0 - (10.0 * t3 - 15.0 * t3 * t + 6.0 * t3 * t2);
    dfc = -(30.0 * t2 - 60.0 * t3 + 30.0 * t3 * t) * iw;
  }
  const double q = m.r0 * ri;
  const double g = q * q;
  const double dg = -2.0 * g * ri;  // d/dr (r0 / r)^2
  u = g * fc;
  du = dg * fc + g * dfc;
}

// sum_b (Gh[b] dH_ab/dd + Gs[b] dS_ab/dd) for one row a of the pair's H and S
// blocks (3-vector), with the weights of that row only.  Written out from the
// two-center forms: with l = d / r, u(r), u'(r) and dl_b/dd_c = (delta_bc -
// l_b l_c) / r,
//   row s:   u' l (P0 + P.l) + (u / r) (P - l (P.l)),
//            P0 = Gh0 Vss + Gs0 Sss, P_b = Gh_{1+b} Vsp + Gs_{1+b} Ssp;
//   row p:   -T0 (u dl_p + l_p u' l) + u (dl_p (Q.l) + l_p (Q - l (Q.l)) / r)
//            + u' l (l_p (Q.l) + R_p),
//            T0 = Gh0 Vsp + Gs0 Ssp, Q_b = Gh_{1+b} (Vpps - Vppp) + Gs_{1+b} (Spps - Sppp),
//            R_p = Gh_{1+p} Vppp + Gs_{1+p} Sppp.
// (iw: 1 / (r_cut - r_on); ri from the reciprocal square root, no division)
__device__ __forceinline__ void pair_row_grad(const SKModelDev& m, double iw, double dx,
                                              double dy, double dz, int a, const double Gh[4],
                                              const double Gs[4], double out[3]) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ri = rsqrt(r2);
  const double r = r2 * ri;
  const double l[3] = {dx * ri, dy * ri, dz * ri};
  double u, du;
  radial_ri(m, r, ri, iw, u, du);
  if (a == 0) {
    const double P0 = Gh[0] * m.vh[0] + Gs[0] * m.vs[0];
    double P[3], pl = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      P[b] = Gh[1 + b] * m.vh[1] + Gs[1 + b] * m.vs[1];
      pl = fma(P[b], l[b], pl);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = du * l[c] * (P0 + pl) + u * ri * (P[c] - l[c] * pl);
  } else {
    const int p = a - 1;
    const double lp = (p == 0) ? l[0] : ((p == 1) ? l[1] : l[2]);
    const double T0 = Gh[0] * m.vh[1] + Gs[0] * m.vs[1];
    const double dh = m.vh[2] - m.vh[3], ds = m.vs[2] - m.vs[3];
    const double Gp_h = (p == 0) ? Gh[1] : ((p == 1) ? Gh[2] : Gh[3]);
    const double Gp_s = (p == 0) ? Gs[1] : ((p == 1) ? Gs[2] : Gs[3]);
    const double Rp = Gp_h * m.vh[3] + Gp_s * m.vs[3];
    double Q[3], ql = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      Q[b] = Gh[1 + b] * dh + Gs[1 + b] * ds;
      ql = fma(Q[b], l[b], ql);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double dlp = ((p == c ? 1.0 : 0.0) - lp * l[c]) * ri;
      out[c] = -T0 * (u * dlp + lp * du * l[c]) + u * (dlp * ql + lp * (Q[c] - l[c] * ql) * ri) +
               du * l[c] * (lp * ql + Rp);
    }
  }
}

}  // namespace mag
