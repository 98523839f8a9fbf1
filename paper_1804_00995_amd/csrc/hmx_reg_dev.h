// hmx_reg_dev.h -- device side of the singular correction (Section 5.2, regularization of the
// kernels): for a close pair (target x, source point q of triangle T) the near-field entry gets
//   ( int_T L_q(y) / |x - y| dy  -  w / |x - y_q| ) / (4 pi)
// (no Gauss term when x = y_q, where the kernel entry is 0), L_q the linear function on T that
// is 1 at the rule's point q and 0 at its other two points.  Close: |x - c_T| <= alpha d_T, c_T
// the centroid and d_T the longest edge.
#pragma once

#include "hmx_dev.h"

namespace hmx {

// Per-triangle record (doubles): v0, v1, v2 at 0..8, centroid at 9..11, (alpha d_T)^2 at 12.
constexpr int TGEO = 16;

// What the near-field assembly needs for the correction: cluster-to-original point map (a point
// with original index o is point o % 3 of triangle o / 3), the triangle records, and the
// coefficients of the three linear functions, L_q = sum_i lag[3 q + i] lambda_i.
struct RegArgs {
  const int32_t* perm;
  const double* tgeo;
  double lag[9];
};

// int_T (c0 lambda_0 + c1 lambda_1 + c2 lambda_2)(y) / |x - y| dy over the flat triangle of the
// record g, lambda_i its barycentric coordinates.  Computed in the triangle's plane with origin
// v0, axes u = (v1 - v0) / |v1 - v0| and w = n x u (n the unit normal of (v1 - v0) x (v2 - v0)),
// where the vertices are p0 = (0, 0), p1 = (|v1 - v0|, 0), p2 = ((v2 - v0).u, (v2 - v0).w) in
// counter-clockwise order.  With rho the projection of x, h its height above the plane and, per
// edge (a, b), its unit direction s, outward normal m, l+- = (b|a - rho).s, P = (a - rho).m,
// R0^2 = P^2 + h^2, R+- = sqrt(R0^2 + l+-^2) and f = ln((R+ + l+) / (R- + l-)), the edge sums of
// Wilton et al. (1984) and Graglia (1993) give
//   I1 = int 1/|x-y|         = sum P f - |h| (atan(P l+ / (R0^2 + |h| R+)) - atan(P l- / (R0^2 + |h| R-)))
//   Ir = int (y - rho)/|x-y| = sum m (R0^2 f + l+ R+ - l- R-) / 2,
// and int lambda_i / |x - y| = lambda_i(rho) I1 + grad(lambda_i) . Ir (lambda_i is affine).
// An edge whose line contains x (R0 = 0) keeps only m (l+ R+ - l- R-) / 2.  R + l is taken as
// R0^2 / (R - l) for l < 0, the same value without cancellation.
__device__ inline double tri_lagrange_inv_r(const double* __restrict__ g, double c0, double c1,
                                            double c2, double x0, double x1, double x2) {
  const double e1x = g[3] - g[0], e1y = g[4] - g[1], e1z = g[5] - g[2];
  const double e2x = g[6] - g[0], e2y = g[7] - g[1], e2z = g[8] - g[2];
  double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const double nn = sqrt(nx * nx + ny * ny + nz * nz);
  nx /= nn;
  ny /= nn;
  nz /= nn;
  const double L1 = sqrt(e1x * e1x + e1y * e1y + e1z * e1z);
  const double ux = e1x / L1, uy = e1y / L1, uz = e1z / L1;
  const double wx = ny * uz - nz * uy, wy = nz * ux - nx * uz, wz = nx * uy - ny * ux;
  const double pu[3] = {0.0, L1, e2x * ux + e2y * uy + e2z * uz};
  const double pw[3] = {0.0, 0.0, e2x * wx + e2y * wy + e2z * wz};
  const double dx = x0 - g[0], dy = x1 - g[1], dz = x2 - g[2];
  const double ru = dx * ux + dy * uy + dz * uz, rw = dx * wx + dy * wy + dz * wz;
  const double h = dx * nx + dy * ny + dz * nz, ah = fabs(h), h2 = h * h;
  double I1 = 0.0, Iu = 0.0, Iw = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int j = i == 2 ? 0 : i + 1;
    const double au = pu[i] - ru, aw = pw[i] - rw, bu = pu[j] - ru, bw = pw[j] - rw;
    double su = pu[j] - pu[i], sw = pw[j] - pw[i];
    const double le = sqrt(su * su + sw * sw);
    su /= le;
    sw /= le;
    const double mu = sw, mw = -su;  // outward: the edge turned clockwise
    const double lp = bu * su + bw * sw, lm = au * su + aw * sw, P = au * mu + aw * mw;
    const double R02 = P * P + h2;
    const double Rp = sqrt(R02 + lp * lp), Rm = sqrt(R02 + lm * lm);
    double c = 0.5 * (lp * Rp - lm * Rm);
    if (R02 > 1e-24 * le * le) {
      const double gp = lp >= 0.0 ? Rp + lp : R02 / (Rp - lp);
      const double gm = lm >= 0.0 ? Rm + lm : R02 / (Rm - lm);
      const double f = log(gp / gm);
      I1 += P * f - ah * (atan(P * lp / (R02 + ah * Rp)) - atan(P * lm / (R02 + ah * Rm)));
      c += 0.5 * R02 * f;
    }
    Iu += c * mu;
    Iw += c * mw;
  }
  // barycentric coordinates of rho and their gradients in the plane (2 area = |v1 - v0| p2.w)
  const double A2 = L1 * pw[2];
  const double cf[3] = {c0, c1, c2};
  double J = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int j = i == 2 ? 0 : i + 1, k = j == 2 ? 0 : j + 1;
    const double lam = ((pu[j] - ru) * (pw[k] - rw) - (pw[j] - rw) * (pu[k] - ru)) / A2;
    const double gu = -(pw[k] - pw[j]) / A2, gw = (pu[k] - pu[j]) / A2;
    J += cf[i] * (lam * I1 + gu * Iu + gw * Iw);
  }
  return J;
}

// The correction of the pair (target t, source point sj with original index o, weight sw) when
// the pair is close, else 0.
__device__ inline double reg_correction(const RegArgs& ra, int32_t o, double tx, double ty,
                                        double tz, double sx, double sy, double sz, double sw) {
  const int32_t t = o / 3, q = o - 3 * t;
  const double* g = ra.tgeo + (int64_t)t * TGEO;
  // closeness in the written order without contraction (the records are built the same way), so
  // the decision is that of the plain definition
  const double cx = tx - g[9], cy = ty - g[10], cz = tz - g[11];
  const double c2 = __dadd_rn(__dadd_rn(__dmul_rn(cx, cx), __dmul_rn(cy, cy)), __dmul_rn(cz, cz));
  if (c2 > g[12]) return 0.0;
  const double J = tri_lagrange_inv_r(g, ra.lag[3 * q], ra.lag[3 * q + 1], ra.lag[3 * q + 2], tx, ty, tz);
  const double dx = tx - sx, dy = ty - sy, dz = tz - sz;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double gauss = r2 == 0.0 ? 0.0 : sw / sqrt(r2);
  return (J - gauss) * INV4PI;
}

}  // namespace hmx
