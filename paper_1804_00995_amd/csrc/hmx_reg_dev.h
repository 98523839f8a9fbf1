// hmx_reg_dev.h -- device side of the singular correction (Section 5.2, regularization of the
// kernels): for a close pair (target x, source point q of triangle T) the near-field entry gets
//   ( int_T L_q(y) / |x - y| dy  -  w / |x - y_q| ) / (4 pi)
// (no Gauss term when x = y_q, where the kernel entry is 0), L_q the linear function on T that
// is 1 at the rule's point q and 0 at its other two points.  One y-integral over T serves the
// pairs of x with all three points of T.  Close: |x - c_T| <= alpha d_T, c_T
// the centroid and d_T the longest edge.
#pragma once

#include "hmx_dev.h"

namespace hmx {

// Per-triangle record (TGEO doubles).  The triangle's plane frame: origin v0 (0..2), axes
// u = (v1 - v0) / |v1 - v0| (3..5) and w = n x u (6..8) with n (13..15) the unit normal of
// (v1 - v0) x (v2 - v0); in it the vertices are p0 = (0, 0), p1 = (L, 0), p2 = (a, b) (L at 16,
// a at 17, b at 18; counter-clockwise, b > 0), 1 / (2 area) = 1 / (L b) at 19, and the unit
// directions (su, sw) of the edges (p0, p1), (p1, p2), (p2, p0) at 20..25 with their squared
// lengths at 26..28.  Closeness: centroid at 9..11 and (alpha d_T)^2 at 12 (d_T the longest edge).
constexpr int TGEO = 32;

// What the near-field correction needs: the cluster-to-original point map and its inverse (a
// point with original index o is point o % 3 of triangle o / 3), the triangle records, and the
// coefficients of the three linear functions, L_q = sum_i lag[3 q + i] lambda_i.
struct RegArgs {
  const int32_t* perm;
  const int32_t* iperm;
  const double* tgeo;
  double lag[9];
};

// J[q] = int_T L_q(y) / |x - y| dy for q = 0, 1, 2 over the flat triangle of the record g,
// L_q = sum_i lag[3 q + i] lambda_i with lambda_i the barycentric coordinates, computed in the
// triangle's plane frame.  With
// rho the projection of x, h its height above the plane and, per edge (a, b), its unit direction
// s, outward normal m, l+- = (b|a - rho).s, P = (a - rho).m, R0^2 = P^2 + h^2, R+- the distances
// from x to b and a, and f = ln((R+ + l+) / (R- + l-)), the edge sums of Wilton et al. (1984)
// and Graglia (1993) give
//   I1 = int 1/|x-y|         = sum P f - |h| (atan(P l+ / (R0^2 + |h| R+)) - atan(P l- / (R0^2 + |h| R-)))
//   Ir = int (y - rho)/|x-y| = sum m (R0^2 f + l+ R+ - l- R-) / 2,
// and int lambda_i / |x - y| = lambda_i(rho) I1 + grad(lambda_i) . Ir (lambda_i is affine).
// The difference of arctangents atan(A / Da) - atan(B / Db) (Da, Db > 0) is the argument of
// (Da + i A)(Db - i B), i.e. atan2(A Db - B Da, Da Db + A B).  An edge whose line contains x
// (R0 = 0) keeps only m (l+ R+ - l- R-) / 2.  R + l is taken as R0^2 / (R - l) for l < 0, the
// same value without cancellation.
__device__ inline void tri_lagrange3(const double* __restrict__ g, const double* lag, double x0,
                                     double x1, double x2, double* J) {
  const double dx = x0 - g[0], dy = x1 - g[1], dz = x2 - g[2];
  const double ru = dx * g[3] + dy * g[4] + dz * g[5];
  const double rw = dx * g[6] + dy * g[7] + dz * g[8];
  const double h = dx * g[13] + dy * g[14] + dz * g[15], ah = fabs(h), h2 = h * h;
  // vertices relative to rho, and their distances to x
  const double au[3] = {-ru, g[16] - ru, g[17] - ru};
  const double aw[3] = {-rw, -rw, g[18] - rw};
  double R[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) R[v] = sqrt(au[v] * au[v] + aw[v] * aw[v] + h2);
  double I1 = 0.0, Iu = 0.0, Iw = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int j = i == 2 ? 0 : i + 1;
    const double su = g[20 + 2 * i], sw = g[21 + 2 * i];
    const double mu = sw, mw = -su;  // outward: the edge turned clockwise
    const double lp = au[j] * su + aw[j] * sw, lm = au[i] * su + aw[i] * sw;
    const double P = au[i] * mu + aw[i] * mw;
    const double R02 = P * P + h2, Rp = R[j], Rm = R[i];
    double c = 0.5 * (lp * Rp - lm * Rm);
    if (R02 > 1e-24 * g[26 + i]) {
      const double gp = lp >= 0.0 ? Rp + lp : R02 / (Rp - lp);
      const double gm = lm >= 0.0 ? Rm + lm : R02 / (Rm - lm);
      const double f = log(gp / gm);
      const double A = P * lp, B = P * lm, Da = R02 + ah * Rp, Db = R02 + ah * Rm;
      I1 += P * f - ah * atan2(A * Db - B * Da, Da * Db + A * B);
      c += 0.5 * R02 * f;
    }
    Iu += c * mu;
    Iw += c * mw;
  }
  // barycentric coordinates of rho (p_k - rho = (au[k], aw[k])) and their gradients
  const double inv2a = g[19];
  double Jb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int j = i == 2 ? 0 : i + 1, k = j == 2 ? 0 : j + 1;
    const double lam = (au[j] * aw[k] - aw[j] * au[k]) * inv2a;
    const double gu = -(aw[k] - aw[j]) * inv2a, gw = (au[k] - au[j]) * inv2a;
    Jb[i] = lam * I1 + gu * Iu + gw * Iw;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) J[q] = lag[3 * q] * Jb[0] + lag[3 * q + 1] * Jb[1] + lag[3 * q + 2] * Jb[2];
}

// Is the pair (target x, triangle t) close: |x - c_T|^2 <= (alpha d_T)^2, evaluated in the
// written order without contraction (the records are built the same way), so the decision is
// that of the plain definition.
__device__ inline bool reg_close(const RegArgs& ra, int32_t t, double tx, double ty, double tz) {
  const double* g = ra.tgeo + (int64_t)t * TGEO;
  const double cx = tx - g[9], cy = ty - g[10], cz = tz - g[11];
  const double c2 = __dadd_rn(__dadd_rn(__dmul_rn(cx, cx), __dmul_rn(cy, cy)), __dmul_rn(cz, cz));
  return c2 <= g[12];
}

}  // namespace hmx
