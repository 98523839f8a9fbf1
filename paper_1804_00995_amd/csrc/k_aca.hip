// k_aca.hip -- partially pivoted adaptive cross approximation of the far blocks.
//
// The paper compresses the kernel matrix to a given accuracy (Section 5.3) without stating the
// method; libhmx uses Bebendorf-style partial pivoting.  For a far block A (m x n, A_ij =
// G(x_{t+i}, x_{s+j}) w_{s+j}), step k with pivot row i_k:
//   (1) residual row R_j = A(i_k, j) - sum_{l<k} u_l[i_k] v_l[j]
//   (2) pivot column j_k = argmax over unused columns of |R_j|^2 (lowest index on ties); a row
//       whose residual maximum is <= 1e-300 is marked used, the lowest unused row is taken and
//       no term is added
//   (3) v_k = R / R_{j_k}
//   (4) u_k[i] = A(i, j_k) - sum_{l<k} v_l[j_k] u_l[i]
//   (5) |S_k|_F^2 = |S_{k-1}|_F^2 + 2 Re sum_{l<k} (u_l^H u_k)(v_l^H v_k) + |u_k|^2 |v_k|^2
//   (6) stop, keeping term k, when |u_k| |v_k| <= tol |S_k|_F has held at ACA_STOP_STEPS (two)
//       consecutive steps; a zero residual row in between neither counts nor resets
//   (7) next pivot row = argmax over unused rows of |u_k[i]|^2 (lowest index on ties).
// A ~ sum_k u_k v_k^T with U (m x cap) and V (n x cap) stored column-major.  Pivot magnitudes,
// norms and the cross terms are accumulated in FP64 in both precisions.
//
// Stored form: column k of V holds the residual row R itself and column k of U holds
// u_k / R_{j_k}, so the product of the two equals u_k v_k^T of steps (3)-(4) without a pass that
// rescales R.  The residual formulas (1) and (4) are unchanged in this form, the norms in (6)
// and the cross terms in (5) are the same products (the scales cancel), and both pivot searches
// use the residual values before any scaling.
//
// Schedule: persistent grids; each workgroup takes the next block from an atomic counter
// (blocks pre-ordered by decreasing size) and runs its whole sequential step chain.  Four
// classes: m + n above a threshold in 512- or 256-thread workgroups, the middle sizes in 128-
// (or 256- / 64-) thread workgroups, small blocks in 64-thread workgroups holding 256
// coefficients, and blocks with m, n <= 64 in single wavefronts (register-resident, below).  The
// classes run on three streams.
//
// Factor storage: segments of interleaved column pairs taken from a device bump pool (atomic
// offset), placed one after the other in per-workgroup arenas so that a finished block keeps
// exactly its columns.  A block that outgrows its segment goes on in a second one; one that
// outgrows both moves to a segment of twice the size.  If the pool is exhausted it saves (rank,
// pivot row, norm) and stops with status OVERFLOW, and the host continues it in a new pool.
// Either way the pivot sequence, and therefore the factors, equal those of one uninterrupted
// run.  A block that needs a term beyond its rank cap is marked DENSE (stored exactly).
#include <limits.h>

#include <algorithm>

#include "hmx_dev.h"
#include "hmx_host.h"

namespace hmx {


// Terms whose Gram sums the large-block kind keeps per wavefront (the sliced passes run for
// ranks up to GB).
constexpr int GB = 64;

// Workgroup state in LDS; NW wavefronts, Gram order GR.
template <int NW, int GR>
struct AcaShared {
  double sv[16];
  int si[16];
  double ssum[32 * (NW + 1)];  // block_sum scratch: N (NW + 1) doubles for N <= 32
  double2 h[GR];  // per previous term: v_l^H (row residual) or u_l^H (column residual)
  int64_t off;
  int q;
};

// sum_{p0 <= p < kk} c_p G[l][p] for one Gram row (8 independent loads per round).
template <class T>
__device__ __forceinline__ double2 gram_row_dot(const double2* __restrict__ row, const T* coef,
                                                int p0, int kk) {
  double2 t = make_double2(0.0, 0.0);
  for (int p = p0; p < kk; p += 8) {
    double2 gv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) gv[q] = p + q < kk ? row[p + q] : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (p + q < kk) {
        const double2 c = to_d2(coef[p + q]);
        t.x += c.x * gv[q].x - c.y * gv[q].y;
        t.y += c.x * gv[q].y + c.y * gv[q].x;
      }
    }
  }
  return t;
}

// Values that are the same in every lane (block fields, pivots, ranks), moved to scalar registers
// so that the factor loads take a scalar base address and a 32-bit lane offset.
__device__ __forceinline__ int ufl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t ufl(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class P>
__device__ __forceinline__ P* ufl(P* p) {
  return (P*)(uintptr_t)ufl((int64_t)(uintptr_t)p);
}

// Gram sums of one window taken by one wavefront over its slice: the 2 GW partial sums are
// reduced over the wavefront and lane u stores term l0 + u in the wavefront's row of gbuf.
template <int GW>
__device__ __forceinline__ void wave_gram_sums(double* g, int lc, int l0, HMX_LDS double2* row,
                                               int lane) {
#pragma unroll
  for (int q = 0; q < 2 * GW; ++q) g[q] = wave_sum(g[q]);
#pragma unroll
  for (int u = 0; u < GW; ++u)
    if (lane == u && u < lc) row[l0 + u] = make_double2(g[2 * u], g[2 * u + 1]);
}

// After the sliced windows of a pass: h[l] = sum over the NW wavefront rows of gbuf, in
// wavefront order (deterministic).  Thread l adds term l; the first barrier makes every row
// visible, the second lets gbuf be written again by the next pass.
template <int NW>
__device__ __forceinline__ void gram_sums_total(HMX_LDS double2* gbuf, int kk, double2* h,
                                                int tid) {
  __syncthreads();
  if (tid < kk) {
    double2 a = gbuf[tid];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const double2 b = gbuf[w * GB + tid];
      a.x += b.x;
      a.y += b.y;
    }
    h[tid] = a;
  }
  __syncthreads();
}

template <class T, int NT, bool BIG, int RL, int CO, class Sh>
__device__ void aca_block(FarDesc* __restrict__ descs, int b, const double* __restrict__ X,
                          const double* __restrict__ Y, const double* __restrict__ Z,
                          const double* __restrict__ W, int kern, const double* kp, double tol,
                          uint8_t* flags, int32_t* rank, int32_t* ipiv, int32_t* status,
                          double* norm2, int fresh, T* gpool, int64_t gcap,
                          unsigned long long* gtop, double2* gram, int gram_min, int64_t arena,
                          int64_t& a_top, int64_t& a_end, T* coef, HMX_LDS T* rbuf,
                          HMX_LDS double2* gbuf, Sh& sh) {
  // terms per Gram window and elements per thread per window round (see aca_rl for the
  // large-block kinds' occupancy)
  constexpr bool F32_256 = sizeof(T) == 8 && NT == 256;
  constexpr int GW = BIG ? (sizeof(T) == 16 || F32_256 ? 6 : 8) : 4;
  constexpr int JW = BIG ? (sizeof(T) == 16 || F32_256 ? 2 : 4) : 1;
  constexpr int JC = 1;                  // elements per thread per round
  constexpr int LU = BIG ? 8 : 4;  // previous terms loaded per round (loads in flight)
  const int tid = threadIdx.x;
  const FarDesc d = descs[b];
  const int m = ufl(d.m), n = ufl(d.n), tb = ufl(d.tb), sb = ufl(d.sb);
  // CO coefficients in LDS bound the rank (the host places only blocks with rank cap <= CO in a
  // kind with CO < ACA_COEF_MAX; the bound only guards the coefficient array)
  const int rcap = min(ufl(d.rcap), CO);
  const double k = kp[tb];  // wavenumber of the block's mesh
  // factor slots are device memory: global-address-space pointers (the slot addresses come from
  // the descriptor in memory, where the compiler cannot infer the space), so that their loads do
  // not count against the LDS counter the coefficient and residual reads wait on
  using gT = HMX_GLOBAL T;
  // Slot layout: interleaved column pairs, ld = m + n; column l of U at colU(l) (m entries) and
  // column l of V at colU(l) + m (n entries).  A slot has at most two segments, columns
  // [0, c0) at S0 and [c0, c0 + c1) at S1, so a block that outgrows its first segment goes on
  // in a second one without moving its columns.  Before its first claim a block has S0 = null
  // and c0 = the initial capacity of its descriptor.
  const int ld = m + n;
  gT* S0 = ufl((gT*)d.U);
  gT* S1 = ufl((gT*)d.U1);
  int c0 = ufl(d.cap), c1 = ufl(d.cap1);
  auto colU = [&](int l) -> gT* {
    return l < c0 ? S0 + (int64_t)l * ld : S1 + (int64_t)(l - c0) * ld;
  };
  auto colV = [&](int l) -> gT* { return colU(l) + m; };
  uint8_t* rused = flags + ufl(d.foff);
  uint8_t* cused = rused + m;
  int kk, ip, hits;
  double nrm2;
  if (fresh) {
    for (int i = tid; i < m + n; i += NT) rused[i] = 0;
    kk = 0;
    ip = 0;
    hits = 0;
    nrm2 = 0.0;
  } else {
    kk = ufl(rank[b]);
    ip = ufl(ipiv[b] & ACA_ROW_MASK);
    hits = ufl(ipiv[b] >> ACA_HIT_SHIFT);
    nrm2 = norm2[b];
  }
  // Gram matrices of the factors, GV[l][p] = v_l^H v_p and GU[l][p] = u_l^H u_p (FP64,
  // GR x GR each, row-major, this workgroup's scratch).  With them the cross terms of step (5)
  // come from dot products taken in the residual passes themselves:
  //   v_l^H R = v_l^H R' - sum_{p in and after l's window} u_p[i_k] GV[l][p],
  // R' the residual before l's window, so the previous columns are read once per step.  Ranks
  // past GR and blocks below gram_min take the direct sums instead.
  constexpr int GR = aca_gram_order(NT, BIG ? ACA_KIND_BIG : ACA_KIND_MID);  // Gram order
  static_assert(GR <= NT, "one Gram row per thread");
  double2* GV = gram;
  double2* GU = gram ? gram + GR * GR : nullptr;
  // (the small-block kind, CO < ACA_COEF_MAX, always takes the direct sums: its blocks lie below
  // the Gram threshold's useful range, and without that code it holds fewer registers and more
  // workgroups per CU)
  bool use_gram = CO >= ACA_COEF_MAX && gram != nullptr && m + n >= gram_min && kk < GR;
  if (use_gram && !fresh && kk > 0) {
    // a block resumed from its saved state: rebuild the Gram matrices of its factors (one
    // wavefront per entry pair)
    const int lane = tid & (WAVE - 1), w = tid / WAVE;
    const int np = kk * (kk + 1) / 2;
    for (int q = w; q < np; q += NT / WAVE) {
      int l = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
      while (l * (l + 1) / 2 > q) --l;
      while ((l + 1) * (l + 2) / 2 <= q) ++l;
      const int p = q - l * (l + 1) / 2;
      double gv[2] = {0.0, 0.0}, gu[2] = {0.0, 0.0};
      for (int j = lane; j < n; j += WAVE) {
        const double2 a = to_d2(colV(l)[j]), c = to_d2(colV(p)[j]);
        gv[0] += a.x * c.x + a.y * c.y;
        gv[1] += a.x * c.y - a.y * c.x;
      }
      for (int i = lane; i < m; i += WAVE) {
        const double2 a = to_d2(colU(l)[i]), c = to_d2(colU(p)[i]);
        gu[0] += a.x * c.x + a.y * c.y;
        gu[1] += a.x * c.y - a.y * c.x;
      }
      gv[0] = wave_sum(gv[0]);
      gv[1] = wave_sum(gv[1]);
      gu[0] = wave_sum(gu[0]);
      gu[1] = wave_sum(gu[1]);
      if (lane == 0) {
        GV[(int64_t)l * GR + p] = make_double2(gv[0], gv[1]);
        GV[(int64_t)p * GR + l] = make_double2(gv[0], -gv[1]);
        GU[(int64_t)l * GR + p] = make_double2(gu[0], gu[1]);
        GU[(int64_t)p * GR + l] = make_double2(gu[0], -gu[1]);
      }
    }
    __syncthreads();
  }
  int st = rcap <= 0 ? ACA_DENSE : ACA_RUNNING;
  bool grew = !fresh && (status[b] & ACA_GREW);
  // Segments.  With arenas (arena > 0) the workgroup takes pool space in arenas of `arena`
  // entries and places its blocks one after the other: a block claims the whole free rest of the
  // arena (up to its rank cap) and, when it stops, keeps exactly the columns it used, so slots
  // are exact without moving factors.  Without arenas every segment is a pool allocation of its
  // own.  claim(need, want, lim) returns the first entry of a segment of at least `need`
  // columns: the rest of the arena when it holds them, else a new arena of max(arena, want ld)
  // entries (the old arena's rest stays unused; without arenas, `want` columns); ncap receives
  // its capacity, at most lim; -1 when the pool is exhausted.
  bool mine = false;     // the last claimed segment lies at the top of this workgroup's arena
  int64_t mine_off = 0;  // its first entry
  auto claim = [&](int need, int want, int lim, int& ncap) -> int64_t {
    if (arena > 0 && a_end - a_top >= (int64_t)need * ld) {
      ncap = (int)min((int64_t)lim, (a_end - a_top) / ld);
      mine = true;
      mine_off = a_top;
      return a_top;
    }
    const int64_t size = arena > 0 ? max(arena, (int64_t)want * ld) : (int64_t)want * ld;
    if (tid == 0) sh.off = (int64_t)atomicAdd(gtop, (unsigned long long)size);
    __syncthreads();
    const int64_t off = ufl(sh.off);
    __syncthreads();  // every thread has read sh.off before it is written again
    if (gpool == nullptr || off + size > gcap) return -1;
    if (arena > 0) {
      a_top = off;
      a_end = off + size;
      ncap = (int)min((int64_t)lim, size / ld);
      mine = true;
      mine_off = off;
    } else {
      ncap = min(want, lim);
      mine = false;
    }
    return off;
  };
  const int want0 = max(min(c0, rcap), 1);  // a first segment of this many columns when new
  if (st == ACA_RUNNING && S0 == nullptr) {
    int ncap = 0;
    const int64_t off = claim(1, want0, rcap, ncap);
    if (off < 0) {
      st = ACA_OVERFLOW;
    } else {
      S0 = (gT*)(gpool + off);
      c0 = ncap;
      S1 = nullptr;
      c1 = 0;
    }
  }
  __syncthreads();
  while (st == ACA_RUNNING) {
    if (kk >= GR) use_gram = false;
    // (1) residual row ip, stored as column kk of V when the slot has room
    for (int l = tid; l < kk; l += NT) coef[l] = colU(l)[ip];
    __syncthreads();
    const double px = X[tb + ip], py = Y[tb + ip], pz = Z[tb + ip];
    const bool store = kk < c0 + c1;
    const bool gstep = use_gram && store;  // this step keeps the Gram matrices
    gT* R = store ? colV(kk) : nullptr;
    double best = -1.0, nv2 = 0.0;
    int bj = INT_MAX;
    // Gram part of v_l^H R for this thread's l (gstep: kk < GR <= NT, one l per thread);
    // it needs only the coefficients, so its loads go out before the row pass
    double2 gcorr = make_double2(0.0, 0.0);
    if (gstep && tid < kk) gcorr = gram_row_dot(GV + (int64_t)tid * GR, coef, (tid / GW) * GW, kk);
    if (gstep) {
      // Windows of GW previous terms.  A thread takes JW elements per round, so that JW GW factor
      // loads are in flight together while the Gram sums and coefficients are shared.  The
      // partial residual between windows lives in LDS for j < RL (RL is a multiple of the round
      // width, so the choice is uniform across a wavefront) and in column kk beyond.
      // Large-block kind with kk <= GB: each wavefront owns a contiguous slice of the row and
      // runs all windows over it without workgroup barriers; its Gram sums go to its own row of
      // gbuf and are added in wavefront order once at the end.  Otherwise elements are
      // interleaved over the workgroup (j0 + q NT) and each window ends in a workgroup sum.
      const bool slice = BIG && kk <= GB;
      const int wv = tid / WAVE, lane = tid & (WAVE - 1);
      const int sl = ((n + NT - 1) / NT) * WAVE;  // slice length, a multiple of 64
      const int e0 = slice ? wv * sl + lane : tid, es = slice ? WAVE : NT;
      const int eend = slice ? min(n, wv * sl + sl) : n;
      for (int l0 = 0; l0 < max(kk, 1); l0 += GW) {
        const int lc = min(GW, kk - l0);
        const bool first = l0 == 0, last = l0 + GW >= kk;
        double g[2 * GW];
#pragma unroll
        for (int q = 0; q < 2 * GW; ++q) g[q] = 0.0;
        gT* vcol[GW];  // the window's columns of V
#pragma unroll
        for (int u = 0; u < GW; ++u) vcol[u] = u < lc ? colV(l0 + u) : nullptr;
        for (int j0 = e0; j0 < eend; j0 += es * JW) {
          T vv[JW][GW], r[JW];
#pragma unroll
          for (int q = 0; q < JW; ++q) {
            const int jc = min(j0 + q * es, eend - 1);  // in bounds; past eend zeroed below
#pragma unroll
            for (int u = 0; u < GW; ++u) vv[q][u] = u < lc ? (T)vcol[u][jc] : czero<T>();
          }
#pragma unroll
          for (int q = 0; q < JW; ++q) {
            const int j = j0 + q * es, jc = min(j, eend - 1);
            const bool inl = j < RL;
            T x = first ? eval_entry<T>(kern, k, px, py, pz, X[sb + jc], Y[sb + jc], Z[sb + jc], W[sb + jc])
                        : inl ? (T)rbuf[inl ? j : 0] : (T)R[jc];
            r[q] = j < eend ? x : czero<T>();
          }
#pragma unroll
          for (int q = 0; q < JW; ++q) {
            const double2 r0 = to_d2(r[q]);
#pragma unroll
            for (int u = 0; u < GW; ++u) {
              const double2 a = to_d2(vv[q][u]);
              g[2 * u] += a.x * r0.x + a.y * r0.y;
              g[2 * u + 1] += a.x * r0.y - a.y * r0.x;
              if (u < lc) cfms(r[q], coef[l0 + u], vv[q][u]);
            }
          }
#pragma unroll
          for (int q = 0; q < JW; ++q) {
            const int j = j0 + q * es;
            if (j < eend) {
              if (last) {
                R[j] = r[q];
                const double a2 = abs2(r[q]);
                nv2 += a2;
                if (!cused[j]) amax_merge(best, bj, a2, j);
              } else if (j < RL) {
                rbuf[j < RL ? j : 0] = r[q];
              } else {
                R[j] = r[q];
              }
            }
          }
        }
        if (lc > 0) {
          if (slice) {
            wave_gram_sums<GW>(g, lc, l0, gbuf + wv * GB, lane);
          } else {
            block_sum<2 * GW, NT>(g, sh.ssum);
#pragma unroll
            for (int u = 0; u < GW; ++u)
              if (tid == u && u < lc) sh.h[l0 + u] = make_double2(g[2 * u], g[2 * u + 1]);
          }
        }
      }
      if (slice) gram_sums_total<NT / WAVE>(gbuf, kk, sh.h, tid);
    } else {
    for (int j0 = tid; j0 < n; j0 += NT * JC) {
      T a[JC];
      int jx[JC];
#pragma unroll
      for (int q = 0; q < JC; ++q) {
        const int j = j0 + q * NT;
        jx[q] = j < n ? j : n - 1;
        a[q] = eval_entry<T>(kern, k, px, py, pz, X[sb + jx[q]], Y[sb + jx[q]], Z[sb + jx[q]],
                             W[sb + jx[q]]);
      }
      int l = 0;
      for (; l + LU <= kk; l += LU) {
        T vv[LU][JC];
#pragma unroll
        for (int u = 0; u < LU; ++u)
#pragma unroll
          for (int q = 0; q < JC; ++q) vv[u][q] = colV(l + u)[jx[q]];
#pragma unroll
        for (int u = 0; u < LU; ++u) {
          const T c = coef[l + u];
#pragma unroll
          for (int q = 0; q < JC; ++q) cfms(a[q], c, vv[u][q]);
        }
      }
      for (; l < kk; ++l) {
        const T c = coef[l];
#pragma unroll
        for (int q = 0; q < JC; ++q) cfms(a[q], c, (T)colV(l)[jx[q]]);
      }
#pragma unroll
      for (int q = 0; q < JC; ++q) {
        const int j = j0 + q * NT;
        if (j < n) {
          const double a2 = abs2(a[q]);
          if (store) R[j] = a[q];
          nv2 += a2;
          if (!cused[j]) amax_merge(best, bj, a2, j);
        }
      }
    }
    }
    block_amax<NT>(best, bj, sh.sv, sh.si);
    bj = ufl(bj);
    if (bj == INT_MAX || best <= 1e-300) {
      // (2') zero residual row: mark it, move to the lowest unused row
      if (tid == 0) rused[ip] = 1;
      __syncthreads();
      int nx = INT_MAX;
      for (int i = tid; i < m; i += NT)
        if (!rused[i]) {
          nx = i;
          break;
        }
      nx = ufl(block_min<NT>(nx, sh.si));
      if (nx == INT_MAX) {
        st = ACA_CONVERGED;
        break;
      }
      ip = nx;
      continue;
    }
    if (!store) {
      if (c0 + c1 >= rcap) {
        st = ACA_DENSE;
        break;
      }
      if (S1 == nullptr) {
        // a second segment; the columns so far stay in the first, which is now full
        if (mine) a_top = mine_off + (int64_t)c0 * ld;
        int ncap = 0;
        const int64_t off = claim(1, max(want0, c0), rcap - c0, ncap);
        if (off < 0) {
          st = ACA_OVERFLOW;
          break;
        }
        S1 = (gT*)(gpool + off);
        c1 = ncap;
      } else {
        // both segments full: one segment of twice the capacity, the columns moved there
        if (mine) a_top = mine_off + (int64_t)c1 * ld;
        const int want = min(rcap, max(2 * (c0 + c1), c0 + c1 + 8));
        int ncap = 0;
        const int64_t off = claim(want, want, rcap, ncap);
        if (off < 0) {
          st = ACA_OVERFLOW;
          break;
        }
        gT* nS = (gT*)(gpool + off);
        const int64_t e0 = (int64_t)c0 * ld, e1 = (int64_t)c1 * ld;
        for (int64_t e = tid; e < e0; e += NT) nS[e] = S0[e];
        for (int64_t e = tid; e < e1; e += NT) nS[e0 + e] = S1[e];
        __syncthreads();
        S0 = nS;
        c0 = ncap;
        S1 = nullptr;
        c1 = 0;
      }
      grew = true;
      continue;  // recompute the residual row into the new slot
    }
    // (3) the scale 1 / R[bj] of v_k, folded into u_k (R stays as stored)
    const double2 pd = to_d2(R[bj]);
    const double den = pd.x * pd.x + pd.y * pd.y;
    const double2 invd = make_double2(pd.x / den, -pd.y / den);
    const T inv = from_d2<T>(invd);
    // v_l^H v_k for this thread's l (gstep: kk < GR <= NT, one l per thread)
    double2 vdot = make_double2(0.0, 0.0);
    if (gstep && tid < kk) vdot = make_double2(sh.h[tid].x - gcorr.x, sh.h[tid].y - gcorr.y);
    if (tid == 0) {
      rused[ip] = 1;
      cused[bj] = 1;
    }
    // (4) residual column bj, stored as column kk of U
    for (int l = tid; l < kk; l += NT) coef[l] = colV(l)[bj];
    __syncthreads();
    const double qx = X[sb + bj], qy = Y[sb + bj], qz = Z[sb + bj], qw = W[sb + bj];
    gT* Uk = colU(kk);
    double ub = -1.0, nu2 = 0.0;
    int ui = INT_MAX;
    double cross = 0.0;
    if (gstep) {
      const double2 ucorr = tid < kk ? gram_row_dot(GU + (int64_t)tid * GR, coef,
                                                    (tid / GW) * GW, kk)
                                     : make_double2(0.0, 0.0);
      const bool slice = BIG && kk <= GB;  // as in the row pass, over the m rows
      const int wv = tid / WAVE, lane = tid & (WAVE - 1);
      const int sl = ((m + NT - 1) / NT) * WAVE;
      const int e0 = slice ? wv * sl + lane : tid, es = slice ? WAVE : NT;
      const int eend = slice ? min(m, wv * sl + sl) : m;
      for (int l0 = 0; l0 < max(kk, 1); l0 += GW) {
        const int lc = min(GW, kk - l0);
        const bool first = l0 == 0, last = l0 + GW >= kk;
        double g[2 * GW];
#pragma unroll
        for (int q = 0; q < 2 * GW; ++q) g[q] = 0.0;
        // JW elements per thread and round, sliced or interleaved as in the row pass
        gT* ucol[GW];  // the window's columns of U
#pragma unroll
        for (int u = 0; u < GW; ++u) ucol[u] = u < lc ? colU(l0 + u) : nullptr;
        for (int i0 = e0; i0 < eend; i0 += es * JW) {
          T uu[JW][GW], r[JW];
#pragma unroll
          for (int q = 0; q < JW; ++q) {
            const int ic = min(i0 + q * es, eend - 1);
#pragma unroll
            for (int u = 0; u < GW; ++u) uu[q][u] = u < lc ? (T)ucol[u][ic] : czero<T>();
          }
#pragma unroll
          for (int q = 0; q < JW; ++q) {
            const int i = i0 + q * es, ic = min(i, eend - 1);
            const bool inl = i < RL;
            T x = first ? eval_entry<T>(kern, k, X[tb + ic], Y[tb + ic], Z[tb + ic], qx, qy, qz, qw)
                        : inl ? (T)rbuf[inl ? i : 0] : (T)Uk[ic];
            r[q] = i < eend ? x : czero<T>();
          }
#pragma unroll
          for (int q = 0; q < JW; ++q) {
            const double2 r0 = to_d2(r[q]);
#pragma unroll
            for (int u = 0; u < GW; ++u) {
              const double2 a = to_d2(uu[q][u]);
              g[2 * u] += a.x * r0.x + a.y * r0.y;
              g[2 * u + 1] += a.x * r0.y - a.y * r0.x;
              if (u < lc) cfms(r[q], coef[l0 + u], uu[q][u]);
            }
          }
#pragma unroll
          for (int q = 0; q < JW; ++q) {
            const int i = i0 + q * es;
            if (i < eend) {
              if (last) {
                if (!rused[i]) amax_merge(ub, ui, abs2(r[q]), i);
                const T us = cmul(r[q], inv);
                Uk[i] = us;
                nu2 += abs2(us);
              } else if (i < RL) {
                rbuf[i < RL ? i : 0] = r[q];
              } else {
                Uk[i] = r[q];
              }
            }
          }
        }
        if (lc > 0) {
          if (slice) {
            wave_gram_sums<GW>(g, lc, l0, gbuf + wv * GB, lane);
          } else {
            block_sum<2 * GW, NT>(g, sh.ssum);
#pragma unroll
            for (int u = 0; u < GW; ++u)
              if (tid == u && u < lc) sh.h[l0 + u] = make_double2(g[2 * u], g[2 * u + 1]);
          }
        }
      }
      if (slice) gram_sums_total<NT / WAVE>(gbuf, kk, sh.h, tid);
      __syncthreads();
      // u_l^H u_k (the window sums hold u_l^H times the unscaled column), the cross term, and
      // the new Gram entries
      double2 udot = make_double2(0.0, 0.0);
      if (tid < kk) {
        const double2 t = make_double2(sh.h[tid].x - ucorr.x, sh.h[tid].y - ucorr.y);
        udot = make_double2(t.x * invd.x - t.y * invd.y, t.x * invd.y + t.y * invd.x);
      }
      double cr[1] = {udot.x * vdot.x - udot.y * vdot.y};
      block_sum<1, NT>(cr, sh.ssum);
      cross = cr[0];
      if (tid < kk) {
        GV[(int64_t)tid * GR + kk] = vdot;
        GV[(int64_t)kk * GR + tid] = make_double2(vdot.x, -vdot.y);
        GU[(int64_t)tid * GR + kk] = udot;
        GU[(int64_t)kk * GR + tid] = make_double2(udot.x, -udot.y);
      }
    } else {
    for (int i0 = tid; i0 < m; i0 += NT * JC) {
      T a[JC];
      int ix[JC];
#pragma unroll
      for (int q = 0; q < JC; ++q) {
        const int i = i0 + q * NT;
        ix[q] = i < m ? i : m - 1;
        a[q] = eval_entry<T>(kern, k, X[tb + ix[q]], Y[tb + ix[q]], Z[tb + ix[q]], qx, qy, qz, qw);
      }
      int l = 0;
      for (; l + LU <= kk; l += LU) {
        T uu[LU][JC];
#pragma unroll
        for (int u = 0; u < LU; ++u)
#pragma unroll
          for (int q = 0; q < JC; ++q) uu[u][q] = colU(l + u)[ix[q]];
#pragma unroll
        for (int u = 0; u < LU; ++u) {
          const T c = coef[l + u];
#pragma unroll
          for (int q = 0; q < JC; ++q) cfms(a[q], c, uu[u][q]);
        }
      }
      for (; l < kk; ++l) {
        const T c = coef[l];
#pragma unroll
        for (int q = 0; q < JC; ++q) cfms(a[q], c, (T)colU(l)[ix[q]]);
      }
#pragma unroll
      for (int q = 0; q < JC; ++q) {
        const int i = i0 + q * NT;
        if (i < m) {
          if (!rused[i]) amax_merge(ub, ui, abs2(a[q]), i);
          const T us = cmul(a[q], inv);
          Uk[i] = us;
          nu2 += abs2(us);
        }
      }
    }
    __syncthreads();
    // (5) cross terms sum_{l<kk} (u_l^H u_k)(v_l^H v_k), LG terms at a time (LG loads in
    // flight per thread per round)
    constexpr int LG = BIG ? 4 : 2;
    constexpr int CJ = 1;  // elements per thread per round in this pass
    for (int l0 = 0; l0 < kk; l0 += LG) {
      const int lc = min(LG, kk - l0);
      double acc[4 * LG];
#pragma unroll
      for (int q = 0; q < 4 * LG; ++q) acc[q] = 0.0;
      for (int i0 = tid; i0 < m; i0 += NT * CJ) {
        double2 uk[CJ];
        T ul[CJ][LG];
#pragma unroll
        for (int c = 0; c < CJ; ++c) {
          const int i = i0 + c * NT;
          const int ix = i < m ? i : m - 1;
          uk[c] = i < m ? to_d2(Uk[ix]) : make_double2(0.0, 0.0);
#pragma unroll
          for (int q = 0; q < LG; ++q) ul[c][q] = q < lc ? (T)colU(l0 + q)[ix] : czero<T>();
        }
#pragma unroll
        for (int c = 0; c < CJ; ++c)
#pragma unroll
          for (int q = 0; q < LG; ++q) {
            const double2 a = to_d2(ul[c][q]);
            acc[2 * q] += a.x * uk[c].x + a.y * uk[c].y;
            acc[2 * q + 1] += a.x * uk[c].y - a.y * uk[c].x;
          }
      }
      for (int j0 = tid; j0 < n; j0 += NT * CJ) {
        double2 vk[CJ];
        T vl[CJ][LG];
#pragma unroll
        for (int c = 0; c < CJ; ++c) {
          const int j = j0 + c * NT;
          const int jx = j < n ? j : n - 1;
          vk[c] = j < n ? to_d2(R[jx]) : make_double2(0.0, 0.0);
#pragma unroll
          for (int q = 0; q < LG; ++q) vl[c][q] = q < lc ? (T)colV(l0 + q)[jx] : czero<T>();
        }
#pragma unroll
        for (int c = 0; c < CJ; ++c)
#pragma unroll
          for (int q = 0; q < LG; ++q) {
            const double2 a = to_d2(vl[c][q]);
            acc[2 * LG + 2 * q] += a.x * vk[c].x + a.y * vk[c].y;
            acc[2 * LG + 2 * q + 1] += a.x * vk[c].y - a.y * vk[c].x;
          }
      }
      block_sum<4 * LG, NT>(acc, sh.ssum);
#pragma unroll
      for (int q = 0; q < LG; ++q)
        if (q < lc)
          cross += acc[2 * q] * acc[2 * LG + 2 * q] - acc[2 * q + 1] * acc[2 * LG + 2 * q + 1];
    }
    }
    double nn2[2] = {nu2, nv2};
    block_sum<2, NT>(nn2, sh.ssum);
    if (gstep && tid == 0) {
      GV[(int64_t)kk * GR + kk] = make_double2(nn2[1], 0.0);
      GU[(int64_t)kk * GR + kk] = make_double2(nn2[0], 0.0);
    }
    nrm2 = nrm2 + 2.0 * cross + nn2[0] * nn2[1];
    kk += 1;
    block_amax<NT>(ub, ui, sh.sv, sh.si);
    ui = ufl(ui);
    // (6) stopping rule (met at ACA_STOP_STEPS consecutive steps), (7) next pivot row
    if (sqrt(nn2[0]) * sqrt(nn2[1]) <= tol * sqrt(nrm2)) {
      if (++hits >= ACA_STOP_STEPS) {
        st = ACA_CONVERGED;
        break;
      }
    } else {
      hits = 0;
    }
    if (ui == INT_MAX) {
      st = ACA_CONVERGED;
      break;
    }
    ip = ui;
  }
  if (mine) {
    // the last segment keeps exactly the columns it used, at the top of the arena (none when the
    // block is stored dense); a block stopped for a later round resumes from them and claims
    // more on its next step
    const int used = st == ACA_DENSE ? 0 : max(S1 != nullptr ? kk - c0 : kk, 0);
    a_top = mine_off + (int64_t)used * ld;
    if (S1 != nullptr)
      c1 = used;
    else
      c0 = used;
  }
  if (tid == 0) {
    descs[b].U = (void*)S0;
    descs[b].U1 = (void*)S1;
    descs[b].cap = c0;
    descs[b].cap1 = c1;
    descs[b].ld = ld;
    rank[b] = kk;
    ipiv[b] = ip | (hits << ACA_HIT_SHIFT);
    norm2[b] = nrm2;
    status[b] = st | (grew ? ACA_GREW : 0);
  }
  __syncthreads();
}

// Length of the LDS residual buffer (a multiple of NT) of the large-block class.  FP64 and
// 512-thread FP32 workgroups keep most of the partial residual in LDS: 7680 / 15360 entries with
// 512 threads (one workgroup per CU), 3328 FP64 entries with 256 threads (two per CU).  FP32
// 256-thread workgroups run three per CU, their registers filling the CU, and keep 4352 entries
// each, as much as three workgroups' LDS allows (52.7 KB each): the residual of blocks up to that
// length no longer goes through the factor slot between windows (1024 entries built the 245 760-
// point sphere 2.5 % and the 3.93M-point share 2.7 % slower).  The other classes keep their
// partial residual in the factor slot.
template <class T, int NT, bool BIG>
constexpr int aca_rl() {
  return !BIG ? 0
         : NT >= 512 ? (sizeof(T) == 16 ? 7680 : 15360)
                     : (sizeof(T) == 16 ? 3328 : 4352);
}
// Minimum waves per SIMD the register allocation has to allow.  The FP32 small-block kind is
// bound by the latency of its steps, not by bandwidth: six waves per SIMD (a few spilled
// registers) run more blocks at once and measured faster than five without spills; in FP64 the
// same limit spills more and gained nothing.
template <class T, int NT, bool BIG, int CO>
constexpr int aca_waves_per_eu() {
  return BIG ? (sizeof(T) == 8 && NT == 256 ? 3 : 2)
             : (CO < ACA_COEF_MAX && sizeof(T) == 8 ? 6 : 3);
}

// BIG: the large-block class (long Gram windows, LDS residual); CO: the coefficient capacity
// (ACA_COEF_SMALL for the small-block class)
template <class T, int NT, bool BIG, int CO = ACA_COEF_MAX>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(aca_waves_per_eu<T, NT, BIG, CO>()))) aca_kernel(FarDesc* __restrict__ desc,
                                                 const int32_t* __restrict__ order, int nb,
                                                 int* counter, const double* __restrict__ X,
                                                 const double* __restrict__ Y,
                                                 const double* __restrict__ Z,
                                                 const double* __restrict__ W, int kern, const double* kp,
                                                 double tol, uint8_t* flags, int32_t* rank,
                                                 int32_t* ipiv, int32_t* status, double* norm2,
                                                 int fresh, T* gpool, int64_t gcap,
                                                 unsigned long long* gtop, double2* gram,
                                                 int gram_min, int64_t arena) {
  constexpr int RL = aca_rl<T, NT, BIG>();
  constexpr int GR = aca_gram_order(NT, BIG ? ACA_KIND_BIG : ACA_KIND_MID);
  __shared__ T coef[CO];
  __shared__ T rbuf[RL > 0 ? RL : 1];
  __shared__ double2 gbuf[BIG ? (NT / WAVE) * GB : 1];  // per-wavefront Gram sums
  __shared__ AcaShared<NT / WAVE, GR> sh;
  double2* my_gram = gram ? gram + (int64_t)blockIdx.x * 2 * GR * GR : nullptr;
  int64_t a_top = 0, a_end = 0;  // this workgroup's arena: free entries [a_top, a_end) of gpool
  for (;;) {
    if (threadIdx.x == 0) sh.q = atomicAdd(counter, 1);
    __syncthreads();
    const int q = ufl(sh.q);
    __syncthreads();
    if (q >= nb) break;
    aca_block<T, NT, BIG, RL, CO>(desc, ufl(order[q]), X, Y, Z, W, kern, kp, tol, flags, rank, ipiv, status,
                         norm2, fresh, gpool, gcap, gtop, my_gram, gram_min, arena, a_top, a_end, coef,
                         (HMX_LDS T*)rbuf, (HMX_LDS double2*)gbuf, sh);
  }
}

// ------------------------------------------------------------------ register-resident ACA
// Blocks with m, n <= 64: one wavefront per block, lane i owns row i of U and column i of V,
// up to RC terms held in registers.  Coefficients u_l[i_k] and v_l[j_k] are broadcast from
// their owner lane with readlane, pivots come from wavefront argmax reductions, and the cross
// term of step (5) is evaluated as sum_i u_k[i] * sum_l conj(u_l[i]) (v_l^H v_k), i.e. k
// wavefront sums for the v_l^H v_k and one for the final sum.  Nothing touches memory between
// loading the points and storing the factors.  A block that needs more than RC terms stores its
// state and stops with status OVERFLOW; the workgroup kernel continues it.
template <class T, int RC>
__global__ void __launch_bounds__(WG) aca_wave_kernel(
    FarDesc* __restrict__ desc, const int32_t* __restrict__ order, int nb,
    const double* __restrict__ X, const double* __restrict__ Y, const double* __restrict__ Z,
    const double* __restrict__ W, int kern, const double* kp, double tol, uint8_t* flags, int32_t* rank,
    int32_t* ipiv, int32_t* status, double* norm2, T* gpool, int64_t gcap,
    unsigned long long* gtop) {
  const int lane = threadIdx.x & (WAVE - 1);
  // static round-robin over the (size-ordered) list: wavefront w takes w, w + nw, ...; the
  // loop carries no lane-dependent control flow
  const int gw = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * NWAVE + threadIdx.x / WAVE));
  const int nw = (int)gridDim.x * NWAVE;
  for (int q = gw; q < nb; q += nw) {
    const int b = order[q];
    const FarDesc d = desc[b];
    const int m = d.m, n = d.n;
    const double k = kp[d.tb];
    const bool hr = lane < m, hc = lane < n;
    const int ir = hr ? lane : 0, ic = hc ? lane : 0;
    const double tx = X[d.tb + ir], ty = Y[d.tb + ir], tz = Z[d.tb + ir];
    const double sx = X[d.sb + ic], sy = Y[d.sb + ic], sz = Z[d.sb + ic], sw = W[d.sb + ic];
    T u[RC], v[RC];
#pragma unroll
    for (int l = 0; l < RC; ++l) u[l] = v[l] = czero<T>();
    bool rused = !hr, cused = !hc;
    int kk = 0, ip = 0, hits = 0;
    double nrm2 = 0.0;
    int st = d.rcap <= 0 ? ACA_DENSE : ACA_RUNNING;
    while (st == ACA_RUNNING) {
      // (1) residual row ip
      const double px = readlane(tx, ip), py = readlane(ty, ip), pz = readlane(tz, ip);
      T a = eval_entry<T>(kern, k, px, py, pz, sx, sy, sz, sw);
#pragma unroll
      for (int l = 0; l < RC; ++l)
        if (l < kk) cfms(a, readlane(u[l], ip), v[l]);
      if (!hc) a = czero<T>();
      // (2) pivot column
      double best = cused ? -1.0 : abs2(a);
      int bj = cused ? INT_MAX : lane;
      wave_amax(best, bj);
      bj = __builtin_amdgcn_readfirstlane(bj);
      const int zero_row = __builtin_amdgcn_readfirstlane((bj == INT_MAX || best <= 1e-300) ? 1 : 0);
      if (zero_row) {
        if (lane == ip) rused = true;
        const int nx = __builtin_amdgcn_readfirstlane(wave_min(rused ? INT_MAX : lane));
        if (nx == INT_MAX) {
          st = ACA_CONVERGED;
          break;
        }
        ip = nx;
        continue;
      }
      if (kk >= d.rcap) {
        st = ACA_DENSE;
        break;
      }
      if (kk >= RC) {
        st = ACA_OVERFLOW;
        break;
      }
      // (3) stored form: v_k is R itself, u_k carries the scale 1 / R[bj]
      const double2 pd = to_d2(readlane(a, bj));
      const double den = pd.x * pd.x + pd.y * pd.y;
      const T inv = from_d2<T>(make_double2(pd.x / den, -pd.y / den));
      const T vn = a;
      if (lane == ip) rused = true;
      if (lane == bj) cused = true;
      // (4) residual column bj
      const double qx = readlane(sx, bj), qy = readlane(sy, bj), qz = readlane(sz, bj),
                   qw = readlane(sw, bj);
      T c = eval_entry<T>(kern, k, tx, ty, tz, qx, qy, qz, qw);
#pragma unroll
      for (int l = 0; l < RC; ++l)
        if (l < kk) cfms(c, readlane(v[l], bj), u[l]);
      const T uraw = hr ? c : czero<T>();
      const T un = cmul(uraw, inv);
      // (5) norms and cross term
      const double nu2 = wave_sum(abs2(un)), nv2 = wave_sum(abs2(vn));
      double2 s = make_double2(0.0, 0.0);
      const double2 und = to_d2(un), vnd = to_d2(vn);
#pragma unroll
      for (int l = 0; l < RC; ++l) {
        if (l < kk) {
          const double2 vl = to_d2(v[l]);
          double2 dv = make_double2(vl.x * vnd.x + vl.y * vnd.y, vl.x * vnd.y - vl.y * vnd.x);
          dv.x = wave_sum(dv.x);
          dv.y = wave_sum(dv.y);
          const double2 ul = to_d2(u[l]);
          // s += conj(u_l[i]) * dv
          s.x += ul.x * dv.x + ul.y * dv.y;
          s.y += ul.x * dv.y - ul.y * dv.x;
        }
      }
      const double cross = wave_sum(und.x * s.x - und.y * s.y);
      nrm2 = nrm2 + 2.0 * cross + nu2 * nv2;
#pragma unroll
      for (int l = 0; l < RC; ++l)
        if (l == kk) {
          u[l] = un;
          v[l] = vn;
        }
      kk += 1;
      // (6) stopping rule, (7) next pivot row
      if (__builtin_amdgcn_readfirstlane(sqrt(nu2) * sqrt(nv2) <= tol * sqrt(nrm2) ? 1 : 0)) {
        if (++hits >= ACA_STOP_STEPS) {
          st = ACA_CONVERGED;
          break;
        }
      } else {
        hits = 0;
      }
      double bu = rused ? -1.0 : abs2(uraw);
      int bi = rused ? INT_MAX : lane;
      wave_amax(bu, bi);
      bi = __builtin_amdgcn_readfirstlane(bi);
      if (bi == INT_MAX) {
        st = ACA_CONVERGED;
        break;
      }
      ip = bi;
    }
    // factors go to a slot of exactly kk columns (or twice RC for a block continued by the
    // workgroup kernel) taken from the device pool, laid out as interleaved column pairs
    // (ld = m + n); if the pool is exhausted the block is restarted from scratch by the
    // workgroup kernel
    const int ld = m + n;
    int scap = st == ACA_OVERFLOW ? min(d.rcap, 2 * RC) : kk;
    using gT = HMX_GLOBAL T;
    gT* Ug = nullptr;
    gT* Vg = nullptr;
    if (scap > 0 && st != ACA_DENSE) {
      const int64_t need = (int64_t)scap * ld;
      // every lane issues the atomic (no lane-dependent branch); only lane 0 adds `need`, and
      // lane 0's return value is the slot offset
      unsigned long long off =
          atomicAdd(gtop, lane == 0 ? (unsigned long long)need : 0ull);
      off = ((unsigned long long)(unsigned int)__builtin_amdgcn_readlane((int)(off >> 32), 0) << 32) |
            (unsigned int)__builtin_amdgcn_readlane((int)(off & 0xffffffffu), 0);
      if (gpool != nullptr && (int64_t)off + need <= gcap) {
        Ug = (gT*)(gpool + off);
        Vg = Ug + m;
      } else {
        st = ACA_OVERFLOW;
        kk = 0;
        ip = 0;
        hits = 0;
        nrm2 = 0.0;
        rused = false;
        cused = false;
      }
    }
    if (Ug != nullptr) {
#pragma unroll
      for (int l = 0; l < RC; ++l) {
        if (l < kk) {
          if (hr) Ug[(int64_t)l * ld + lane] = u[l];
          if (hc) Vg[(int64_t)l * ld + lane] = v[l];
        }
      }
    }
    if (st == ACA_OVERFLOW) {
      uint8_t* rf = flags + d.foff;
      if (hr) rf[lane] = rused ? 1 : 0;
      if (hc) rf[m + lane] = cused ? 1 : 0;
    }
    if (lane == 0) {
      desc[b].U = (void*)Ug;
      desc[b].U1 = nullptr;
      desc[b].cap = Ug ? scap : d.cap;
      desc[b].cap1 = 0;
      desc[b].ld = ld;
    }
    if (lane == 0) {
      rank[b] = kk;
      ipiv[b] = ip | (hits << ACA_HIT_SHIFT);
      norm2[b] = nrm2;
      status[b] = st;
    }
  }
}

template <class T>
void launch_aca_wave(FarDesc* d, const int32_t* order, int nb, const double* X,
                     const double* Y, const double* Z, const double* W, int kern, const double* kp,
                     double tol, uint8_t* flags, int32_t* rank, int32_t* ipiv, int32_t* status,
                     double* norm2, T* gpool, int64_t gcap, unsigned long long* gtop,
                     hipStream_t s) {
  if (nb <= 0) return;
  int dev = 0, ncu = 0;
  HMX_HIP(hipGetDevice(&dev));
  HMX_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int grid = std::min((nb + NWAVE - 1) / NWAVE, 8 * ncu);
  hipLaunchKernelGGL((aca_wave_kernel<T, ACA_WAVE_RC>), dim3(grid), dim3(WG), 0, s, d, order, nb,
                     X, Y, Z, W, kern, kp, tol, flags, rank, ipiv, status, norm2, gpool, gcap,
                     gtop);
  HMX_LAUNCHED();
}

// Workgroups of a persistent ACA grid of one kind (ACA_KIND_BIG: 512 or 256 threads;
// ACA_KIND_MID: 256, 128 or 64; ACA_KIND_SMALL: 64): as many as can be resident at once.
template <class T>
int aca_grid(int threads, int kind) {
  int dev = 0, ncu = 0, occ = 0;
  HMX_HIP(hipGetDevice(&dev));
  HMX_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
#define HMX_ACA_OCC(...) \
  HMX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, __VA_ARGS__, threads, 0))
  if (kind == ACA_KIND_SMALL)
    HMX_ACA_OCC(aca_kernel<T, 64, false, ACA_COEF_SMALL>);
  else if (kind == ACA_KIND_BIG && threads == 512)
    HMX_ACA_OCC(aca_kernel<T, 512, true>);
  else if (kind == ACA_KIND_BIG)
    HMX_ACA_OCC(aca_kernel<T, 256, true>);
  else if (threads == 256)
    HMX_ACA_OCC(aca_kernel<T, 256, false>);
  else if (threads == 128)
    HMX_ACA_OCC(aca_kernel<T, 128, false>);
  else
    HMX_ACA_OCC(aca_kernel<T, 64, false>);
#undef HMX_ACA_OCC
  return std::max(1, occ) * ncu;
}

template <class T>
void launch_aca(FarDesc* d, const int32_t* order, int nb, int* counter, int threads, int kind,
                const double* X, const double* Y, const double* Z, const double* W, int kern,
                const double* kp, double tol, uint8_t* flags, int32_t* rank, int32_t* ipiv,
                int32_t* status, double* norm2, int fresh, T* gpool, int64_t gcap,
                unsigned long long* gtop, double2* gram, int gram_min, int64_t arena,
                hipStream_t s) {
  if (nb <= 0) return;
  // `gram` (when given) holds 2 aca_gram_order(threads, kind)^2 entries for each of
  // aca_grid(threads, kind) workgroups; blocks with m + n >= gram_min use the Gram matrices;
  // arena > 0: slots placed in per-workgroup arenas of that many entries
  const int grid = std::min(nb, aca_grid<T>(threads, kind));
#define HMX_ACA_LAUNCH(NT_, ...)                                                                 \
  hipLaunchKernelGGL((__VA_ARGS__), dim3(grid), dim3(NT_), 0, s, d, order, nb, counter, X, Y, Z, \
                     W, kern, kp, tol, flags, rank, ipiv, status, norm2, fresh, gpool, gcap,     \
                     gtop, gram, gram_min, arena)
  if (kind == ACA_KIND_SMALL)
    HMX_ACA_LAUNCH(64, aca_kernel<T, 64, false, ACA_COEF_SMALL>);
  else if (kind == ACA_KIND_BIG && threads == 512)
    HMX_ACA_LAUNCH(512, aca_kernel<T, 512, true>);
  else if (kind == ACA_KIND_BIG)
    HMX_ACA_LAUNCH(256, aca_kernel<T, 256, true>);
  else if (threads == 256)
    HMX_ACA_LAUNCH(256, aca_kernel<T, 256, false>);
  else if (threads == 128)
    HMX_ACA_LAUNCH(128, aca_kernel<T, 128, false>);
  else
    HMX_ACA_LAUNCH(64, aca_kernel<T, 64, false>);
#undef HMX_ACA_LAUNCH
  HMX_LAUNCHED();
}

#define HMX_INST(T)                                                                              \
  template void launch_aca_wave<T>(FarDesc*, const int32_t*, int, const double*,                \
                                   const double*, const double*, const double*, int,             \
                                   const double*, double, uint8_t*, int32_t*, int32_t*, int32_t*, double*, T*,  \
                                   int64_t, unsigned long long*, hipStream_t);                   \
  template void launch_aca<T>(FarDesc*, const int32_t*, int, int*, int, int, const double*,      \
                              const double*, const double*, const double*, int, const double*,   \
                              double, uint8_t*, int32_t*, int32_t*, int32_t*, double*, int, T*,  \
                              int64_t, unsigned long long*, double2*, int, int64_t, hipStream_t); \
  template int aca_grid<T>(int, int);                                                            \

HMX_INST(double2)
HMX_INST(float2)
#undef HMX_INST

}  // namespace hmx
