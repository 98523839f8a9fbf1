// hmx_api.hip -- the C ABI of libhmx: argument checks, build orchestration, product dispatch,
// queries.  All arithmetic of the operator runs in the kernels of the k_*.hip units; this file
// only sizes buffers, launches kernels and moves small index arrays.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "hmx_host.h"
#include "hmx_reg_dev.h"

using namespace hmx;

namespace {

thread_local std::string g_err;

hmx_status fail(hmx_status c, const std::string& m) {
  g_err = m;
  return c;
}

}  // namespace

void hmx::set_last_error(const std::string& m) { g_err = m; }

namespace {

#define API_TRY try {
#define API_CATCH                                            \
  }                                                          \
  catch (const hmx::Error& e) {                              \
    return fail(e.code, e.what());                           \
  }                                                          \
  catch (const std::bad_alloc&) {                            \
    return fail(HMX_ENOMEM, "host allocation failed");       \
  }                                                          \
  catch (const std::exception& e) {                          \
    return fail(HMX_EINTERNAL, e.what());                    \
  }

void defaults(hmx_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->struct_size = (int32_t)sizeof(hmx_params);
  p->tol = 1e-3;
  p->leaf_size = 64;
  p->eta = 1.5;
  p->precision = HMX_FP64;
  p->rank_model = HMX_RANK_ADAPTIVE;
  p->initial_rank = 16;
  p->force_pred_scale = 1.0;
  p->force_rank_cap = 0;
  p->pool_limit_bytes = 0;
  p->aca_big_mn = 4096;
  p->aca_gram_min_mn = 1024;
  p->aca_serial = 0;
  p->aca_mid_threads = 128;
  p->aca_big_threads = 0;
  p->aca_small_mn = 1024;
  p->aca_wave = 0;
  p->aca_arena = 1;
  p->row_shares = 1;
  p->row_share = 0;
  p->force_pool_bytes = 0;
  p->max_far_mn = 12288;
  p->regularize = 0;
  p->reg_radius = 2.0;
  p->near_mode = 0;
  p->force_block_cap = 0;
}

hmx_params resolve(const hmx_params* in) {
  hmx_params p;
  defaults(&p);
  if (in) {
    HMX_REQUIRE(in->struct_size == (int32_t)sizeof(hmx_params), HMX_EINVAL,
                "hmx_params.struct_size does not match this library (use hmx_params_default)");
    p = *in;
  }
  HMX_REQUIRE(std::isfinite(p.tol), HMX_EINVAL, "tol must be finite");
  HMX_REQUIRE(p.leaf_size >= 1, HMX_EINVAL, "leaf_size must be >= 1");
  HMX_REQUIRE(p.leaf_size <= 256, HMX_EUNSUPPORTED, "leaf_size above 256 is not supported");
  HMX_REQUIRE(std::isfinite(p.eta) && p.eta > 0, HMX_EINVAL, "eta must be finite and > 0");
  HMX_REQUIRE(p.precision == HMX_FP64 || p.precision == HMX_FP32_MIXED, HMX_EINVAL,
              "unknown precision");
  HMX_REQUIRE(p.rank_model == HMX_RANK_ADAPTIVE || p.rank_model == HMX_RANK_LEARNED, HMX_EINVAL,
              "unknown rank_model");
  HMX_REQUIRE(p.initial_rank >= 1, HMX_EINVAL, "initial_rank must be >= 1");
  HMX_REQUIRE(std::isfinite(p.force_pred_scale) && p.force_pred_scale >= 0, HMX_EINVAL,
              "force_pred_scale must be finite and >= 0");
  HMX_REQUIRE(p.force_rank_cap >= 0, HMX_EINVAL, "force_rank_cap must be >= 0");
  HMX_REQUIRE(p.pool_limit_bytes >= 0, HMX_EINVAL, "pool_limit_bytes must be >= 0");
  HMX_REQUIRE(p.aca_big_mn >= 2, HMX_EINVAL, "aca_big_mn must be >= 2");
  HMX_REQUIRE(p.aca_gram_min_mn >= 0, HMX_EINVAL, "aca_gram_min_mn must be >= 0");
  HMX_REQUIRE(p.aca_serial == 0 || p.aca_serial == 1, HMX_EINVAL, "aca_serial must be 0 or 1");
  HMX_REQUIRE(p.aca_arena == 0 || p.aca_arena == 1, HMX_EINVAL, "aca_arena must be 0 or 1");
  HMX_REQUIRE(p.aca_mid_threads == 256 || p.aca_mid_threads == 128 || p.aca_mid_threads == 64,
              HMX_EINVAL, "aca_mid_threads must be 256, 128 or 64");
  HMX_REQUIRE(p.aca_big_threads == 0 || p.aca_big_threads == 512 || p.aca_big_threads == 256,
              HMX_EINVAL, "aca_big_threads must be 0, 512 or 256");
  // 0: by precision (measured on the 245 760-point sphere: FP64 streams 16-byte factor entries
  // and runs best with one 512-thread workgroup per CU, FP32 with two 256-thread ones)
  if (p.aca_big_threads == 0) p.aca_big_threads = p.precision == HMX_FP64 ? 512 : 256;
  HMX_REQUIRE(p.aca_small_mn >= 0, HMX_EINVAL, "aca_small_mn must be >= 0");
  HMX_REQUIRE(p.aca_wave == 0 || p.aca_wave == 1, HMX_EINVAL, "aca_wave must be 0 or 1");
  HMX_REQUIRE(p.row_shares >= 1 && p.row_shares <= (1 << 20) &&
                  (p.row_shares & (p.row_shares - 1)) == 0,
              HMX_EINVAL, "row_shares must be a power of two in [1, 2^20]");
  HMX_REQUIRE(p.row_share >= 0 && p.row_share < p.row_shares, HMX_EINVAL,
              "row_share must be in [0, row_shares)");
  HMX_REQUIRE(p.force_pool_bytes >= 0, HMX_EINVAL, "force_pool_bytes must be >= 0");
  HMX_REQUIRE(p.max_far_mn >= 0, HMX_EINVAL, "max_far_mn must be >= 0");
  HMX_REQUIRE(p.row_shares == 1 || p.tol > 0, HMX_EUNSUPPORTED,
              "row shares need an H-matrix operator (tol > 0)");
  HMX_REQUIRE(p.regularize == 0 || p.regularize == 1, HMX_EINVAL, "regularize must be 0 or 1");
  HMX_REQUIRE(std::isfinite(p.reg_radius) && p.reg_radius > 0, HMX_EINVAL,
              "reg_radius must be finite and > 0");
  HMX_REQUIRE(p.regularize == 0 || p.tol > 0, HMX_EUNSUPPORTED,
              "the singular correction needs an H-matrix operator (tol > 0)");
  HMX_REQUIRE(p.near_mode == 0 || p.near_mode == 1, HMX_EINVAL, "near_mode must be 0 or 1");
  HMX_REQUIRE(p.force_block_cap >= 0, HMX_EINVAL, "force_block_cap must be >= 0");
  HMX_REQUIRE(p.near_mode == 0 || p.regularize == 0, HMX_EUNSUPPORTED,
              "near_mode 1 (near field computed in the product) cannot carry the singular "
              "correction, which is assembled into stored near blocks");
  return p;
}

Rule make_rule(const double* q_bary, const double* q_w, int32_t nq) {
  HMX_REQUIRE(q_bary && q_w, HMX_EINVAL, "null quadrature rule");
  HMX_REQUIRE(nq >= 1, HMX_EINVAL, "n_q must be >= 1");
  HMX_REQUIRE(nq <= MAX_NQ, HMX_EUNSUPPORTED, "n_q above 32 is not supported");
  Rule r{};
  r.nq = nq;
  double ws = 0.0;
  for (int q = 0; q < nq; ++q) {
    double s = 0.0;
    for (int j = 0; j < 3; ++j) {
      double l = q_bary[3 * q + j];
      HMX_REQUIRE(std::isfinite(l) && l >= -1e-12, HMX_EINVAL,
                  "barycentric coordinates must lie in the triangle");
      r.b[q][j] = l;
      s += l;
    }
    HMX_REQUIRE(std::fabs(s - 1.0) <= 1e-12, HMX_EINVAL, "barycentric coordinates must sum to 1");
    HMX_REQUIRE(std::isfinite(q_w[q]), HMX_EINVAL, "non-finite quadrature weight");
    r.w[q] = q_w[q];
    ws += q_w[q];
  }
  HMX_REQUIRE(std::fabs(ws - 1.0) <= 1e-12, HMX_EINVAL, "reference weights must sum to 1");
  return r;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

void check_build_args(int32_t kern, double k) {
  HMX_REQUIRE(kern == HMX_LAPLACE || kern == HMX_HELMHOLTZ || kern == HMX_GRADY_X ||
                  kern == HMX_GRADY_Y || kern == HMX_GRADY_Z || kern == HMX_TEST_POLY2,
              HMX_EINVAL, "unknown kernel");
  HMX_REQUIRE(std::isfinite(k) && k >= 0, HMX_EINVAL, "k must be finite and >= 0");
}

// Singular correction (Section 5.2): the rule's three points carry one linear function per
// triangle; lag[3 q + i] is the coefficient of lambda_i in L_q, the function equal to 1 at point
// q and 0 at the two others.  With B[q][i] the barycentric coordinates of point q,
// L_q(point p) = sum_i lag[q][i] B[p][i] = delta_qp, so lag = (B^-1)^T (inverse by cofactors).
void setup_reg(hmx_op* op, const Rule& r, int32_t kern) {
  HMX_REQUIRE(kern == HMX_LAPLACE || kern == HMX_HELMHOLTZ, HMX_EINVAL,
              "the singular correction needs the Laplace or Helmholtz kernel");
  HMX_REQUIRE(r.nq == 3, HMX_EINVAL, "the singular correction needs a 3-point rule");
  const double(*B)[3] = r.b;
  double cof[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      cof[i][j] = B[i1][j1] * B[i2][j2] - B[i1][j2] * B[i2][j1];
    }
  const double det = B[0][0] * cof[0][0] + B[0][1] * cof[0][1] + B[0][2] * cof[0][2];
  HMX_REQUIRE(std::fabs(det) > 1e-9, HMX_EINVAL,
              "the singular correction needs three non-collinear rule points");
  // (B^-1)[i][q] = cof[q][i] / det, so lag[q][i] = (B^-1)[i][q] = cof[q][i] / det
  for (int q = 0; q < 3; ++q)
    for (int i = 0; i < 3; ++i) op->reg_lag[3 * q + i] = cof[q][i] / det;
  op->reg = true;
}

}  // namespace

int64_t hmx_op::bytes() const {
  size_t b = X.bytes() + Y.bytes() + Z.bytes() + W.bytes() + perm.bytes() + nbegin.bytes() +
             nend.bytes() + nlevel.bytes() + child0.bytes() + child1.bytes() + parent.bytes() +
             box.bytes() + leaves.bytes() + leaf_of_node.bytes() + nearL.bytes() + near_tb.bytes() +
             near_m.bytes() + near_sb.bytes() + near_n.bytes() + near_off.bytes() +
             near_ptr.bytes() + near_pool.bytes() + farL.bytes() + far.bytes() +
             dense_pool.bytes() + far_ptr.bytes() + far_list.bytes() + xp.bytes() + tbuf.bytes() +
             partial.bytes() + tgeo.bytes();
  for (const auto& p : far_pools) b += p.bytes();
  return (int64_t)b;
}

extern "C" {

hmx_status hmx_params_default(hmx_params* p) {
  if (!p) return fail(HMX_EINVAL, "null params");
  defaults(p);
  return HMX_OK;
}

hmx_status hmx_quad_points(const double* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                           const double* q_bary, const double* q_w, int32_t n_q, double* xyzw,
                           void* stream) {
  API_TRY
  HMX_REQUIRE(vtx && tri && xyzw, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(n_vtx >= 1 && n_tri >= 1, HMX_EINVAL, "empty mesh");
  Rule r = make_rule(q_bary, q_w, n_q);
  hipStream_t s = as_stream(stream);
  const int64_t M = n_tri * n_q;
  DevBuf<int> err(1);
  fill_i32(err.p, 0, 1, s);
  launch_quad(vtx, n_vtx, tri, n_tri, r, xyzw, xyzw + M, xyzw + 2 * M, xyzw + 3 * M, err.p, s);
  int e = read1(err.p, s);
  HMX_REQUIRE(!(e & 1), HMX_EINVAL, "triangle vertex index out of range");
  HMX_REQUIRE(!(e & 2), HMX_EINVAL, "non-finite vertex coordinate");
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_build(const double* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                     const double* q_bary, const double* q_w, int32_t n_q, int32_t kern, double k,
                     const hmx_params* p, void* stream, hmx_op** out) {
  API_TRY
  HMX_REQUIRE(vtx && tri && out, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(n_vtx >= 1 && n_tri >= 1, HMX_EINVAL, "empty mesh");
  check_build_args(kern, k);
  hmx_params prm = resolve(p);
  Rule r = make_rule(q_bary, q_w, n_q);
  hipStream_t s = as_stream(stream);
  auto op = std::make_unique<hmx_op>();
  op->M = n_tri * n_q;
  op->kern = kern;
  op->k = k;
  op->p = prm;
  op->prec = prm.precision;
  if (prm.regularize) setup_reg(op.get(), r, kern);  // host checks before any device work
  op->X.alloc(op->M);
  op->Y.alloc(op->M);
  op->Z.alloc(op->M);
  op->W.alloc(op->M);
  DevBuf<int> err(1);
  fill_i32(err.p, 0, 1, s);
  launch_quad(vtx, n_vtx, tri, n_tri, r, op->X.p, op->Y.p, op->Z.p, op->W.p, err.p, s);
  int e = read1(err.p, s);
  HMX_REQUIRE(!(e & 1), HMX_EINVAL, "triangle vertex index out of range");
  HMX_REQUIRE(!(e & 2), HMX_EINVAL, "non-finite vertex coordinate");
  if (prm.regularize) {
    // triangle records (the indices were checked above)
    op->tgeo.alloc((size_t)n_tri * TGEO);
    launch_tri_geom(vtx, tri, n_tri, prm.reg_radius, op->tgeo.p, s);
  }
  finish_build(op.get(), s);
  *out = op.release();
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_build_points(const double* xyzw, int64_t M, int32_t kern, double k,
                            const hmx_params* p, void* stream, hmx_op** out) {
  API_TRY
  HMX_REQUIRE(xyzw && out, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(M >= 1, HMX_EINVAL, "M must be >= 1");
  check_build_args(kern, k);
  hmx_params prm = resolve(p);
  HMX_REQUIRE(!prm.regularize, HMX_EINVAL, "the singular correction needs the mesh (hmx_build)");
  hipStream_t s = as_stream(stream);
  auto op = std::make_unique<hmx_op>();
  op->M = M;
  op->kern = kern;
  op->k = k;
  op->p = prm;
  op->prec = prm.precision;
  op->X.alloc(M);
  op->Y.alloc(M);
  op->Z.alloc(M);
  op->W.alloc(M);
  HMX_HIP(hipMemcpyAsync(op->X.p, xyzw, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipMemcpyAsync(op->Y.p, xyzw + M, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipMemcpyAsync(op->Z.p, xyzw + 2 * M, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipMemcpyAsync(op->W.p, xyzw + 3 * M, M * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipStreamSynchronize(s));
  finish_build(op.get(), s);
  *out = op.release();
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_build_rect(const double* txyz, int64_t Mt, const double* xyzw, int64_t Ms,
                          int32_t kern, double k, const hmx_params* p, void* stream,
                          hmx_op** out) {
  API_TRY
  HMX_REQUIRE(txyz && xyzw && out, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(Mt >= 1 && Ms >= 1, HMX_EINVAL, "Mt and Ms must be >= 1");
  check_build_args(kern, k);
  hmx_params prm = resolve(p);
  HMX_REQUIRE(!prm.regularize, HMX_EINVAL, "the singular correction needs the mesh (hmx_build)");
  HMX_REQUIRE(prm.row_shares == 1, HMX_EUNSUPPORTED,
              "row shares of an operator between different point sets");
  hipStream_t s = as_stream(stream);
  auto op = std::make_unique<hmx_op>();
  op->M = Mt + Ms;
  op->kern = kern;
  op->k = k;
  op->p = prm;
  op->prec = prm.precision;
  op->rect = true;
  op->rows = Mt;
  op->cols = Ms;
  op->x_off = Mt;
  // targets first (weight 0: they are never sources), then the sources; one tree root each
  op->mesh_off = {0, Mt, Mt + Ms};
  op->mesh_k = {k, k};
  op->X.alloc(op->M);
  op->Y.alloc(op->M);
  op->Z.alloc(op->M);
  op->W.alloc(op->M);
  double* dst[3] = {op->X.p, op->Y.p, op->Z.p};
  for (int d = 0; d < 3; ++d) {
    HMX_HIP(hipMemcpyAsync(dst[d], txyz + d * Mt, Mt * 8, hipMemcpyDeviceToDevice, s));
    HMX_HIP(hipMemcpyAsync(dst[d] + Mt, xyzw + d * Ms, Ms * 8, hipMemcpyDeviceToDevice, s));
  }
  fill_f64(op->W.p, 0.0, Mt, s);
  HMX_HIP(hipMemcpyAsync(op->W.p + Mt, xyzw + 3 * Ms, Ms * 8, hipMemcpyDeviceToDevice, s));
  HMX_HIP(hipStreamSynchronize(s));
  finish_build(op.get(), s);
  *out = op.release();
  return HMX_OK;
  API_CATCH
}

namespace {
// The product's launches (no synchronisation, no allocation: capturable).
static void enqueue_matvec(const hmx_op* op, const void* x, void* y, hipStream_t s) {
  if (op->dense) {
    if (op->prec == HMX_FP64)
      launch_dense_otf<double2>(op->X.p, op->Y.p, op->Z.p, op->W.p, op->rows, op->x_off, op->cols,
                                op->kern, op->k, (const double2*)x, (double2*)op->partial.p,
                                (double2*)y, s);
    else
      launch_dense_otf<float2>(op->X.p, op->Y.p, op->Z.p, op->W.p, op->rows, op->x_off, op->cols,
                               op->kern, op->k, (const float2*)x, (float2*)op->partial.p,
                               (float2*)y, s);
    return;
  }
  auto run = [&](auto tag) {
    using T = decltype(tag);
    T* xp = (T*)op->xp.p;
    T* t = (T*)op->tbuf.p;
    launch_gather<T>((const T*)x, op->perm.p, xp, op->M, op->x_off, s);
    launch_far_vt<T>(op->far.p, op->n_far, xp, t, s);
    const NearOtfArgs otf{op->X.p, op->Y.p, op->Z.p, op->W.p, op->kern, op->kpt.p};
    launch_leaf_apply<T>(op->n_leaves, op->leaves.p, op->nbegin.p, op->nend.p, op->near_ptr.p,
                         op->near_sb.p, op->near_n.p, op->near_off.p, (const T*)op->near_pool.p,
                         op->far_ptr.p, op->far_list.p, op->far.p, t, xp, op->perm.p, op->rows,
                         (T*)y, op->max_leaf_rows, s, op->p.near_mode == 1 ? &otf : nullptr);
  };
  if (op->prec == HMX_FP64) run(double2{});
  else run(float2{});
}
}  // namespace

hmx_status hmx_matvec(const hmx_op* op, const void* x, void* y, void* stream) {
  API_TRY
  HMX_REQUIRE(op && x && y, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(x != y, HMX_EINVAL, "x and y must not alias");
  enqueue_matvec(op, x, y, as_stream(stream));
  return HMX_OK;
  API_CATCH
}

namespace {
// Scratch of the several-vector product: 4 permuted vectors and 4 vectors of far-block
// coefficients V^H x (each group holds at most four vectors).
static size_t multi_work_bytes(const hmx_op* op) {
  return op->dense ? 0 : (size_t)4 * (op->M + std::max<int64_t>(op->t_len, 1)) * op->elem;
}
}  // namespace

hmx_status hmx_matvec_multi_work_bytes(const hmx_op* op, size_t* bytes) {
  if (!op || !bytes) return fail(HMX_EINVAL, "null pointer");
  *bytes = multi_work_bytes(op);
  return HMX_OK;
}

namespace {
// Argument checks of the several-vector product (host only, before any enqueue).
static void check_multi_args(const hmx_op* op, int32_t nr, const void* const* x,
                             void* const* y) {
  HMX_REQUIRE(op && x && y, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(nr >= 1, HMX_EINVAL, "nr must be >= 1");
  for (int r = 0; r < nr; ++r) HMX_REQUIRE(x[r] && y[r], HMX_EINVAL, "null vector pointer");
  // vectors run in successive groups, so an output that is also an input (of any vector) or
  // that appears twice would be overwritten before it is read or write over another result
  for (int r = 0; r < nr; ++r)
    for (int q = 0; q < nr; ++q) {
      HMX_REQUIRE((const void*)y[r] != x[q], HMX_EINVAL, "an output vector aliases an input vector");
      HMX_REQUIRE(q <= r || y[r] != y[q], HMX_EINVAL, "an output vector appears twice");
    }
}

// The several-vector product's launches on `work` (no synchronisation, no allocation).
static void enqueue_multi(const hmx_op* op, int32_t nr, const void* const* x, void* const* y,
                          void* work, hipStream_t s) {
  auto run = [&](auto tag) {
    using T = decltype(tag);
    T* xpm = (T*)work;
    T* tm = xpm + 4 * op->M;
    for (int r0 = 0; r0 < nr;) {
      const int left = nr - r0;
      // (an operator whose near field is computed in the product takes one vector at a time)
      const int g = op->dense || op->p.near_mode == 1 ? 1 : (left >= 4 ? 4 : left >= 2 ? 2 : 1);
      if (g == 1) {
        enqueue_matvec(op, x[r0], y[r0], s);
      } else {
        const T* xs[4];
        T* ys[4];
        for (int r = 0; r < g; ++r) {
          xs[r] = (const T*)x[r0 + r];
          ys[r] = (T*)y[r0 + r];
        }
        launch_matvec_multi<T>(op, g, xs, ys, xpm, tm, s);
      }
      r0 += g;
    }
  };
  if (op->prec == HMX_FP64) run(double2{});
  else run(float2{});
}
}  // namespace

hmx_status hmx_matvec_multi(const hmx_op* op, int32_t nr, const void* const* x, void* const* y,
                            void* work, void* stream) {
  API_TRY
  check_multi_args(op, nr, x, y);
  HMX_REQUIRE(op->dense || work, HMX_EINVAL, "an H-matrix operator needs the work buffer");
  enqueue_multi(op, nr, x, y, work, as_stream(stream));
  return HMX_OK;
  API_CATCH
}

// ------------------------------------------------------------ product without allocation
// Scratch of hmx_matvec_multi_static: a file-scope device array, one copy on every device the
// library runs on, held until the process ends.  Host code never passes the array's name to a
// kernel (on the host it only stands for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[HMX_STATIC_WORK_BYTES];

namespace {
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
static void* static_scratch() {
  int dev = 0;
  HMX_HIP(hipGetDevice(&dev));
  HMX_REQUIRE(dev >= 0 && dev < kMaxDevices, HMX_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      throw Error(HMX_EDEVICE, std::string("hipGetSymbolAddress of the static scratch: ") +
                                   hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

hmx_status hmx_matvec_multi_static(const hmx_op* op, int32_t nr, const void* const* x,
                                   void* const* y, void* stream) {
  API_TRY
  check_multi_args(op, nr, x, y);
  const size_t need = multi_work_bytes(op);
  HMX_REQUIRE(need <= HMX_STATIC_WORK_BYTES, HMX_EINVAL,
              "the operator's product needs " + std::to_string(need) +
                  " bytes of scratch, more than the static scratch holds (" +
                  std::to_string((size_t)HMX_STATIC_WORK_BYTES) + " bytes)");
  void* work = need > 0 ? static_scratch() : nullptr;
  enqueue_multi(op, nr, x, y, work, as_stream(stream));
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_graph_create(const hmx_op* op, const void* x, void* y, hmx_graph** out) {
  API_TRY
  HMX_REQUIRE(op && x && y && out, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(x != y, HMX_EINVAL, "x and y must not alias");
  auto g = std::make_unique<hmx_graph>();
  hipStream_t cs = nullptr;
  HMX_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  try {
    HMX_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      enqueue_matvec(op, x, y, cs);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(cs, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    HMX_HIP(hipStreamEndCapture(cs, &g->graph));
    HMX_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  } catch (...) {
    (void)hipStreamDestroy(cs);
    throw;
  }
  HMX_HIP(hipStreamDestroy(cs));
  *out = g.release();
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_graph_launch(hmx_graph* g, int32_t reps, void* stream) {
  API_TRY
  HMX_REQUIRE(g && g->exec, HMX_EINVAL, "null graph");
  HMX_REQUIRE(reps >= 0, HMX_EINVAL, "reps must be >= 0");
  for (int32_t r = 0; r < reps; ++r) HMX_HIP(hipGraphLaunch(g->exec, as_stream(stream)));
  return HMX_OK;
  API_CATCH
}

void hmx_graph_destroy(hmx_graph* g) { delete g; }

hmx_status hmx_build_batch(const hmx_mesh* meshes, int32_t n_meshes, const double* q_bary,
                           const double* q_w, int32_t n_q, int32_t kern, const hmx_params* p,
                           void* stream, hmx_op** out) {
  API_TRY
  HMX_REQUIRE(meshes && out, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(n_meshes >= 1, HMX_EINVAL, "n_meshes must be >= 1");
  hmx_params prm = resolve(p);
  HMX_REQUIRE(prm.tol > 0, HMX_EINVAL, "a batch operator needs tol > 0");
  HMX_REQUIRE(prm.row_shares == 1, HMX_EUNSUPPORTED, "row shares of a batch operator");
  Rule r = make_rule(q_bary, q_w, n_q);
  auto op = std::make_unique<hmx_op>();
  op->mesh_off.assign(1, 0);
  for (int32_t i = 0; i < n_meshes; ++i) {
    const hmx_mesh& m = meshes[i];
    HMX_REQUIRE(m.vtx && m.tri, HMX_EINVAL, "null mesh pointer");
    HMX_REQUIRE(m.n_vtx >= 1 && m.n_tri >= 1, HMX_EINVAL, "empty mesh");
    check_build_args(kern, m.k);
    HMX_REQUIRE(m.n_tri <= (int64_t(1) << 23), HMX_EUNSUPPORTED,
                "H-matrix mode supports at most 2^23 - 1 points");
    op->mesh_off.push_back(op->mesh_off.back() + m.n_tri * n_q);
    op->mesh_k.push_back(m.k);
  }
  hipStream_t s = as_stream(stream);
  op->M = op->mesh_off.back();
  HMX_REQUIRE(op->M < (int64_t(1) << 23), HMX_EUNSUPPORTED,
              "H-matrix mode supports at most 2^23 - 1 points");
  op->kern = kern;
  op->k = op->mesh_k[0];
  op->p = prm;
  op->prec = prm.precision;
  if (prm.regularize) setup_reg(op.get(), r, kern);  // host checks before any device work
  op->X.alloc(op->M);
  op->Y.alloc(op->M);
  op->Z.alloc(op->M);
  op->W.alloc(op->M);
  DevBuf<int> err(1);
  fill_i32(err.p, 0, 1, s);
  for (int32_t i = 0; i < n_meshes; ++i) {
    const int64_t o = op->mesh_off[i];
    launch_quad(meshes[i].vtx, meshes[i].n_vtx, meshes[i].tri, meshes[i].n_tri, r, op->X.p + o,
                op->Y.p + o, op->Z.p + o, op->W.p + o, err.p, s);
  }
  int e = read1(err.p, s);
  HMX_REQUIRE(!(e & 1), HMX_EINVAL, "triangle vertex index out of range");
  HMX_REQUIRE(!(e & 2), HMX_EINVAL, "non-finite vertex coordinate");
  if (prm.regularize) {
    // the records of all meshes, concatenated like their points (triangle o / 3 of point o)
    op->tgeo.alloc((size_t)(op->M / n_q) * TGEO);
    for (int32_t i = 0; i < n_meshes; ++i)
      launch_tri_geom(meshes[i].vtx, meshes[i].tri, meshes[i].n_tri, prm.reg_radius,
                      op->tgeo.p + (op->mesh_off[i] / n_q) * TGEO, s);
  }
  finish_build(op.get(), s);
  *out = op.release();
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_mesh_offsets(const hmx_op* op, int64_t* off, int32_t cap, int32_t* n_meshes) {
  if (!op || !n_meshes) return fail(HMX_EINVAL, "null pointer");
  // an operator between different point sets has one source set: offsets {0, cols} of x
  const std::vector<int64_t> rect_off = {0, op->cols};
  const std::vector<int64_t>& mo = op->rect ? rect_off : op->mesh_off;
  const int32_t n = (int32_t)mo.size() - 1;
  if (off) {
    if (cap < n + 1) return fail(HMX_EINVAL, "offset array too small");
    std::memcpy(off, mo.data(), sizeof(int64_t) * (n + 1));
  }
  *n_meshes = n;
  return HMX_OK;
}

hmx_status hmx_info(const hmx_op* op, hmx_info_t* out) {
  if (!op || !out) return fail(HMX_EINVAL, "null pointer");
  std::memset(out, 0, sizeof(*out));
  out->n_points = op->M;
  out->n_nodes = op->n_nodes;
  out->n_leaves = op->n_leaves;
  out->n_near = op->n_near;
  out->n_far = op->n_far;
  out->near_entries = op->near_entries;
  out->far_entries = op->far_entries;
  out->dense_far = op->dense_far;
  out->dense_far_entries = op->dense_far_entries;
  out->max_rank = op->max_rank;
  out->sum_rank = op->sum_rank;
  out->overflow_blocks = op->overflow_blocks;
  out->bytes = op->bytes();
  out->precision = op->prec;
  out->is_dense = op->dense ? 1 : 0;
  out->t_tree_ms = op->t_tree;
  out->t_blocks_ms = op->t_blocks;
  out->t_near_ms = op->t_near;
  out->t_aca_ms = op->t_aca;
  out->t_total_ms = op->t_total;
  out->kernel_evals = op->kernel_evals;
  out->factor_bytes = op->pool_used_bytes;
  out->predicted_entries = op->predicted_entries;
  for (int c = 0; c < 4; ++c) {
    out->aca_blocks[c] = op->aca_blocks[c];
    out->aca_ms[c] = op->aca_ms[c];
    out->aca_bytes[c] = op->aca_bytes[c];
  }
  out->aca_rounds = op->aca_rounds;
  out->row_begin = op->dense ? 0 : op->row_begin;
  out->row_end = op->dense ? op->M : op->row_end;
  out->n_rows = op->rows;
  out->n_cols = op->cols;
  out->pool_reserved_bytes = op->pool_reserved_bytes;
  return HMX_OK;
}

hmx_status hmx_export_tree(const hmx_op* op, int32_t* perm, int64_t* begin, int64_t* end,
                           int32_t* level, int32_t* child0, int32_t* child1, double* box) {
  API_TRY
  HMX_REQUIRE(op, HMX_EINVAL, "null operator");
  HMX_REQUIRE(!op->dense, HMX_EINVAL, "dense operators have no tree");
  hipStream_t s = nullptr;
  const int n = op->n_nodes;
  std::vector<int32_t> tmp;
  if (perm) {
    to_host(tmp, op->perm.p, op->M, s);
    std::memcpy(perm, tmp.data(), op->M * 4);
  }
  if (begin) {
    to_host(tmp, op->nbegin.p, n, s);
    for (int i = 0; i < n; ++i) begin[i] = tmp[i];
  }
  if (end) {
    to_host(tmp, op->nend.p, n, s);
    for (int i = 0; i < n; ++i) end[i] = tmp[i];
  }
  if (level) {
    to_host(tmp, op->nlevel.p, n, s);
    std::memcpy(level, tmp.data(), n * 4);
  }
  if (child0) {
    to_host(tmp, op->child0.p, n, s);
    std::memcpy(child0, tmp.data(), n * 4);
  }
  if (child1) {
    to_host(tmp, op->child1.p, n, s);
    std::memcpy(child1, tmp.data(), n * 4);
  }
  if (box) {
    std::vector<double> hb;
    to_host(hb, op->box.p, 6 * (size_t)n, s);
    std::memcpy(box, hb.data(), 6 * (size_t)n * 8);
  }
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_export_blocks(const hmx_op* op, int64_t* near_rc, int64_t* far_rc, int32_t* ranks) {
  API_TRY
  HMX_REQUIRE(op, HMX_EINVAL, "null operator");
  HMX_REQUIRE(!op->dense, HMX_EINVAL, "dense operators have no blocks");
  hipStream_t s = nullptr;
  if (near_rc && op->n_near) {
    std::vector<int32_t> a, b, c, d;
    to_host(a, op->near_tb.p, op->n_near, s);
    to_host(b, op->near_m.p, op->n_near, s);
    to_host(c, op->near_sb.p, op->n_near, s);
    to_host(d, op->near_n.p, op->n_near, s);
    for (int64_t i = 0; i < op->n_near; ++i) {
      near_rc[4 * i] = a[i];
      near_rc[4 * i + 1] = a[i] + b[i];
      near_rc[4 * i + 2] = c[i];
      near_rc[4 * i + 3] = c[i] + d[i];
    }
  }
  std::vector<FarRec> rec;
  to_host(rec, op->far.p, op->n_far, s);
  for (int64_t i = 0; i < op->n_far; ++i) {
    const FarRec& f = rec[i];
    if (far_rc) {
      far_rc[4 * i] = f.tb;
      far_rc[4 * i + 1] = f.tb + f.m;
      far_rc[4 * i + 2] = f.sb;
      far_rc[4 * i + 3] = f.sb + f.n;
    }
    if (ranks) ranks[i] = f.dense ? -1 : f.r;
  }
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_export_far(const hmx_op* op, int64_t b, void* U, void* V, int32_t* rank) {
  API_TRY
  HMX_REQUIRE(op && U && rank, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(!op->dense, HMX_EINVAL, "dense operators have no far blocks");
  HMX_REQUIRE(b >= 0 && b < op->n_far, HMX_EINVAL, "far block index out of range");
  FarRec f;
  HMX_HIP(hipMemcpy(&f, op->far.p + b, sizeof(FarRec), hipMemcpyDeviceToHost));
  if (f.dense) {
    HMX_HIP(hipMemcpy(U, f.U, (size_t)f.m * f.n * op->elem, hipMemcpyDeviceToHost));
    *rank = -1;
  } else {
    HMX_REQUIRE(V || f.r == 0, HMX_EINVAL, "null V");
    if (f.r) {
      // columns of stride ldu / ldv in up to two segments on the device, packed column-major on
      // the host
      const size_t es = op->elem;
      const int r0 = std::min(f.r, f.split), r1 = f.r - r0;
      unsigned char* hu = (unsigned char*)U;
      unsigned char* hv = (unsigned char*)V;
      HMX_HIP(hipMemcpy2D(hu, (size_t)f.m * es, f.U, (size_t)f.ldu * es, (size_t)f.m * es, r0,
                          hipMemcpyDeviceToHost));
      HMX_HIP(hipMemcpy2D(hv, (size_t)f.n * es, f.V, (size_t)f.ldv * es, (size_t)f.n * es, r0,
                          hipMemcpyDeviceToHost));
      if (r1 > 0) {
        HMX_HIP(hipMemcpy2D(hu + (size_t)r0 * f.m * es, (size_t)f.m * es, f.U1, (size_t)f.ldu * es,
                            (size_t)f.m * es, r1, hipMemcpyDeviceToHost));
        HMX_HIP(hipMemcpy2D(hv + (size_t)r0 * f.n * es, (size_t)f.n * es, f.V1, (size_t)f.ldv * es,
                            (size_t)f.n * es, r1, hipMemcpyDeviceToHost));
      }
    }
    *rank = f.r;
  }
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_import_far(hmx_op* op, const int32_t* ranks, const void* U, const void* V) {
  API_TRY
  HMX_REQUIRE(op && ranks, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(!op->dense, HMX_EINVAL, "dense operators have no far blocks");
  const int64_t nf = op->n_far;
  std::vector<FarRec> rec;
  to_host(rec, op->far.p, nf, (hipStream_t) nullptr);
  int64_t total = 0, trun = 0;
  for (int64_t b = 0; b < nf; ++b) {
    const FarRec& f = rec[b];
    if (f.dense) {
      HMX_REQUIRE(ranks[b] == -1, HMX_EINVAL, "a far block stored dense must be given rank -1");
      continue;
    }
    HMX_REQUIRE(ranks[b] >= 0 && ranks[b] <= std::min(f.m, f.n), HMX_EINVAL,
                "rank out of range for a low-rank far block");
    total += (int64_t)ranks[b] * (f.m + f.n);
  }
  HMX_REQUIRE(total == 0 || (U && V), HMX_EINVAL, "null factors");
  // factors in one new pool: U_b then V_b for every low-rank block in turn
  DevBuf<unsigned char> pool(std::max<int64_t>(total, 1) * op->elem);
  int64_t ou = 0, ov = 0, off = 0;
  const unsigned char* hu = (const unsigned char*)U;
  const unsigned char* hv = (const unsigned char*)V;
  op->far_entries = op->sum_rank = op->max_rank = 0;
  for (int64_t b = 0; b < nf; ++b) {
    FarRec& f = rec[b];
    f.toff = trun;
    if (f.dense) {
      trun += f.n;
      continue;
    }
    const int64_t r = ranks[b];
    unsigned char* du = pool.p + off * op->elem;
    unsigned char* dv = du + r * f.m * op->elem;
    if (r) {
      HMX_HIP(hipMemcpy(du, hu + ou * op->elem, r * f.m * op->elem, hipMemcpyHostToDevice));
      HMX_HIP(hipMemcpy(dv, hv + ov * op->elem, r * f.n * op->elem, hipMemcpyHostToDevice));
    }
    ou += r * f.m;
    ov += r * f.n;
    off += r * (f.m + f.n);
    f.r = (int32_t)r;
    f.U = du;
    f.V = dv;
    f.ldu = f.m;
    f.ldv = f.n;
    f.split = (int32_t)r;
    f.U1 = nullptr;
    f.V1 = nullptr;
    trun += r;
    op->far_entries += r * (f.m + f.n);
    op->sum_rank += r;
    op->max_rank = std::max<int64_t>(op->max_rank, r);
  }
  HMX_HIP(hipMemcpy(op->far.p, rec.data(), nf * sizeof(FarRec), hipMemcpyHostToDevice));
  op->far_pools.push_back(std::move(pool));
  op->t_len = trun;
  op->tbuf.alloc(std::max<size_t>((size_t)trun * op->elem, op->elem));
  return HMX_OK;
  API_CATCH
}

void hmx_destroy(hmx_op* op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  delete op;
}

}  // extern "C"

// ------------------------------------------------------------------ Galerkin P1 and GMRES
// The P1 space of the mesh an operator was built on: the rule, the point weights (original
// order), the triangles and, per vertex, its incidences (3 t + j, increasing t), plus scratch
// vectors of M entries for the Galerkin product.
struct hmx_p1 {
  const hmx_op* op = nullptr;
  int64_t nv = 0, nt = 0, M = 0;
  hmx::P1Rule rule{};
  hmx::DevBuf<int32_t> tri, inc;
  hmx::DevBuf<int64_t> ptr;
  hmx::DevBuf<double> w;
  hmx::DevBuf<unsigned char> zp, kp;
};

namespace {

template <class T>
void galerkin_enqueue(const hmx_p1* P, const T* xv, T* yv, hipStream_t s) {
  launch_p1_interp<T>(P->tri.p, P->nt, P->rule, xv, (T*)P->zp.p, s);
  enqueue_matvec(P->op, P->zp.p, P->kp.p, s);
  launch_p1_project<T>(P->ptr.p, P->inc.p, P->nv, P->rule, P->w.p, (const T*)P->kp.p, yv, s);
}

// Restarted GMRES(m) for A x = b (apply(v, out): out = A v on the stream), from x = 0:
// classical Gram-Schmidt with one reorthogonalisation (two batched dot launches per step, the
// coefficients applied from device memory, one copy to the host per step), complex Givens
// rotations on the host, stop when the residual estimate falls to tol ||b|| or after max_it
// products; each cycle starts from the true residual b - A x, which is also what is reported.
template <class T, class Apply>
void gmres_run(Apply apply, int64_t n, const T* b, T* x, int m, int max_it, double tol,
               hipStream_t s, int32_t* iters, double* relres) {
  using cd = std::complex<double>;
  DevBuf<T> V((size_t)n * (m + 1)), w(n), r(n);
  DevBuf<double2> partial((size_t)mdot_chunks(n) * (m + 1)), dd(m + 1), hd(m + 1);
  // one step's Gram-Schmidt coefficients (two passes) and the new vector's squared norm stay on
  // the device between the kernels and come back to the host in one copy
  DevBuf<double2> step_d((size_t)2 * (m + 1) + 1);
  std::vector<double2> hbuf(m + 1), step_h(2 * (m + 1) + 1);
  auto col = [&](int c) { return V.p + (int64_t)c * n; };
  auto norm = [&](const T* vec) {
    launch_mdot<T>(vec, n, 1, vec, n, partial.p, dd.p, s);
    double2 v;
    HMX_HIP(hipMemcpyAsync(&v, dd.p, sizeof(double2), hipMemcpyDeviceToHost, s));
    HMX_HIP(hipStreamSynchronize(s));
    return std::sqrt(std::max(v.x, 0.0));
  };
  auto subtract = [&](const std::vector<cd>& h, int nc, T* vec, double sign) {
    for (int c = 0; c < nc; ++c) hbuf[c] = make_double2(h[c].real(), h[c].imag());
    HMX_HIP(hipMemcpyAsync(hd.p, hbuf.data(), nc * sizeof(double2), hipMemcpyHostToDevice, s));
    launch_gemv_update<T>(V.p, n, hd.p, nc, sign, vec, n, s);
  };
  HMX_HIP(hipMemsetAsync(x, 0, n * sizeof(T), s));
  const double bnorm = norm(b);
  int it = 0;
  double res = 0.0;
  if (bnorm == 0.0) {
    *iters = 0;
    *relres = 0.0;
    return;
  }
  std::vector<cd> H((size_t)(m + 1) * m), g(m + 1), sn(m), y(m);
  std::vector<double> cs(m);
  auto Hc = [&](int i, int j) -> cd& { return H[(size_t)i * m + j]; };
  for (;;) {
    if (it == 0) {
      HMX_HIP(hipMemcpyAsync(r.p, b, n * sizeof(T), hipMemcpyDeviceToDevice, s));
    } else {
      apply(x, w.p);
      launch_vec<T>(w.p, b, 0.0, 1, r.p, n, s);  // r = b - A x
    }
    const double beta = norm(r.p);
    res = beta / bnorm;
    if (res <= tol || it >= max_it) break;
    launch_vec<T>(r.p, nullptr, 1.0 / beta, 0, col(0), n, s);
    std::fill(g.begin(), g.end(), cd(0.0));
    g[0] = beta;
    int k = 0;  // columns of this cycle
    while (k < m) {
      const int j = k;
      apply(col(j), w.p);
      ++it;
      double2* d1 = step_d.p;
      double2* d2 = step_d.p + (m + 1);
      double2* dn = step_d.p + 2 * (m + 1);
      launch_mdot<T>(V.p, n, j + 1, w.p, n, partial.p, d1, s);  // h = V^H w
      launch_gemv_update<T>(V.p, n, d1, j + 1, -1.0, w.p, n, s);
      launch_mdot<T>(V.p, n, j + 1, w.p, n, partial.p, d2, s);  // reorthogonalisation
      launch_gemv_update<T>(V.p, n, d2, j + 1, -1.0, w.p, n, s);
      launch_mdot<T>(w.p, n, 1, w.p, n, partial.p, dn, s);
      HMX_HIP(hipMemcpyAsync(step_h.data(), step_d.p, step_h.size() * sizeof(double2),
                             hipMemcpyDeviceToHost, s));
      HMX_HIP(hipStreamSynchronize(s));
      for (int c = 0; c <= j; ++c)
        Hc(c, j) = cd(step_h[c].x, step_h[c].y) + cd(step_h[m + 1 + c].x, step_h[m + 1 + c].y);
      const double hn = std::sqrt(std::max(step_h[2 * (m + 1)].x, 0.0));
      Hc(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {  // previous rotations
        const cd t = cs[i] * Hc(i, j) + sn[i] * Hc(i + 1, j);
        Hc(i + 1, j) = -std::conj(sn[i]) * Hc(i, j) + cs[i] * Hc(i + 1, j);
        Hc(i, j) = t;
      }
      const cd a = Hc(j, j), bb = Hc(j + 1, j);
      const double t = std::sqrt(std::norm(a) + std::norm(bb));
      if (std::abs(a) == 0.0) {
        cs[j] = 0.0;
        sn[j] = 1.0;
      } else {
        cs[j] = std::abs(a) / t;
        sn[j] = (a / std::abs(a)) * std::conj(bb) / t;
      }
      Hc(j, j) = cs[j] * a + sn[j] * bb;
      Hc(j + 1, j) = 0.0;
      g[j + 1] = -std::conj(sn[j]) * g[j];
      g[j] = cs[j] * g[j];
      ++k;
      if (hn > 0.0) launch_vec<T>(w.p, nullptr, 1.0 / hn, 0, col(j + 1), n, s);
      if (std::abs(g[j + 1]) <= tol * bnorm || it >= max_it || hn == 0.0) break;
    }
    for (int i = k - 1; i >= 0; --i) {  // H y = g, upper triangular
      cd acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= Hc(i, l) * y[l];
      y[i] = acc / Hc(i, i);
    }
    subtract(y, k, x, 1.0);  // x += V y
  }
  *iters = it;
  *relres = res;
}

}  // namespace

extern "C" {

hmx_status hmx_p1_create(const hmx_op* op, const double* vtx, int64_t n_vtx, const int32_t* tri,
                         int64_t n_tri, const double* q_bary, const double* q_w, int32_t n_q,
                         void* stream, hmx_p1** out) {
  API_TRY
  HMX_REQUIRE(op && vtx && tri && out, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(n_vtx >= 1 && n_tri >= 1, HMX_EINVAL, "empty mesh");
  HMX_REQUIRE(!op->rect, HMX_EINVAL, "the P1 space needs an operator on the mesh's own points");
  HMX_REQUIRE(op->M == n_tri * (int64_t)n_q, HMX_EINVAL,
              "the operator's points are not this mesh's quadrature points (M != n_q n_tri)");
  HMX_REQUIRE(op->dense || op->p.row_shares == 1, HMX_EUNSUPPORTED,
              "the Galerkin product needs all rows of the operator (no row share)");
  Rule r = make_rule(q_bary, q_w, n_q);
  hipStream_t s = as_stream(stream);
  auto P = std::make_unique<hmx_p1>();
  P->op = op;
  P->nv = n_vtx;
  P->nt = n_tri;
  P->M = op->M;
  P->rule.nq = n_q;
  for (int q = 0; q < n_q; ++q)
    for (int j = 0; j < 3; ++j) P->rule.b[q][j] = r.b[q][j];
  // point weights in the original order (and the range check of the triangles)
  DevBuf<double> X(P->M), Y(P->M), Z(P->M);
  P->w.alloc(P->M);
  DevBuf<int> err(1);
  fill_i32(err.p, 0, 1, s);
  launch_quad(vtx, n_vtx, tri, n_tri, r, X.p, Y.p, Z.p, P->w.p, err.p, s);
  const int e = read1(err.p, s);
  HMX_REQUIRE(!(e & 1), HMX_EINVAL, "triangle vertex index out of range");
  HMX_REQUIRE(!(e & 2), HMX_EINVAL, "non-finite vertex coordinate");
  P->tri.alloc(3 * n_tri);
  HMX_HIP(hipMemcpyAsync(P->tri.p, tri, 3 * n_tri * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  // vertex incidences (counting sort on the host: increasing t within each vertex)
  std::vector<int32_t> ht;
  to_host(ht, tri, 3 * n_tri, s);
  std::vector<int64_t> hp(n_vtx + 1, 0);
  for (int64_t i = 0; i < 3 * n_tri; ++i) hp[ht[i] + 1]++;
  for (int64_t v = 0; v < n_vtx; ++v) hp[v + 1] += hp[v];
  std::vector<int32_t> hi(3 * n_tri);
  std::vector<int64_t> fillp(hp.begin(), hp.end() - 1);
  for (int64_t i = 0; i < 3 * n_tri; ++i) hi[fillp[ht[i]]++] = (int32_t)i;
  P->ptr.alloc(n_vtx + 1);
  P->inc.alloc(3 * n_tri);
  HMX_HIP(hipMemcpyAsync(P->ptr.p, hp.data(), hp.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  HMX_HIP(hipMemcpyAsync(P->inc.p, hi.data(), hi.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  P->zp.alloc((size_t)P->M * op->elem);
  P->kp.alloc((size_t)P->M * op->elem);
  HMX_HIP(hipStreamSynchronize(s));
  *out = P.release();
  return HMX_OK;
  API_CATCH
}

void hmx_p1_destroy(hmx_p1* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  delete p;
}

hmx_status hmx_p1_interp(const hmx_p1* p, const void* xv, void* xp, void* stream) {
  if (!p || !xv || !xp) return fail(HMX_EINVAL, "null pointer");
  API_TRY
  if (p->op->prec == HMX_FP64)
    launch_p1_interp<double2>(p->tri.p, p->nt, p->rule, (const double2*)xv, (double2*)xp, as_stream(stream));
  else
    launch_p1_interp<float2>(p->tri.p, p->nt, p->rule, (const float2*)xv, (float2*)xp, as_stream(stream));
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_p1_project(const hmx_p1* p, const void* zp, void* yv, void* stream) {
  if (!p || !zp || !yv) return fail(HMX_EINVAL, "null pointer");
  API_TRY
  if (p->op->prec == HMX_FP64)
    launch_p1_project<double2>(p->ptr.p, p->inc.p, p->nv, p->rule, p->w.p, (const double2*)zp,
                               (double2*)yv, as_stream(stream));
  else
    launch_p1_project<float2>(p->ptr.p, p->inc.p, p->nv, p->rule, p->w.p, (const float2*)zp,
                              (float2*)yv, as_stream(stream));
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_galerkin_matvec(const hmx_p1* p, const void* xv, void* yv, void* stream) {
  if (!p || !xv || !yv) return fail(HMX_EINVAL, "null pointer");
  API_TRY
  if (p->op->prec == HMX_FP64)
    galerkin_enqueue<double2>(p, (const double2*)xv, (double2*)yv, as_stream(stream));
  else
    galerkin_enqueue<float2>(p, (const float2*)xv, (float2*)yv, as_stream(stream));
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_gmres(const hmx_p1* p, const void* b, void* x, int32_t restart, int32_t max_iter,
                     double tol, void* stream, int32_t* iters, double* relres) {
  API_TRY
  HMX_REQUIRE(p && b && x && iters && relres, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(restart >= 1 && restart <= 1000, HMX_EINVAL, "restart must be in [1, 1000]");
  HMX_REQUIRE(max_iter >= 0, HMX_EINVAL, "max_iter must be >= 0");
  HMX_REQUIRE(std::isfinite(tol) && tol >= 0, HMX_EINVAL, "tol must be finite and >= 0");
  hipStream_t s = as_stream(stream);
  if (p->op->prec == HMX_FP64)
    gmres_run<double2>([&](const double2* v, double2* out) { galerkin_enqueue<double2>(p, v, out, s); },
                       p->nv, (const double2*)b, (double2*)x, restart, max_iter, tol, s, iters, relres);
  else
    gmres_run<float2>([&](const float2* v, float2* out) { galerkin_enqueue<float2>(p, v, out, s); },
                      p->nv, (const float2*)b, (float2*)x, restart, max_iter, tol, s, iters, relres);
  return HMX_OK;
  API_CATCH
}

const char* hmx_last_error(void) { return g_err.c_str(); }

void hmx_release_cache(void) { dev_release_cache(); }

}  // extern "C"

// ------------------------------------------------------------------ RWG elements, EFIE/MFIE/CFIE
// The RWG space of a closed, consistently oriented mesh: per triangle the edge of each local
// vertex (tedge), its orientation and a geometry record; per edge its two incidences 3 t + j
// (the triangle running along it a -> b first); the point weights; and the operators: the
// single layer for the EFIE terms, the three gradient kernels for the MFIE term.  Scratch: 14
// vectors of M entries (the RWG field and its divergence, the four single-layer products, the
// six gradient products).
struct hmx_rwg {
  const hmx_op* single = nullptr;
  const hmx_op* grad[3] = {nullptr, nullptr, nullptr};
  const hmx_op* any = nullptr;
  int64_t nt = 0, ne = 0, M = 0;
  double k = 0.0;
  int32_t prec = HMX_FP64;
  hmx::P1Rule rule{};
  hmx::DevBuf<int32_t> tedge, einc, edges;
  hmx::DevBuf<double> rec, w;
  hmx::DevBuf<unsigned char> scratch;
  // several-vector products: nr permuted inputs and nr intermediate vectors V^T x of one operator
  hmx::DevBuf<unsigned char> xpm, tm;
  template <class T>
  T* vec(int i) const {
    return (T*)scratch.p + (int64_t)i * M;
  }
};

namespace {

// y = A x, A = -beta T + (1 - beta) (Id / 2 - NxK):
//   T = i k sum_d Psi_d^T W K Psi_d - (i / k) D^T W K D      (K the single layer)
//   NxK x = <n x psi_i, c>,  c_e = G_{e+1} u_{e+2} - G_{e+2} u_{e+1}  (G_d the gradient kernels)
// y_r = K x_r for nr vectors: one several-vector product on an H-matrix operator (its entries
// read once), one product per vector on a dense one or on one whose near field is computed in
// the product
template <class T>
void matvec_n(const hmx_rwg* R, const hmx_op* op, int nr, const T* const* x, T* const* y,
              hipStream_t s) {
  if (op->dense || op->p.near_mode == 1) {
    for (int r = 0; r < nr; ++r) enqueue_matvec(op, x[r], y[r], s);
    return;
  }
  launch_matvec_multi<T>(op, nr, x, y, (T*)R->xpm.p, (T*)R->tm.p, s);
}

template <class T>
void cfie_enqueue(const hmx_rwg* R, double beta, const T* x, T* y, hipStream_t s) {
  T* u = R->vec<T>(0);  // u_0..u_2 = Psi x, u_3 = D x  (slots 0..3)
  launch_rwg_interp<T>(R->rec.p, R->tedge.p, R->nt, R->rule, x, u, s);
  RwgTerms<T> a;
  if (beta != 0.0) {
    const T* in[4] = {R->vec<T>(0), R->vec<T>(1), R->vec<T>(2), R->vec<T>(3)};
    T* out[4] = {R->vec<T>(4), R->vec<T>(5), R->vec<T>(6), R->vec<T>(7)};
    matvec_n<T>(R, R->single, 4, in, out, s);
    for (int d = 0; d < 3; ++d) a.ku[d] = R->vec<T>(4 + d);
    a.kv = R->vec<T>(7);
    a.aT = make_double2(0.0, -beta * R->k);
    a.aD = make_double2(0.0, beta / R->k);
  }
  if (beta != 1.0) {
    // c_e = G_{e+1} u_{e+2} - G_{e+2} u_{e+1} (slots 8 + e and 11 + e): operator G_d takes
    // u_{d+1} into slot 8 + (d - 1) and u_{d+2} into slot 11 + (d + 1)
    for (int d = 0; d < 3; ++d) {
      const T* in[2] = {R->vec<T>((d + 1) % 3), R->vec<T>((d + 2) % 3)};
      T* out[2] = {R->vec<T>(8 + (d + 2) % 3), R->vec<T>(11 + (d + 1) % 3)};
      matvec_n<T>(R, R->grad[d], 2, in, out, s);
    }
    for (int e = 0; e < 3; ++e) {
      a.u[e] = R->vec<T>(e);
      a.cp[e] = R->vec<T>(8 + e);
      a.cm[e] = R->vec<T>(11 + e);
    }
    a.aI = 0.5 * (1.0 - beta);
    a.aN = -(1.0 - beta);
  }
  launch_rwg_project<T>(R->einc.p, R->ne, R->rec.p, R->rule, R->w.p, a, y, s);
}

void check_beta(const hmx_rwg* R, double beta) {
  HMX_REQUIRE(std::isfinite(beta) && beta >= 0.0 && beta <= 1.0, HMX_EINVAL,
              "beta must be in [0, 1]");
  HMX_REQUIRE(beta == 0.0 || R->single, HMX_EINVAL, "beta > 0 needs the single-layer operator");
  HMX_REQUIRE(beta == 1.0 || R->grad[0], HMX_EINVAL, "beta < 1 needs the gradient operators");
}

}  // namespace

extern "C" {

hmx_status hmx_rwg_create(const hmx_op* single, const hmx_op* grad_x, const hmx_op* grad_y,
                          const hmx_op* grad_z, const double* vtx, int64_t n_vtx,
                          const int32_t* tri, int64_t n_tri, const double* q_bary,
                          const double* q_w, int32_t n_q, void* stream, hmx_rwg** out) {
  API_TRY
  HMX_REQUIRE(vtx && tri && out, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(n_vtx >= 3 && n_tri >= 2, HMX_EINVAL, "empty mesh");
  const int ng = (grad_x != nullptr) + (grad_y != nullptr) + (grad_z != nullptr);
  HMX_REQUIRE(ng == 0 || ng == 3, HMX_EINVAL, "give all three gradient operators or none");
  HMX_REQUIRE(single || ng == 3, HMX_EINVAL, "no operator given");
  const hmx_op* ops[4] = {single, grad_x, grad_y, grad_z};
  const hmx_op* any = single ? single : grad_x;
  for (int i = 0; i < 4; ++i) {
    const hmx_op* op = ops[i];
    if (!op) continue;
    HMX_REQUIRE(op->kern == (i == 0 ? HMX_HELMHOLTZ : HMX_GRADY_X + i - 1), HMX_EINVAL,
                "the operators must be the Helmholtz single layer and its y-gradients x, y, z");
    HMX_REQUIRE(!op->rect && op->mesh_off.size() <= 2, HMX_EINVAL,
                "the RWG space needs operators on one mesh's own points");
    HMX_REQUIRE(op->M == n_tri * (int64_t)n_q, HMX_EINVAL,
                "the operator's points are not this mesh's quadrature points (M != n_q n_tri)");
    HMX_REQUIRE(op->dense || op->p.row_shares == 1, HMX_EUNSUPPORTED,
                "the RWG products need all rows of the operators (no row share)");
    HMX_REQUIRE(op->prec == any->prec, HMX_EINVAL, "the operators differ in precision");
    HMX_REQUIRE(op->k == any->k, HMX_EINVAL, "the operators differ in wavenumber");
  }
  HMX_REQUIRE(any->k > 0.0, HMX_EINVAL, "the electromagnetic equations need k > 0");
  Rule r = make_rule(q_bary, q_w, n_q);
  hipStream_t s = as_stream(stream);
  auto R = std::make_unique<hmx_rwg>();
  R->single = single;
  R->grad[0] = grad_x;
  R->grad[1] = grad_y;
  R->grad[2] = grad_z;
  R->any = any;
  R->nt = n_tri;
  R->M = any->M;
  R->k = any->k;
  R->prec = any->prec;
  R->rule.nq = n_q;
  for (int q = 0; q < n_q; ++q)
    for (int j = 0; j < 3; ++j) R->rule.b[q][j] = r.b[q][j];
  // point weights in the original order (and the range check of the triangles)
  DevBuf<double> X(R->M), Y(R->M), Z(R->M);
  R->w.alloc(R->M);
  DevBuf<int> err(1);
  fill_i32(err.p, 0, 1, s);
  launch_quad(vtx, n_vtx, tri, n_tri, r, X.p, Y.p, Z.p, R->w.p, err.p, s);
  const int e = read1(err.p, s);
  HMX_REQUIRE(!(e & 1), HMX_EINVAL, "triangle vertex index out of range");
  HMX_REQUIRE(!(e & 2), HMX_EINVAL, "non-finite vertex coordinate");
  // edges: sort the 3 n_tri (triangle, local vertex) slots by the vertex pair of their edge
  std::vector<int32_t> ht;
  to_host(ht, tri, 3 * n_tri, s);
  const int64_t ns = 3 * n_tri;
  std::vector<uint64_t> key(ns);
  for (int64_t i = 0; i < ns; ++i) {
    const int64_t t = i / 3;
    const int j = (int)(i % 3);
    const uint32_t a = (uint32_t)ht[3 * t + (j + 1) % 3], b = (uint32_t)ht[3 * t + (j + 2) % 3];
    key[i] = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
  }
  std::vector<int64_t> order(ns);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    return key[x] != key[y] ? key[x] < key[y] : x < y;
  });
  std::vector<int32_t> tedge(ns), tsign(ns), einc, edges;
  einc.reserve(ns);
  edges.reserve(ns);
  for (int64_t i = 0; i < ns;) {
    int64_t j = i;
    while (j < ns && key[order[j]] == key[order[i]]) ++j;
    HMX_REQUIRE(j - i == 2, HMX_EINVAL, "every edge must belong to exactly two triangles");
    const int64_t ed = (int64_t)edges.size() / 2;
    int32_t plus = -1, minus = -1;
    for (int64_t l = i; l < j; ++l) {
      const int64_t slot = order[l], t = slot / 3;
      const int jj = (int)(slot % 3);
      const bool fwd = ht[3 * t + (jj + 1) % 3] < ht[3 * t + (jj + 2) % 3];
      tedge[slot] = (int32_t)ed;
      tsign[slot] = fwd ? 1 : -1;
      (fwd ? plus : minus) = (int32_t)slot;
    }
    HMX_REQUIRE(plus >= 0 && minus >= 0, HMX_EINVAL,
                "the two triangles of an edge must run along it in opposite directions");
    einc.push_back(plus);
    einc.push_back(minus);
    edges.push_back((int32_t)(key[order[i]] >> 32));
    edges.push_back((int32_t)(key[order[i]] & 0xffffffffu));
    i = j;
  }
  R->ne = (int64_t)edges.size() / 2;
  R->tedge.alloc(ns);
  R->einc.alloc(einc.size());
  R->edges.alloc(edges.size());
  DevBuf<int32_t> dsign(ns);
  HMX_HIP(hipMemcpyAsync(R->tedge.p, tedge.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HMX_HIP(hipMemcpyAsync(dsign.p, tsign.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HMX_HIP(hipMemcpyAsync(R->einc.p, einc.data(), einc.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, s));
  HMX_HIP(hipMemcpyAsync(R->edges.p, edges.data(), edges.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, s));
  R->rec.alloc((size_t)RWG_REC * n_tri);
  launch_rwg_geom(vtx, tri, dsign.p, n_tri, R->rec.p, s);
  R->scratch.alloc((size_t)14 * R->M * any->elem);
  int64_t tmax = 1;
  for (int i = 0; i < 4; ++i)
    if (ops[i]) tmax = std::max<int64_t>(tmax, ops[i]->t_len);
  R->xpm.alloc((size_t)4 * R->M * any->elem);
  R->tm.alloc((size_t)4 * tmax * any->elem);
  HMX_HIP(hipStreamSynchronize(s));
  *out = R.release();
  return HMX_OK;
  API_CATCH
}

void hmx_rwg_destroy(hmx_rwg* r) {
  if (!r) return;
  (void)hipDeviceSynchronize();
  delete r;
}

hmx_status hmx_rwg_n_edges(const hmx_rwg* r, int64_t* n_edges) {
  if (!r || !n_edges) return fail(HMX_EINVAL, "null pointer");
  *n_edges = r->ne;
  return HMX_OK;
}

hmx_status hmx_rwg_edges(const hmx_rwg* r, int32_t* edges, void* stream) {
  if (!r || !edges) return fail(HMX_EINVAL, "null pointer");
  API_TRY
  HMX_HIP(hipMemcpyAsync(edges, r->edges.p, 2 * r->ne * sizeof(int32_t), hipMemcpyDeviceToDevice,
                         as_stream(stream)));
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_rwg_interp(const hmx_rwg* r, const void* x, void* u, void* stream) {
  if (!r || !x || !u) return fail(HMX_EINVAL, "null pointer");
  API_TRY
  if (r->prec == HMX_FP64)
    launch_rwg_interp<double2>(r->rec.p, r->tedge.p, r->nt, r->rule, (const double2*)x,
                               (double2*)u, as_stream(stream));
  else
    launch_rwg_interp<float2>(r->rec.p, r->tedge.p, r->nt, r->rule, (const float2*)x, (float2*)u,
                              as_stream(stream));
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_rwg_rhs(const hmx_rwg* r, double beta, const void* e_inc, const void* h_inc,
                       void* b, void* stream) {
  API_TRY
  HMX_REQUIRE(r && b, HMX_EINVAL, "null pointer");
  HMX_REQUIRE(std::isfinite(beta) && beta >= 0.0 && beta <= 1.0, HMX_EINVAL,
              "beta must be in [0, 1]");
  HMX_REQUIRE(beta == 0.0 || e_inc, HMX_EINVAL, "beta > 0 needs the incident electric field");
  HMX_REQUIRE(beta == 1.0 || h_inc, HMX_EINVAL, "beta < 1 needs the incident magnetic field");
  auto run = [&](auto tag) {
    using T = decltype(tag);
    RwgTerms<T> a;
    for (int d = 0; d < 3; ++d) {
      if (beta != 0.0) a.u[d] = (const T*)e_inc + d * r->M;
      if (beta != 1.0) a.cp[d] = (const T*)h_inc + d * r->M;
    }
    a.aI = beta;
    a.aN = -(1.0 - beta);
    launch_rwg_project<T>(r->einc.p, r->ne, r->rec.p, r->rule, r->w.p, a, (T*)b, as_stream(stream));
  };
  if (r->prec == HMX_FP64)
    run(double2{});
  else
    run(float2{});
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_cfie_matvec(const hmx_rwg* r, double beta, const void* x, void* y, void* stream) {
  API_TRY
  HMX_REQUIRE(r && x && y, HMX_EINVAL, "null pointer");
  check_beta(r, beta);
  if (r->prec == HMX_FP64)
    cfie_enqueue<double2>(r, beta, (const double2*)x, (double2*)y, as_stream(stream));
  else
    cfie_enqueue<float2>(r, beta, (const float2*)x, (float2*)y, as_stream(stream));
  return HMX_OK;
  API_CATCH
}

hmx_status hmx_cfie_gmres(const hmx_rwg* r, double beta, const void* b, void* x, int32_t restart,
                          int32_t max_iter, double tol, void* stream, int32_t* iters,
                          double* relres) {
  API_TRY
  HMX_REQUIRE(r && b && x && iters && relres, HMX_EINVAL, "null pointer");
  check_beta(r, beta);
  HMX_REQUIRE(restart >= 1 && restart <= 1000, HMX_EINVAL, "restart must be in [1, 1000]");
  HMX_REQUIRE(max_iter >= 0, HMX_EINVAL, "max_iter must be >= 0");
  HMX_REQUIRE(std::isfinite(tol) && tol >= 0, HMX_EINVAL, "tol must be finite and >= 0");
  hipStream_t s = as_stream(stream);
  if (r->prec == HMX_FP64)
    gmres_run<double2>([&](const double2* v, double2* o) { cfie_enqueue<double2>(r, beta, v, o, s); },
                       r->ne, (const double2*)b, (double2*)x, restart, max_iter, tol, s, iters, relres);
  else
    gmres_run<float2>([&](const float2* v, float2* o) { cfie_enqueue<float2>(r, beta, v, o, s); },
                      r->ne, (const float2*)b, (float2*)x, restart, max_iter, tol, s, iters, relres);
  return HMX_OK;
  API_CATCH
}

}  // extern "C"
