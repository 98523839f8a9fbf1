// hmx_host.h -- host-side internals of libhmx: errors, device buffers, the operator object and
// the kernel launchers implemented in the k_*.hip translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hmx.h"

namespace hmx {

struct Error : std::runtime_error {
  hmx_status code;
  Error(hmx_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void hip_fail(hipError_t e, const char* what, const char* file, int line) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e) + " (" + file + ":" +
                  std::to_string(line) + ")";
  throw Error(e == hipErrorOutOfMemory ? HMX_ENOMEM : HMX_EDEVICE, m);
}
#define HMX_HIP(x)                                                   \
  do {                                                               \
    hipError_t e_ = (x);                                             \
    if (e_ != hipSuccess) ::hmx::hip_fail(e_, #x, __FILE__, __LINE__); \
  } while (0)
#define HMX_LAUNCHED() HMX_HIP(hipGetLastError())
#define HMX_REQUIRE(cond, code, msg)   \
  do {                                 \
    if (!(cond)) throw ::hmx::Error(code, msg); \
  } while (0)

// Device memory: a caching allocator (freed buffers stay mapped and are reused, so that
// repeated builds do not map and unmap memory; dev_free waits for the device first, as hipFree
// does).  dev_shrink keeps the first `bytes` of a buffer and hands the rest to later
// allocations; dev_release_cache returns the entirely free blocks to the runtime.
void* dev_alloc(size_t bytes);
void* dev_alloc_block(size_t bytes);  // a block of its own, for a buffer that will be shrunk
size_t dev_shrink(void* p, size_t bytes);
void dev_free(void* p);
void dev_release_cache();
size_t dev_cached_bytes();  // bytes of free blocks the cache holds on the current device

// Message returned by hmx_last_error on this thread.
void set_last_error(const std::string& m);

// Owning device buffer (move-only).
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { reset(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { reset(); }
  void alloc(size_t count) {
    reset();
    if (count == 0) return;
    p = (T*)dev_alloc(count * sizeof(T));
    n = count;
  }
  void reset() {
    if (p) dev_free(p);
    p = nullptr;
    n = 0;
  }
  // A buffer that will be shrunk: a block of its own, so that the shrink frees only its tail.
  void alloc_block(size_t count) {
    reset();
    if (count == 0) return;
    p = (T*)dev_alloc_block(count * sizeof(T));
    n = count;
  }
  // Keeps the first `count` elements (at least one) and gives the rest back to the allocator.
  void shrink(size_t count) {
    count = count < 1 ? 1 : count;
    if (!p || count >= n) return;
    dev_shrink(p, count * sizeof(T));
    n = count;
  }
  size_t bytes() const { return n * sizeof(T); }
  T* get() const { return p; }
};

template <class T>
void to_host(std::vector<T>& h, const T* d, size_t n, hipStream_t s) {
  h.resize(n);
  if (n) HMX_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
  HMX_HIP(hipStreamSynchronize(s));
}
template <class T>
T read1(const T* d, hipStream_t s) {
  T v;
  HMX_HIP(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, s));
  HMX_HIP(hipStreamSynchronize(s));
  return v;
}

constexpr int MAX_NQ = 32;
struct Rule {
  double b[MAX_NQ][3];
  double w[MAX_NQ];
  int nq;
};

// Far-block descriptor used by ACA and by the compaction step.
struct FarDesc {
  int32_t tb, m, sb, n;
  int32_t rcap;  // rank cap: min(floor(m n / (m + n)), coefficient limit, forced cap)
  int32_t cap;   // columns of the first segment (before ACA: the initial capacity wanted)
  void* U;       // first segment: column l of U at U + l ld (m entries), of V at that + m
  void* U1;      // second segment (columns cap .. cap + cap1 - 1), or null
  int64_t foff;  // byte offset of the row/column used-flags (m + n bytes)
  int32_t ld;    // column stride of both factors: m + n (interleaved column pairs)
  int32_t cap1;  // columns of the second segment
};

// Final far-block record used by the product.
struct FarRec {
  int32_t tb, m, sb, n;
  int32_t r;      // rank, or n for a block stored dense (then U is the m x n block)
  int32_t dense;  // 1 when stored dense
  const void* U;  // m x r, column stride ldu (or the m x n block when dense, ldu = m);
  const void* V;  // n x r, column stride ldv (unused when dense);
  int64_t toff;   // offset of t_b = V^T x_s in the product scratch
  int32_t ldu, ldv;
  int32_t split;  // columns >= split live in the second segment: column l of U at
  int32_t pad_;   // U1 + (l - split) ldu, of V at V1 + (l - split) ldv
  const void* U1;
  const void* V1;
};

constexpr int ACA_COEF_MAX = 1024;  // largest ACA rank (coefficients of a step held in LDS)
// The small-block class (m + n below aca_small_mn, not a wavefront block) keeps at most this
// many coefficients: its blocks have rank cap floor(m n / (m + n)) <= (m + n) / 4 <= 256 for
// m + n < 1024, and only blocks with rank cap <= ACA_COEF_SMALL are placed in the class.
constexpr int ACA_COEF_SMALL = 256;
enum AcaStatus : int32_t { ACA_RUNNING = 0, ACA_CONVERGED = 1, ACA_OVERFLOW = 2, ACA_DENSE = 3 };
// added to a block's saved status word once ACA has moved it to a larger pool slot
constexpr int32_t ACA_GREW = 0x100;
// ACA stops once |u_k| |v_k| <= tol |S_k|_F has held at this many consecutive steps (one step
// can meet it by accident when its pivot row lies where the block is already well approximated).
// A block's saved state keeps the count of steps met so far in the ACA_HIT_SHIFT bits of its
// next-pivot-row word.
constexpr int ACA_STOP_STEPS = 2;
constexpr int ACA_HIT_SHIFT = 28;
constexpr int32_t ACA_ROW_MASK = (1 << ACA_HIT_SHIFT) - 1;
static_assert(ACA_STOP_STEPS < 8, "hit count fits the saved state word");

// ------------------------------------------------------------------------------- launchers
// k_quad.hip
void launch_quad(const double* vtx, int64_t nv, const int32_t* tri, int64_t nt, const Rule& rule,
                 double* X, double* Y, double* Z, double* W, int* err, hipStream_t s);
// k_scan.hip
void scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);  // out[n] = total
// the same without synchronisation, on caller scratch of scan_work_len(n) entries
int64_t scan_work_len(int64_t n);
void scan_excl_i64_work(const int64_t* in, int64_t* out, int64_t n, int64_t* work, hipStream_t s);
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);
void fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);
void fill_f64(double* p, double v, int64_t n, hipStream_t s);
void iota_i32(int32_t* p, int64_t n, hipStream_t s);
// k_sort.hip: ascending radix sort of pairs on key bits [0, end_bit); `tmp` holds the sort's
// scratch and must outlive the enqueued sort (the caller synchronises before dropping it)
void radix_sort_u64_pairs(const uint64_t* kin, uint64_t* kout, const int32_t* vin, int32_t* vout,
                          int64_t n, int end_bit, DevBuf<unsigned char>& tmp, hipStream_t s);
// k_tree.hip
void launch_tree_level(int first, int count, const int32_t* nbegin, const int32_t* nend, int leaf,
                       const double* cx, const double* cy, const double* cz, const double* cw,
                       const int32_t* cperm, double* nx, double* ny, double* nz, double* nw,
                       int32_t* nperm, double* box, int32_t* nleft, hipStream_t s);
// multi-workgroup variant for levels of few large nodes; max_chunks >= sum ceil(n / 2048)
void launch_tree_level_chunked(int first, int count, int max_chunks, const int32_t* nbegin,
                               const int32_t* nend, int leaf, const double* cx, const double* cy,
                               const double* cz, const double* cw, const int32_t* cperm,
                               double* nx, double* ny, double* nz, double* nw, int32_t* nperm,
                               double* box, int32_t* nleft, int32_t* choff, double* pbox,
                               int32_t* saxis, double* smid, int32_t* ccnt, int32_t* cleft,
                               hipStream_t s);
constexpr int TREE_CHUNK_PTS = 2048;  // points per chunk of launch_tree_level_chunked
void launch_tree_children(int first, int count, int next_first, const int32_t* nleft,
                          int32_t* nbegin, int32_t* nend, int32_t* level, int32_t* child0,
                          int32_t* child1, int32_t* parent, int* next_count, hipStream_t s);
void launch_leaf_marks(int n_nodes, const int32_t* nbegin, const int32_t* child0,
                       int64_t* pos_flag, hipStream_t s);
void launch_leaf_list(int64_t M, const int64_t* pos_flag, const int64_t* pos_scan,
                      const int32_t* start_node, int32_t* leaves, hipStream_t s);
void launch_start_node(int n_nodes, const int32_t* nbegin, const int32_t* child0,
                       int32_t* start_node, hipStream_t s);
void launch_leaf_index(int n_leaves, const int32_t* leaves, int32_t* leaf_of_node, hipStream_t s);
// k_blocks.hip
// one level of the block recursion; nfront is a device counter (see k_blocks.hip)
void launch_block_level(const int2* front, const int* nfront, int64_t front_cap,
                        const double* box, const int32_t* child0, const int32_t* child1,
                        const int32_t* nbegin, const int32_t* nend, int rb, int re, double eta2,
                        int max_mn, int2* next, int64_t next_cap, int* next_cnt, int2* nearL,
                        int64_t near_cap, int* near_cnt, int2* farL, int64_t far_cap,
                        int* far_cnt, int* err, hipStream_t s);
void launch_node_rank(const int32_t* nbegin, const int32_t* level, int n_nodes, int64_t M,
                      int64_t* cnt, int64_t* start, int32_t* deep, int32_t* rank, hipStream_t s);
void launch_pair_rank_keys(const int2* pairs, int64_t n, const int32_t* rank, int64_t n_nodes,
                           uint64_t list_bit, int64_t offset, uint64_t* key, int32_t* val,
                           hipStream_t s);
void launch_pair_gather2(const int2* a, int64_t na, const int2* b, const int32_t* idx, int64_t n,
                         int2* out, hipStream_t s);
void launch_near_prep(const int2* nearL, int64_t n, const int32_t* nbegin, const int32_t* nend,
                      const int32_t* leaf_of_node, int64_t* sizes, int64_t* leaf_cnt, hipStream_t s);
void launch_far_prep(const int2* farL, int64_t n, const int32_t* nbegin, const int32_t* nend,
                     int32_t* far_tb, int32_t* far_m, int32_t* far_sb, int32_t* far_n,
                     int64_t* node_cnt, int32_t* node_first, hipStream_t s);
void launch_leaf_far_count(int n_leaves, const int32_t* leaves, const int32_t* parent,
                           const int64_t* node_cnt, int64_t* leaf_cnt, hipStream_t s);
void launch_pair_ranges(const int2* pairs, int64_t n, const int32_t* nbegin, const int32_t* nend,
                        int32_t* tb, int32_t* m, int32_t* sb, int32_t* nn, hipStream_t s);
void launch_leaf_far_fill(int n_leaves, const int32_t* leaves, const int32_t* parent,
                          const int64_t* node_cnt, const int32_t* node_first,
                          const int64_t* leaf_ptr, int32_t* list, hipStream_t s);
// k_near.hip  (T = double2 or float2); reg: the singular correction of close pairs, or null
struct RegArgs;
template <class T>
void launch_assemble(const int32_t* tb, const int32_t* m, const int32_t* sb, const int32_t* n,
                     const int64_t* off, int64_t nblk, const double* X, const double* Y,
                     const double* Z, const double* W, int kern, const double* kp, T* pool,
                     const RegArgs* reg, hipStream_t s);
// k_p1.hip: P1 basis at the quadrature points and the GMRES vector kernels
struct P1Rule {
  double b[MAX_NQ][3];  // barycentric coordinates of the rule's points
  int nq;
};
template <class T>
void launch_p1_interp(const int32_t* tri, int64_t nt, const P1Rule& r, const T* xv, T* xp,
                      hipStream_t s);
template <class T>
void launch_p1_project(const int64_t* ptr, const int32_t* inc, int64_t nv, const P1Rule& r,
                       const double* w, const T* zp, T* yv, hipStream_t s);
int mdot_chunks(int64_t n);
template <class T>
void launch_mdot(const T* V, int64_t ld, int nc, const T* w, int64_t n, double2* partial,
                 double2* d, hipStream_t s);
template <class T>
void launch_gemv_update(const T* V, int64_t ld, const double2* h, int nc, double sign, T* w,
                        int64_t n, hipStream_t s);
template <class T>
void launch_vec(const T* x, const T* b, double a, int sub, T* y, int64_t n, hipStream_t s);
// k_matvec.hip: y_r = K x_r for nr = 2 or 4 vectors, the operator's entries read once; scratch
// xpm of nr M and tm of nr max(t_len, 1) entries (H-matrix operators only)
template <class T>
void launch_matvec_multi(const hmx_op* op, int nr, const T* const* x, T* const* y, T* xpm, T* tm,
                         hipStream_t s);
// k_rwg.hip: RWG elements at the quadrature points (records of RWG_REC doubles per triangle)
constexpr int RWG_REC = 16;
// Terms of the projection onto the RWG functions: coefficients and point vectors (M entries,
// original point order); ku, kv for the single layer, u for the identity, cp - cm for n x psi.
template <class T>
struct RwgTerms {
  double2 aT{0.0, 0.0}, aD{0.0, 0.0};
  double aI = 0.0, aN = 0.0;
  const T* ku[3] = {nullptr, nullptr, nullptr};
  const T* kv = nullptr;
  const T* u[3] = {nullptr, nullptr, nullptr};
  const T* cp[3] = {nullptr, nullptr, nullptr};
  const T* cm[3] = {nullptr, nullptr, nullptr};
};
void launch_rwg_geom(const double* vtx, const int32_t* tri, const int32_t* tsign, int64_t nt,
                     double* rec, hipStream_t s);
template <class T>
void launch_rwg_interp(const double* rec, const int32_t* tedge, int64_t nt, const P1Rule& r,
                       const T* x, T* u, hipStream_t s);
template <class T>
void launch_rwg_project(const int32_t* einc, int64_t ne, const double* rec, const P1Rule& r,
                        const double* w, const RwgTerms<T>& a, T* y, hipStream_t s);
// k_reg.hip: per-triangle records of the singular correction (TGEO doubles each)
void launch_tri_geom(const double* vtx, const int32_t* tri, int64_t nt, double alpha,
                     double* tgeo, hipStream_t s);
void launch_iperm(const int32_t* perm, int64_t M, int32_t* iperm, hipStream_t s);
// k_aca.hip
template <class T>
void launch_aca(FarDesc* d, const int32_t* order, int nb, int* counter, int threads, int kind,
                const double* X, const double* Y, const double* Z, const double* W, int kern,
                const double* kp, double tol, uint8_t* flags, int32_t* rank, int32_t* ipiv,
                int32_t* status, double* norm2, int fresh, T* gpool, int64_t gcap,
                unsigned long long* gtop, double2* gram, int gram_min, int64_t arena,
                hipStream_t s);
// arena size (entries) of a workgroup of the large-block and of the smaller ACA kernels
constexpr int64_t ACA_ARENA_BIG = int64_t(1) << 20;
constexpr int64_t ACA_ARENA_MID = int64_t(1) << 16;
constexpr int64_t ACA_ARENA_SMALL = int64_t(1) << 15;
// ACA workgroup kinds: the middle class (256, 128 or 64 threads), the large-block class (512 or
// 256 threads) and the small-block class (64 threads, ACA_COEF_SMALL coefficients)
enum AcaKind : int { ACA_KIND_MID = 0, ACA_KIND_BIG = 1, ACA_KIND_SMALL = 2 };
// workgroups of the persistent grid of the ACA kernel of this kind and size
template <class T>
int aca_grid(int threads, int kind);
// Gram-matrix order per workgroup of the large-block and the middle ACA kernels (steps past it
// use direct cross sums)
constexpr int ACA_GRAM_R = 256;
constexpr int ACA_GRAM_R_MID = 128;
// order of a kind's per-workgroup Gram matrices (one row per thread, at most the workgroup
// size); a workgroup's Gram scratch holds 2 order^2 FP64 complex entries
constexpr int aca_gram_order(int threads, int kind) {
  return kind == ACA_KIND_BIG ? ACA_GRAM_R : threads >= 128 ? ACA_GRAM_R_MID : threads;
}
constexpr int ACA_BIG = 4096;  // block size (m + n) from which first rank slots are enlarged
constexpr int ACA_WAVE_N = 64; // blocks with m, n <= ACA_WAVE_N run one per wavefront
constexpr int ACA_WAVE_RC = 16; // terms a wavefront block holds in registers
template <class T>
void launch_aca_wave(FarDesc* d, const int32_t* order, int nb, const double* X,
                     const double* Y, const double* Z, const double* W, int kern,
                     const double* kp, double tol, uint8_t* flags, int32_t* rank, int32_t* ipiv, int32_t* status,
                     double* norm2, T* gpool, int64_t gcap, unsigned long long* gtop,
                     hipStream_t s);
// k_mlp.hip -- block-rank MLP (4 -> 64 -> 64 -> 1, ReLU, FP32)
constexpr int MLP_IN = 4, MLP_H = 64, MLP_NPARAMS = 4545;
void launch_mlp_features(const int2* pairs, int64_t n, const int32_t* nbegin, const int32_t* nend,
                         const double* box, const double* kp, float* feat, hipStream_t s);
void launch_mlp_predict(const float* theta, const float* norm, const float* feat, int64_t n,
                        float* out, hipStream_t s);
size_t mlp_cache_floats(int B);
void launch_mlp_grad(const float* theta, const float* X, const float* y, int64_t b0, int B,
                     float* cache, float* grad, hipStream_t s);
void launch_mlp_adam(float* theta, const float* grad, float* m, float* v, int t, float lr,
                     hipStream_t s);
// model used by builds with HMX_RANK_LEARNED (hmx_mlp.hip)
struct RankModel {
  bool set = false;
  float theta[MLP_NPARAMS];
  float norm[8];
  float alpha = 1.0f, beta = 0.0f;
};
RankModel get_rank_model();

// k_far.hip: far-field bookkeeping around ACA
void launch_far_desc(const int2* pairs, int64_t nf, const int32_t* nbegin, const int32_t* nend,
                     int initial_rank, int force_cap, int use_wave, FarDesc* desc, int64_t* mn,
                     int64_t* est, uint8_t* wave, int64_t* work, hipStream_t s);
void launch_far_foff(FarDesc* desc, const int64_t* foff, int64_t nf, hipStream_t s);
void launch_far_pred(const float* pred, const FarDesc* desc, int64_t nf, double alpha,
                     int64_t beta, double scale, int64_t* ramn, int64_t* work, hipStream_t s);
constexpr int FAR_ORDER_KEYS = 4 * 64;  // class * 64 + (63 - floor(log2 work))
void launch_far_order(const FarDesc* desc, const uint8_t* wave, const int64_t* work, int64_t nf,
                      int64_t big_mn, int64_t small_mn, int* hist, int* cursor, int32_t* order,
                      hipStream_t s);
void launch_count_status(const int32_t* status, int64_t nf, int code, int* count, hipStream_t s);
constexpr int FAR_STATS = 15;
void launch_far_rec(const FarDesc* desc, const int32_t* rank, const int32_t* status,
                    const uint8_t* continued, const uint8_t* wave, int64_t big_mn,
                    int64_t small_mn, int es,
                    int64_t nf, FarRec* rec, int64_t* tcount, int64_t* dcount, int64_t* dflag,
                    unsigned long long* stats, int* bad, hipStream_t s);
template <class T>
void launch_far_rec_finish(FarRec* rec, const int64_t* toff, const int64_t* doff,
                           const int64_t* dpos, int64_t nf, T* dense_pool, int32_t* dtb,
                           int32_t* dm, int32_t* dsb, int32_t* dn, int64_t* dofs, hipStream_t s);

// k_matvec.hip
template <class T>
void launch_gather(const T* x, const int32_t* perm, T* xp, int64_t M, int64_t x_off,
                   hipStream_t s);
template <class T>
void launch_far_vt(const FarRec* rec, int64_t nf, const T* xp, T* t, hipStream_t s);
// The points and kernel of an operator whose near field is computed in the product.
struct NearOtfArgs {
  const double* X;
  const double* Y;
  const double* Z;
  const double* W;
  int kern;
  const double* kp;
};
// otf: null for stored near blocks (near_pool), else the near field is evaluated in the kernel
template <class T>
void launch_leaf_apply(int n_leaves, const int32_t* leaves, const int32_t* nbegin,
                       const int32_t* nend, const int64_t* near_ptr, const int32_t* near_sb,
                       const int32_t* near_n, const int64_t* near_off, const T* near_pool,
                       const int64_t* far_ptr, const int32_t* far_list, const FarRec* far,
                       const T* tbuf, const T* xp, const int32_t* perm, int64_t y_rows, T* y,
                       int max_leaf_rows, hipStream_t s, const NearOtfArgs* otf = nullptr);
template <class T>
void launch_dense_otf(const double* X, const double* Y, const double* Z, const double* W,
                      int64_t rows, int64_t so, int64_t cols, int kern, double k, const T* x,
                      T* partial, T* y, hipStream_t s);
int64_t dense_otf_partial_len(int64_t rows, int64_t cols);

}  // namespace hmx

// The operator object.
struct hmx_op {
  int64_t M = 0;
  // product shape: y has `rows` entries and x `cols`.  An operator between different point sets
  // (hmx_build_rect) holds its targets as points [0, rows) and its sources as points
  // [x_off, x_off + cols); the others have rows = cols = M and x_off = 0.
  bool rect = false;
  int64_t rows = 0, cols = 0, x_off = 0;
  int32_t kern = 1;
  double k = 0.0;
  hmx_params p{};
  bool dense = false;
  int32_t prec = HMX_FP64;
  size_t elem = 16;  // bytes per complex entry
  // points (cluster order for H operators, original order for dense ones)
  hmx::DevBuf<double> X, Y, Z, W;
  hmx::DevBuf<int32_t> perm;
  // wavenumber at each point (that of the point's mesh; the same in both point orders since
  // cluster ranges never cross a mesh boundary)
  hmx::DevBuf<double> kpt;
  // meshes of a batched operator: points [mesh_off[i], mesh_off[i + 1]) belong to mesh i
  std::vector<int64_t> mesh_off;
  std::vector<double> mesh_k;
  // rows held (cluster positions [row_begin, row_end)); all rows unless built as a row share
  int64_t row_begin = 0, row_end = 0;
  // tree (breadth-first node numbering)
  int n_nodes = 0, n_leaves = 0, depth = 0;
  int max_leaf_rows = 0;  // points of the largest leaf (at most 256)
  hmx::DevBuf<int32_t> nbegin, nend, nlevel, child0, child1, parent;
  hmx::DevBuf<double> box;
  hmx::DevBuf<int32_t> leaves, leaf_of_node;
  // near field
  int64_t n_near = 0, near_entries = 0;
  hmx::DevBuf<int2> nearL;
  hmx::DevBuf<int32_t> near_tb, near_m, near_sb, near_n;
  hmx::DevBuf<int64_t> near_off, near_ptr;
  hmx::DevBuf<unsigned char> near_pool;
  // far field
  int64_t n_far = 0, far_entries = 0, dense_far = 0, dense_far_entries = 0, max_rank = 0,
          sum_rank = 0, overflow_blocks = 0, t_len = 0, pool_used_bytes = 0,
          pool_reserved_bytes = 0, predicted_entries = 0;
  hmx::DevBuf<int2> farL;
  hmx::DevBuf<hmx::FarRec> far;
  std::vector<hmx::DevBuf<unsigned char>> far_pools;  // factor slots (ACA writes in place)
  hmx::DevBuf<unsigned char> dense_pool;               // far blocks stored dense
  hmx::DevBuf<int64_t> far_ptr;
  hmx::DevBuf<int32_t> far_list;
  // product scratch (allocated at build; the product allocates nothing)
  hmx::DevBuf<unsigned char> xp, tbuf, partial;
  // build statistics
  double t_tree = 0, t_blocks = 0, t_near = 0, t_aca = 0, t_total = 0;
  // ACA by block class (0: m + n >= aca_big_mn, 1: other workgroup blocks, 2: wavefront blocks)
  int64_t aca_blocks[4] = {0, 0, 0, 0}, aca_bytes[4] = {0, 0, 0, 0};
  double aca_ms[4] = {0, 0, 0, 0};
  int32_t aca_rounds = 0;
  int64_t kernel_evals = 0;
  // singular correction of the near field (Section 5.2): triangle records of the points'
  // meshes and the Lagrange coefficients of the 3-point rule
  bool reg = false;
  double reg_lag[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  hmx::DevBuf<double> tgeo;
  int64_t bytes() const;
};

// A captured product (hmx_graph_create).
struct hmx_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~hmx_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace hmx {
// hmx_build.hip: builds the operator from its points (dense when tol <= 0, else H-matrix).
void finish_build(hmx_op* op, hipStream_t s);
}  // namespace hmx
