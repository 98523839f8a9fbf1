// hmx_tune.hip -- autotuner of the build schedule (hmx_autotune).  A client of the library's own
// entry points: it builds the caller's operator under a grid of schedule settings, times each
// build, and keeps the fastest.  Results are cached in a small JSON file keyed by device
// architecture and problem class, so a later call for the same class returns at once.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "hmx_host.h"

namespace {

struct Choice {
  int big = 4096, gram = 1024, serial = 0, maxmn = 12288, mid = 128, bigt = 0, small = 1024,
      wave = 0;
  double ms = 0.0;
};

// "<arch>|<precision>|<kernel>|M2^<floor(log2 M)>|tol1e<round(log10 tol)>|leaf<L>|eta<eta>",
// with "|batch<n>" after the kernel for a batch of n meshes and "|learned" at the end for the
// learned layout
std::string class_key(int64_t M, int32_t kern, const hmx_params& p, int32_t n_meshes = 0) {
  int dev = 0;
  HMX_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HMX_HIP(hipGetDeviceProperties(&prop, dev));
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  int lm = 0;
  while ((int64_t(1) << (lm + 1)) <= M) ++lm;
  const long te = std::lround(std::log10(p.tol));
  std::ostringstream o;
  o << arch << "|" << (p.precision == HMX_FP64 ? "fp64" : "fp32") << "|"
    << (kern == HMX_LAPLACE ? "laplace" : kern == HMX_HELMHOLTZ ? "helmholtz" : "poly2");
  if (n_meshes > 0) o << "|batch" << n_meshes;
  o << "|M2^" << lm << "|tol1e" << te << "|leaf" << p.leaf_size << "|eta" << p.eta;
  if (p.rank_model == HMX_RANK_LEARNED) o << "|learned";
  if (p.near_mode == 1) o << "|nearotf";  // no near-field assembly in the timed builds
  return o.str();
}

// The cache file is one JSON object of entries
//   "key": {"max_far_mn": N, "aca_big_mn": N, "aca_gram_min_mn": N, "aca_mid_threads": N,
//           "aca_big_threads": N, "aca_small_mn": N, "aca_wave": N, "aca_serial": N, "ms": X}
// written by this file; the reader accepts exactly that shape.
double field(const std::string& body, const char* name, double dflt) {
  const std::string pat = std::string("\"") + name + "\":";
  size_t i = body.find(pat);
  if (i == std::string::npos) return dflt;
  return std::strtod(body.c_str() + i + pat.size(), nullptr);
}

std::map<std::string, Choice> read_cache(const char* path) {
  std::map<std::string, Choice> out;
  if (!path) return out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t pos = 0;
  for (;;) {
    const size_t q0 = t.find('"', pos);
    if (q0 == std::string::npos) break;
    const size_t q1 = t.find('"', q0 + 1);
    const size_t b0 = t.find('{', q1);
    const size_t b1 = t.find('}', b0);
    if (q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
    const std::string key = t.substr(q0 + 1, q1 - q0 - 1);
    const std::string body = t.substr(b0, b1 - b0 + 1);
    Choice c;
    c.big = (int)field(body, "aca_big_mn", 4096);
    c.gram = (int)field(body, "aca_gram_min_mn", 1024);
    c.serial = (int)field(body, "aca_serial", 0);
    c.maxmn = (int)field(body, "max_far_mn", 12288);
    c.mid = (int)field(body, "aca_mid_threads", 128);
    c.bigt = (int)field(body, "aca_big_threads", 0);
    c.small = (int)field(body, "aca_small_mn", 1024);
    c.wave = (int)field(body, "aca_wave", 0);
    c.ms = field(body, "ms", 0.0);
    out[key] = c;
    pos = b1 + 1;
  }
  return out;
}

void write_cache(const char* path, const std::map<std::string, Choice>& m) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    HMX_REQUIRE(bool(f), HMX_EINVAL, "cannot write the autotuner cache file");
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
      char buf[320];
      std::snprintf(buf, sizeof(buf),
                    "{\"max_far_mn\": %d, \"aca_big_mn\": %d, \"aca_gram_min_mn\": %d, "
                    "\"aca_mid_threads\": %d, \"aca_big_threads\": %d, \"aca_small_mn\": %d, "
                    "\"aca_wave\": %d, \"aca_serial\": %d, \"ms\": %.3f}",
                    kv.second.maxmn, kv.second.big, kv.second.gram, kv.second.mid, kv.second.bigt,
                    kv.second.small, kv.second.wave, kv.second.serial, kv.second.ms);
      f << "  \"" << kv.first << "\": " << buf << (++i < m.size() ? ",\n" : "\n");
    }
    f << "}\n";
  }
  HMX_REQUIRE(std::rename(tmp.c_str(), path) == 0, HMX_EINVAL,
              "cannot replace the autotuner cache file");
}

// Best of `reps` synchronous builds, in ms (wall clock around the synchronous call);
// build(p, &op) makes one operator.
template <class Build>
double time_build(Build build, const hmx_params& p, int reps) {
  double best = 1e300;
  for (int r = 0; r < reps; ++r) {
    hmx_op* op = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    const hmx_status st = build(p, &op);
    const auto t1 = std::chrono::steady_clock::now();
    if (st != HMX_OK) throw hmx::Error(st, hmx_last_error());
    hmx_destroy(op);
    best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
  }
  return best;
}

// The search: the far-block size bound first (default schedule), then the class thresholds
// (concurrent classes), the two workgroup sizes, the small-block bound, the other wavefront
// setting, then serial vs concurrent at the best; each setting the best of two builds.
template <class Build>
Choice search(Build build, const hmx_params& base) {
  const int maxmns[] = {0, 32768, 16384, 12288, 8192};
  const int bigs[] = {2048, 4096, 8192, 1 << 30};
  const int grams[] = {0, 1024, 4096, 1 << 30};
  const int mids[] = {256, 128, 64};
  const int bigts[] = {512, 256};
  const int smalls[] = {512, 2048, 0};
  hmx_params q = base;
  q.aca_serial = 0;
  (void)time_build(build, q, 1);  // warm the allocator and the code
  Choice best{q.aca_big_mn, q.aca_gram_min_mn, 0, q.max_far_mn, q.aca_mid_threads,
              q.aca_big_threads, q.aca_small_mn, q.aca_wave, 1e300};
  auto trial = [&](const hmx_params& t) {
    const double ms = time_build(build, t, 2);
    if (ms < best.ms)
      best = Choice{t.aca_big_mn, t.aca_gram_min_mn, t.aca_serial, t.max_far_mn,
                    t.aca_mid_threads, t.aca_big_threads, t.aca_small_mn, t.aca_wave, ms};
  };
  for (int mx : maxmns) {
    q.max_far_mn = mx;
    trial(q);
  }
  q.max_far_mn = best.maxmn;
  for (int b : bigs)
    for (int g : grams) {
      q.aca_big_mn = b;
      q.aca_gram_min_mn = g;
      trial(q);
    }
  q.aca_big_mn = best.big;
  q.aca_gram_min_mn = best.gram;
  for (int mt : mids) {
    q.aca_mid_threads = mt;
    trial(q);
  }
  q.aca_mid_threads = best.mid;
  for (int bt : bigts) {
    q.aca_big_threads = bt;
    trial(q);
  }
  q.aca_big_threads = best.bigt;
  for (int sm : smalls) {
    q.aca_small_mn = sm;
    trial(q);
  }
  q.aca_small_mn = best.small;
  q.aca_wave = 1 - q.aca_wave;
  trial(q);
  q.aca_wave = best.wave;
  q.aca_serial = 1;
  trial(q);
  return best;
}

hmx_params resolve_base(const hmx_params* p) {
  hmx_params base;
  if (p) {
    base = *p;
  } else {
    const hmx_status st = hmx_params_default(&base);
    if (st != HMX_OK) throw hmx::Error(st, hmx_last_error());
  }
  HMX_REQUIRE(base.struct_size == (int32_t)sizeof(hmx_params), HMX_EINVAL,
              "hmx_params.struct_size does not match this library (use hmx_params_default)");
  HMX_REQUIRE(base.tol > 0, HMX_EINVAL, "the autotuner needs an H-matrix build (tol > 0)");
  return base;
}

// The cached or searched choice for `key`, written into *out (the caller's base otherwise).
template <class Build>
void tune(Build build, const hmx_params& base, const std::string& key, const char* cache_path,
          hmx_params* out, double* best_ms) {
  auto cache = read_cache(cache_path);
  auto hit = cache.find(key);
  Choice best;
  if (hit != cache.end()) {
    best = hit->second;
  } else {
    best = search(build, base);
    cache[key] = best;
    write_cache(cache_path, cache);
  }
  *out = base;
  out->aca_big_mn = best.big;
  out->aca_gram_min_mn = best.gram;
  out->aca_serial = best.serial;
  out->max_far_mn = best.maxmn;
  out->aca_mid_threads = best.mid;
  out->aca_big_threads = best.bigt;
  out->aca_small_mn = best.small;
  out->aca_wave = best.wave;
  if (best_ms) *best_ms = best.ms;
}

}  // namespace

extern "C" hmx_status hmx_autotune(const double* xyzw, int64_t M, int32_t kern, double k,
                                   const hmx_params* p, const char* cache_path, void* stream,
                                   hmx_params* out, double* best_ms) {
  try {
    HMX_REQUIRE(xyzw && out, HMX_EINVAL, "null pointer");
    HMX_REQUIRE(M >= 1, HMX_EINVAL, "M must be >= 1");
    const hmx_params base = resolve_base(p);
    auto build = [&](const hmx_params& q, hmx_op** op) {
      return hmx_build_points(xyzw, M, kern, k, &q, stream, op);
    };
    tune(build, base, class_key(M, kern, base), cache_path, out, best_ms);
    return HMX_OK;
  } catch (const hmx::Error& e) {
    hmx::set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    hmx::set_last_error(e.what());
    return HMX_EINTERNAL;
  }
}

extern "C" hmx_status hmx_autotune_batch(const hmx_mesh* meshes, int32_t n_meshes,
                                         const double* q_bary, const double* q_w, int32_t n_q,
                                         int32_t kern, const hmx_params* p,
                                         const char* cache_path, void* stream, hmx_params* out,
                                         double* best_ms) {
  try {
    HMX_REQUIRE(meshes && q_bary && q_w && out, HMX_EINVAL, "null pointer");
    HMX_REQUIRE(n_meshes >= 1, HMX_EINVAL, "n_meshes must be >= 1");
    HMX_REQUIRE(n_q >= 1, HMX_EINVAL, "n_q must be >= 1");
    const hmx_params base = resolve_base(p);
    int64_t M = 0;
    for (int32_t i = 0; i < n_meshes; ++i) M += (int64_t)n_q * meshes[i].n_tri;
    HMX_REQUIRE(M >= 1, HMX_EINVAL, "the batch has no points");
    auto build = [&](const hmx_params& q, hmx_op** op) {
      return hmx_build_batch(meshes, n_meshes, q_bary, q_w, n_q, kern, &q, stream, op);
    };
    tune(build, base, class_key(M, kern, base, n_meshes), cache_path, out, best_ms);
    return HMX_OK;
  } catch (const hmx::Error& e) {
    hmx::set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    hmx::set_last_error(e.what());
    return HMX_EINTERNAL;
  }
}
