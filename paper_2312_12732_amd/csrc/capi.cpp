// C ABI of the mf library: argument validation, algorithm handles, plan
// lookup, workspace and the launch sequence of one fast product.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <mutex>
#include <vector>
#include <cstring>
#include <string>

#include "mf_internal.h"

namespace mf {

namespace {
thread_local std::string t_err;
std::atomic<uint64_t> g_next_id{1};
}  // namespace

mf_status fail(mf_status st, const std::string& msg) {
  t_err = msg;
  return st;
}
void clear_error() { t_err.clear(); }

namespace {

constexpr int64_t kMaxN = 1 << 20;
// Largest lda / ldb of mf_gemm: the GEMM addresses a 128-row operand tile
// with 32-bit byte offsets from the tile origin (128 x 2^21 x 8 B = 2^31).
constexpr int64_t kMaxLdAB = 1 << 21;

mf_status new_handle(const Algo& a, mf_algo** out) {
  const int64_t bad = brent_violations(a);
  if (bad != 0)
    return fail(MF_ERR_BRENT, "the Brent equations fail for " + std::to_string(bad) + " index triples");
  mf_algo* h = new (std::nothrow) mf_algo;
  if (!h) return fail(MF_ERR_NOMEM, "host allocation failed");
  h->a = a;
  h->id = g_next_id.fetch_add(1);
  *out = h;
  return MF_OK;
}

}  // namespace

// Byte ranges [x, x + xb) and [y, y + yb) intersect.
bool overlaps(const void* x, size_t xb, const void* y, size_t yb) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(x), b = reinterpret_cast<uintptr_t>(y);
  return a < b + yb && b < a + xb;
}
bool overlaps(const void* x, const void* y, size_t bytes) { return overlaps(x, bytes, y, bytes); }

mf_status check_request(const mf_algo* algo, bool need_algo, int depth, int cutoff, const void* A,
                        const void* B, void* C, int64_t n, int dtype) {
  if (need_algo && !algo) return fail(MF_ERR_ARG, "algo is NULL");
  if (depth < 0) return fail(MF_ERR_ARG, "depth must be >= 0");
  if (cutoff < 0) return fail(MF_ERR_ARG, "cutoff must be >= 0");
  if (n < 0) return fail(MF_ERR_ARG, "n must be >= 0");
  if (n > kMaxN) return fail(MF_ERR_SHAPE, "n exceeds the supported maximum (2^20)");
  const int storage = dtype & 0xff, leaf = (dtype >> 8) & 0xff;
  if ((dtype & ~(0xffff | MF_SCHED_FUSED)) != 0 || (storage != MF_F64 && storage != MF_F32) || leaf > 3)
    return fail(MF_ERR_ARG, "unknown dtype code");
  if (storage == MF_F64 && leaf != 0)
    return fail(MF_ERR_UNSUPPORTED, "reduced-precision leaves need FP32 storage");
  if (n == 0) return MF_OK;
  if (!A || !B || !C) return fail(MF_ERR_ARG, "A, B and C must be non-NULL");
  const size_t elem = storage == MF_F64 ? 8 : 4;
  const uintptr_t mask = elem - 1;
  if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) | reinterpret_cast<uintptr_t>(C)) & mask)
    return fail(MF_ERR_ARG, "A, B and C must be aligned to the element size");
  const size_t bytes = (size_t)n * (size_t)n * elem;
  if (overlaps(C, A, bytes) || overlaps(C, B, bytes)) return fail(MF_ERR_ARG, "C overlaps A or B");
  return MF_OK;
}

mf_status plan_for(const mf_algo* algo, int depth, int cutoff, int64_t n, int dtype, std::shared_ptr<const Plan>* pl,
                   bool copy_in) {
  Shape sh = Shape::sq(n);
  sh.copy_in = copy_in;
  return get_plan(depth > 0 ? algo : nullptr, depth, cutoff, sh, dtype, kStandaloneMinWorkgroups, pl);
}

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Phase timing: when enabled, every call records a HIP event on its stream
// before each phase and after the last; reading sums the elapsed times.
struct PhaseTiming {
  std::mutex mu;
  bool enabled = false;
  std::vector<std::array<hipEvent_t, kPhases + 1>> calls;
};
PhaseTiming& timing() {
  static auto* t = new PhaseTiming();
  return *t;
}

}  // namespace

// Enqueues the phases of one product on stream s.  desc: device address of a
// copy of the plan's descriptor image; ws: the plan's workspace.
mf_status run_at(const Plan& pl, const char* desc, const void* A, const void* B, void* C, void* ws, hipStream_t s,
                 bool may_time, double alpha, double beta) {
  // Rows start on 16-byte boundaries when the bases do and a row is a whole
  // number of 16-byte units.
  const Shape& sh = pl.shape;
  const int64_t eb = (int64_t)pl.elem;
  const bool vec_in = (sh.lda * eb) % 16 == 0 && (sh.ldb * eb) % 16 == 0 && aligned16(A) && aligned16(B);
  const bool vec_c = (sh.ldc * eb) % 16 == 0 && aligned16(C);
  CScale sc;
  sc.alpha = alpha;
  sc.beta = beta;
  const int leaf = (pl.dtype >> 8) & 0xff;
  // Timing events of this call; destroyed on every early return, handed to
  // the timing list once the whole call has been enqueued.
  struct Events {
    std::array<hipEvent_t, kPhases + 1> ev{};
    bool keep = false;
    ~Events() {
      if (!keep)
        for (hipEvent_t x : ev)
          if (x) (void)hipEventDestroy(x);
    }
  } events;
  auto& ev = events.ev;
  bool timed = false;
  {
    std::lock_guard<std::mutex> lk(timing().mu);
    timed = timing().enabled && may_time;
  }
  if (timed) {
    for (auto& x : ev)
      if (hipEventCreate(&x) != hipSuccess) {
        x = nullptr;
        return fail(MF_ERR_HIP, "hipEventCreate failed");
      }
  }
  for (int ph = 0; ph < kPhases; ++ph) {
    if (timed && hipEventRecord(ev[ph], s) != hipSuccess) return fail(MF_ERR_HIP, "hipEventRecord failed");
    hipError_t e = hipSuccess;
    if (ph == 0) {
      for (const CombineStage& st : pl.pre)
        if (e == hipSuccess) e = launch_combine(st, desc, (int)pl.elem, A, B, C, ws, vec_in, vec_c, sc, s);
      // BF16 leaves: the last pre-addition level, fused with the staging
      if (e == hipSuccess && (leaf == 2 || leaf == 3))
        e = launch_stage_bf16(pl, desc, leaf == 3, A, B, C, ws, vec_in, s);
    } else if (ph == 2) {
      for (const CombineStage& st : pl.post)
        if (e == hipSuccess) e = launch_combine(st, desc, (int)pl.elem, A, B, C, ws, vec_in, vec_c, sc, s);
    } else if (pl.elem == 8)
      e = launch_gemm_f64(pl, desc, A, B, C, ws, vec_in, sc, s);
    else if (leaf == 2 || leaf == 3)
      e = launch_gemm_bf16(pl, desc, leaf == 3, A, B, C, ws, vec_in, s);
    else
      e = launch_gemm_f32(pl, desc, A, B, C, ws, vec_in, sc, s);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  }
  if (timed) {
    if (hipEventRecord(ev[kPhases], s) != hipSuccess) return fail(MF_ERR_HIP, "hipEventRecord failed");
    std::lock_guard<std::mutex> lk(timing().mu);
    timing().calls.push_back(ev);
    events.keep = true;
  }
  return MF_OK;
}

namespace {

// run_at() with the plan's own device copy of its descriptors.
mf_status run(const Plan& pl, const void* A, const void* B, void* C, void* ws, hipStream_t s, double alpha = 1.0,
              double beta = 0.0) {
  mf_status st = ensure_device(pl);
  if (st != MF_OK) return st;
  return run_at(pl, pl.desc(), A, B, C, ws, s, true, alpha, beta);
}

// One pool per device, made on first use and kept until the process ends.
hipMemPool_t device_pool(int dev) {
  static std::mutex mu;
  static hipMemPool_t pools[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!pools[dev]) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    uint64_t keep = UINT64_MAX;
    if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipMemPoolDestroy(pool);
      return nullptr;
    }
    pools[dev] = pool;
  }
  return pools[dev];
}

}  // namespace

hipError_t workspace_alloc(void** p, size_t bytes, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipMemPool_t pool = device_pool(dev);
  if (!pool) return hipErrorOutOfMemory;
  return hipMallocFromPoolAsync(p, bytes, pool, s);
}

hipError_t workspace_free(void* p, hipStream_t s) { return hipFreeAsync(p, s); }

namespace {

// run() with the workspace taken from the library's pool for the call.
mf_status run_with_pool(const Plan& pl, const void* A, const void* B, void* C, hipStream_t s, double alpha = 1.0,
                        double beta = 0.0) {
  void* ws = nullptr;
  if (pl.ws_bytes > 0) {
    hipError_t e = workspace_alloc(&ws, pl.ws_bytes, s);
    if (e != hipSuccess || !ws) {
      (void)hipGetLastError();
      return fail(MF_ERR_NOMEM, "workspace allocation of " + std::to_string(pl.ws_bytes) + " bytes failed");
    }
  }
  mf_status st = run(pl, A, B, C, ws, s, alpha, beta);
  if (ws) {
    hipError_t e = workspace_free(ws, s);
    if (e != hipSuccess && st == MF_OK) st = fail(MF_ERR_HIP, "workspace release failed");
  }
  return st;
}

}  // namespace
}  // namespace mf

using namespace mf;

extern "C" {

const char* mf_last_error(void) { return t_err.c_str(); }

mf_status mf_algo_from_uvw(int n0, int R, const double* U, const double* V, const double* W, int w_convention,
                           mf_algo** out) {
  clear_error();
  if (!out) return fail(MF_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n0 < 1 || n0 > 8) return fail(MF_ERR_ARG, "n0 must be in [1, 8]");
  if (R < 1 || R > 4096) return fail(MF_ERR_ARG, "R must be in [1, 4096]");
  if (!U || !V || !W) return fail(MF_ERR_ARG, "U, V and W must be non-NULL");
  if (w_convention != MF_W_ROWMAJOR_C && w_convention != MF_W_DEEPMIND_CT)
    return fail(MF_ERR_ARG, "unknown W convention");
  const int P2 = n0 * n0;
  const size_t cnt = (size_t)P2 * R;
  for (size_t i = 0; i < cnt; ++i)
    if (!std::isfinite(U[i]) || !std::isfinite(V[i]) || !std::isfinite(W[i]))
      return fail(MF_ERR_ARG, "coefficients must be finite");
  Algo a;
  a.set_shape(n0, n0, n0);
  a.R = R;
  a.U.assign(U, U + cnt);
  a.V.assign(V, V + cnt);
  a.W.assign((size_t)P2 * R, 0.0);
  for (int t = 0; t < P2; ++t) {
    // DeepMind-style rows index C transposed: row t = (x, y) belongs to C_(y, x).
    const int c = w_convention == MF_W_DEEPMIND_CT ? (t % n0) * n0 + (t / n0) : t;
    memcpy(&a.W[(size_t)c * R], &W[(size_t)t * R], sizeof(double) * R);
  }
  return new_handle(a, out);
}

mf_status mf_algo_builtin(const char* name, mf_algo** out) {
  clear_error();
  if (!out || !name) return fail(MF_ERR_ARG, "NULL argument");
  *out = nullptr;
  Algo a;
  if (!builtin(name, &a)) return fail(MF_ERR_ARG, std::string("unknown built-in algorithm: ") + name);
  return new_handle(a, out);
}

mf_status mf_algo_compose(const mf_algo* outer, const mf_algo* inner, mf_algo** out) {
  clear_error();
  if (!outer || !inner || !out) return fail(MF_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (outer->a.m0 * inner->a.m0 > 8 || outer->a.k0 * inner->a.k0 > 8 || outer->a.n0 * inner->a.n0 > 8)
    return fail(MF_ERR_ARG, "composed split factors must be <= 8");
  if ((int64_t)outer->a.R * inner->a.R > 4096) return fail(MF_ERR_ARG, "composed R must be <= 4096");
  return new_handle(compose(outer->a, inner->a), out);
}

mf_status mf_algo_rebase(const mf_algo* a, const int64_t* X, const int64_t* Y, const int64_t* Z, mf_algo** out) {
  clear_error();
  if (!a || !X || !Y || !Z || !out) return fail(MF_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (!a->a.square()) return fail(MF_ERR_UNSUPPORTED, "re-basis is defined for square algorithms");
  Algo b;
  if (!rebase(a->a, X, Y, Z, &b)) return fail(MF_ERR_ARG, "X, Y and Z must be unimodular integer matrices");
  return new_handle(b, out);
}

mf_status mf_algo_info(const mf_algo* a, int* n0, int* R, int* nnz_u, int* nnz_v, int* nnz_w) {
  clear_error();
  if (!a) return fail(MF_ERR_ARG, "algo is NULL");
  auto nnz = [](const std::vector<double>& x) {
    int c = 0;
    for (double v : x) c += v != 0.0;
    return c;
  };
  if (n0) *n0 = a->a.p;
  if (R) *R = a->a.R;
  if (nnz_u) *nnz_u = nnz(a->a.U);
  if (nnz_v) *nnz_v = nnz(a->a.V);
  if (nnz_w) *nnz_w = nnz(a->a.W);
  return MF_OK;
}

mf_status mf_algo_get_uvw(const mf_algo* a, double* U, double* V, double* W) {
  clear_error();
  if (!a) return fail(MF_ERR_ARG, "algo is NULL");
  if (U) memcpy(U, a->a.U.data(), a->a.U.size() * sizeof(double));
  if (V) memcpy(V, a->a.V.data(), a->a.V.size() * sizeof(double));
  if (W) memcpy(W, a->a.W.data(), a->a.W.size() * sizeof(double));
  return MF_OK;
}

void mf_algo_free(mf_algo* a) {
  if (!a) return;
  drop_plans(a->id);
  delete a;
}

mf_status mf_workspace_bytes(const mf_algo* algo, int depth, int cutoff, int64_t n, int dtype, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(MF_ERR_ARG, "bytes is NULL");
  *bytes = 0;
  // Validate everything except the pointers.
  static const double dummy[3] = {0, 0, 0};
  mf_status st = check_request(algo, true, depth, cutoff, &dummy[0], &dummy[1], (void*)&dummy[2], 0, dtype);
  if (st != MF_OK) return st;
  if (n < 0) return fail(MF_ERR_ARG, "n must be >= 0");
  if (n > kMaxN) return fail(MF_ERR_SHAPE, "n exceeds the supported maximum (2^20)");
  if (n == 0) return MF_OK;
  std::shared_ptr<const Plan> pl;
  st = plan_for(algo, depth, cutoff, n, dtype, &pl);
  if (st != MF_OK) return st;
  *bytes = pl->ws_bytes;
  return MF_OK;
}

mf_status mf_plan_query(const mf_algo* algo, int depth, int cutoff, int64_t n, int dtype, mf_plan_info* out) {
  clear_error();
  if (!out) return fail(MF_ERR_ARG, "out is NULL");
  *out = mf_plan_info{};
  static const double dummy[3] = {0, 0, 0};
  mf_status st = check_request(algo, depth > 0, depth, cutoff, &dummy[0], &dummy[1], (void*)&dummy[2], 0, dtype);
  if (st != MF_OK) return st;
  if (n < 1) return fail(MF_ERR_ARG, "n must be >= 1");
  if (n > kMaxN) return fail(MF_ERR_SHAPE, "n exceeds the supported maximum (2^20)");
  std::shared_ptr<const Plan> pl;
  st = plan_for(algo, depth, cutoff, n, dtype, &pl);
  if (st != MF_OK) return st;
  auto stage_bytes = [&](const std::vector<CombineStage>& stages) {
    double b = 0;
    for (const CombineStage& cs : stages)
      for (const CombSet& set : cs.sets) {
        for (int k = 0; k < cs.nin; ++k) b += (double)cs.ins[set.in_beg + k].vr * cs.ins[set.in_beg + k].vc;
        for (int o = set.out_beg; o < set.out_end; ++o) b += (double)cs.outs[o].vr * cs.outs[o].vc;
      }
    return b * (double)pl->elem;
  };
  out->levels = pl->levels;
  out->levels_outer = pl->levels_outer;
  out->groups = pl->groups;
  out->pre_stages = (int)pl->pre.size();
  out->post_stages = (int)pl->post.size();
  out->leaf_m = pl->m;
  out->products = (int64_t)pl->prods.size();
  // MFMA work as executed: every 128 x 128 output tile of every product,
  // over the product's valid inner size in whole K steps of 16 (the FP64 /
  // FP32 kernel stops there; the BF16 and fused-operand kernels run the
  // padded K)
  const int leaf = (pl->dtype >> 8) & 0xff;
  const bool padded_k = leaf == 2 || leaf == 3 || pl->fused_terms > 0;
  const double tm = (double)((pl->m + kLeafTile - 1) / kLeafTile * kLeafTile);
  const double tn = (double)((pl->leaf_n + kLeafTile - 1) / kLeafTile * kLeafTile);
  double flops = 0.0;
  for (const ProdDesc& pd : pl->prods) {
    const int64_t k = padded_k ? pl->leaf_k
                               : std::min<int64_t>(pl->leaf_k, std::min<int64_t>(pd.a_vc, pd.b_vr));
    flops += 2.0 * tm * tn * (double)((k + 15) / 16 * 16);
  }
  out->gemm_flops = flops;
  out->pre_bytes = stage_bytes(pl->pre);
  out->post_bytes = stage_bytes(pl->post);
  out->ws_bytes = pl->ws_bytes;
  return MF_OK;
}

mf_status mf_fastmm_ws(const mf_algo* algo, int depth, int cutoff, const void* A, const void* B, void* C,
                       int64_t n, int dtype, void* workspace, size_t ws_bytes, mf_stream stream) {
  clear_error();
  mf_status st = check_request(algo, true, depth, cutoff, A, B, C, n, dtype);
  if (st != MF_OK || n == 0) return st;
  std::shared_ptr<const Plan> pl;
  st = plan_for(algo, depth, cutoff, n, dtype, &pl);
  if (st != MF_OK) return st;
  if (pl->ws_bytes > 0) {
    if (!workspace) return fail(MF_ERR_ARG, "workspace is NULL");
    if (ws_bytes < pl->ws_bytes) return fail(MF_ERR_SHAPE, "workspace too small");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(MF_ERR_ARG, "workspace must be 256-byte aligned");
    const size_t mat = (size_t)n * (size_t)n * pl->elem;
    if (overlaps(workspace, pl->ws_bytes, A, mat) || overlaps(workspace, pl->ws_bytes, B, mat) ||
        overlaps(workspace, pl->ws_bytes, C, mat))
      return fail(MF_ERR_ARG, "workspace overlaps A, B or C");
  }
  return run(*pl, A, B, C, workspace, static_cast<hipStream_t>(stream));
}

mf_status mf_fastmm(const mf_algo* algo, int depth, int cutoff, const void* A, const void* B, void* C, int64_t n,
                    int dtype, mf_stream stream) {
  clear_error();
  mf_status st = check_request(algo, true, depth, cutoff, A, B, C, n, dtype);
  if (st != MF_OK || n == 0) return st;
  std::shared_ptr<const Plan> pl;
  st = plan_for(algo, depth, cutoff, n, dtype, &pl, !aligned16(A) || !aligned16(B));
  if (st != MF_OK) return st;
  return run_with_pool(*pl, A, B, C, static_cast<hipStream_t>(stream));
}

mf_status mf_classical_mm(const void* A, const void* B, void* C, int64_t n, int dtype, mf_stream stream) {
  clear_error();
  mf_status st = check_request(nullptr, false, 0, 0, A, B, C, n, dtype);
  if (st != MF_OK || n == 0) return st;
  std::shared_ptr<const Plan> pl;
  st = plan_for(nullptr, 0, 0, n, dtype, &pl, !aligned16(A) || !aligned16(B));
  if (st != MF_OK) return st;
  return run_with_pool(*pl, A, B, C, static_cast<hipStream_t>(stream));
}

mf_status mf_algo_from_uvw_rect(int m0, int k0, int n0, int R, const double* U, const double* V, const double* W,
                                mf_algo** out) {
  clear_error();
  if (!out) return fail(MF_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (m0 < 1 || k0 < 1 || n0 < 1 || m0 > 8 || k0 > 8 || n0 > 8) return fail(MF_ERR_ARG, "m0, k0, n0 must be in [1, 8]");
  if (R < 1 || R > 4096) return fail(MF_ERR_ARG, "R must be in [1, 4096]");
  if (!U || !V || !W) return fail(MF_ERR_ARG, "U, V and W must be non-NULL");
  Algo a;
  a.set_shape(m0, k0, n0);
  a.R = R;
  a.U.assign(U, U + (size_t)m0 * k0 * R);
  a.V.assign(V, V + (size_t)k0 * n0 * R);
  a.W.assign(W, W + (size_t)m0 * n0 * R);
  for (const std::vector<double>* x : {&a.U, &a.V, &a.W})
    for (double v : *x)
      if (!std::isfinite(v)) return fail(MF_ERR_ARG, "coefficients must be finite");
  return new_handle(a, out);
}

mf_status mf_algo_classical(int m0, int k0, int n0, mf_algo** out) {
  clear_error();
  if (!out) return fail(MF_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (m0 < 1 || k0 < 1 || n0 < 1 || m0 > 8 || k0 > 8 || n0 > 8) return fail(MF_ERR_ARG, "m0, k0, n0 must be in [1, 8]");
  return new_handle(classical_algo(m0, k0, n0), out);
}

mf_status mf_algo_concat(const mf_algo* a, const mf_algo* b, int axis, mf_algo** out) {
  clear_error();
  if (!a || !b || !out) return fail(MF_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (axis < 0 || axis > 2) return fail(MF_ERR_ARG, "axis must be 0 (m), 1 (k) or 2 (n)");
  if ((int64_t)a->a.R + b->a.R > 4096) return fail(MF_ERR_ARG, "R must be <= 4096");
  Algo c;
  if (!concat(a->a, b->a, axis, &c)) return fail(MF_ERR_ARG, "the other two dimensions of the algorithms differ");
  if (c.m0 > 8 || c.k0 > 8 || c.n0 > 8) return fail(MF_ERR_ARG, "split factors must be <= 8");
  return new_handle(c, out);
}

mf_status mf_algo_shape(const mf_algo* a, int* m0, int* k0, int* n0, int* R) {
  clear_error();
  if (!a) return fail(MF_ERR_ARG, "algo is NULL");
  if (m0) *m0 = a->a.m0;
  if (k0) *k0 = a->a.k0;
  if (n0) *n0 = a->a.n0;
  if (R) *R = a->a.R;
  return MF_OK;
}

mf_status mf_gemm(const mf_algo* algo, int depth, int cutoff, int64_t M, int64_t N, int64_t K, double alpha,
                  const void* A, int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc, int dtype,
                  mf_stream stream) {
  clear_error();
  if (depth > 0 && !algo) return fail(MF_ERR_ARG, "algo is NULL with depth > 0");
  if (depth < 0 || cutoff < 0) return fail(MF_ERR_ARG, "depth and cutoff must be >= 0");
  if (M < 0 || N < 0 || K < 0) return fail(MF_ERR_ARG, "M, N, K must be >= 0");
  const int base = dtype & ~MF_SCHED_FUSED;
  if ((base != MF_F64 && base != MF_F32))
    return fail(MF_ERR_UNSUPPORTED, "mf_gemm takes MF_F64 or MF_F32 with leaves in the storage type");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(MF_ERR_ARG, "alpha and beta must be finite");
  if (M == 0 || N == 0) return MF_OK;
  if (K == 0) return fail(MF_ERR_SHAPE, "K must be >= 1");
  if (M > kMaxN || N > kMaxN || K > kMaxN) return fail(MF_ERR_SHAPE, "dimensions exceed the supported maximum (2^20)");
  if (lda < K || ldb < N || ldc < N) return fail(MF_ERR_ARG, "leading dimensions must be >= the row lengths");
  if (lda > kMaxLdAB || ldb > kMaxLdAB) return fail(MF_ERR_SHAPE, "lda and ldb must be at most 2^21");
  if (ldc > INT32_MAX) return fail(MF_ERR_SHAPE, "ldc exceeds 2^31 - 1");
  if (!A || !B || !C) return fail(MF_ERR_ARG, "A, B and C must be non-NULL");
  const size_t elem = base == MF_F64 ? 8 : 4;
  if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) | reinterpret_cast<uintptr_t>(C)) & (elem - 1))
    return fail(MF_ERR_ARG, "A, B and C must be aligned to the element size");
  const size_t ba = ((size_t)(M - 1) * lda + K) * elem, bb = ((size_t)(K - 1) * ldb + N) * elem,
               bc = ((size_t)(M - 1) * ldc + N) * elem;
  if (overlaps(C, bc, A, ba) || overlaps(C, bc, B, bb)) return fail(MF_ERR_ARG, "C overlaps A or B");
  Shape sh;
  sh.M = M;
  sh.N = N;
  sh.K = K;
  sh.lda = lda;
  sh.ldb = ldb;
  sh.ldc = ldc;
  sh.copy_in = !aligned16(A) || !aligned16(B);
  std::shared_ptr<const Plan> pl;
  mf_status st = get_plan(depth > 0 ? algo : nullptr, depth, cutoff, sh, dtype, kStandaloneMinWorkgroups, &pl);
  if (st != MF_OK) return st;
  return run_with_pool(*pl, A, B, C, static_cast<hipStream_t>(stream), alpha, beta);
}

mf_status mf_phase_timing(int enable) {
  clear_error();
  std::lock_guard<std::mutex> lk(timing().mu);
  timing().enabled = enable != 0;
  return MF_OK;
}

mf_status mf_phase_timing_read(double* ms, int* calls) {
  clear_error();
  std::vector<std::array<hipEvent_t, kPhases + 1>> evs;
  {
    std::lock_guard<std::mutex> lk(timing().mu);
    evs.swap(timing().calls);
  }
  double acc[kPhases] = {0, 0, 0};
  mf_status st = MF_OK;
  for (auto& ev : evs) {
    if (hipEventSynchronize(ev[kPhases]) != hipSuccess) st = fail(MF_ERR_HIP, "hipEventSynchronize failed");
    for (int ph = 0; ph < kPhases && st == MF_OK; ++ph) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, ev[ph], ev[ph + 1]) != hipSuccess)
        st = fail(MF_ERR_HIP, "hipEventElapsedTime failed");
      acc[ph] += t;
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
  }
  if (ms)
    for (int ph = 0; ph < kPhases; ++ph) ms[ph] = acc[ph];
  if (calls) *calls = (int)evs.size();
  return st;
}

}  // extern "C"
