// Batched execution: many independent products C_i = A_i B_i, each with its
// own algorithm, depth and size, planned as one task list in topological
// order and run as one launch per phase over all instances
// (kernels_batch.hip).
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "mf_internal.h"

struct mf_batch {
  int count = 0;
  int dtype = MF_F64;
  bool persistent = false;  // MF_BATCH_PERSISTENT: one launch; else one launch per phase
  size_t elem = 8;
  std::vector<int64_t> n;
  std::vector<std::shared_ptr<const mf::Plan>> plans;
  std::vector<size_t> ws_off;  // bytes, per instance
  size_t ws_bytes = 0;
  std::vector<mf::BatchTask> tasks;
  // phases of the task list, in order: [begin, end) and whether GEMM tiles
  std::vector<std::pair<int, int>> phase_range;
  std::vector<bool> phase_gemm;
  int nctr = 0;
  // record tables: stage records (plan, pre stage s >= 0 or post stage -1-q)
  // and GEMM records (plan), in the index order the tasks use
  std::vector<std::pair<const mf::Plan*, int>> stage_list;
  std::vector<const mf::Plan*> gemm_list;
  // device state, made on the first run: tasks, stage records, GEMM records
  // (immutable); instance table and counters (rewritten by every run)
  mutable std::once_flag uploaded;
  mutable mf_status upload_status = MF_OK;
  mutable std::string upload_error;
  mutable int grid = 0;
  mutable void* dev = nullptr;
  mutable mf::BatchTask* d_tasks = nullptr;
  mutable mf::StageRec* d_stages = nullptr;
  mutable mf::GemmRec* d_gemms = nullptr;
  mutable void* run_dev = nullptr;
  mutable mf::BatchInst* d_insts = nullptr;
  mutable int* d_ctr = nullptr;
  mutable mf::BatchInst* h_insts = nullptr;  // pinned staging of the instance table
  mutable hipEvent_t copied = nullptr;        // the last run's table copy has executed
  mutable hipEvent_t finished = nullptr;      // the last run's kernels have executed
  mutable std::mutex run_mu;                  // serialises runs issued from several host threads
  ~mf_batch() {
    if (finished) (void)hipEventSynchronize(finished);
    if (finished) (void)hipEventDestroy(finished);
    if (copied) (void)hipEventSynchronize(copied);
    if (copied) (void)hipEventDestroy(copied);
    if (h_insts) (void)hipHostFree(h_insts);
    if (dev) (void)hipFree(dev);
    if (run_dev) (void)hipFree(run_dev);
  }
};

namespace mf {
namespace {

constexpr int64_t kChunk = 32768;  // elements per combination task

mf_status build_batch(mf_batch* b, const std::vector<const mf_algo*>& algos, const int* depth, const int* cutoff) {
  struct Recs {
    std::vector<int> pre, post;
    int gemm = -1;
  };
  std::map<const Plan*, Recs> recs;
  for (int i = 0; i < b->count; ++i) {
    std::shared_ptr<const Plan> pl;
    mf_status st = get_plan(depth[i] > 0 ? algos[i] : nullptr, depth[i], cutoff[i], b->n[i], b->dtype,
                            kStandaloneMinWorkgroups, &pl);
    if (st != MF_OK) return st;
    if (!pl->square) return fail(MF_ERR_UNSUPPORTED, "batches take square algorithms");
    for (const CombineStage& cs : pl->pre)
      if (cs.kron3 || !batch_stage_supported(cs.nin, cs.nout_max, b->persistent))
        return fail(MF_ERR_UNSUPPORTED, "algorithm shape not supported in batches");
    for (const CombineStage& cs : pl->post)
      if (cs.kron3 || !batch_stage_supported(cs.nin, cs.nout_max, b->persistent))
        return fail(MF_ERR_UNSUPPORTED, "algorithm shape not supported in batches");
    b->plans.push_back(pl);
    if (!recs.count(pl.get())) {
      Recs r;
      for (size_t q = 0; q < pl->pre.size(); ++q) {
        r.pre.push_back((int)b->stage_list.size());
        b->stage_list.push_back({pl.get(), (int)q});
      }
      for (size_t q = 0; q < pl->post.size(); ++q) {
        r.post.push_back((int)b->stage_list.size());
        b->stage_list.push_back({pl.get(), -1 - (int)q});
      }
      r.gemm = (int)b->gemm_list.size();
      b->gemm_list.push_back(pl.get());
      recs[pl.get()] = r;
    }
  }
  // workspace and counters
  std::vector<int> ctr_base(b->count);
  for (int i = 0; i < b->count; ++i) {
    b->ws_off.push_back(b->ws_bytes);
    b->ws_bytes += (b->plans[i]->ws_bytes + 255) / 256 * 256;
    ctr_base[i] = b->nctr;
    b->nctr += (int)b->plans[i]->pre.size() + 1 + (int)b->plans[i]->post.size();
  }
  // tasks per (instance, stage), then the global topological order:
  // pre level 0 of every instance, pre level 1, ..., GEMM work items (larger
  // leaves first), post stages in launch order.
  auto stage_tasks = [&](int i, const CombineStage& cs, int rec, int wait_ctr, int wait_val, int done_ctr,
                         std::vector<BatchTask>* out) {
    const int64_t mm = cs.m * cs.m;
    for (size_t s = 0; s < cs.sets.size(); ++s)
      for (int64_t e0 = 0; e0 < mm; e0 += kChunk) {
        BatchTask t{};
        t.type = 0;
        t.inst = i;
        t.rec = rec;
        t.wait_ctr = wait_ctr;
        t.wait_val = wait_val;
        t.done_ctr = done_ctr;
        t.a = (int32_t)s;
        t.e0 = e0;
        t.e1 = std::min(mm, e0 + kChunk);
        out->push_back(t);
      }
  };
  auto count_stage = [&](const CombineStage& cs) {
    return (int)(cs.sets.size() * ((cs.m * cs.m + kChunk - 1) / kChunk));
  };
  int max_pre = 0, max_post = 0;
  for (auto& pl : b->plans) {
    max_pre = std::max(max_pre, (int)pl->pre.size());
    max_post = std::max(max_post, (int)pl->post.size());
  }
  std::vector<std::vector<BatchTask>> pre_phase(max_pre), post_phase(max_post);
  std::vector<std::pair<int64_t, std::vector<BatchTask>>> gemm_phase;
  for (int i = 0; i < b->count; ++i) {
    const Plan& pl = *b->plans[i];
    const Recs& r = recs[&pl];
    const int P = (int)pl.pre.size();
    int wait_ctr = -1, wait_val = 0;
    for (int s = 0; s < P; ++s) {
      stage_tasks(i, pl.pre[s], r.pre[s], wait_ctr, wait_val, ctr_base[i] + s, &pre_phase[s]);
      wait_ctr = ctr_base[i] + s;
      wait_val = count_stage(pl.pre[s]);
    }
    std::vector<BatchTask> gt;
    const int tiles = (int)((pl.m + kLeafTile - 1) / kLeafTile);
    for (int g = 0; g < pl.groups; ++g)
      for (int ti = 0; ti < tiles; ++ti)
        for (int tj = 0; tj < tiles; ++tj) {
          BatchTask t{};
          t.type = 1;
          t.inst = i;
          t.rec = r.gemm;
          t.wait_ctr = wait_ctr;
          t.wait_val = wait_val;
          t.done_ctr = ctr_base[i] + P;
          t.a = g;
          t.b = ti;
          t.c = tj;
          gt.push_back(t);
        }
    const int64_t work = (int64_t)(pl.prods.size()) * pl.m * pl.m * pl.m / std::max(1, pl.groups * tiles * tiles);
    wait_ctr = ctr_base[i] + P;
    wait_val = (int)gt.size();
    gemm_phase.push_back({work, std::move(gt)});
    for (int q = 0; q < (int)pl.post.size(); ++q) {
      stage_tasks(i, pl.post[q], r.post[q], wait_ctr, wait_val, ctr_base[i] + P + 1 + q, &post_phase[q]);
      wait_ctr = ctr_base[i] + P + 1 + q;
      wait_val = count_stage(pl.post[q]);
    }
  }
  std::stable_sort(gemm_phase.begin(), gemm_phase.end(),
                   [](const auto& x, const auto& y) { return x.first > y.first; });
  auto add_phase = [&](const std::vector<BatchTask>& v, bool gemm) {
    const int beg = (int)b->tasks.size();
    b->tasks.insert(b->tasks.end(), v.begin(), v.end());
    if ((int)b->tasks.size() > beg) {
      b->phase_range.push_back({beg, (int)b->tasks.size()});
      b->phase_gemm.push_back(gemm);
    }
  };
  for (auto& v : pre_phase) add_phase(v, false);
  std::vector<BatchTask> all_gemm;
  for (auto& v : gemm_phase) all_gemm.insert(all_gemm.end(), v.second.begin(), v.second.end());
  add_phase(all_gemm, true);
  for (auto& v : post_phase) add_phase(v, false);

  return MF_OK;
}

// Device state of a batch: plan descriptors, record tables, task list, run
// buffers.
mf_status upload_batch(const mf_batch* b) {
  std::vector<StageRec> stage_recs;
  std::vector<GemmRec> gemm_recs;
  for (const auto& sp : b->stage_list) {
    mf_status st = ensure_device(*sp.first);
    if (st != MF_OK) return st;
    const CombineStage& cs = sp.second >= 0 ? sp.first->pre[sp.second] : sp.first->post[-1 - sp.second];
    const char* d = sp.first->desc();
    stage_recs.push_back(StageRec{img_at<CombSet>(d, cs.img_sets), img_at<CombIn>(d, cs.img_ins),
                                  img_at<CombOut>(d, cs.img_outs), img_at<double>(d, cs.img_coef), cs.nin,
                                  (int32_t)cs.m});
  }
  for (const Plan* pl : b->gemm_list) {
    mf_status st = ensure_device(*pl);
    if (st != MF_OK) return st;
    const char* d = pl->desc();
    gemm_recs.push_back(GemmRec{img_at<ProdDesc>(d, pl->img_prods), img_at<EpiDesc>(d, pl->img_epis),
                                img_at<int32_t>(d, pl->img_group_beg), pl->groups, (int32_t)pl->m,
                                (int32_t)((pl->m + kLeafTile - 1) / kLeafTile), 0});
  }
  auto align = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t st_ = align(b->tasks.size() * sizeof(BatchTask));
  const size_t ss_ = align(std::max<size_t>(1, stage_recs.size()) * sizeof(StageRec));
  const size_t sg_ = align(gemm_recs.size() * sizeof(GemmRec));
  std::vector<char> host(st_ + ss_ + sg_, 0);
  memcpy(host.data(), b->tasks.data(), b->tasks.size() * sizeof(BatchTask));
  if (!stage_recs.empty()) memcpy(host.data() + st_, stage_recs.data(), stage_recs.size() * sizeof(StageRec));
  memcpy(host.data() + st_ + ss_, gemm_recs.data(), gemm_recs.size() * sizeof(GemmRec));
  if (hipMalloc(&b->dev, host.size()) != hipSuccess) {
    (void)hipGetLastError();
    b->dev = nullptr;
    return fail(MF_ERR_NOMEM, "device allocation of the batch task list failed");
  }
  if (hipMemcpy(b->dev, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail(MF_ERR_HIP, "copy of the batch task list failed");
  char* d = static_cast<char*>(b->dev);
  b->d_tasks = reinterpret_cast<BatchTask*>(d);
  b->d_stages = reinterpret_cast<StageRec*>(d + st_);
  b->d_gemms = reinterpret_cast<GemmRec*>(d + st_ + ss_);
  const size_t run_bytes = align((size_t)b->count * sizeof(BatchInst)) + (size_t)(b->nctr + 2) * sizeof(int);
  if (hipMalloc(&b->run_dev, run_bytes) != hipSuccess) {
    (void)hipGetLastError();
    b->run_dev = nullptr;
    return fail(MF_ERR_NOMEM, "device allocation of the batch run state failed");
  }
  b->d_insts = static_cast<BatchInst*>(b->run_dev);
  if (hipHostMalloc(reinterpret_cast<void**>(&b->h_insts), (size_t)b->count * sizeof(BatchInst), hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreateWithFlags(&b->copied, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->finished, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MF_ERR_NOMEM, "pinned staging allocation of the batch failed");
  }
  b->d_ctr = reinterpret_cast<int*>(static_cast<char*>(b->run_dev) + align((size_t)b->count * sizeof(BatchInst)));
  int dev_id = 0, cus = 256;
  if (hipGetDevice(&dev_id) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id);
  b->grid = (int)std::min<int64_t>((int64_t)b->tasks.size(), 2 * (int64_t)cus);
  return MF_OK;
}

}  // namespace
}  // namespace mf

using namespace mf;

extern "C" {

mf_status mf_batch_create(int count, const int64_t* n, const mf_algo* const* algos, const int* depth,
                          const int* cutoff, int dtype, mf_batch** out) {
  return mf_batch_create_form(count, n, algos, depth, cutoff, dtype, MF_BATCH_PHASES, out);
}

mf_status mf_batch_create_form(int count, const int64_t* n, const mf_algo* const* algos, const int* depth,
                               const int* cutoff, int dtype, int form, mf_batch** out) {
  clear_error();
  if (!out) return fail(MF_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (form != MF_BATCH_PHASES && form != MF_BATCH_PERSISTENT) return fail(MF_ERR_ARG, "unknown batch form");
  if (count < 1 || !n || !depth || !cutoff) return fail(MF_ERR_ARG, "count must be >= 1 and arrays non-NULL");
  if (dtype != MF_F64 && dtype != MF_F32) return fail(MF_ERR_UNSUPPORTED, "batches support FP64 and FP32 (native leaves)");
  std::vector<const mf_algo*> al(count, nullptr);
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > (1 << 16)) return fail(MF_ERR_SHAPE, "batch sizes must be in [1, 65536]");
    if (depth[i] < 0 || cutoff[i] < 0) return fail(MF_ERR_ARG, "depth and cutoff must be >= 0");
    al[i] = algos ? algos[i] : nullptr;
    if (depth[i] > 0 && !al[i]) return fail(MF_ERR_ARG, "depth > 0 needs an algorithm");
  }
  mf_batch* b = new (std::nothrow) mf_batch;
  if (!b) return fail(MF_ERR_NOMEM, "host allocation failed");
  b->count = count;
  b->dtype = dtype;
  b->persistent = form == MF_BATCH_PERSISTENT;
  b->elem = dtype == MF_F64 ? 8 : 4;
  b->n.assign(n, n + count);
  const mf_status st = build_batch(b, al, depth, cutoff);
  if (st != MF_OK) {
    delete b;
    return st;
  }
  *out = b;
  return MF_OK;
}

mf_status mf_batch_workspace_bytes(const mf_batch* b, size_t* bytes) {
  clear_error();
  if (!b || !bytes) return fail(MF_ERR_ARG, "NULL argument");
  *bytes = b->ws_bytes;
  return MF_OK;
}

mf_status mf_batch_tasks(const mf_batch* b, int* ntasks, int* nctr, int32_t* desc) {
  clear_error();
  if (!b) return fail(MF_ERR_ARG, "batch is NULL");
  if (ntasks) *ntasks = (int)b->tasks.size();
  if (nctr) *nctr = b->nctr;
  if (desc)
    for (size_t t = 0; t < b->tasks.size(); ++t) {
      const BatchTask& k = b->tasks[t];
      int32_t* o = desc + 5 * t;
      o[0] = k.type;
      o[1] = k.inst;
      o[2] = k.wait_ctr;
      o[3] = k.wait_val;
      o[4] = k.done_ctr;
    }
  return MF_OK;
}

mf_status mf_batch_run(const mf_batch* b, const void* const* A, const void* const* B, void* const* C, void* workspace,
                       size_t ws_bytes, mf_stream stream) {
  clear_error();
  if (!b || !A || !B || !C) return fail(MF_ERR_ARG, "NULL argument");
  std::call_once(b->uploaded, [&]() {
    b->upload_status = upload_batch(b);
    if (b->upload_status != MF_OK) b->upload_error = mf_last_error();
  });
  if (b->upload_status != MF_OK) return fail(b->upload_status, "batch device setup failed: " + b->upload_error);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<BatchInst> insts(b->count);
  const uintptr_t mask = b->elem - 1;
  for (int i = 0; i < b->count; ++i) {
    if (!A[i] || !B[i] || !C[i]) return fail(MF_ERR_ARG, "NULL matrix pointer in the batch");
    const uintptr_t a = reinterpret_cast<uintptr_t>(A[i]), bb = reinterpret_cast<uintptr_t>(B[i]),
                    c = reinterpret_cast<uintptr_t>(C[i]);
    if ((a | bb | c) & mask) return fail(MF_ERR_ARG, "matrices must be aligned to the element size");
    const size_t bytes = (size_t)b->n[i] * (size_t)b->n[i] * b->elem;
    if ((c < a + bytes && a < c + bytes) || (c < bb + bytes && bb < c + bytes))
      return fail(MF_ERR_ARG, "C overlaps A or B in instance " + std::to_string(i));
    const bool rows16 = ((size_t)b->n[i] * b->elem) % 16 == 0;
    insts[i].A = A[i];
    insts[i].B = B[i];
    insts[i].C = C[i];
    insts[i].vec_in = rows16 && ((a | bb) & 15) == 0;
    insts[i].vec_out = rows16 && (c & 15) == 0;
  }
  void* ws = workspace;
  bool own = false;
  if (b->ws_bytes > 0) {
    if (workspace) {
      if (ws_bytes < b->ws_bytes) return fail(MF_ERR_SHAPE, "workspace too small");
      if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(MF_ERR_ARG, "workspace must be 256-byte aligned");
      // the part of the workspace a run uses must not overlap any operand
      const uintptr_t w0 = reinterpret_cast<uintptr_t>(workspace), w1 = w0 + b->ws_bytes;
      for (int i = 0; i < b->count; ++i) {
        const size_t bytes = (size_t)b->n[i] * (size_t)b->n[i] * b->elem;
        for (const void* p : {A[i], B[i], static_cast<const void*>(C[i])}) {
          const uintptr_t x = reinterpret_cast<uintptr_t>(p);
          if (x < w1 && w0 < x + bytes)
            return fail(MF_ERR_ARG, "workspace overlaps A, B or C of instance " + std::to_string(i));
        }
      }
    } else {
      if (workspace_alloc(&ws, b->ws_bytes, s) != hipSuccess || !ws) {
        (void)hipGetLastError();
        return fail(MF_ERR_NOMEM, "batch workspace allocation failed");
      }
      own = true;
    }
  }
  for (int i = 0; i < b->count; ++i) insts[i].ws = static_cast<char*>(ws) + b->ws_off[i];
  mf_status st = MF_OK;
  // One instance table per batch, rewritten by every run.  Runs are ordered:
  // host threads take the lock; the pinned staging buffer is reused once the
  // previous run's copy out of it has executed; and the device table is
  // overwritten only after the previous run's kernels (on whatever stream
  // they were issued) have finished reading it.
  std::lock_guard<std::mutex> lk(b->run_mu);
  if (hipEventSynchronize(b->copied) != hipSuccess) {
    if (own) (void)workspace_free(ws, s);
    return fail(MF_ERR_HIP, "waiting for the previous run failed");
  }
  memcpy(b->h_insts, insts.data(), insts.size() * sizeof(BatchInst));
  hipError_t e = hipStreamWaitEvent(s, b->finished, 0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_insts, b->h_insts, insts.size() * sizeof(BatchInst), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(b->copied, s);
  if (b->persistent) {
    if (e == hipSuccess) e = launch_fill_zero(b->d_ctr, b->nctr + 2, s);
    if (e == hipSuccess)
      e = launch_batch((int)b->elem, b->d_tasks, (int)b->tasks.size(), b->d_stages, b->d_gemms, b->d_insts,
                       b->d_ctr, b->nctr, b->grid, s);
  } else {
    for (size_t p = 0; p < b->phase_range.size() && e == hipSuccess; ++p)
      e = launch_batch_phase((int)b->elem, b->phase_gemm[p], b->d_tasks, b->phase_range[p].first,
                             b->phase_range[p].second - b->phase_range[p].first, b->d_stages, b->d_gemms,
                             b->d_insts, s);
  }
  if (e == hipSuccess) e = hipEventRecord(b->finished, s);
  if (e != hipSuccess) st = fail(MF_ERR_HIP, std::string("batch launch failed: ") + hipGetErrorString(e));
  if (own && workspace_free(ws, s) != hipSuccess && st == MF_OK) st = fail(MF_ERR_HIP, "workspace release failed");
  return st;
}

mf_status mf_batch_aborted(const mf_batch* b, int* aborted) {
  clear_error();
  if (!b || !aborted) return fail(MF_ERR_ARG, "NULL argument");
  int flag = 0;
  if (hipDeviceSynchronize() != hipSuccess) return fail(MF_ERR_HIP, "synchronisation failed");
  if (!b->d_ctr || !b->persistent) {  // the phase form has no waits to abort
    *aborted = 0;
    return MF_OK;
  }
  if (hipMemcpy(&flag, b->d_ctr + b->nctr + 1, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(MF_ERR_HIP, "reading the abort flag failed");
  *aborted = flag;
  return MF_OK;
}

mf_status mf_batch_phases(const mf_batch* b, int* nphases, int32_t* desc) {
  clear_error();
  if (!b || !nphases) return fail(MF_ERR_ARG, "NULL argument");
  *nphases = (int)b->phase_range.size();
  if (desc)
    for (size_t p = 0; p < b->phase_range.size(); ++p) {
      desc[3 * p] = b->phase_range[p].first;
      desc[3 * p + 1] = b->phase_range[p].second;
      desc[3 * p + 2] = b->phase_gemm[p] ? 1 : 0;
    }
  return MF_OK;
}

void mf_batch_free(mf_batch* b) { delete b; }

}  // extern "C"
