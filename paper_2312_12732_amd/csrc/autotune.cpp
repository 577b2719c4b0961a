// Autotuner of the batched form: for each product size it measures every
// candidate plan (classical, or a given algorithm at depth 1..max_depth)
// where it will run - many products of that size in one batch, which runs
// as one launch per phase - and picks the plan with the least device time per
// product.
//
// The GEMM tile shape is fixed (128 x 128, one compiled shape per element
// type), so the tuned parameters are the algorithm and the recursion depth;
// a depth that the level rule would not take for a size (the leaves would
// fall to the tile size or below, or the cutoff stops it) repeats a shallower
// plan and is skipped.
#include <algorithm>
#include <cmath>
#include <vector>

#include "mf_internal.h"

namespace mf {

constexpr double kMinGain = 0.05;  // least relative gain of a fast plan over the classical one

hipError_t launch_fill_uniform(void* p, int64_t count, int elem, uint64_t seed, hipStream_t s);

namespace {

// Device buffers of one tuning batch, freed on every exit path.
struct Buffers {
  void* a = nullptr;
  void* b = nullptr;
  void* c = nullptr;
  ~Buffers() {
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (c) (void)hipFree(c);
  }
};

struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

struct BatchGuard {
  mf_batch* b = nullptr;
  ~BatchGuard() { mf_batch_free(b); }
};

constexpr size_t kMaxTuneBytes = size_t(8) << 30;  // operands, and workspace, of one tuning batch

}  // namespace

}  // namespace mf

using namespace mf;

extern "C" {

mf_status mf_autotune_batch(int nsizes, const int64_t* n, int dtype, const mf_algo* const* algos, int nalgos,
                            int max_depth, double work_flops, int max_copies, int reps, mf_stream stream,
                            int* out_choice, double* out_ms) {
  clear_error();
  if (nsizes < 1 || !n || !out_choice || !out_ms) return fail(MF_ERR_ARG, "nsizes >= 1 and non-NULL arrays needed");
  if (dtype != MF_F64 && dtype != MF_F32) return fail(MF_ERR_UNSUPPORTED, "batches support FP64 and FP32");
  if (nalgos < 0 || (nalgos > 0 && !algos) || max_depth < 0 || max_depth > 8)
    return fail(MF_ERR_ARG, "nalgos >= 0 with an algos array, 0 <= max_depth <= 8");
  if (!(work_flops > 0) || max_copies < 1 || reps < 1) return fail(MF_ERR_ARG, "work, copies and reps must be > 0");
  for (int j = 0; j < nalgos; ++j)
    if (!algos[j]) return fail(MF_ERR_ARG, "NULL algorithm handle");
  for (int i = 0; i < nsizes; ++i)
    if (n[i] < 1 || n[i] > (1 << 16)) return fail(MF_ERR_SHAPE, "sizes must be in [1, 65536]");
  const int ncand = 1 + nalgos * max_depth;
  const size_t elem = dtype == MF_F64 ? 8 : 4;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Events ev;
  if (hipEventCreate(&ev.e0) != hipSuccess || hipEventCreate(&ev.e1) != hipSuccess)
    return fail(MF_ERR_HIP, "hipEventCreate failed");

  for (int i = 0; i < nsizes; ++i) {
    const int64_t ni = n[i];
    const double flops = 2.0 * (double)ni * ni * ni;
    const size_t mat = (size_t)ni * ni * elem;
    int copies = (int)std::min<double>(max_copies, std::ceil(work_flops / flops));
    copies = (int)std::max<size_t>(1, std::min<size_t>(copies, kMaxTuneBytes / (3 * mat)));
    Buffers buf;
    if (hipMalloc(&buf.a, mat * copies) != hipSuccess || hipMalloc(&buf.b, mat * copies) != hipSuccess ||
        hipMalloc(&buf.c, mat * copies) != hipSuccess)
      return fail(MF_ERR_NOMEM, "device allocation for tuning failed");
    const int64_t count = (int64_t)ni * ni * copies;
    if (launch_fill_uniform(buf.a, count, (int)elem, 0x51ull + 2 * (uint64_t)i, s) != hipSuccess ||
        launch_fill_uniform(buf.b, count, (int)elem, 0x52ull + 2 * (uint64_t)i, s) != hipSuccess)
      return fail(MF_ERR_HIP, "operand fill failed");
    std::vector<const void*> pa(copies), pb(copies);
    std::vector<void*> pc(copies);
    for (int k = 0; k < copies; ++k) {
      pa[k] = static_cast<const char*>(buf.a) + mat * k;
      pb[k] = static_cast<const char*>(buf.b) + mat * k;
      pc[k] = static_cast<char*>(buf.c) + mat * k;
    }
    double best = -1.0;
    int best_c = 0;
    for (int c = 0; c < ncand; ++c) {
      double* slot = out_ms + (size_t)i * ncand + c;
      *slot = -1.0;
      const mf_algo* al = nullptr;
      int depth = 0;
      if (c > 0) {
        al = algos[(c - 1) / max_depth];
        depth = 1 + (c - 1) % max_depth;
        if (levels_for(ni, ni, ni, al->a.m0, al->a.k0, al->a.n0, al->a.R, depth, 0) != depth) continue;  // repeats a shallower plan
      }
      // the copies this candidate runs: as many as its workspace allows
      // within the tuning budget (the operands of the others stay unused)
      size_t ws1 = 0;
      if (al) {
        const mf_status wst = mf_workspace_bytes(al, depth, 0, ni, dtype, &ws1);
        if (wst != MF_OK) return wst;
      }
      const int cc = (int)std::max<size_t>(1, std::min<size_t>((size_t)copies, ws1 ? kMaxTuneBytes / ws1 : copies));
      std::vector<const mf_algo*> av(cc, al);
      std::vector<int> dv(cc, depth), cv(cc, 0);
      std::vector<int64_t> nv(cc, ni);
      BatchGuard bg;
      mf_status st = mf_batch_create(cc, nv.data(), av.data(), dv.data(), cv.data(), dtype, &bg.b);
      if (st != MF_OK) return st;
      st = mf_batch_run(bg.b, pa.data(), pb.data(), pc.data(), nullptr, 0, stream);  // untimed: upload, pool
      if (st != MF_OK) return st;
      if (hipEventRecord(ev.e0, s) != hipSuccess) return fail(MF_ERR_HIP, "hipEventRecord failed");
      for (int r = 0; r < reps; ++r) {
        st = mf_batch_run(bg.b, pa.data(), pb.data(), pc.data(), nullptr, 0, stream);
        if (st != MF_OK) return st;
      }
      if (hipEventRecord(ev.e1, s) != hipSuccess || hipEventSynchronize(ev.e1) != hipSuccess)
        return fail(MF_ERR_HIP, "event wait failed");
      int aborted = 0;
      st = mf_batch_aborted(bg.b, &aborted);
      if (st != MF_OK) return st;
      if (aborted) return fail(MF_ERR_HIP, "a tuning batch aborted (wait limit exceeded)");
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev.e0, ev.e1) != hipSuccess) return fail(MF_ERR_HIP, "hipEventElapsedTime failed");
      *slot = (double)ms / reps / cc;
      if (best < 0 || *slot < best) {
        best = *slot;
        best_c = c;
      }
    }
    // A fast plan must beat the classical GEMM by kMinGain: measured in a
    // batch of its own size, it does not pay for the launches its addition
    // phases add to a mixed batch (FP64, 512 sizes in [128, 2048]: plans won
    // by 2-3% made the mixed batch 2% slower than all-classical).
    const double classical = out_ms[(size_t)i * ncand];
    if (best_c != 0 && classical > 0.0 && best > (1.0 - kMinGain) * classical) best_c = 0;
    out_choice[i] = best_c;
  }
  return MF_OK;
}

}  // extern "C"
