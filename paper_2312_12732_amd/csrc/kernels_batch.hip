// Persistent batched kernel (gfx950): all tasks of many independent fast
// products - chunks of their pre-/post-addition stages and the work items
// of their grouped leaf GEMMs - run in one launch.
//
// Scheduling.  Tasks are stored in topological order (every task a task
// waits on has a smaller index).  A workgroup takes the next index from a
// global ticket, waits until its prerequisite counter reaches the required
// value, runs the task and increments its own counter.  A task only waits on
// tasks with smaller tickets, which were taken earlier by workgroups that are
// running, so the smallest unfinished task can always proceed: no deadlock,
// whatever the number of resident workgroups.  Every wait is bounded: past
// the spin limit (or once another workgroup has aborted) the workgroup sets
// the abort flag and exits, and so does every workgroup that takes a ticket
// afterwards; the host reports the abort.
//
// Memory ordering.  A task's results are published by an agent-scope
// release fence in every wave followed by the counter increment; a waiting
// workgroup polls the counter with relaxed agent-scope loads (vector loads
// that bypass the non-coherent caches without invalidating anything), sleeping
// between polls, and once it has seen the value every wave executes one
// agent-scope acquire fence (which invalidates the XCD-local caches) before
// reading the results, so producers and consumers may sit on different XCDs.
// Polling with acquire loads would invalidate the L2 on every poll and, with
// hundreds of waiting workgroups, starve the producers.
#include "combine_body.h"
#include "gemm_tile.h"

namespace mf {

namespace {

// Polls (each after a sleep of about 2000 cycles) before a wait gives up:
// a few seconds, far beyond any legitimate wait.
constexpr int kSpinLimit = 1 << 21;

struct BatchArgs {
  const BatchTask* tasks;
  const StageRec* stages;
  const GemmRec* gemms;
  const BatchInst* insts;
  int* ctr;  // nctr counters, then the ticket, then the abort flag
  int nctr;
  int ntasks;
};

__device__ __forceinline__ int load_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// WIDE: also the many-input combinations (27, 49, 64 inputs), through the
// register-accumulating body (the phase form has the registers for them).
template <class T, bool WIDE>
__device__ __forceinline__ void run_combine(const BatchArgs& g, const BatchTask& tk) {
  const StageRec st = load_uniform(g.stages + tk.rec);
  const BatchInst in = load_uniform(g.insts + tk.inst);
  CombArgs<T> a;
  a.A = static_cast<const T*>(in.A);
  a.B = static_cast<const T*>(in.B);
  a.C = static_cast<T*>(in.C);
  a.ws = static_cast<T*>(in.ws);
  a.sets = st.sets;
  a.ins = st.ins;
  a.outs = st.outs;
  a.coef = st.coef;
  a.m = st.m;
  a.vec_in = in.vec_in;
  a.vec_out = in.vec_out;
  a.scale_c = 0;
  a.alpha = T(1);
  a.beta = T(0);
  const CombSet set = load_uniform(st.sets + tk.a);
  const bool full = set.full && in.vec_in && in.vec_out;
  auto chunk = [&](auto body, int vec) {
    for (int64_t e = tk.e0 + (int64_t)threadIdx.x * vec; e < tk.e1; e += (int64_t)Tile128::NTHREADS * vec) {
      const int i = (int)(e / st.m), j = (int)(e % st.m);
      body(i, j);
    }
  };
  if constexpr (WIDE) {
    if (st.nin >= 27) {
      auto wide = [&](auto nin_c, auto nout_c) {
        constexpr int NIN = decltype(nin_c)::value, NOUT = decltype(nout_c)::value;
        if (full)
          chunk([&](int i, int j) { combine_acc_body<T, NIN, NOUT, 2, true>(a, set, i, j); }, 2);
        else
          chunk([&](int i, int j) { combine_acc_body<T, NIN, NOUT, 2, false>(a, set, i, j); }, 2);
      };
      if (st.nin == 27) wide(std::integral_constant<int, 27>(), std::integral_constant<int, 9>());
      if (st.nin == 49) wide(std::integral_constant<int, 49>(), std::integral_constant<int, 16>());
      if (st.nin == 64) wide(std::integral_constant<int, 64>(), std::integral_constant<int, 16>());
      return;
    }
  }
  with_nin(st.nin, [&](auto nin_c) {
    constexpr int NIN = decltype(nin_c)::value;
    constexpr int VEC = NIN <= 4 ? 4 : (NIN <= 9 ? 2 : 1);
    if (full)
      chunk([&](int i, int j) { combine_body<T, NIN, VEC, true>(a, set, i, j); }, VEC);
    else
      chunk([&](int i, int j) { combine_body<T, NIN, VEC, false>(a, set, i, j); }, VEC);
  });
}

template <class T>
__device__ __forceinline__ void run_gemm(const BatchArgs& g, const BatchTask& tk, T* lds) {
  const GemmRec gr = load_uniform(g.gemms + tk.rec);
  const BatchInst in = load_uniform(g.insts + tk.inst);
  GemmArgs<T> a;
  a.A = static_cast<const T*>(in.A);
  a.B = static_cast<const T*>(in.B);
  a.C = static_cast<T*>(in.C);
  a.ws = static_cast<T*>(in.ws);
  a.prods = gr.prods;
  a.epis = gr.epis;
  a.group_beg = gr.group_beg;
  a.terms = nullptr;
  a.groups = gr.groups;
  a.m = a.n = a.k = gr.m;
  a.tiles_m = gr.tiles;
  a.tiles_n = gr.tiles;
  a.vec_in = in.vec_in;
  a.scale_c = 0;
  a.alpha = T(1);
  a.beta = T(0);
  gemm_tile<T, Tile128>(a, tk.a, tk.b, tk.c, lds);
}

// Wave 0 of a workgroup claims its next task: it publishes the completion of
// the previous one (done counter prev_done, -1 for none), takes a ticket and
// waits until the task's prerequisite counter is reached.  Returns the task
// index, g.ntasks when the list is exhausted, or -1 after an abort.  All 64
// lanes run this with identical control flow: every branch and loop condition
// is a value broadcast with readfirstlane (all lanes poll the same address),
// and the one lane that issues an atomic does it in a region with no loop and
// no barrier, so the wave never splits around the polling loop.
__device__ __forceinline__ int claim_task(const BatchArgs& g, int prev_done, int lane) {
  int* ticket = g.ctr + g.nctr;
  int* abort_flag = ticket + 1;
  int t = 0;
  if (lane == 0) {
    if (prev_done >= 0) __hip_atomic_fetch_add(&g.ctr[prev_done], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    t = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  t = __builtin_amdgcn_readfirstlane(t);
  if (t >= g.ntasks) return g.ntasks;
  if (__builtin_amdgcn_readfirstlane(load_relaxed(abort_flag)) != 0) return -1;
  const BatchTask tk = load_uniform(g.tasks + t);
  if (tk.wait_ctr < 0) return t;
  bool ok = true;
  for (int spins = 0;; ++spins) {
    if (__builtin_amdgcn_readfirstlane(load_relaxed(&g.ctr[tk.wait_ctr])) >= tk.wait_val) break;
    if (__builtin_amdgcn_readfirstlane(load_relaxed(abort_flag)) != 0 || spins >= kSpinLimit) {
      ok = false;
      break;
    }
    __builtin_amdgcn_s_sleep(32);
  }
  if (ok) return t;
  if (lane == 0) __hip_atomic_exchange(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return -1;
}

// Persistent form: one launch; workgroups take tasks in ticket order and wait
// on per-instance stage counters.  Only wave 0 touches the counters
// (claim_task); it hands the task index to the other waves through LDS across
// one barrier.  The task loop's condition is that broadcast index, so the
// loop, like every barrier in it, is wave-uniform.  (An earlier form let
// thread 0 alone publish and fetch in separate regions; the compiler turned
// the loop into a nested one that lane 0 left to fetch a ticket while lanes
// 1-63 of wave 0 kept re-running the barrier and the old task: the launch
// never finished.)
template <class T>
__global__ void __launch_bounds__(Tile128::NTHREADS, Tile128::WAVES_PER_SIMD) batch_persistent(BatchArgs g) {
  __shared__ T lds[Geom<T, Tile128>::ELEMS];
  __shared__ int s_task;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = (int)(threadIdx.x & 63);
  int prev_done = -1;
  for (;;) {
    if (wave == 0) {
      const int t = claim_task(g, prev_done, lane);
      if (lane == 0) s_task = t;
    }
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_task);
    if (t < 0 || t >= g.ntasks) break;
    const BatchTask tk = load_uniform(g.tasks + t);
    if (tk.wait_ctr >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (tk.type == 0)
      run_combine<T, false>(g, tk);
    else
      run_gemm<T>(g, tk, lds);
    // every wave's results reach agent scope before wave 0 publishes them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    prev_done = tk.done_ctr;
  }
}

// Phase form: one launch per phase (a pre-addition level of every instance,
// all GEMM tiles, a post-addition level of every instance); workgroup b runs
// task task0 + b.  No counters and no waits: launch order on the stream
// orders the phases.
template <class T>
__global__ void __launch_bounds__(Tile128::NTHREADS) batch_combine_phase(BatchArgs g, int task0) {
  const BatchTask tk = load_uniform(g.tasks + task0 + blockIdx.x);
  run_combine<T, true>(g, tk);
}

template <class T>
__global__ void __launch_bounds__(Tile128::NTHREADS, Tile128::WAVES_PER_SIMD) batch_gemm_phase(BatchArgs g, int task0) {
  __shared__ T lds[Geom<T, Tile128>::ELEMS];
  const BatchTask tk = load_uniform(g.tasks + task0 + blockIdx.x);
  run_gemm<T>(g, tk, lds);
}

__global__ void fill_zero(int* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

}  // namespace

bool batch_stage_supported(int nin, int nout_max, bool persistent) {
  if (nin == 1 || nin == 4 || nin == 7 || nin == 8 || nin == 9 || nin == 16) return true;
  if (persistent) return false;
  return (nin == 27 && nout_max <= 9) || ((nin == 49 || nin == 64) && nout_max <= 16);
}

hipError_t launch_fill_zero(int* p, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_batch(int elem, const BatchTask* tasks, int ntasks, const StageRec* stages, const GemmRec* gemms,
                        const BatchInst* insts, int* ctr, int nctr, int grid, hipStream_t s) {
  BatchArgs g;
  g.tasks = tasks;
  g.stages = stages;
  g.gemms = gemms;
  g.insts = insts;
  g.ctr = ctr;
  g.nctr = nctr;
  g.ntasks = ntasks;
  if (elem == 8)
    hipLaunchKernelGGL(batch_persistent<double>, dim3(grid), dim3(Tile128::NTHREADS), 0, s, g);
  else
    hipLaunchKernelGGL(batch_persistent<float>, dim3(grid), dim3(Tile128::NTHREADS), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_batch_phase(int elem, bool gemm, const BatchTask* tasks, int task0, int count,
                              const StageRec* stages, const GemmRec* gemms, const BatchInst* insts, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  BatchArgs g{};
  g.tasks = tasks;
  g.stages = stages;
  g.gemms = gemms;
  g.insts = insts;
  g.ntasks = task0 + count;
  const dim3 grid((unsigned)count), block(Tile128::NTHREADS);
  if (elem == 8) {
    if (gemm)
      hipLaunchKernelGGL(batch_gemm_phase<double>, grid, block, 0, s, g, task0);
    else
      hipLaunchKernelGGL(batch_combine_phase<double>, grid, block, 0, s, g, task0);
  } else {
    if (gemm)
      hipLaunchKernelGGL(batch_gemm_phase<float>, grid, block, 0, s, g, task0);
    else
      hipLaunchKernelGGL(batch_combine_phase<float>, grid, block, 0, s, g, task0);
  }
  return hipGetLastError();
}

}  // namespace mf
