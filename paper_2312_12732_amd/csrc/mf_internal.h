// Internal data structures of the mf library: the algorithm handle, the
// execution plan and the descriptors the kernels read.  Host and device code
// both include this header; nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "mf.h"

namespace mf {

// ---------------------------------------------------------------------------
// Algorithms
// ---------------------------------------------------------------------------

// A canonical <m0,k0,n0;R> algorithm: A is split into m0 x k0 blocks, B into
// k0 x n0 and C into m0 x n0, each numbered row-major; U is (m0 k0) x R, V is
// (k0 n0) x R and W is (m0 n0) x R, row-major, with row c of W belonging to
// C_c.  A square algorithm <p,p,p;R> has p = m0 = k0 = n0; p is 0 otherwise.
struct Algo {
  int p = 0;
  int m0 = 0, k0 = 0, n0 = 0;
  int R = 0;
  std::vector<double> U, V, W;
  // A Kronecker composition (compose, power) keeps its factors, outermost
  // first, each without factors of its own; empty for any other algorithm.
  std::vector<Algo> factors;
  double u(int k, int r) const { return U[(size_t)k * R + r]; }
  double v(int k, int r) const { return V[(size_t)k * R + r]; }
  double w(int k, int r) const { return W[(size_t)k * R + r]; }
  bool square() const { return m0 == k0 && k0 == n0; }
  void set_shape(int m, int k, int n) {
    m0 = m;
    k0 = k;
    n0 = n;
    p = square() ? m : 0;
  }
};

// Number of failing Brent equations (exact for integer coefficients).
int64_t brent_violations(const Algo& a);
Algo compose(const Algo& outer, const Algo& inner);
Algo power(const Algo& a, int d);
// Direct sum along one dimension (axis 0: rows of A and C, 1: the inner
// dimension, 2: columns of B and C); false if the other dimensions differ.
bool concat(const Algo& a, const Algo& b, int axis, Algo* out);
// Re-base by unimodular X, Y, Z (p x p, row-major); false if not unimodular.
bool rebase(const Algo& a, const int64_t* X, const int64_t* Y, const int64_t* Z, Algo* out);
bool builtin(const std::string& name, Algo* out);
// The textbook partitioned product <m0,k0,n0; m0 k0 n0>.
Algo classical_algo(int m0, int k0, int n0);

}  // namespace mf

struct mf_algo {
  mf::Algo a;
  uint64_t id = 0;  // unique per handle; keys the plan cache
};

namespace mf {

// ---------------------------------------------------------------------------
// Device descriptors
// ---------------------------------------------------------------------------

// Source (or destination) of a view: the caller's A, B or C, or the
// workspace.
enum Src : int32_t { SRC_A = 0, SRC_B = 1, SRC_C = 2, SRC_WS = 3 };

// One leaf product P_r = X_r Y_r of size m x m x m, where X_r and Y_r are
// views (src, offset, ld) of the inputs or of workspace blocks.  Entries of
// a view at row >= vr or column >= vc are zero (virtual padding).
struct ProdDesc {
  int64_t a_off, b_off;      // element offsets of the view origins
  int32_t a_src, b_src;      // Src
  int32_t lda, ldb;          // leading dimensions (elements)
  int32_t a_vr, a_vc;        // valid rows / columns of the A view
  int32_t b_vr, b_vc;        // valid rows / columns of the B view
  int32_t epi_beg, epi_end;  // range in the epilogue list
  // Fused-operand plans: the A operand is sum_t coef_t X_t over a_terms
  // views X_t = terms[a_term0 + t] of the A source (the pre-addition done in
  // the operand load), and so for B; 0 terms: the single view above.
  int32_t a_terms, b_terms;
  int32_t a_term0, b_term0;
};

// One term of a fused operand: coef times the view of its product's source
// at `off` with leading dimension lda (ldb), valid over vr x vc.
struct TermDesc {
  int64_t off;
  double coef;
  int32_t vr, vc;
};

// One post-addition term of the GEMM epilogue: output block (dst, offset,
// ld) gets coef * P_r.  first = 1: the product writes the block first (in
// product order) and stores; 0: accumulates; 2: stores zeros (a block that
// no product feeds, which happens only through padding).
struct EpiDesc {
  int64_t c_off;
  int32_t c_src;  // SRC_C or SRC_WS
  int32_t ldc;
  int32_t c_vr, c_vc;
  int32_t first;
  int32_t pad_;
  double coef;
};

// Input view of a linear-combination stage.
struct CombIn {
  int64_t off;
  int32_t src;
  int32_t ld;
  int32_t vr, vc;  // zero outside (vr = vc = 0: an all-zero input)
};

// Output of a linear-combination stage: out = sum_k coef[k] * in_k.
struct CombOut {
  int64_t off;
  int32_t dst;
  int32_t ld;
  int32_t vr, vc;  // only this extent is written
  int32_t coef_off;
  int32_t pad_;
};

// One operand set of a linear-combination stage: `nin` input views starting
// at ins[in_beg] and the outputs [out_beg, out_end), all of rows x cols
// elements.  full: every view covers its whole block (no virtual padding).
struct CombSet {
  int32_t in_beg;
  int32_t out_beg, out_end;
  int32_t full;
  int32_t rows, cols;
};

// A linear-combination launch: one operand set per blockIdx.y, each over
// blocks of its own shape (m x m for the Kronecker-factored and batched
// stages, which are square).
struct CombineStage {
  // kron3 = 1: a level of a three-factor Kronecker composition of <2,2,2;7>
  // algorithms (<8,8,8;343>).  Each set then lists its inputs and outputs in
  // factor order (index t = 16 t1 + 4 t2 + t3 over the factors' 2 x 2 block
  // indices, r = 49 r1 + 7 r2 + r3 over their products; outputs that are
  // not stored have an empty extent), and its coefficients are the three
  // 4 x 7 factor matrices, starting at the first output's coef_off.  kpost:
  // the post-addition (inputs are products, outputs blocks) rather than the
  // pre-addition.
  int kron3 = 0;
  int kpost = 0;
  int nin = 0;
  int nout_max = 0;  // most outputs of any set
  int64_t m = 0;         // block size of a square stage
  int64_t elems_max = 0;  // largest rows x cols of any set
  std::vector<CombSet> sets;
  std::vector<CombIn> ins;
  std::vector<CombOut> outs;
  std::vector<double> coef;
  // byte offsets of sets, ins, outs and coef in the plan's descriptor image
  size_t img_sets = 0, img_ins = 0, img_outs = 0, img_coef = 0;
};

// Device pointer to an entry of a descriptor image: `base` is where the image
// sits in device memory, `off` the entry's byte offset in it.
template <class T>
inline const T* img_at(const char* base, size_t off) {
  return reinterpret_cast<const T*>(base + off);
}

// BF16 leaves: the last pre-addition level runs fused with the BF16 staging.
// One set per block of the level above: its nin quarters are the inputs, and
// each child that is a leaf operand is staged operand z = sum_k coef[k] in_k
// (z < products: the A operand of product z, by rows; otherwise the B
// operand of product z - products, transposed).
struct StageSet {
  int32_t in_beg;
  int32_t out_beg, out_end;
  int32_t side;  // 0: A operands, 1: B operands
};

struct StageOut {
  int32_t z;
  int32_t coef_off;  // nin coefficients, one per input (zeros included)
};

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------

// Execution plan of one request, a recursive data flow of `levels` levels of
// the algorithm (split factor p, R products per level):
//  - pre-addition stages, one launch per level: every block of the level
//    above is split into p^2 quarters and each of its R children is either a
//    (scaled) view of one quarter or a materialised linear combination;
//  - one grouped GEMM over all R^levels leaf products.  The products are
//    grouped by the first `levels_outer` levels: group g computes the result
//    P_g of its sub-problem, with the post-additions of the remaining inner
//    levels fused into the GEMM epilogue (composed coefficients);
//  - post-addition stages, one launch per outer level, innermost first,
//    combining R child results into the p^2 blocks of their parent (C at the
//    top).  With levels_outer = 0 the epilogue writes C directly.
// Shape of one product C (M x N) = A (M x K) B (K x N): row-major with
// leading dimensions lda, ldb, ldc (elements).
struct Shape {
  int64_t M = 0, N = 0, K = 0;
  int64_t lda = 0, ldb = 0, ldc = 0;
  // operands with unaligned rows are read in place rather than copied into
  // aligned workspace blocks (plans that must fit a fixed workspace)
  bool no_copy = false;
  // the caller's A or B base is not 16-byte aligned: copy as for unaligned
  // rows (plans whose workspace the library allocates)
  bool copy_in = false;
  static Shape sq(int64_t n) { return Shape{n, n, n, n, n, n}; }
  bool square() const { return M == N && N == K && lda == M && ldb == M && ldc == M; }
};

struct Plan {
  Shape shape;          // the request
  bool square = true;   // shape.square() and only square algorithm levels
  int64_t n = 0;        // true size (M)
  int64_t npad = 0;     // padded size = P * m (square plans)
  int64_t m = 0;        // leaf rows (multiple of the GEMM tile); every leaf size of a square plan
  int64_t leaf_n = 0, leaf_k = 0;  // leaf columns and inner size
  int64_t m_outer = 0;  // size of a group's output block (P_inner * m)
  int levels = 0, levels_outer = 0;
  int P = 1, P_outer = 1;
  int R = 1, groups = 1;
  int dtype = MF_F64;
  size_t elem = 8;
  size_t ws_bytes = 0;
  std::vector<ProdDesc> prods;   // ordered by group
  std::vector<EpiDesc> epis;
  std::vector<TermDesc> terms;   // fused-operand plans: operand terms
  int fused_terms = 0;           // most terms of any fused operand (0: not fused)
  std::vector<int32_t> group_beg;  // groups + 1 entries
  std::vector<CombineStage> pre, post;  // in launch order
  // BF16 leaves: every leaf operand is staged once as BF16 (two planes, hi
  // and lo, for split-BF16x3) in the workspace from this byte offset on: the
  // A operands of the products in product order, then their B operands
  // transposed (row j holds column j), each plane m x m in the block order of
  // the BF16 GEMM (16 x 32 blocks, k-block major).
  int64_t bf_base = -1;
  int bf_planes = 0;
  // The staging sets (see StageSet): every staged operand is the output of
  // exactly one set; bf_nin inputs per set, each quarter of size m.
  int bf_nin = 0;
  std::vector<StageSet> bf_sets;
  std::vector<CombIn> bf_ins;
  std::vector<StageOut> bf_outs;
  std::vector<float> bf_coef;
  // Descriptor image: every descriptor array above, each at a 256-byte
  // aligned byte offset, as the kernels read it from device memory.  Made
  // when the plan is built; the kernels get the device address of a copy of
  // it (the plan's own, or one the caller's call placed elsewhere).
  std::vector<char> image;
  size_t img_prods = 0, img_epis = 0, img_group_beg = 0, img_terms = 0;
  size_t img_bf_sets = 0, img_bf_ins = 0, img_bf_outs = 0, img_bf_coef = 0;
  // the plan's own device copy of the image (one allocation, owned by the
  // plan), made on first use
  mutable std::once_flag uploaded;
  mutable mf_status upload_status = MF_OK;
  mutable void* dev = nullptr;
  const char* desc() const { return static_cast<const char*>(dev); }
  ~Plan();
};

// ---------------------------------------------------------------------------
// Batched execution: many independent products in one persistent launch
// ---------------------------------------------------------------------------

// Device record of one combination stage of a plan (pointers into the plan's
// device descriptors).
struct StageRec {
  const CombSet* sets;
  const CombIn* ins;
  const CombOut* outs;
  const double* coef;
  int32_t nin;
  int32_t m;
};

// Device record of the grouped GEMM of a plan.
struct GemmRec {
  const ProdDesc* prods;
  const EpiDesc* epis;
  const int32_t* group_beg;
  int32_t groups;
  int32_t m;
  int32_t tiles;
  int32_t pad_;
};

// Per-run pointers of one instance.
struct BatchInst {
  const void* A;
  const void* B;
  void* C;
  void* ws;
  int32_t vec_in, vec_out;
};

// One task of the persistent kernel, in topological order: a chunk
// [e0, e1) of one set of a combination stage (type 0) or one (group, tile)
// work item of a grouped GEMM (type 1).  The task waits until counter
// wait_ctr reaches wait_val (no wait if wait_ctr < 0) and increments done_ctr
// when it has finished.
struct BatchTask {
  int32_t type;
  int32_t inst;
  int32_t rec;  // StageRec or GemmRec index
  int32_t wait_ctr, wait_val, done_ctr;
  int32_t a, b, c;  // combination: set; GEMM: group, ti, tj
  int32_t pad_;
  int64_t e0, e1;
};

// Builds (or fetches from the cache) the plan for a request.  Outer levels
// are split into groups while the grouped GEMM has fewer than min_wg
// workgroups.  A standalone product takes every level as an outer level:
// each leaf product is stored once and the post-additions run as separate
// HBM-bound launches.  Fusing inner post-additions into the GEMM epilogue
// moves fewer bytes but its read-modify-writes stall the MFMA pipes; on
// MI355X at n = 8192 (FP64 Winograd) storing every product is faster at
// depth 1 / 2 / 3: 14.82 / 14.30 / 15.05 ms against 15.13 / 14.86 / 16.23 ms
// with outer levels only until 1024 workgroups.  Batches use the same plans,
// so an instance's result is bitwise that of the standalone call.
// Returns an mf_status and sets the thread's error message on failure.
constexpr int64_t kStandaloneMinWorkgroups = int64_t(1) << 62;
mf_status get_plan(const mf_algo* algo, int depth, int cutoff, const Shape& shape, int dtype, int64_t min_wg,
                   std::shared_ptr<const Plan>* out);
inline mf_status get_plan(const mf_algo* algo, int depth, int cutoff, int64_t n, int dtype, int64_t min_wg,
                          std::shared_ptr<const Plan>* out) {
  return get_plan(algo, depth, cutoff, Shape::sq(n), dtype, min_wg, out);
}

// Copies the plan's descriptor image to the device once (host-only queries
// such as the workspace size never touch the device); afterwards pl.desc()
// is its device address.
mf_status ensure_device(const Plan& pl);

// Releases the cached plans of an algorithm handle that is being freed.
void drop_plans(uint64_t algo_id);

// Leaf tile granularity: every leaf size is a multiple of this.
constexpr int kLeafTile = 128;
// Leaf sizes of plans with FP64 / FP32 leaves and stored products are
// multiples of kLeafStep (whole K steps of the GEMM, 16-byte rows); the GEMM
// covers a leaf with ceil(size / 128) tiles, the last one moved inside the
// block.  BF16 leaves and fused-operand plans use whole tiles (kLeafTile).
constexpr int kLeafStep = 16;

// Number of recursion levels the plan of a product of this shape takes for
// an algorithm with splits (m0, k0, n0) and rank R at the requested depth and
// cutoff: one more while levels remain, every dimension the algorithm splits
// exceeds the cutoff and the leaf tile, and the leaf count stays within the
// limit (sizes rounded up at each split).
int levels_for(int64_t M, int64_t K, int64_t N, int m0, int k0, int n0, int R, int depth, int cutoff);
inline int levels_for(int64_t n, int p, int R, int depth, int cutoff) {
  return levels_for(n, n, n, p, p, p, R, depth, cutoff);
}

// ---------------------------------------------------------------------------
// Launchers (kernels.hip)
// ---------------------------------------------------------------------------

// Kernel launchers.  vec_in / vec_out: rows of A and B / of C start on
// 16-byte boundaries.
constexpr int kPhases = 3;  // pre-addition, grouped GEMM, outer post-addition
// Scaling of the results written into C: C = alpha (sum) + beta C (beta = 0:
// C is not read).  Outputs into the workspace are never scaled.
struct CScale {
  double alpha = 1.0, beta = 0.0;
  bool plain() const { return alpha == 1.0 && beta == 0.0; }
};
// desc: device address of a copy of the plan's descriptor image.
hipError_t launch_combine(const CombineStage& cs, const char* desc, int elem, const void* A, const void* B, void* C,
                          void* ws, bool vec_in, bool vec_out, const CScale& sc, hipStream_t s);
hipError_t launch_gemm_f64(const Plan& pl, const char* desc, const void* A, const void* B, void* C, void* ws,
                           bool vec_in, const CScale& sc, hipStream_t s);
hipError_t launch_gemm_f32(const Plan& pl, const char* desc, const void* A, const void* B, void* C, void* ws,
                           bool vec_in, const CScale& sc, hipStream_t s);
// BF16 leaves: the staging launch (the last pre-addition level fused with the
// conversion to BF16 planes), then the grouped GEMM on the staged planes
// (square plans only; results are written unscaled, see capi).
hipError_t launch_stage_bf16(const Plan& pl, const char* desc, bool x3, const void* A, const void* B, void* C,
                             void* ws, bool vec_in, hipStream_t s);
hipError_t launch_gemm_bf16(const Plan& pl, const char* desc, bool x3, const void* A, const void* B, void* C,
                            void* ws, bool vec_in, hipStream_t s);
// Input counts with a compiled linear-combination kernel.
bool combine_supported(int nin);
// BF16 staging sets exist for this many inputs per set.
bool stage_supported(int nin);

// Persistent batched kernel: runs `ntasks` tasks with `grid` workgroups.
// ctr holds nctr counters, then the ticket, then the abort flag (all must be
// zero at launch); abort is set if a wait exceeds its spin limit.
hipError_t launch_batch(int elem, const BatchTask* tasks, int ntasks, const StageRec* stages, const GemmRec* gemms,
                        const BatchInst* insts, int* ctr, int nctr, int grid, hipStream_t s);
hipError_t launch_fill_zero(int* p, int count, hipStream_t s);
// One phase of a batch (tasks [task0, task0 + count), all of one type) as
// its own launch, one workgroup per task.
hipError_t launch_batch_phase(int elem, bool gemm, const BatchTask* tasks, int task0, int count,
                              const StageRec* stages, const GemmRec* gemms, const BatchInst* insts, hipStream_t s);
// Whether a combination stage can run inside a batch (the persistent form
// supports only the narrow shapes).
bool batch_stage_supported(int nin, int nout_max, bool persistent);

// Request checks shared by the entry points of one product: arguments,
// sizes, dtype code, alignment and overlap of C with A or B (sets the
// thread's error message on failure).
mf_status check_request(const mf_algo* algo, bool need_algo, int depth, int cutoff, const void* A, const void* B,
                        void* C, int64_t n, int dtype);
// The plan of a standalone product (classical when depth is 0); copy_in:
// the caller's A or B base is not 16-byte aligned, and the call allocates
// the workspace itself.
mf_status plan_for(const mf_algo* algo, int depth, int cutoff, int64_t n, int dtype,
                   std::shared_ptr<const Plan>* pl, bool copy_in = false);
// Enqueues the phases of one product on stream s.  desc: device address of
// a copy of the plan's descriptor image; ws: the plan's workspace.  may_time:
// whether the call may record phase-timing events (creating them).
// alpha, beta: C = alpha A B + beta C (beta = 0: C is not read).
mf_status run_at(const Plan& pl, const char* desc, const void* A, const void* B, void* C, void* ws, hipStream_t s,
                 bool may_time = true, double alpha = 1.0, double beta = 0.0);
// Byte ranges [x, x + xb) and [y, y + yb) intersect.
bool overlaps(const void* x, size_t xb, const void* y, size_t yb);
constexpr int kMaxDevices = 64;

// Workspace for one call, from the library's stream-ordered pool on the
// current device.  The pool keeps the memory it has reserved (release
// threshold at its maximum), so repeated calls reuse it instead of mapping
// fresh device memory each time.
hipError_t workspace_alloc(void** p, size_t bytes, hipStream_t s);
hipError_t workspace_free(void* p, hipStream_t s);

// Thread-local error message.
mf_status fail(mf_status st, const std::string& msg);
void clear_error();

}  // namespace mf
