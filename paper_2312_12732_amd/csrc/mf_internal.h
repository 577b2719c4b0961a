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

// A canonical <p,p,p;R> algorithm: U, V, W are p^2 x R, row-major, with row c
// of W belonging to C_c (blocks numbered row-major).
struct Algo {
  int p = 0;
  int R = 0;
  std::vector<double> U, V, W;
  double u(int k, int r) const { return U[(size_t)k * R + r]; }
  double v(int k, int r) const { return V[(size_t)k * R + r]; }
  double w(int k, int r) const { return W[(size_t)k * R + r]; }
};

// Number of failing Brent equations (exact for integer coefficients).
int64_t brent_violations(const Algo& a);
Algo compose(const Algo& outer, const Algo& inner);
Algo power(const Algo& a, int d);
// Re-base by unimodular X, Y, Z (p x p, row-major); false if not unimodular.
bool rebase(const Algo& a, const int64_t* X, const int64_t* Y, const int64_t* Z, Algo* out);
bool builtin(const std::string& name, Algo* out);

}  // namespace mf

struct mf_algo {
  mf::Algo a;
  uint64_t id = 0;  // unique per handle; keys the plan cache
};

namespace mf {

// ---------------------------------------------------------------------------
// Device descriptors
// ---------------------------------------------------------------------------

// Source of an operand view: the caller's A, B or C, or the workspace.
enum Src : int32_t { SRC_A = 0, SRC_B = 1, SRC_WS = 2 };

// One leaf product P_r = scale * X_r Y_r of size m x m x m, where X_r and Y_r
// are views (src, offset, ld) of the inputs or of workspace blocks.  Entries
// of a view at row >= vr or column >= vc are zero (virtual padding).
struct ProdDesc {
  int64_t a_off, b_off;   // element offsets of the view origins
  int32_t a_src, b_src;   // Src
  int32_t lda, ldb;       // leading dimensions (elements)
  int32_t a_vr, a_vc;     // valid rows / columns of the A view
  int32_t b_vr, b_vc;     // valid rows / columns of the B view
  int32_t epi_beg, epi_end;  // range in the epilogue list
};

// One post-addition term: C block c (view of C) gets coef * P_r.  `first`
// is set for the product that writes the block first (in product order).
struct EpiDesc {
  int64_t c_off;
  int32_t c_vr, c_vc;
  int32_t first;
  int32_t pad_;
  double coef;
};

// One materialised pre-addition output: out = sum_k coef[k] * in_k over the
// p^2 input block views; written densely (ld = m) at ws offset out_off.
struct PreOut {
  int64_t out_off;
  int32_t coef_off;  // offset into the coefficient array (P2 entries)
  int32_t nnz;
};

// Input block view k of the pre-addition (same for every output).
struct PreIn {
  int64_t off;
  int32_t vr, vc;
};

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------

struct Plan {
  int64_t n = 0;      // true size
  int64_t npad = 0;   // padded size = P * m
  int64_t m = 0;      // leaf size (multiple of the GEMM tile)
  int levels = 0;     // recursion levels taken
  int P = 1;          // split factor of the fused level (p^levels)
  int R = 1;          // number of leaf products
  int dtype = MF_F64;
  size_t elem = 8;
  size_t ws_bytes = 0;
  int n_pre_a = 0, n_pre_b = 0;  // materialised T / S outputs
  // host copies
  std::vector<ProdDesc> prods;
  std::vector<EpiDesc> epis;
  std::vector<PreOut> pre_out;   // A outputs first, then B outputs
  std::vector<PreIn> pre_in;     // A inputs (P2), then B inputs (P2)
  std::vector<double> pre_coef;
  // device copy (one allocation, owned by the plan), made on first use
  mutable std::once_flag uploaded;
  mutable mf_status upload_status = MF_OK;
  mutable void* dev = nullptr;
  mutable ProdDesc* d_prods = nullptr;
  mutable EpiDesc* d_epis = nullptr;
  mutable PreOut* d_pre_out = nullptr;
  mutable PreIn* d_pre_in = nullptr;
  mutable double* d_pre_coef = nullptr;
  ~Plan();
};

// Builds (or fetches from the cache) the plan for a request.  Returns an
// mf_status and sets the thread's error message on failure.
mf_status get_plan(const mf_algo* algo, int depth, int cutoff, int64_t n, int dtype,
                   std::shared_ptr<const Plan>* out);

// Copies the plan's descriptors to the device once (host-only queries such as
// the workspace size never touch the device).
mf_status ensure_device(const Plan& pl);

// Releases the cached plans of an algorithm handle that is being freed.
void drop_plans(uint64_t algo_id);

// Leaf tile granularity: every leaf size is a multiple of this.
constexpr int kLeafTile = 128;

// ---------------------------------------------------------------------------
// Launchers (kernels.hip)
// ---------------------------------------------------------------------------

// vec_in: rows of A and B are 16-byte aligned (vector loads allowed).
hipError_t launch_preadd_f64(const Plan& pl, const void* A, const void* B, void* ws, bool vec_in, hipStream_t s);
hipError_t launch_gemm_f64(const Plan& pl, const void* A, const void* B, void* C, void* ws, bool vec_in,
                           hipStream_t s);

// Thread-local error message.
mf_status fail(mf_status st, const std::string& msg);
void clear_error();

}  // namespace mf
