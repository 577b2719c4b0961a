// Grouped leaf GEMM kernel on FP64 or FP32 MFMA for gfx950, with the inner
// post-addition fused into its epilogue.
//
// One launch covers all leaf products of a plan (equation "strassen",
// Section 2 of the paper).  Workgroup (group g, tile position): for each
// product r of group g in order, acc = T_r S_r (MFMA), then
// Out_c (tile) = / += W[c,r] * acc for each output block c it feeds.  With one
// group Out is C itself; otherwise Out is the group's workspace block P_g (the
// inner product result) and linear-combination launches apply the outer
// post-additions.
#include "gemm_tile.h"

namespace mf {

template <class T>
__global__ void __launch_bounds__(NTHREADS, MF_GEMM_WAVES_PER_SIMD) gemm_grouped(GemmArgs<T> g) {
  __shared__ T lds[2][2][BK * LDS_STRIDE];  // [buffer][A|B][k][col]
  int grp, ti, tj;
  work_of(blockIdx.x, g.tiles, g.groups, &grp, &ti, &tj);
  gemm_tile<T>(g, grp, ti, tj, lds);
}

template <class T>
static hipError_t launch_gemm_t(const Plan& pl, const void* A, const void* B, void* C, void* ws, bool vec_in,
                                hipStream_t s) {
  GemmArgs<T> g;
  g.A = static_cast<const T*>(A);
  g.B = static_cast<const T*>(B);
  g.C = static_cast<T*>(C);
  g.ws = static_cast<T*>(ws);
  g.prods = pl.d_prods;
  g.epis = pl.d_epis;
  g.group_beg = pl.d_group_beg;
  g.groups = pl.groups;
  g.m = (int)pl.m;
  g.tiles = (int)(pl.m / BM);
  g.vec_in = vec_in ? 1 : 0;
  const unsigned grid = (unsigned)g.tiles * (unsigned)g.tiles * (unsigned)g.groups;
  hipLaunchKernelGGL(gemm_grouped<T>, dim3(grid), dim3(NTHREADS), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const Plan& pl, const void* A, const void* B, void* C, void* ws, bool vec_in,
                           hipStream_t s) {
  return launch_gemm_t<double>(pl, A, B, C, ws, vec_in, s);
}

hipError_t launch_gemm_f32(const Plan& pl, const void* A, const void* B, void* C, void* ws, bool vec_in,
                           hipStream_t s) {
  return launch_gemm_t<float>(pl, A, B, C, ws, vec_in, s);
}

}  // namespace mf
