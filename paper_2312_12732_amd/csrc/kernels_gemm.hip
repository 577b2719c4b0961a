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

// Tile choice.  Tile128: 128 x 128 tiles, two workgroups of eight 64 x 32
// waves per CU.  Tile256: 256 x 128 tiles, one workgroup of eight 128 x 32
// waves per CU (a quarter less operand traffic per flop).  Measured on
// MI355X at n = 8192 (FP64 classical / Winograd depth 1 / depth 2), Tile256
// is slower (16.9 / 16.1 / 18.1 ms against 16.0 / 15.1 / 14.9 ms): with two
// waves per SIMD the barrier of each K step stalls the MFMA pipes.  It is
// kept as an option: MF_GEMM_BIG_TILES = 1 takes it where its work items
// fill whole rounds of the CUs, 2 wherever the leaf size allows, 0 (default)
// never.
#ifndef MF_GEMM_BIG_TILES
#define MF_GEMM_BIG_TILES 0
#endif

namespace mf {

template <class T, class Cfg>
__global__ void __launch_bounds__(Cfg::NTHREADS, Cfg::WAVES_PER_SIMD) gemm_grouped(GemmArgs<T> g) {
  __shared__ T lds[Cfg::LDS_ELEMS];  // [A buffer 0 | A buffer 1 | B buffer 0 | B buffer 1], k-major
  int grp, ti, tj;
  work_of(blockIdx.x, g.tiles_m, g.tiles_n, g.groups, &grp, &ti, &tj);
  gemm_tile<T, Cfg>(g, grp, ti, tj, lds);
}

template <class T, class Cfg>
static hipError_t launch_cfg(GemmArgs<T> g, int64_t m, hipStream_t s) {
  g.tiles_m = (int)(m / Cfg::BM);
  g.tiles_n = (int)(m / Cfg::BN);
  const unsigned grid = (unsigned)g.tiles_m * (unsigned)g.tiles_n * (unsigned)g.groups;
  hipLaunchKernelGGL((gemm_grouped<T, Cfg>), dim3(grid), dim3(Cfg::NTHREADS), 0, s, g);
  return hipGetLastError();
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
  g.vec_in = vec_in ? 1 : 0;
  int cus = 256;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t big_items = (pl.m / Tile256::BM) * (pl.m / Tile256::BN) * (int64_t)pl.groups;
  const bool big_ok = pl.m % Tile256::BM == 0 && big_items >= cus;
  const bool big_fills = big_items % cus == 0 || big_items >= 8 * (int64_t)cus;
  if (big_ok && (MF_GEMM_BIG_TILES == 2 || (MF_GEMM_BIG_TILES == 1 && big_fills)))
    return launch_cfg<T, Tile256>(g, pl.m, s);
  return launch_cfg<T, Tile128>(g, pl.m, s);
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
