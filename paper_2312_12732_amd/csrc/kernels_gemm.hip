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

// Tile: 128 x 128 output tiles, two workgroups of eight 64 x 32 waves per CU
// (Tile128).

namespace mf {

template <class T, class Cfg, bool FULL>
__global__ void __launch_bounds__(Cfg::NTHREADS, Cfg::WAVES_PER_SIMD) gemm_grouped(GemmArgs<T> g) {
  __shared__ T lds[Geom<T, Cfg>::ELEMS];  // [A buffer 0 | A buffer 1 | B buffer 0 | B buffer 1]
  int grp, ti, tj;
  work_of(blockIdx.x, g.tiles_m, g.tiles_n, g.groups, &grp, &ti, &tj);
  gemm_tile<T, Cfg, FULL>(g, grp, ti, tj, lds);
}

// FP32 plans without edge tiles: the same tile on a budget of six waves per
// SIMD (80 VGPRs, no spill; 33 KiB of LDS), so three workgroups share a CU.
// At n = 16384 its leaf GEMMs ran 1-2% faster than at four waves per SIMD.
// The general FP32 kernel needs 120 VGPRs and keeps Tile128.
using Tile128F32 = TileCfg<128, 128, 2, 4, 6>;

// Fused-operand plans: the same tile on a register budget of two waves per
// SIMD (one workgroup per CU), so that the loads of every operand term stay
// in flight during the MFMAs of the previous K step.
using Tile128F = TileCfg<128, 128, 2, 4, 2>;

template <class T, class Cfg, int NT, bool FULL>
__global__ void __launch_bounds__(Cfg::NTHREADS, Cfg::WAVES_PER_SIMD) gemm_fused(GemmArgs<T> g) {
  __shared__ T lds[Geom<T, Cfg>::ELEMS];
  int grp, ti, tj;
  work_of(blockIdx.x, g.tiles_m, g.tiles_n, g.groups, &grp, &ti, &tj);
  gemm_tile_fused<T, Cfg, NT, FULL>(g, grp, ti, tj, lds);
}

// Whether every term of a fused-operand plan covers its whole block with
// 16-byte aligned rows and every epilogue output its whole block.
static bool fused_full(const Plan& pl, size_t elem, bool vec_in) {
  if (!vec_in || (pl.shape.lda * (int64_t)elem) % 16 || (pl.shape.ldb * (int64_t)elem) % 16) return false;
  for (const ProdDesc& pd : pl.prods) {
    for (int u = 0; u < pd.a_terms; ++u) {
      const TermDesc& td = pl.terms[(size_t)pd.a_term0 + u];
      if (td.vr < pl.m || td.vc < pl.leaf_k || (td.off * (int64_t)elem) % 16) return false;
    }
    for (int u = 0; u < pd.b_terms; ++u) {
      const TermDesc& td = pl.terms[(size_t)pd.b_term0 + u];
      if (td.vr < pl.leaf_k || td.vc < pl.leaf_n || (td.off * (int64_t)elem) % 16) return false;
    }
  }
  for (const EpiDesc& ed : pl.epis)
    if (ed.c_vr < pl.m || ed.c_vc < pl.leaf_n) return false;
  return true;
}

template <class T, int NT>
static hipError_t launch_fused(GemmArgs<T> g, bool full, hipStream_t s) {
  using Cfg = Tile128F;
  g.tiles_m = g.m / Cfg::BM;
  g.tiles_n = g.n / Cfg::BN;
  const unsigned grid = (unsigned)g.tiles_m * (unsigned)g.tiles_n * (unsigned)g.groups;
  if (full)
    hipLaunchKernelGGL((gemm_fused<T, Cfg, NT, true>), dim3(grid), dim3(Cfg::NTHREADS), 0, s, g);
  else
    hipLaunchKernelGGL((gemm_fused<T, Cfg, NT, false>), dim3(grid), dim3(Cfg::NTHREADS), 0, s, g);
  return hipGetLastError();
}

// Whether the leaves are whole tiles and every operand view and epilogue
// output of the plan covers its whole m x m block with 16-byte aligned rows
// (then the kernel without the masked paths runs; true for sizes the splits
// divide into whole tiles).
static bool plan_full(const Plan& pl, size_t elem, bool vec_in) {
  const int64_t m = pl.m, n = pl.leaf_n, k = pl.leaf_k;
  if (m % kLeafTile || n % kLeafTile) return false;  // edge tiles: the general kernel
  for (const ProdDesc& pd : pl.prods) {
    const bool va = pd.a_src == SRC_WS || vec_in, vb = pd.b_src == SRC_WS || vec_in;
    if (!va || !vb || pd.a_vr < m || pd.a_vc < k || pd.b_vr < k || pd.b_vc < n) return false;
    if ((pd.lda * elem) % 16 || (pd.ldb * elem) % 16 || (pd.a_off * elem) % 16 || (pd.b_off * elem) % 16) return false;
  }
  for (const EpiDesc& ed : pl.epis)
    if (ed.c_vr < m || ed.c_vc < n) return false;
  return true;
}

template <class T, class Cfg, bool FULL>
static hipError_t launch_tiles(GemmArgs<T> g, hipStream_t s) {
  g.tiles_m = (g.m + Cfg::BM - 1) / Cfg::BM;
  g.tiles_n = (g.n + Cfg::BN - 1) / Cfg::BN;
  const unsigned grid = (unsigned)g.tiles_m * (unsigned)g.tiles_n * (unsigned)g.groups;
  hipLaunchKernelGGL((gemm_grouped<T, Cfg, FULL>), dim3(grid), dim3(Cfg::NTHREADS), 0, s, g);
  return hipGetLastError();
}

template <class T>
static hipError_t launch_gemm_t(const Plan& pl, const char* desc, const void* A, const void* B, void* C, void* ws,
                                bool vec_in, const CScale& sc, hipStream_t s) {
  GemmArgs<T> g;
  g.A = static_cast<const T*>(A);
  g.B = static_cast<const T*>(B);
  g.C = static_cast<T*>(C);
  g.ws = static_cast<T*>(ws);
  g.prods = img_at<ProdDesc>(desc, pl.img_prods);
  g.epis = img_at<EpiDesc>(desc, pl.img_epis);
  g.group_beg = img_at<int32_t>(desc, pl.img_group_beg);
  g.terms = img_at<TermDesc>(desc, pl.img_terms);
  g.groups = pl.groups;
  g.m = (int)pl.m;
  g.n = (int)pl.leaf_n;
  g.k = (int)pl.leaf_k;
  g.vec_in = vec_in ? 1 : 0;
  g.scale_c = sc.plain() ? 0 : 1;
  g.alpha = (T)sc.alpha;
  g.beta = (T)sc.beta;
  if (pl.fused_terms > 0) {
    const bool full = fused_full(pl, sizeof(T), vec_in);
    if (pl.fused_terms <= 4) return launch_fused<T, 4>(g, full, s);
    if (pl.fused_terms <= 16) return launch_fused<T, 16>(g, full, s);
    return hipErrorInvalidValue;
  }
  const bool full = plan_full(pl, sizeof(T), vec_in);
  if constexpr (sizeof(T) == 4)
    return full ? launch_tiles<T, Tile128F32, true>(g, s) : launch_tiles<T, Tile128, false>(g, s);
  else
    return full ? launch_tiles<T, Tile128, true>(g, s) : launch_tiles<T, Tile128, false>(g, s);
}

hipError_t launch_gemm_f64(const Plan& pl, const char* desc, const void* A, const void* B, void* C, void* ws,
                           bool vec_in, const CScale& sc, hipStream_t s) {
  return launch_gemm_t<double>(pl, desc, A, B, C, ws, vec_in, sc, s);
}

hipError_t launch_gemm_f32(const Plan& pl, const char* desc, const void* A, const void* B, void* C, void* ws,
                           bool vec_in, const CScale& sc, hipStream_t s) {
  return launch_gemm_t<float>(pl, desc, A, B, C, ws, vec_in, sc, s);
}

}  // namespace mf
