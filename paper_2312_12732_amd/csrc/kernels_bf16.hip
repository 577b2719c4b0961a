// Grouped leaf GEMM with BF16 MFMA leaves for FP32 storage (gfx950).
//
// Same data flow as the FP64/FP32 grouped GEMM (one workgroup owns a tile
// position of every output block of its group; the post-addition is fused
// into the epilogue in FP32).  The leaf product runs on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation:
//   BF16:    operands rounded to BF16 (round to nearest even);
//   BF16x3:  split-BF16 compensated product: x = hi + lo with
//            hi = bf16(x), lo = bf16(x - hi); the product is accumulated as
//            hi_a lo_b + lo_a hi_b + hi_a hi_b (the lo_a lo_b term dropped),
//            recovering close to FP32 product accuracy.
//
// Two launches.  The staging kernel converts every leaf operand once: the A
// operand of each product to row-major BF16 planes, the B operand transposed
// (so that both have k contiguous), zero beyond the view's valid extent, into
// the plan's BF16 region of the workspace.  The GEMM kernel then streams
// 16-byte BF16 rows straight into LDS: no conversion, no masking, and half
// the operand bytes of FP32 per plane.
//
// MFMA lane layout (16 x 16 x 32): lane l holds A[l % 16][8 (l / 16) + t] and
// B[8 (l / 16) + t][l % 16] for t = 0..7; element v of the result is
// D[4 (l / 16) + v][l % 16].  Both LDS tiles are stored with k contiguous
// (A row-major, B transposed) so a fragment is one 16-byte read.
#include <type_traits>

#include "gemm_tile.h"

namespace mf {

namespace bf {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BK = 32;
constexpr int KS = BK + 8;     // bf16 elements per LDS row: 80 bytes, 16-byte aligned, conflict-free reads
constexpr int NTHREADS = 256;  // 4 waves, 2 x 2

// ---------------------------------------------------------------------------
// Staging: FP32 leaf operand views -> BF16 planes
// ---------------------------------------------------------------------------

constexpr int ST = 64;  // staging tile (ST x ST elements per workgroup of 256 threads)

// Block (x, y, z): columns x*64.., rows y*64.. of operand z (z < nprod: A of
// product z; otherwise B of product z - nprod, written transposed).
template <bool X3>
__global__ void __launch_bounds__(256) stage_bf16(GemmArgs<float> g, __bf16* dst_base, int nprod, int64_t plane) {
  __shared__ float tile[ST][ST + 1];
  const int z = blockIdx.z;
  const bool bside = z >= nprod;
  const ProdDesc pd = load_uniform(g.prods + (bside ? z - nprod : z));
  const float* src = bside ? src_ptr(g, pd.b_src) + pd.b_off : src_ptr(g, pd.a_src) + pd.a_off;
  const int ld = bside ? pd.ldb : pd.lda;
  const int vr = bside ? pd.b_vr : pd.a_vr, vc = bside ? pd.b_vc : pd.a_vc;
  const int r0 = blockIdx.y * ST, c0 = blockIdx.x * ST;
  const int t = threadIdx.x;
  const int m = g.m;
  __bf16* hi = dst_base + (size_t)z * (X3 ? 2 : 1) * plane;
  __bf16* lo = hi + plane;
  // thread t reads 4 consecutive columns of rows t / 16 + 16 q
  const int cc = (t % 16) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rr = t / 16 + 16 * q;
    const int i = r0 + rr;
    f4 v;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = c0 + cc + u;
      v[u] = (i < vr && j < vc) ? src[(size_t)i * ld + j] : 0.f;
    }
    if (!bside) {
      bf4 h, l;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        h[u] = (__bf16)v[u];
        l[u] = (__bf16)(v[u] - (float)h[u]);
      }
      *reinterpret_cast<bf4*>(hi + (size_t)i * m + c0 + cc) = h;
      if (X3) *reinterpret_cast<bf4*>(lo + (size_t)i * m + c0 + cc) = l;
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) tile[rr][cc + u] = v[u];
    }
  }
  if (!bside) return;  // uniform per workgroup
  __syncthreads();
  // transposed: output row c0 + c holds column c of the tile; thread t writes
  // 4 consecutive k (tile rows) of output rows t / 16 + 16 q
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = t / 16 + 16 * q;
    const int kk = (t % 16) * 4;
    bf4 h, l;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float x = tile[kk + u][c];
      h[u] = (__bf16)x;
      l[u] = (__bf16)(x - (float)h[u]);
    }
    *reinterpret_cast<bf4*>(hi + (size_t)(c0 + c) * m + r0 + kk) = h;
    if (X3) *reinterpret_cast<bf4*>(lo + (size_t)(c0 + c) * m + r0 + kk) = l;
  }
}

// ---------------------------------------------------------------------------
// GEMM on staged BF16 operands
// ---------------------------------------------------------------------------

// Tile geometry: a BM_ x BN_ output tile per workgroup of 4 waves (2 x 2),
// each wave (BM_ / 2) x (BN_ / 2) = WTM x WTN MFMA tiles of 16 x 16.
//   Cfg128: 128 x 128, waves of 64 x 64 (BF16 and split-BF16x3);
//   Cfg256: 256 x 128, waves of 128 x 64: per MFMA a quarter fewer LDS
//           fragment reads and operand loads (BF16 only: the x3 form would
//           need more registers than two waves per SIMD have).
template <int BM_, int BN_>
struct BfCfg {
  static constexpr int BM = BM_, BN = BN_;
  static constexpr int WTM = BM / 32, WTN = BN / 32;  // 16 x 16 tiles per wave
  static constexpr int A_LOADS = BM * BK / 8 / NTHREADS, B_LOADS = BN * BK / 8 / NTHREADS;
  static_assert(A_LOADS * 8 * NTHREADS == BM * BK && B_LOADS * 8 * NTHREADS == BN * BK, "whole 16-byte pieces");
};
using Cfg128 = BfCfg<128, 128>;
using Cfg256 = BfCfg<256, 128>;

template <class C, bool X3>
struct Lds {
  __bf16 a[2][X3 ? 2 : 1][C::BM * KS];  // [buffer][hi|lo][row][k]
  __bf16 b[2][X3 ? 2 : 1][C::BN * KS];  // [buffer][hi|lo][col][k]
};

constexpr int PLANES_MAX = 2;

// 16-byte piece idx of a rows x 32 tile -> (row, first k).
__device__ __forceinline__ void piece(int idx, int& row, int& kc) {
  row = idx / (BK / 8);
  kc = (idx % (BK / 8)) * 8;
}

template <class C, bool X3>
__device__ __forceinline__ void load_stage(const __bf16* a, const __bf16* b, int64_t plane, int m, int i0, int j0,
                                           int k0, int t, bf8 (&ra)[PLANES_MAX][C::A_LOADS],
                                           bf8 (&rb)[PLANES_MAX][C::B_LOADS]) {
  constexpr int P = X3 ? 2 : 1;
#pragma unroll
  for (int pl = 0; pl < P; ++pl) {
    const __amdgpu_buffer_rsrc_t sa = raw_rsrc(a + pl * plane + (size_t)i0 * m + k0);
    const __amdgpu_buffer_rsrc_t sb = raw_rsrc(b + pl * plane + (size_t)j0 * m + k0);
#pragma unroll
    for (int q = 0; q < C::A_LOADS; ++q) {
      int row, kc;
      piece(t + NTHREADS * q, row, kc);
      const int off = (row * m + kc) * 2;  // row < 256, m <= 2^19: below 2^31 bytes
      ra[pl][q] = __builtin_bit_cast(bf8, __builtin_amdgcn_raw_buffer_load_b128(sa, off, 0, 0));
    }
#pragma unroll
    for (int q = 0; q < C::B_LOADS; ++q) {
      int row, kc;
      piece(t + NTHREADS * q, row, kc);
      const int off = (row * m + kc) * 2;
      rb[pl][q] = __builtin_bit_cast(bf8, __builtin_amdgcn_raw_buffer_load_b128(sb, off, 0, 0));
    }
  }
}

template <class C, bool X3>
__device__ __forceinline__ void store_stage(Lds<C, X3>& L, int buf, int t, const bf8 (&ra)[PLANES_MAX][C::A_LOADS],
                                            const bf8 (&rb)[PLANES_MAX][C::B_LOADS]) {
  constexpr int P = X3 ? 2 : 1;
#pragma unroll
  for (int pl = 0; pl < P; ++pl) {
#pragma unroll
    for (int q = 0; q < C::A_LOADS; ++q) {
      int row, kc;
      piece(t + NTHREADS * q, row, kc);
      *reinterpret_cast<bf8*>(&L.a[buf][pl][row * KS + kc]) = ra[pl][q];
    }
#pragma unroll
    for (int q = 0; q < C::B_LOADS; ++q) {
      int row, kc;
      piece(t + NTHREADS * q, row, kc);
      *reinterpret_cast<bf8*>(&L.b[buf][pl][row * KS + kc]) = rb[pl][q];
    }
  }
}

template <class C, bool X3>
__device__ __forceinline__ void k_loop(Lds<C, X3>& L, const __bf16* a, const __bf16* b, int64_t plane, int m, int i0,
                                       int j0, int t, int wm, int wn, int lr, int lk,
                                       f4 (&acc)[C::WTM][C::WTN]) {
  constexpr int WTM = C::WTM, WTN = C::WTN;
  bf8 ra[PLANES_MAX][C::A_LOADS], rb[PLANES_MAX][C::B_LOADS];
  const int KT = m / BK;
  load_stage<C, X3>(a, b, plane, m, i0, j0, 0, t, ra, rb);
  store_stage<C, X3>(L, 0, t, ra, rb);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < KT;
    if (more) load_stage<C, X3>(a, b, plane, m, i0, j0, (kt + 1) * BK, t, ra, rb);
    bf8 ah[WTM], bh[WTN];
#pragma unroll
    for (int mi = 0; mi < WTM; ++mi)
      ah[mi] = *reinterpret_cast<const bf8*>(&L.a[cur][0][(wm + 16 * mi + lr) * KS + 8 * lk]);
#pragma unroll
    for (int ni = 0; ni < WTN; ++ni)
      bh[ni] = *reinterpret_cast<const bf8*>(&L.b[cur][0][(wn + 16 * ni + lr) * KS + 8 * lk]);
    if constexpr (X3) {
      bf8 al[WTM], bl[WTN];
#pragma unroll
      for (int mi = 0; mi < WTM; ++mi)
        al[mi] = *reinterpret_cast<const bf8*>(&L.a[cur][1][(wm + 16 * mi + lr) * KS + 8 * lk]);
#pragma unroll
      for (int ni = 0; ni < WTN; ++ni)
        bl[ni] = *reinterpret_cast<const bf8*>(&L.b[cur][1][(wn + 16 * ni + lr) * KS + 8 * lk]);
#pragma unroll
      for (int mi = 0; mi < WTM; ++mi)
#pragma unroll
        for (int ni = 0; ni < WTN; ++ni) {
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bl[ni], acc[mi][ni], 0, 0, 0);
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mi], bh[ni], acc[mi][ni], 0, 0, 0);
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bh[ni], acc[mi][ni], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int mi = 0; mi < WTM; ++mi)
#pragma unroll
        for (int ni = 0; ni < WTN; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bh[ni], acc[mi][ni], 0, 0, 0);
    }
    if (more) store_stage<C, X3>(L, cur ^ 1, t, ra, rb);
    __syncthreads();
  }
}

template <class C, bool X3>
__global__ void __launch_bounds__(NTHREADS, 2)
    gemm_bf16_grouped(GemmArgs<float> g, const __bf16* __restrict__ staged, int nprod, int64_t plane) {
  __shared__ Lds<C, X3> L;
  constexpr int WTM = C::WTM, WTN = C::WTN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * (C::BM / 2), wn = (wave & 1) * (C::BN / 2);
  const int lr = lane & 15, lk = lane >> 4;
  int grp, ti, tj;
  work_of(blockIdx.x, g.tiles_m, g.tiles_n, g.groups, &grp, &ti, &tj);
  const int i0 = ti * C::BM, j0 = tj * C::BN;
  const int r_beg = load_uniform(g.group_beg + grp), r_end = load_uniform(g.group_beg + grp + 1);
  constexpr int P = X3 ? 2 : 1;

  for (int r = r_beg; r < r_end; ++r) {
    const ProdDesc pd = load_uniform(g.prods + r);
    const __bf16* a = staged + (size_t)r * P * plane;
    const __bf16* b = staged + (size_t)(nprod + r) * P * plane;
    f4 acc[WTM][WTN];
#pragma unroll
    for (int mi = 0; mi < WTM; ++mi)
#pragma unroll
      for (int ni = 0; ni < WTN; ++ni) acc[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
    k_loop<C, X3>(L, a, b, plane, g.m, i0, j0, t, wm, wn, lr, lk, acc);

    for (int e = pd.epi_beg; e < pd.epi_end; ++e) {
      const EpiDesc ed = load_uniform(g.epis + e);
      float* pc = dst_ptr(g, ed.c_src) + ed.c_off;
      const bool full = (i0 + C::BM <= ed.c_vr) && (j0 + C::BN <= ed.c_vc);
      const float coef = (float)ed.coef;
#pragma unroll
      for (int mi = 0; mi < WTM; ++mi)
#pragma unroll
        for (int ni = 0; ni < WTN; ++ni)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = i0 + wm + 16 * mi + 4 * lk + v;
            const int col = j0 + wn + 16 * ni + lr;
            if (full || (row < ed.c_vr && col < ed.c_vc))
              epi_apply<float>(pc + (size_t)row * ed.ldc + col, ed.first, coef, acc[mi][ni][v]);
          }
    }
  }
}

}  // namespace bf

#ifndef MF_BF16_BIG_TILES
#define MF_BF16_BIG_TILES 1
#endif

hipError_t launch_gemm_bf16(const Plan& pl, bool x3, const void* A, const void* B, void* C, void* ws, bool vec_in,
                            hipStream_t s) {
  (void)vec_in;  // the staged operands are always aligned and whole
  GemmArgs<float> g;
  g.A = static_cast<const float*>(A);
  g.B = static_cast<const float*>(B);
  g.C = static_cast<float*>(C);
  g.ws = static_cast<float*>(ws);
  g.prods = pl.d_prods;
  g.epis = pl.d_epis;
  g.group_beg = pl.d_group_beg;
  g.groups = pl.groups;
  g.m = (int)pl.m;
  g.vec_in = 0;
  if (pl.bf_base < 0 || !ws) return hipErrorInvalidValue;
  __bf16* staged = reinterpret_cast<__bf16*>(static_cast<char*>(ws) + pl.bf_base);
  const int nprod = (int)pl.prods.size();
  const int64_t plane = pl.m * pl.m;
  const dim3 sgrid((unsigned)(pl.m / bf::ST), (unsigned)(pl.m / bf::ST), (unsigned)(2 * nprod));
  if (x3)
    hipLaunchKernelGGL(bf::stage_bf16<true>, sgrid, dim3(256), 0, s, g, staged, nprod, plane);
  else
    hipLaunchKernelGGL(bf::stage_bf16<false>, sgrid, dim3(256), 0, s, g, staged, nprod, plane);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const __bf16* st = staged;
  auto launch = [&](auto cfg, auto x3c) {
    typedef decltype(cfg) Cf;
    constexpr bool X = decltype(x3c)::value;
    g.tiles_m = (int)(pl.m / Cf::BM);
    g.tiles_n = (int)(pl.m / Cf::BN);
    const unsigned grid = (unsigned)g.tiles_m * (unsigned)g.tiles_n * (unsigned)g.groups;
    hipLaunchKernelGGL((bf::gemm_bf16_grouped<Cf, X>), dim3(grid), dim3(bf::NTHREADS), 0, s, g, st, nprod, plane);
  };
  if (x3)
    launch(bf::Cfg128{}, std::true_type{});
  else if (MF_BF16_BIG_TILES && pl.m % bf::Cfg256::BM == 0)
    launch(bf::Cfg256{}, std::false_type{});
  else
    launch(bf::Cfg128{}, std::false_type{});
  return hipGetLastError();
}

}  // namespace mf
