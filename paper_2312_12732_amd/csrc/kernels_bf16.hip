// Grouped leaf GEMM with BF16 MFMA leaves for FP32 storage (gfx950).
//
// Same data flow as the FP64/FP32 grouped GEMM (one workgroup owns a tile
// position of every output block of its group; the post-addition is fused
// into the epilogue in FP32).  The leaf product runs on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation:
//   BF16:    operands rounded to BF16 (round to nearest even) when staged
//            into LDS;
//   BF16x3:  split-BF16 compensated product: x = hi + lo with
//            hi = bf16(x), lo = bf16(x - hi); the product is accumulated as
//            hi_a lo_b + lo_a hi_b + hi_a hi_b (the lo_a lo_b term dropped),
//            recovering close to FP32 product accuracy.
// MFMA lane layout (16 x 16 x 32): lane l holds A[l % 16][8 (l / 16) + t] and
// B[8 (l / 16) + t][l % 16] for t = 0..7; element v of the result is
// D[4 (l / 16) + v][l % 16].  Both LDS tiles are therefore stored with k
// contiguous (A row-major, B transposed) so a fragment is one 16-byte read.
#include "gemm_common.h"

namespace mf {

namespace bf {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BM = kLeafTile, BN = kLeafTile, BK = 32;
constexpr int KS = BK + 8;           // bf16 elements per LDS row (16-byte aligned, conflict-free reads)
constexpr int NTHREADS = 256;        // 4 waves, 2 x 2, each 64 x 64
constexpr int WT = 4;                // 16 x 16 tiles per wave side
constexpr int A_LOADS = BM * BK / 4 / NTHREADS;  // float4 loads of A per thread (4)
constexpr int B_COLS_PER_T = 1;                  // B: one column, BK / 2 consecutive k per thread
static_assert(A_LOADS == 4, "A staging assumes 4 float4 loads per thread");

template <bool X3>
struct Lds {
  __bf16 a[2][X3 ? 2 : 1][BM * KS];  // [buffer][hi|lo][row][k]
  __bf16 b[2][X3 ? 2 : 1][BN * KS];  // [buffer][hi|lo][col][k]
};

// Round to BF16 and, for the split form, the BF16 residual.
__device__ __forceinline__ void split(float x, __bf16* hi, __bf16* lo) {
  const __bf16 h = (__bf16)x;
  *hi = h;
  *lo = (__bf16)(x - (float)h);
}

template <bool MASKED>
__device__ __forceinline__ void load_a(const float* __restrict__ pa, int lda, int vr, int vc, int i0, int k0, int t,
                                       f4 (&ra)[A_LOADS]) {
#pragma unroll
  for (int q = 0; q < A_LOADS; ++q) {
    const int idx = t + NTHREADS * q;
    const int row = idx / (BK / 4), kq = (idx % (BK / 4)) * 4;
    const int gi = i0 + row, gk = k0 + kq;
    if (!MASKED) {
      ra[q] = *reinterpret_cast<const f4*>(pa + (size_t)gi * lda + gk);
    } else {
      f4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (gi < vr && gk + u < vc) v[u] = pa[(size_t)gi * lda + gk + u];
      ra[q] = v;
    }
  }
}

// B: thread t stages column j = t % BN, k = (t / BN) * (BK / 2) + 0..15.
template <bool MASKED>
__device__ __forceinline__ void load_b(const float* __restrict__ pb, int ldb, int vr, int vc, int j0, int k0, int t,
                                       float (&rb)[BK / 2]) {
  const int j = j0 + t % BN, kb = k0 + (t / BN) * (BK / 2);
#pragma unroll
  for (int u = 0; u < BK / 2; ++u) {
    if (!MASKED)
      rb[u] = pb[(size_t)(kb + u) * ldb + j];
    else
      rb[u] = (kb + u < vr && j < vc) ? pb[(size_t)(kb + u) * ldb + j] : 0.f;
  }
}

template <bool X3>
__device__ __forceinline__ void store_ab(Lds<X3>& L, int buf, int t, const f4 (&ra)[A_LOADS],
                                         const float (&rb)[BK / 2]) {
#pragma unroll
  for (int q = 0; q < A_LOADS; ++q) {
    const int idx = t + NTHREADS * q;
    const int row = idx / (BK / 4), kq = (idx % (BK / 4)) * 4;
    bf4 h, l;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      __bf16 hh, ll;
      split(ra[q][u], &hh, &ll);
      h[u] = hh;
      l[u] = ll;
    }
    *reinterpret_cast<bf4*>(&L.a[buf][0][row * KS + kq]) = h;
    if (X3) *reinterpret_cast<bf4*>(&L.a[buf][X3 ? 1 : 0][row * KS + kq]) = l;
  }
  const int j = t % BN, kb = (t / BN) * (BK / 2);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    bf8 h, l;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      __bf16 hh, ll;
      split(rb[8 * half + u], &hh, &ll);
      h[u] = hh;
      l[u] = ll;
    }
    *reinterpret_cast<bf8*>(&L.b[buf][0][j * KS + kb + 8 * half]) = h;
    if (X3) *reinterpret_cast<bf8*>(&L.b[buf][X3 ? 1 : 0][j * KS + kb + 8 * half]) = l;
  }
}

template <bool X3, bool MASKED>
__device__ __forceinline__ void k_loop(Lds<X3>& L, const float* __restrict__ pa, int lda, int a_vr, int a_vc,
                                       const float* __restrict__ pb, int ldb, int b_vr, int b_vc, int i0, int j0,
                                       int KT, int t, int wm, int wn, int lr, int lk, f4 (&acc)[WT][WT]) {
  f4 ra[A_LOADS];
  float rb[BK / 2];
  load_a<MASKED>(pa, lda, a_vr, a_vc, i0, 0, t, ra);
  load_b<MASKED>(pb, ldb, b_vr, b_vc, j0, 0, t, rb);
  store_ab<X3>(L, 0, t, ra, rb);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < KT;
    if (more) {
      load_a<MASKED>(pa, lda, a_vr, a_vc, i0, (kt + 1) * BK, t, ra);
      load_b<MASKED>(pb, ldb, b_vr, b_vc, j0, (kt + 1) * BK, t, rb);
    }
    bf8 ah[WT], bh[WT];
#pragma unroll
    for (int mi = 0; mi < WT; ++mi)
      ah[mi] = *reinterpret_cast<const bf8*>(&L.a[cur][0][(wm + 16 * mi + lr) * KS + 8 * lk]);
#pragma unroll
    for (int ni = 0; ni < WT; ++ni)
      bh[ni] = *reinterpret_cast<const bf8*>(&L.b[cur][0][(wn + 16 * ni + lr) * KS + 8 * lk]);
    if (X3) {
      bf8 al[WT], bl[WT];
#pragma unroll
      for (int mi = 0; mi < WT; ++mi)
        al[mi] = *reinterpret_cast<const bf8*>(&L.a[cur][X3 ? 1 : 0][(wm + 16 * mi + lr) * KS + 8 * lk]);
#pragma unroll
      for (int ni = 0; ni < WT; ++ni)
        bl[ni] = *reinterpret_cast<const bf8*>(&L.b[cur][X3 ? 1 : 0][(wn + 16 * ni + lr) * KS + 8 * lk]);
#pragma unroll
      for (int mi = 0; mi < WT; ++mi)
#pragma unroll
        for (int ni = 0; ni < WT; ++ni) {
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bl[ni], acc[mi][ni], 0, 0, 0);
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mi], bh[ni], acc[mi][ni], 0, 0, 0);
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bh[ni], acc[mi][ni], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int mi = 0; mi < WT; ++mi)
#pragma unroll
        for (int ni = 0; ni < WT; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mi], bh[ni], acc[mi][ni], 0, 0, 0);
    }
    if (more) store_ab<X3>(L, cur ^ 1, t, ra, rb);
    __syncthreads();
  }
}

template <bool X3>
__global__ void __launch_bounds__(NTHREADS, 2) gemm_bf16_grouped(GemmArgs<float> g) {
  __shared__ Lds<X3> L;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int lr = lane & 15, lk = lane >> 4;
  int grp, ti, tj;
  work_of(blockIdx.x, g.tiles_m, g.tiles_n, g.groups, &grp, &ti, &tj);
  const int i0 = ti * BM, j0 = tj * BN;
  const int KT = g.m / BK;
  const int r_beg = g.group_beg[grp], r_end = g.group_beg[grp + 1];

  for (int r = r_beg; r < r_end; ++r) {
    const ProdDesc pd = g.prods[r];
    const float* pa = src_ptr(g, pd.a_src) + pd.a_off;
    const float* pb = src_ptr(g, pd.b_src) + pd.b_off;
    const bool vec_a = pd.a_src == SRC_WS || g.vec_in;
    f4 acc[WT][WT];
#pragma unroll
    for (int mi = 0; mi < WT; ++mi)
#pragma unroll
      for (int ni = 0; ni < WT; ++ni) acc[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
    const bool interior = vec_a && i0 + BM <= pd.a_vr && pd.a_vc >= g.m && pd.b_vr >= g.m && j0 + BN <= pd.b_vc;
    if (interior)
      k_loop<X3, false>(L, pa, pd.lda, pd.a_vr, pd.a_vc, pb, pd.ldb, pd.b_vr, pd.b_vc, i0, j0, KT, t, wm, wn, lr, lk,
                        acc);
    else
      k_loop<X3, true>(L, pa, pd.lda, pd.a_vr, pd.a_vc, pb, pd.ldb, pd.b_vr, pd.b_vc, i0, j0, KT, t, wm, wn, lr, lk,
                       acc);

    for (int e = pd.epi_beg; e < pd.epi_end; ++e) {
      const EpiDesc ed = g.epis[e];
      float* pc = dst_ptr(g, ed.c_src) + ed.c_off;
      const bool full = (i0 + BM <= ed.c_vr) && (j0 + BN <= ed.c_vc);
      const float coef = (float)ed.coef;
#pragma unroll
      for (int mi = 0; mi < WT; ++mi)
#pragma unroll
        for (int ni = 0; ni < WT; ++ni)
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

hipError_t launch_gemm_bf16(const Plan& pl, bool x3, const void* A, const void* B, void* C, void* ws, bool vec_in,
                            hipStream_t s) {
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
  g.tiles_m = (int)(pl.m / bf::BM);
  g.tiles_n = (int)(pl.m / bf::BN);
  g.vec_in = vec_in ? 1 : 0;
  const unsigned grid = (unsigned)g.tiles_m * (unsigned)g.tiles_n * (unsigned)g.groups;
  if (x3)
    hipLaunchKernelGGL(bf::gemm_bf16_grouped<true>, dim3(grid), dim3(bf::NTHREADS), 0, s, g);
  else
    hipLaunchKernelGGL(bf::gemm_bf16_grouped<false>, dim3(grid), dim3(bf::NTHREADS), 0, s, g);
  return hipGetLastError();
}

}  // namespace mf
