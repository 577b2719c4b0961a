// FP64 kernels for gfx950: the fused pre-addition (GEMA over operand
// blocks) and the grouped leaf GEMM on FP64 MFMA with the post-addition fused
// into its epilogue.
//
// Data flow of one fused level (equation "strassen", Section 2 of the paper):
//   preadd:  T_r = sum_k U[k,r] A_k, S_r = sum_l V[l,r] B_l for every product
//            whose combination has more than one term (one-term columns are
//            read in place as views of A or B);
//   gemm:    for each output tile position, for r = 0..R-1 in order:
//            acc = T_r S_r (MFMA), then C_c (tile) = / += W[c,r] * acc for
//            each c with W[c,r] != 0.  One workgroup owns a tile position of
//            every C block, so the read-modify-write is race-free and its
//            summation order is fixed (bitwise reproducible).
#include "mf_internal.h"

namespace mf {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// GEMM tile geometry: 128 x 128 output tile per workgroup of 256 threads
// (4 waves of 64, 2 x 2 waves of 64 x 64), K step 16 (4 MFMA k-steps of 4),
// LDS double-buffered.  The MFMA is v_mfma_f64_16x16x4_f64:
//   A operand: lane l holds A[l % 16][l / 16]   (16 x 4)
//   B operand: lane l holds B[l / 16][l % 16]   (4 x 16)
//   D: element v of lane l is D[l / 16 + 4 v][l % 16]
// ---------------------------------------------------------------------------
constexpr int BM = 128, BN = 128, BK = 16;
constexpr int LDS_STRIDE = BM + 16;  // doubles per LDS row (k-major A and B tiles)
constexpr int NTHREADS = 256;
#ifndef MF_GEMM_WAVES_PER_SIMD
#define MF_GEMM_WAVES_PER_SIMD 2
#endif

struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  double* ws;
  const ProdDesc* prods;
  const EpiDesc* epis;
  int nprod;
  int m;          // M = N = K of every leaf product
  int tiles;      // tiles per side (m / BM)
  int64_t ldc;    // leading dimension of C (= n)
  int vec_in;     // A and B rows are 16-byte aligned
};

__device__ __forceinline__ const double* src_ptr(const GemmArgs& g, int src) {
  return src == SRC_A ? g.A : (src == SRC_B ? g.B : g.ws);
}

// Map a workgroup id to a tile position.  Workgroups are dealt round-robin to
// the 8 XCDs; regroup so that each XCD works on a contiguous range of
// positions, and walk positions in bands of 8 tile rows so that concurrently
// running tiles share operand panels in the XCD's L2.
__device__ __forceinline__ void tile_of(int b, int tiles, int* ti, int* tj) {
  const int G = tiles * tiles;
  int L = b;
  if ((G & 7) == 0) L = (b & 7) * (G >> 3) + (b >> 3);
  constexpr int BAND = 8;
  const int per_band = BAND * tiles;
  const int band = L / per_band;
  const int first = band * BAND;
  const int rows = min(BAND, tiles - first);
  const int in = L - band * per_band;
  *ti = first + in % rows;
  *tj = in / rows;
}

// Load the BM x BK tile of the A view (rows i0.., cols k0..) and the BK x BN
// tile of the B view into registers.  Out-of-view entries are zero.
__device__ __forceinline__ void load_tiles(const double* __restrict__ pa, int lda, int a_vr, int a_vc,
                                           const double* __restrict__ pb, int ldb, int b_vr, int b_vc,
                                           int i0, int j0, int k0, bool vec_a, bool vec_b, int t,
                                           d2 (&ra)[4], d2 (&rb)[4]) {
  // A: 128 rows x 8 pairs; B: 16 rows x 64 pairs.
  const bool a_full = vec_a && (i0 + BM <= a_vr) && (k0 + BK <= a_vc);
  const bool b_full = vec_b && (k0 + BK <= b_vr) && (j0 + BN <= b_vc);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = t + NTHREADS * q;
    const int row = idx >> 3, kp = (idx & 7) * 2;
    const int gi = i0 + row, gk = k0 + kp;
    if (a_full) {
      ra[q] = *reinterpret_cast<const d2*>(pa + (size_t)gi * lda + gk);
    } else {
      d2 v = {0.0, 0.0};
      if (gi < a_vr) {
        if (gk < a_vc) v.x = pa[(size_t)gi * lda + gk];
        if (gk + 1 < a_vc) v.y = pa[(size_t)gi * lda + gk + 1];
      }
      ra[q] = v;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = t + NTHREADS * q;
    const int kr = idx >> 6, cp = (idx & 63) * 2;
    const int gk = k0 + kr, gj = j0 + cp;
    if (b_full) {
      rb[q] = *reinterpret_cast<const d2*>(pb + (size_t)gk * ldb + gj);
    } else {
      d2 v = {0.0, 0.0};
      if (gk < b_vr) {
        if (gj < b_vc) v.x = pb[(size_t)gk * ldb + gj];
        if (gj + 1 < b_vc) v.y = pb[(size_t)gk * ldb + gj + 1];
      }
      rb[q] = v;
    }
  }
}

__device__ __forceinline__ void store_tiles(double* As, double* Bs, int t, const d2 (&ra)[4], const d2 (&rb)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = t + NTHREADS * q;
    const int row = idx >> 3, kp = (idx & 7) * 2;
    As[kp * LDS_STRIDE + row] = ra[q].x;
    As[(kp + 1) * LDS_STRIDE + row] = ra[q].y;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = t + NTHREADS * q;
    const int kr = idx >> 6, cp = (idx & 63) * 2;
    *reinterpret_cast<d2*>(Bs + kr * LDS_STRIDE + cp) = rb[q];
  }
}

__global__ void __launch_bounds__(NTHREADS, MF_GEMM_WAVES_PER_SIMD) gemm_f64_grouped(GemmArgs g) {
  __shared__ double lds[2][2][BK * LDS_STRIDE];  // [buffer][A|B][k][col]
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int lr = lane & 15, lk = lane >> 4;
  int ti, tj;
  tile_of(blockIdx.x, g.tiles, &ti, &tj);
  const int i0 = ti * BM, j0 = tj * BN;
  const int KT = g.m / BK;

  for (int r = 0; r < g.nprod; ++r) {
    const ProdDesc pd = g.prods[r];
    const double* pa = src_ptr(g, pd.a_src) + pd.a_off;
    const double* pb = src_ptr(g, pd.b_src) + pd.b_off;
    const bool vec_a = pd.a_src == SRC_WS || g.vec_in;
    const bool vec_b = pd.b_src == SRC_WS || g.vec_in;

    d4 acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};

    d2 ra[4], rb[4];
    load_tiles(pa, pd.lda, pd.a_vr, pd.a_vc, pb, pd.ldb, pd.b_vr, pd.b_vc, i0, j0, 0, vec_a, vec_b, t, ra, rb);
    store_tiles(lds[0][0], lds[0][1], t, ra, rb);
    __syncthreads();

    for (int kt = 0; kt < KT; ++kt) {
      const int cur = kt & 1;
      const bool more = kt + 1 < KT;
      if (more)
        load_tiles(pa, pd.lda, pd.a_vr, pd.a_vc, pb, pd.ldb, pd.b_vr, pd.b_vc, i0, j0, (kt + 1) * BK, vec_a,
                   vec_b, t, ra, rb);
      const double* As = lds[cur][0];
      const double* Bs = lds[cur][1];
#pragma unroll
      for (int s = 0; s < BK / 4; ++s) {
        double fa[4], fb[4];
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) fa[mi] = As[(4 * s + lk) * LDS_STRIDE + wm + 16 * mi + lr];
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) fb[ni] = Bs[(4 * s + lk) * LDS_STRIDE + wn + 16 * ni + lr];
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
          for (int ni = 0; ni < 4; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[mi], fb[ni], acc[mi][ni], 0, 0, 0);
      }
      if (more) store_tiles(lds[cur ^ 1][0], lds[cur ^ 1][1], t, ra, rb);
      __syncthreads();
    }

    // Epilogue: post-addition into every C block this product feeds.
    for (int e = pd.epi_beg; e < pd.epi_end; ++e) {
      const EpiDesc ed = g.epis[e];
      double* pc = g.C + ed.c_off;
      const bool full = (i0 + BM <= ed.c_vr) && (j0 + BN <= ed.c_vc);
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = i0 + wm + 16 * mi + lk + 4 * v;
            const int col = j0 + wn + 16 * ni + lr;
            if (full || (row < ed.c_vr && col < ed.c_vc)) {
              double* p = pc + (size_t)row * g.ldc + col;
              if (ed.first == 1)
                *p = ed.coef * acc[mi][ni][v];
              else if (ed.first == 2)
                *p = 0.0;
              else
                *p = __builtin_fma(ed.coef, acc[mi][ni][v], *p);
            }
          }
    }
  }
}

// ---------------------------------------------------------------------------
// Pre-addition: every thread owns VEC consecutive elements at one position
// (i, j) of the m x m blocks, reads that position of all P2 input blocks once
// and writes it to every materialised output of its operand.
// ---------------------------------------------------------------------------
struct PreArgs {
  const double* A;
  const double* B;
  double* ws;
  const PreOut* outs;
  const PreIn* ins;
  const double* coef;
  int n_out_a, n_out_b;
  int m;
  int64_t ld_in;
  int vec_in;
};

template <int P2, int VEC>
__global__ void __launch_bounds__(256) preadd_f64(PreArgs g) {
  typedef double dv __attribute__((ext_vector_type(VEC)));
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int64_t mm = (int64_t)g.m * g.m;
  if (e >= mm) return;
  const int i = (int)(e / g.m), j = (int)(e % g.m);
  const int op = blockIdx.y;
  const double* base = op == 0 ? g.A : g.B;
  const PreIn* ins = g.ins + op * P2;
  const int o_beg = op == 0 ? 0 : g.n_out_a;
  const int o_end = op == 0 ? g.n_out_a : g.n_out_a + g.n_out_b;

  dv in[P2];
#pragma unroll
  for (int k = 0; k < P2; ++k) {
    const PreIn v = ins[k];
    const double* p = base + v.off + (int64_t)i * g.ld_in + j;
    if (g.vec_in && i < v.vr && j + VEC <= v.vc) {
      in[k] = *reinterpret_cast<const dv*>(p);
    } else {
      dv x;
#pragma unroll
      for (int q = 0; q < VEC; ++q) x[q] = (i < v.vr && j + q < v.vc) ? p[q] : 0.0;
      in[k] = x;
    }
  }
  for (int o = o_beg; o < o_end; ++o) {
    const PreOut po = g.outs[o];
    const double* c = g.coef + po.coef_off;
    dv acc;
    bool started = false;
#pragma unroll
    for (int k = 0; k < P2; ++k) {
      const double ck = c[k];
      if (ck != 0.0) {
        if (!started) {
          acc = ck == 1.0 ? in[k] : ck * in[k];
          started = true;
        } else {
#pragma unroll
          for (int q = 0; q < VEC; ++q) acc[q] = __builtin_fma(ck, in[k][q], acc[q]);
        }
      }
    }
    if (!started) acc = (dv)(0.0);
    *reinterpret_cast<dv*>(g.ws + po.out_off + (int64_t)i * g.m + j) = acc;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_preadd_f64(const Plan& pl, const void* A, const void* B, void* ws, bool vec_in, hipStream_t s) {
  if (pl.n_pre_a + pl.n_pre_b == 0) return hipSuccess;
  PreArgs g;
  g.A = static_cast<const double*>(A);
  g.B = static_cast<const double*>(B);
  g.ws = static_cast<double*>(ws);
  g.outs = pl.d_pre_out;
  g.ins = pl.d_pre_in;
  g.coef = pl.d_pre_coef;
  g.n_out_a = pl.n_pre_a;
  g.n_out_b = pl.n_pre_b;
  g.m = (int)pl.m;
  g.ld_in = pl.n;
  g.vec_in = vec_in ? 1 : 0;
  const int P2 = pl.P * pl.P;
  const int64_t mm = pl.m * pl.m;
  auto grid = [&](int vec) { return dim3((unsigned)((mm / vec + 255) / 256), 2, 1); };
  switch (P2) {
    case 4: hipLaunchKernelGGL((preadd_f64<4, 2>), grid(2), dim3(256), 0, s, g); break;
    case 9: hipLaunchKernelGGL((preadd_f64<9, 2>), grid(2), dim3(256), 0, s, g); break;
    case 16: hipLaunchKernelGGL((preadd_f64<16, 2>), grid(2), dim3(256), 0, s, g); break;
    case 36: hipLaunchKernelGGL((preadd_f64<36, 1>), grid(1), dim3(256), 0, s, g); break;
    case 64: hipLaunchKernelGGL((preadd_f64<64, 1>), grid(1), dim3(256), 0, s, g); break;
    case 81: hipLaunchKernelGGL((preadd_f64<81, 1>), grid(1), dim3(256), 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const Plan& pl, const void* A, const void* B, void* C, void* ws, bool vec_in,
                           hipStream_t s) {
  GemmArgs g;
  g.A = static_cast<const double*>(A);
  g.B = static_cast<const double*>(B);
  g.C = static_cast<double*>(C);
  g.ws = static_cast<double*>(ws);
  g.prods = pl.d_prods;
  g.epis = pl.d_epis;
  g.nprod = (int)pl.prods.size();
  g.m = (int)pl.m;
  g.tiles = (int)(pl.m / BM);
  g.ldc = pl.n;
  g.vec_in = vec_in ? 1 : 0;
  const unsigned grid = (unsigned)g.tiles * (unsigned)g.tiles;
  hipLaunchKernelGGL(gemm_f64_grouped, dim3(grid), dim3(NTHREADS), 0, s, g);
  return hipGetLastError();
}

}  // namespace mf
