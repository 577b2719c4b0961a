// FP64 kernels for gfx950: the linear-combination kernel (GEMA over blocks,
// used for the pre-additions and for the outer post-addition) and the grouped
// leaf GEMM on FP64 MFMA with the inner post-addition fused into its epilogue.
//
// Data flow of one fused level (equation "strassen", Section 2 of the paper),
// for an algorithm split as outer levels x inner levels:
//   combine (pre):  T_r = sum_k U[k,r] A_k, S_r = sum_l V[l,r] B_l for every
//                   product whose combination has more than one term
//                   (one-term columns are read in place as views of A or B);
//   gemm:           workgroup (group g, tile position): for each product r of
//                   group g in order, acc = T_r S_r (MFMA), then
//                   Out_c (tile) = / += W[c,r] * acc for each c it feeds.
//                   With one group Out is C itself; otherwise Out is the
//                   group's workspace block P_g (the inner product result).
//                   A workgroup owns its tile position of every block it
//                   writes, so the read-modify-write is race-free and its
//                   summation order is fixed (bitwise reproducible);
//   combine (post): C_c = sum_g W_outer[c,g] P_g  (only with several groups).
#include "mf_internal.h"

namespace mf {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// GEMM tile geometry: 128 x 128 output tile per workgroup of 256 threads
// (4 waves of 64 arranged 2 x 2, each wave 64 x 64 = 4 x 4 MFMA tiles),
// K step 16 (4 MFMA k-steps of 4), LDS double-buffered.  The MFMA is
// v_mfma_f64_16x16x4_f64 with the lane layout
//   A operand: lane l holds A[l % 16][l / 16]   (16 x 4)
//   B operand: lane l holds B[l / 16][l % 16]   (4 x 16)
//   D: element v of lane l is D[l / 16 + 4 v][l % 16].
// Both LDS tiles are stored k-major (A transposed on the way in) so that the
// 16 lanes of a fragment row read 16 consecutive doubles.
// ---------------------------------------------------------------------------
constexpr int BM = 128, BN = 128, BK = 16;
constexpr int LDS_STRIDE = BM + 16;  // doubles per LDS row
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
  const int32_t* group_beg;  // products of group g: [group_beg[g], group_beg[g+1])
  int groups;
  int m;          // M = N = K of every leaf product
  int tiles;      // tiles per side (m / BM)
  int vec_in;     // A and B rows are 16-byte aligned
};

__device__ __forceinline__ const double* src_ptr(const GemmArgs& g, int src) {
  return src == SRC_A ? g.A : (src == SRC_B ? g.B : (src == SRC_C ? g.C : g.ws));
}
__device__ __forceinline__ double* dst_ptr(const GemmArgs& g, int src) { return src == SRC_C ? g.C : g.ws; }

// Map a workgroup id to (group, tile position).  Workgroups are dealt
// round-robin to the 8 XCDs; regroup so that each XCD works on a contiguous
// range of (group, position) pairs, and walk positions in bands of 8 tile
// rows so that concurrently running tiles share operand panels in the XCD's
// L2.
__device__ __forceinline__ void work_of(int b, int tiles, int groups, int* grp, int* ti, int* tj) {
  const int G = tiles * tiles;
  const int total = G * groups;
  int L = b;
  if ((total & 7) == 0) L = (b & 7) * (total >> 3) + (b >> 3);
  *grp = L / G;
  L -= *grp * G;
  constexpr int BAND = 8;
  const int per_band = BAND * tiles;
  const int band = L / per_band;
  const int first = band * BAND;
  const int rows = min(BAND, tiles - first);
  const int in = L - band * per_band;
  *ti = first + in % rows;
  *tj = in / rows;
}

// Global -> register prefetch of one BM x BK tile of the A view and one
// BK x BN tile of the B view.  MASKED: entries outside the view's valid
// rows/columns are zero and only valid elements are read.
template <bool MASKED>
__device__ __forceinline__ void load_tiles(const double* __restrict__ pa, int lda, int a_vr, int a_vc,
                                           const double* __restrict__ pb, int ldb, int b_vr, int b_vc,
                                           int i0, int j0, int k0, int t, d2 (&ra)[4], d2 (&rb)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = t + NTHREADS * q;
    const int row = idx >> 3, kp = (idx & 7) * 2;
    const int gi = i0 + row, gk = k0 + kp;
    if (!MASKED) {
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
    if (!MASKED) {
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

// acc = A_view(i0.., :) * B_view(:, j0..) over K = KT * BK.
template <bool MASKED>
__device__ __forceinline__ void k_loop(double (*lds)[2][BK * LDS_STRIDE], const double* __restrict__ pa, int lda,
                                       int a_vr, int a_vc, const double* __restrict__ pb, int ldb, int b_vr,
                                       int b_vc, int i0, int j0, int KT, int t, int wm, int wn, int lr, int lk,
                                       d4 (&acc)[4][4]) {
  d2 ra[4], rb[4];
  load_tiles<MASKED>(pa, lda, a_vr, a_vc, pb, ldb, b_vr, b_vc, i0, j0, 0, t, ra, rb);
  store_tiles(lds[0][0], lds[0][1], t, ra, rb);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < KT;
    if (more) load_tiles<MASKED>(pa, lda, a_vr, a_vc, pb, ldb, b_vr, b_vc, i0, j0, (kt + 1) * BK, t, ra, rb);
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
}

__global__ void __launch_bounds__(NTHREADS, MF_GEMM_WAVES_PER_SIMD) gemm_f64_grouped(GemmArgs g) {
  __shared__ double lds[2][2][BK * LDS_STRIDE];  // [buffer][A|B][k][col]
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int lr = lane & 15, lk = lane >> 4;
  int grp, ti, tj;
  work_of(blockIdx.x, g.tiles, g.groups, &grp, &ti, &tj);
  const int i0 = ti * BM, j0 = tj * BN;
  const int KT = g.m / BK;
  const int r_beg = g.group_beg[grp], r_end = g.group_beg[grp + 1];

  for (int r = r_beg; r < r_end; ++r) {
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

    const bool interior = vec_a && vec_b && i0 + BM <= pd.a_vr && pd.a_vc >= g.m && pd.b_vr >= g.m &&
                          j0 + BN <= pd.b_vc;
    if (interior)
      k_loop<false>(lds, pa, pd.lda, pd.a_vr, pd.a_vc, pb, pd.ldb, pd.b_vr, pd.b_vc, i0, j0, KT, t, wm, wn, lr, lk,
                    acc);
    else
      k_loop<true>(lds, pa, pd.lda, pd.a_vr, pd.a_vc, pb, pd.ldb, pd.b_vr, pd.b_vc, i0, j0, KT, t, wm, wn, lr, lk,
                   acc);

    // Epilogue: post-addition into every output block this product feeds.
    for (int e = pd.epi_beg; e < pd.epi_end; ++e) {
      const EpiDesc ed = g.epis[e];
      double* pc = dst_ptr(g, ed.c_src) + ed.c_off;
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
              double* p = pc + (size_t)row * ed.ldc + col;
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
// Linear combination of blocks (GEMA): every thread owns VEC consecutive
// elements at one position (i, j) of the m x m blocks, reads that position of
// all NIN input views once and writes it to every output of its operand set
// (blockIdx.y selects the set).  Inputs outside a view's valid extent are
// zero; outputs outside a view's valid extent are not written.
// ---------------------------------------------------------------------------
struct CombArgs {
  const double* src[4];  // indexed by Src
  double* dst[4];
  const CombIn* ins;     // NIN per operand set
  const CombOut* outs;
  const double* coef;    // NIN per output
  int out_beg[3];        // outputs of set y: [out_beg[y], out_beg[y+1])
  int m;
  int vec_in;            // input views with src A/B/C have 16-byte aligned rows
  int vec_out;           // output views with dst C have 16-byte aligned rows
};

template <int NIN, int VEC>
__global__ void __launch_bounds__(256) combine_f64(CombArgs g) {
  typedef double dv __attribute__((ext_vector_type(VEC)));
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int64_t mm = (int64_t)g.m * g.m;
  if (e >= mm) return;
  const int i = (int)(e / g.m), j = (int)(e % g.m);
  const int op = blockIdx.y;
  const CombIn* ins = g.ins + op * NIN;

  dv in[NIN];
#pragma unroll
  for (int k = 0; k < NIN; ++k) {
    const CombIn v = ins[k];
    const double* p = g.src[v.src] + v.off + (int64_t)i * v.ld + j;
    const bool vec = v.src == SRC_WS || g.vec_in;
    if (vec && i < v.vr && j + VEC <= v.vc) {
      in[k] = *reinterpret_cast<const dv*>(p);
    } else {
      dv x;
#pragma unroll
      for (int q = 0; q < VEC; ++q) x[q] = (i < v.vr && j + q < v.vc) ? p[q] : 0.0;
      in[k] = x;
    }
  }
  for (int o = g.out_beg[op]; o < g.out_beg[op + 1]; ++o) {
    const CombOut po = g.outs[o];
    const double* c = g.coef + po.coef_off;
    dv acc;
    bool started = false;
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
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
    if (i >= po.vr) continue;
    double* p = g.dst[po.dst] + po.off + (int64_t)i * po.ld + j;
    const bool vec = po.dst == SRC_WS || g.vec_out;
    if (vec && j + VEC <= po.vc) {
      *reinterpret_cast<dv*>(p) = acc;
    } else {
#pragma unroll
      for (int q = 0; q < VEC; ++q)
        if (j + q < po.vc) p[q] = acc[q];
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static hipError_t launch_combine(const CombineStage& cs, int m, const void* A, const void* B, void* C, void* ws,
                                 bool vec_in, bool vec_out, hipStream_t s) {
  if (cs.n_sets == 0) return hipSuccess;
  CombArgs g;
  g.src[SRC_A] = static_cast<const double*>(A);
  g.src[SRC_B] = static_cast<const double*>(B);
  g.src[SRC_C] = static_cast<const double*>(C);
  g.src[SRC_WS] = static_cast<const double*>(ws);
  g.dst[SRC_A] = nullptr;
  g.dst[SRC_B] = nullptr;
  g.dst[SRC_C] = static_cast<double*>(C);
  g.dst[SRC_WS] = static_cast<double*>(ws);
  g.ins = cs.d_ins;
  g.outs = cs.d_outs;
  g.coef = cs.d_coef;
  for (int y = 0; y < 3; ++y) g.out_beg[y] = cs.out_beg[y];
  g.m = m;
  g.vec_in = vec_in ? 1 : 0;
  g.vec_out = vec_out ? 1 : 0;
  const int64_t mm = (int64_t)m * m;
  auto grid = [&](int vec) { return dim3((unsigned)((mm / vec + 255) / 256), (unsigned)cs.n_sets, 1); };
  switch (cs.nin) {
#define MF_COMB_CASE(N, V) \
  case N: hipLaunchKernelGGL((combine_f64<N, V>), grid(V), dim3(256), 0, s, g); break;
    MF_COMB_CASE(4, 2)
    MF_COMB_CASE(7, 2)
    MF_COMB_CASE(9, 2)
    MF_COMB_CASE(16, 2)
    MF_COMB_CASE(27, 1)
    MF_COMB_CASE(36, 1)
    MF_COMB_CASE(49, 1)
    MF_COMB_CASE(64, 1)
    MF_COMB_CASE(81, 1)
#undef MF_COMB_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool combine_supported(int nin) {
  switch (nin) {
    case 4: case 7: case 9: case 16: case 27: case 36: case 49: case 64: case 81: return true;
    default: return false;
  }
}

hipError_t launch_phase_f64(const Plan& pl, int phase, const void* A, const void* B, void* C, void* ws, bool vec_in,
                            bool vec_c, hipStream_t s) {
  if (phase == 0) return launch_combine(pl.pre, (int)pl.m, A, B, C, ws, vec_in, vec_c, s);
  if (phase == 2) return launch_combine(pl.post, (int)pl.m_outer, A, B, C, ws, vec_in, vec_c, s);
  GemmArgs g;
  g.A = static_cast<const double*>(A);
  g.B = static_cast<const double*>(B);
  g.C = static_cast<double*>(C);
  g.ws = static_cast<double*>(ws);
  g.prods = pl.d_prods;
  g.epis = pl.d_epis;
  g.group_beg = pl.d_group_beg;
  g.groups = pl.groups;
  g.m = (int)pl.m;
  g.tiles = (int)(pl.m / BM);
  g.vec_in = vec_in ? 1 : 0;
  const unsigned grid = (unsigned)g.tiles * (unsigned)g.tiles * (unsigned)g.groups;
  hipLaunchKernelGGL(gemm_f64_grouped, dim3(grid), dim3(NTHREADS), 0, s, g);
  return hipGetLastError();
}

}  // namespace mf
