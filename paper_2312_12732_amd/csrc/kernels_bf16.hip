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
// Two launches.  The staging kernel converts every leaf operand once into the
// plan's BF16 region of the workspace: the A operand of each product by rows,
// the B operand transposed (so that both run along k), zero beyond the view's
// valid extent, in the block order described below.  The GEMM kernel then
// copies contiguous 1 KiB blocks straight into LDS: no conversion, no
// masking, and half the operand bytes of FP32 per plane.
//
// MFMA lane layout (16 x 16 x 32): lane l holds A[l % 16][8 (l / 16) + t] and
// B[8 (l / 16) + t][l % 16] for t = 0..7; element v of the result is
// D[4 (l / 16) + v][l % 16].  Both LDS tiles hold k contiguous in 16-byte
// groups (A by rows, B transposed) so a fragment is one 16-byte read.
#include <type_traits>

#include "gemm_tile.h"

namespace mf {

namespace bf {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BK = 32;
// Operand layout, shared by the staged planes in HBM and the LDS tiles.  A
// plane (m x m; its rows are the rows of A or the columns of B, k runs along
// each row) is cut into blocks of 16 rows x 32 k (1 KiB), stored k-block
// major: block (K, R) starts at element 512 (K (m / 16) + R).  Inside a
// block, row r holds its 64 bytes in four 16-byte slots, k group g
// (k = 8g .. 8g + 7) in slot g ^ ((r >> 1) & 3).
//   * The operand tile of one K step (BM rows) is BM / 16 consecutive blocks:
//     each wave load instruction reads 1 KiB of contiguous bytes (8 whole
//     cache lines), and its LDS image is a plain copy.  With row-major planes
//     every load instruction touched 16 rows in 16 cache lines and the
//     texture data path was 97% busy at 0.44 MFMA utilisation.
//   * The MFMA fragment reads (lanes 0-15 on 16 rows of one k group; lane
//     group l / 16 on k group l / 16) and the linear LDS writes run with no
//     bank conflict on gfx950 (measured SQ_LDS_BANK_CONFLICT = 0 for each
//     pattern; rows padded to 80 bytes cost 4 conflict cycles per fragment
//     read and 8 per write).
constexpr int KS = BK;  // bf16 elements per LDS row (64 bytes)

// Element offset of k group g (8 elements) of row r inside a block-ordered tile.
__device__ __forceinline__ int lds_slot(int r, int g) { return r * KS + 8 * (g ^ ((r >> 1) & 3)); }

// Element offset in a staged plane (leaf size m) of element (row i, k).
__device__ __forceinline__ int64_t staged_off(int i, int k, int m) {
  return ((int64_t)(k / BK) * (m / 16) + i / 16) * (16 * BK) + lds_slot(i % 16, (k % BK) / 8) + k % 8;
}

// ---------------------------------------------------------------------------
// Staging: the last pre-addition level, fused with the BF16 conversion
// ---------------------------------------------------------------------------


constexpr int ST = 32;  // staging tile: ST x ST elements of every input of a set per workgroup

template <int NIN>
struct CoefRow {
  float c[NIN];
};

// Block (x, y): tile x (row-major over the m x m quarter) of staging set y.
// Thread t owns 4 elements of the tile: for A operands (side 0) row lr and
// columns lc .. lc + 3 of every input (staged row r0 + lr, k = c0 + lc ..);
// for B operands (side 1) column lr and rows lc .. lc + 3 (staged row
// c0 + lr, k = r0 + lc ..), so that the transposition happens in the loads
// and every input value is read once, into registers (zero outside a view's
// valid extent).  Each output of the set is then z = sum_k coef[k] in_k in
// FP32, in input order, the first nonzero term scaled and the others added by
// fused multiply-add (an exact add or subtract for the coefficients +-1),
// rounded to BF16 (and the BF16 rest for split-BF16x3) and written in the
// block order of the staged planes.  vec_in: views of the caller's A and B
// may be read as aligned 16-byte vectors (workspace views always can).
template <int NIN, bool X3>
__global__ void __launch_bounds__(256)
    stage_sets(GemmArgs<float> g, __bf16* dst_base, int64_t plane, const StageSet* __restrict__ sets,
               const CombIn* __restrict__ ins, const StageOut* __restrict__ outs, const float* __restrict__ coef,
               int vec_in) {
  const StageSet ss = load_uniform(sets + blockIdx.y);
  const int m = g.m;
  const int tiles_x = m / ST;
  const int r0 = (int)(blockIdx.x / tiles_x) * ST, c0 = (int)(blockIdx.x % tiles_x) * ST;
  const int t = threadIdx.x;
  const int lr = t / 8, lc = (t % 8) * 4;
  const bool bside = ss.side != 0;
  f4 x[NIN];
#pragma unroll
  for (int k = 0; k < NIN; ++k) {
    const CombIn in = load_uniform(ins + ss.in_beg + k);
    const float* src = src_ptr(g, in.src) + in.off;
    if (!bside) {
      const int i = r0 + lr, j = c0 + lc;
      if (r0 + ST <= in.vr && c0 + ST <= in.vc && (vec_in || in.src == SRC_WS)) {
        x[k] = *reinterpret_cast<const f4*>(src + (size_t)i * in.ld + j);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) x[k][u] = (i < in.vr && j + u < in.vc) ? src[(size_t)i * in.ld + j + u] : 0.f;
      }
    } else {
      const int j = c0 + lr;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = r0 + lc + u;
        x[k][u] = (i < in.vr && j < in.vc) ? src[(size_t)i * in.ld + j] : 0.f;
      }
    }
  }
  const int srow = bside ? c0 + lr : r0 + lr, sk = bside ? r0 + lc : c0 + lc;
  for (int o = ss.out_beg; o < ss.out_end; ++o) {
    const StageOut so = load_uniform(outs + o);
    const CoefRow<NIN> cr = load_uniform(reinterpret_cast<const CoefRow<NIN>*>(coef + so.coef_off));
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    bool first = true;
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      const float c = cr.c[k];
      if (c == 0.f) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = first ? c * x[k][u] : __builtin_fmaf(c, x[k][u], acc[u]);
      first = false;
    }
    __bf16* hi = dst_base + (size_t)so.z * (X3 ? 2 : 1) * plane;
    bf4 h, l;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      h[u] = (__bf16)acc[u];
      l[u] = (__bf16)(acc[u] - (float)h[u]);
    }
    *reinterpret_cast<bf4*>(hi + staged_off(srow, sk, m)) = h;
    if (X3) *reinterpret_cast<bf4*>(hi + plane + staged_off(srow, sk, m)) = l;
  }
}

// ---------------------------------------------------------------------------
// GEMM on staged BF16 operands
// ---------------------------------------------------------------------------

// Tile geometry: a BM_ x BN_ output tile per workgroup of WM_ x WN_ waves,
// each wave (BM_ / WM_) x (BN_ / WN_) = WTM x WTN MFMA tiles of 16 x 16; two
// waves per SIMD either way.
//   Cfg128: 128 x 128, 2 x 2 waves of 64 x 64, two workgroups per CU (either
//           form; leaves that the larger tiles do not divide);
//   CfgSq:  256 x 256, 2 x 4 waves of 128 x 64, one workgroup per CU (either
//           form).  The LDS bytes a wave reads per MFMA fall as its tile
//           grows: for split-BF16x3 (hi and lo planes, 244 VGPRs, 64 KiB per
//           K step) the 128 x 64 wave tile moved the GEMM from 0.52 to 0.64
//           of the peak at n = 16384, against 256 x 128 tiles of 64 x 64
//           waves, which kept LDS about 90% busy.  (BF16 on four 128 x 128
//           waves, one per SIMD with 256 accumulator registers, halves those
//           bytes again but measured 5-11% slower: one wave per SIMD leaves
//           its stalls uncovered.)
template <int BM_, int BN_, int WM_, int WN_, int WPE_ = 2>
struct BfCfg {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_;
  static constexpr int NT = 64 * WM * WN;                       // threads per workgroup
  static constexpr int WPE = WPE_;                              // waves per SIMD (register budget)
  static constexpr int ONE_PER_CU = BM * BN >= 256 * 256;       // LDS holds one workgroup
  static constexpr int WTM = BM / WM / 16, WTN = BN / WN / 16;  // 16 x 16 tiles per wave
  static constexpr int A_LOADS = BM * BK / 8 / NT, B_LOADS = BN * BK / 8 / NT;
  static_assert(A_LOADS * 8 * NT == BM * BK && B_LOADS * 8 * NT == BN * BK, "whole 16-byte pieces");
};
using Cfg128 = BfCfg<128, 128, 2, 2>;
using CfgSq = BfCfg<256, 256, 2, 4>;

// LDS ring of NBUF K-step buffers: four for the BF16 256 x 256 tile (128
// KiB, fragment prefetch with the loads two steps ahead, k_loop_pf), two for
// split-BF16x3 on that tile (64 KiB per step, 128 KiB) and for Cfg128, whose
// two workgroups per CU share the LDS.
template <class C, bool X3>
constexpr int nbuf() {
  return C::ONE_PER_CU && !X3 ? 4 : 2;
}

template <class C, bool X3>
struct Lds {
  static constexpr int NBUF = nbuf<C, X3>();
  __bf16 a[NBUF][X3 ? 2 : 1][C::BM * KS];  // [buffer][hi|lo][block order, as staged]
  __bf16 b[NBUF][X3 ? 2 : 1][C::BN * KS];
};

constexpr int PLANES_MAX = 2;

// The operand tiles of one K step are contiguous in the staged planes and
// in LDS (same block order): thread t moves 16-byte pieces t + NT q.  They go
// straight from memory to LDS (buffer_load ... lds, 16 bytes per lane: lane
// l of a wave lands at the wave's LDS base + 16 l, measured on the device),
// so no registers hold them and no LDS store instructions run.
template <class C, bool X3>
__device__ __forceinline__ void dma_stage(Lds<C, X3>& L, int buf, const __bf16* a, const __bf16* b, int64_t plane,
                                          int m, int i0, int j0, int k0, int t) {
  constexpr int P = X3 ? 2 : 1;
  const int64_t kb = (int64_t)(k0 / BK) * (m / 16);
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // the LDS base is per wave
#pragma unroll
  for (int pl = 0; pl < P; ++pl) {
    const __amdgpu_buffer_rsrc_t sa = raw_rsrc(a + pl * plane + (kb + i0 / 16) * (16 * BK));
    const __amdgpu_buffer_rsrc_t sb = raw_rsrc(b + pl * plane + (kb + j0 / 16) * (16 * BK));
#pragma unroll
    for (int q = 0; q < C::A_LOADS; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(sa, &L.a[buf][pl][(64 * w + C::NT * q) * 8], 16,
                                               (t + C::NT * q) * 16, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < C::B_LOADS; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(sb, &L.b[buf][pl][(64 * w + C::NT * q) * 8], 16,
                                               (t + C::NT * q) * 16, 0, 0, 0);
  }
}

// Wait until at most N of this thread's memory loads are outstanding
// (s_waitcnt vmcnt(N); N < 64), leaving LDS and export counters alone.
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}

// MFMA work of one K step from LDS buffer cur.
template <class C, bool X3>
__device__ __forceinline__ void mma_step(const Lds<C, X3>& L, int cur, int wm, int wn, int lr, int lk,
                                         f4 (&acc)[C::WTM][C::WTN]) {
  constexpr int WTM = C::WTM, WTN = C::WTN;
  bf8 ah[WTM], bh[WTN];
#pragma unroll
  for (int mi = 0; mi < WTM; ++mi)
    ah[mi] = *reinterpret_cast<const bf8*>(&L.a[cur][0][lds_slot(wm + 16 * mi + lr, lk)]);
#pragma unroll
  for (int ni = 0; ni < WTN; ++ni)
    bh[ni] = *reinterpret_cast<const bf8*>(&L.b[cur][0][lds_slot(wn + 16 * ni + lr, lk)]);
  if constexpr (X3) {
    bf8 al[WTM], bl[WTN];
#pragma unroll
    for (int mi = 0; mi < WTM; ++mi)
      al[mi] = *reinterpret_cast<const bf8*>(&L.a[cur][1][lds_slot(wm + 16 * mi + lr, lk)]);
#pragma unroll
    for (int ni = 0; ni < WTN; ++ni)
      bl[ni] = *reinterpret_cast<const bf8*>(&L.b[cur][1][lds_slot(wn + 16 * ni + lr, lk)]);
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
}

// K loop over an LDS ring of NBUF buffers: the loads of step k + NBUF - 1 go
// to LDS at the start of step k (into the buffer step k - 1 read, freed by the
// barrier that ended it), so NBUF - 1 steps of MFMA work cover their latency;
// each step ends by waiting for the next step's loads and a barrier.  (Staging
// through registers instead - two register sets, loads two steps ahead and
// stored to LDS one step ahead - measured the same: 0.47 of the BF16 peak at
// n = 16384 classical either way.)
template <class C, bool X3>
__device__ __forceinline__ void k_loop(Lds<C, X3>& L, const __bf16* a, const __bf16* b, int64_t plane, int m, int i0,
                                       int j0, int t, int wm, int wn, int lr, int lk,
                                       f4 (&acc)[C::WTM][C::WTN]) {
  constexpr int NB = Lds<C, X3>::NBUF, D = NB - 1;
  constexpr int LPS = (X3 ? 2 : 1) * (C::A_LOADS + C::B_LOADS);  // loads per thread and step
  const int KT = m / BK;
  for (int d = 0; d < D; ++d)
    if (d < KT) dma_stage<C, X3>(L, d, a, b, plane, m, i0, j0, d * BK, t);
  if (D > 1 && KT > 1)
    wait_vm<(D > 1 ? LPS : 0)>();  // step 0 landed, step 1 may still fly
  else
    wait_vm<0>();
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const bool ahead = kt + D < KT;
    if (ahead) dma_stage<C, X3>(L, (kt + D) % NB, a, b, plane, m, i0, j0, (kt + D) * BK, t);
    mma_step<C, X3>(L, kt % NB, wm, wn, lr, lk, acc);
    // step kt + 1 must have landed; later steps may still fly
    if (D > 1 && ahead)
      wait_vm<(D > 1 ? LPS : 0)>();
    else
      wait_vm<0>();
    __syncthreads();
  }
}

// Fragments of one K step (hi, and lo for split-BF16x3).
template <class C, bool X3>
struct Frags {
  bf8 ah[C::WTM], bh[C::WTN];
  bf8 al[X3 ? C::WTM : 1], bl[X3 ? C::WTN : 1];
};

template <class C, bool X3>
__device__ __forceinline__ void read_frags(const Lds<C, X3>& L, int cur, int wm, int wn, int lr, int lk,
                                           Frags<C, X3>& F) {
#pragma unroll
  for (int mi = 0; mi < C::WTM; ++mi)
    F.ah[mi] = *reinterpret_cast<const bf8*>(&L.a[cur][0][lds_slot(wm + 16 * mi + lr, lk)]);
#pragma unroll
  for (int ni = 0; ni < C::WTN; ++ni)
    F.bh[ni] = *reinterpret_cast<const bf8*>(&L.b[cur][0][lds_slot(wn + 16 * ni + lr, lk)]);
  if constexpr (X3) {
#pragma unroll
    for (int mi = 0; mi < C::WTM; ++mi)
      F.al[mi] = *reinterpret_cast<const bf8*>(&L.a[cur][1][lds_slot(wm + 16 * mi + lr, lk)]);
#pragma unroll
    for (int ni = 0; ni < C::WTN; ++ni)
      F.bl[ni] = *reinterpret_cast<const bf8*>(&L.b[cur][1][lds_slot(wn + 16 * ni + lr, lk)]);
  }
}

template <class C, bool X3>
__device__ __forceinline__ void mma_frags(const Frags<C, X3>& F, f4 (&acc)[C::WTM][C::WTN]) {
#pragma unroll
  for (int mi = 0; mi < C::WTM; ++mi)
#pragma unroll
    for (int ni = 0; ni < C::WTN; ++ni) {
      if constexpr (X3) {
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.ah[mi], F.bl[ni], acc[mi][ni], 0, 0, 0);
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.al[mi], F.bh[ni], acc[mi][ni], 0, 0, 0);
      }
      acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.ah[mi], F.bh[ni], acc[mi][ni], 0, 0, 0);
    }
}

// K loop with the fragments of step k + 1 read while the MFMAs of step k
// run (the BF16 256 x 256 tile, NBUF = 4).  Step k starts by waiting for
// the tiles of step k + 1 and a barrier: every wave then has all of step
// k + 1 in LDS and has finished reading buffer (k - 1) % NBUF (its fragments
// were in registers before step k - 1's MFMAs), so the loads of step
// k + NBUF - 1 go there; then the fragments of step k + 1 are read and the
// MFMAs of step k issued.  BF16 at n = 16384: leaf GEMMs of depth 1-3 4-6%
// faster than k_loop, classical unchanged.  (On a three-buffer ring, split-
// BF16x3 on 256 x 128 tiles, the loads ran only one step ahead and the x3
// GEMM was 3% slower.)
template <class C, bool X3>
__device__ __forceinline__ void k_loop_pf(Lds<C, X3>& L, const __bf16* a, const __bf16* b, int64_t plane, int m,
                                          int i0, int j0, int t, int wm, int wn, int lr, int lk,
                                          f4 (&acc)[C::WTM][C::WTN]) {
  constexpr int NB = Lds<C, X3>::NBUF;
  static_assert(NB == 3 || NB == 4, "a ring of 3 or 4 buffers");
  constexpr int LPS = (X3 ? 2 : 1) * (C::A_LOADS + C::B_LOADS);  // loads per thread and step
  const int KT = m / BK;
  for (int d = 0; d < NB - 1; ++d)
    if (d < KT) dma_stage<C, X3>(L, d, a, b, plane, m, i0, j0, d * BK, t);
  // step 0 landed; steps 1 .. NB - 2 may still fly
  if (NB == 4 && KT > 2)
    wait_vm<(NB == 4 ? 2 * LPS : 0)>();
  else if (KT > 1)
    wait_vm<LPS>();
  else
    wait_vm<0>();
  __syncthreads();
  Frags<C, X3> F, Fn;
  read_frags<C, X3>(L, 0, wm, wn, lr, lk, F);
  for (int kt = 0; kt < KT; ++kt) {
    // step kt + 1 landed; with four buffers step kt + 2 may still fly
    if (NB == 4 && kt + 2 < KT)
      wait_vm<(NB == 4 ? LPS : 0)>();
    else
      wait_vm<0>();
    __syncthreads();
    if (kt + NB - 1 < KT) dma_stage<C, X3>(L, (kt + NB - 1) % NB, a, b, plane, m, i0, j0, (kt + NB - 1) * BK, t);
    if (kt + 1 < KT) read_frags<C, X3>(L, (kt + 1) % NB, wm, wn, lr, lk, Fn);
    mma_frags<C, X3>(F, acc);
    F = Fn;
  }
}

// XCD bands of 4 tile rows: at n = 16384 2-3% faster than 8 (and than 2) for
// the 256-row tiles, one workgroup per CU.
constexpr int kBand = 4;

template <class C, bool X3>
__global__ void __launch_bounds__(C::NT, C::WPE)
    gemm_bf16_grouped(GemmArgs<float> g, const __bf16* __restrict__ staged, int nprod, int64_t plane) {
  __shared__ Lds<C, X3> L;
  constexpr int WTM = C::WTM, WTN = C::WTN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = (wave / C::WN) * (C::BM / C::WM), wn = (wave % C::WN) * (C::BN / C::WN);
  const int lr = lane & 15, lk = lane >> 4;
  int grp, ti, tj;
  work_of<kBand>(blockIdx.x, g.tiles_m, g.tiles_n, g.groups, &grp, &ti, &tj);
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
    if constexpr (Lds<C, X3>::NBUF == 4)
      k_loop_pf<C, X3>(L, a, b, plane, g.m, i0, j0, t, wm, wn, lr, lk, acc);
    else
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

bool stage_supported(int nin) { return nin == 1 || nin == 4 || nin == 9 || nin == 16; }


namespace {

GemmArgs<float> bf_args(const Plan& pl, const char* desc, const void* A, const void* B, void* C, void* ws) {
  GemmArgs<float> g;
  g.A = static_cast<const float*>(A);
  g.B = static_cast<const float*>(B);
  g.C = static_cast<float*>(C);
  g.ws = static_cast<float*>(ws);
  g.prods = img_at<ProdDesc>(desc, pl.img_prods);
  g.epis = img_at<EpiDesc>(desc, pl.img_epis);
  g.group_beg = img_at<int32_t>(desc, pl.img_group_beg);
  g.groups = pl.groups;
  g.m = g.n = g.k = (int)pl.m;
  g.terms = nullptr;
  g.scale_c = 0;
  g.alpha = 1.0f;
  g.beta = 0.0f;
  g.vec_in = 0;
  return g;
}

bool bf_plan_ok(const Plan& pl, const void* ws) {
  return pl.bf_base >= 0 && ws && pl.bf_outs.size() == 2 * pl.prods.size();
}

}  // namespace

hipError_t launch_stage_bf16(const Plan& pl, const char* desc, bool x3, const void* A, const void* B, void* C,
                             void* ws, bool vec_in, hipStream_t s) {
  if (!bf_plan_ok(pl, ws)) return hipErrorInvalidValue;
  const GemmArgs<float> g = bf_args(pl, desc, A, B, C, ws);
  const StageSet* sets = img_at<StageSet>(desc, pl.img_bf_sets);
  const CombIn* ins = img_at<CombIn>(desc, pl.img_bf_ins);
  const StageOut* outs = img_at<StageOut>(desc, pl.img_bf_outs);
  const float* coef = img_at<float>(desc, pl.img_bf_coef);
  __bf16* staged = reinterpret_cast<__bf16*>(static_cast<char*>(ws) + pl.bf_base);
  const int64_t plane = pl.m * pl.m;
  const dim3 sgrid((unsigned)((pl.m / bf::ST) * (pl.m / bf::ST)), (unsigned)pl.bf_sets.size());
  const int vin = vec_in ? 1 : 0;
  bool staged_ok = false;
  auto stage = [&](auto nin) {
    constexpr int N = decltype(nin)::value;
    if (pl.bf_nin != N) return;
    staged_ok = true;
    if (x3)
      hipLaunchKernelGGL((bf::stage_sets<N, true>), sgrid, dim3(256), 0, s, g, staged, plane, sets, ins, outs,
                         coef, vin);
    else
      hipLaunchKernelGGL((bf::stage_sets<N, false>), sgrid, dim3(256), 0, s, g, staged, plane, sets, ins, outs,
                         coef, vin);
  };
  stage(std::integral_constant<int, 1>{});
  stage(std::integral_constant<int, 4>{});
  stage(std::integral_constant<int, 9>{});
  stage(std::integral_constant<int, 16>{});
  if (!staged_ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gemm_bf16(const Plan& pl, const char* desc, bool x3, const void* A, const void* B, void* C,
                            void* ws, bool vec_in, hipStream_t s) {
  (void)vec_in;  // the staged operands are aligned and whole
  if (!bf_plan_ok(pl, ws)) return hipErrorInvalidValue;
  GemmArgs<float> g = bf_args(pl, desc, A, B, C, ws);
  const __bf16* st = reinterpret_cast<const __bf16*>(static_cast<char*>(ws) + pl.bf_base);
  const int nprod = (int)pl.prods.size();
  const int64_t plane = pl.m * pl.m;
  auto launch = [&](auto cfg, auto x3c) {
    typedef decltype(cfg) Cf;
    constexpr bool X = decltype(x3c)::value;
    g.tiles_m = (int)(pl.m / Cf::BM);
    g.tiles_n = (int)(pl.m / Cf::BN);
    const unsigned grid = (unsigned)g.tiles_m * (unsigned)g.tiles_n * (unsigned)g.groups;
    hipLaunchKernelGGL((bf::gemm_bf16_grouped<Cf, X>), dim3(grid), dim3(Cf::NT), 0, s, g, st, nprod, plane);
  };
  // CfgSq; Cfg128 for leaves the larger tile does not divide
  if (x3) {
    if (pl.m % bf::CfgSq::BM == 0)
      launch(bf::CfgSq{}, std::true_type{});
    else
      launch(bf::Cfg128{}, std::true_type{});
  } else {
    if (pl.m % bf::CfgSq::BM == 0)
      launch(bf::CfgSq{}, std::false_type{});
    else
      launch(bf::Cfg128{}, std::false_type{});
  }
  return hipGetLastError();
}

}  // namespace mf
