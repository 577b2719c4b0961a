// Device code of the grouped leaf GEMM on FP64 / FP32 MFMA (gfx950), shared
// by the grouped-GEMM kernel and the persistent batched kernel.
//
// Tile geometry (TileCfg): a BM x BN output tile per workgroup of
// WAVES_M x WAVES_N waves, each wave (BM / WAVES_M) x (BN / WAVES_N) made of
// 16 x 16 MFMA tiles, K step 16 (4 MFMA k-steps of 4), LDS double-buffered.
// Tile128: 128 x 128, 8 waves of 64 x 32, two workgroups per CU (4 waves per
// SIMD).  Both MFMAs used (v_mfma_f64_16x16x4_f64, v_mfma_f32_16x16x4_f32) take
//   A operand: lane l holds A[l % 16][l / 16]   (16 x 4)
//   B operand: lane l holds B[l / 16][l % 16]   (4 x 16)
// and return 4 values per lane:
//   f64: element v of lane l is D[l / 16 + 4 v][l % 16]
//   f32: element v of lane l is D[4 (l / 16) + v][l % 16].
// Two ways to fill LDS:
//   * FP64 interior tiles (k_loop_dma): both operands straight from memory to
//     LDS (no registers, no LDS stores); A stays row-major with its 16-byte
//     pieces swizzled per row, B k-major.
//   * Edge tiles, FP32 and fused operands (k_loop, k_loop_fused): through
//     registers; both LDS tiles k-major (A transposed on the way in) so that
//     the 16 lanes of a fragment row read 16 consecutive elements.  The A tile
//     is loaded so that the lanes one LDS cycle serves write consecutive rows
//     of one k-row pair (a_slot), which keeps the transposing stores free of
//     bank conflicts.
// All paths feed the MFMA k slots in the same order (kslot).
//
// A work item owns one tile position of every output block of its group and
// runs the group's products in order: the first product feeding a block
// stores, later ones accumulate by FMA (race-free, fixed order).
#pragma once

#include "gemm_common.h"

namespace mf {

template <int BM_, int BN_, int WAVES_M_, int WAVES_N_, int WAVES_PER_SIMD_>
struct TileCfg {
  static constexpr int BM = BM_, BN = BN_, BK = 16;
  static constexpr int WAVES_M = WAVES_M_, WAVES_N = WAVES_N_;
  static constexpr int NTHREADS = 64 * WAVES_M * WAVES_N;
  static constexpr int WAVES_PER_SIMD = WAVES_PER_SIMD_;  // occupancy the register budget is sized for
  static constexpr int WM_T = BM / (16 * WAVES_M), WN_T = BN / (16 * WAVES_N);  // MFMA tiles per wave
  static constexpr int LPT_A = BM * BK / 2 / NTHREADS;  // element-pair loads per thread and K step
  static constexpr int LPT_B = BK * BN / 2 / NTHREADS;
  static_assert(LPT_A >= 1 && LPT_B >= 1 && BM * BK / 2 % NTHREADS == 0 && BK * BN / 2 % NTHREADS == 0,
                "tile loads must divide evenly");
  static_assert(BM % kLeafTile == 0 && BN % kLeafTile == 0, "tiles are multiples of the leaf granularity");
};
using Tile128 = TileCfg<128, 128, 2, 4, 4>;

// LDS geometry of one element type: two A buffers, then two B buffers.
//   A, register-staged path: k-major, k row k at k * SA.
//   A, LDS-direct path: row-major, BM rows of BK elements (same space).
//   B, both paths: k-major rows of BN elements, at b_row(k) on the
//   LDS-direct path and at b_row_r(k) on the register-staged one.
// LDS has 32 four-byte banks and serves 128 bytes per cycle: an FP64
// fragment read serves 16 lanes (one k row) per cycle, an FP32 one 32 lanes,
// i.e. the k rows of row groups lk and lk + 1, which kslot puts 4 apart.  For
// FP32 those rows start 16 banks apart: A stride BM + 4, and B stored as
// pairs of k rows (a pair is what one LDS-direct instruction moves) 2 BN + 8
// apart.
template <class T, class Cfg>
struct Geom {
  static constexpr bool F64 = sizeof(T) == 8;
  static constexpr int SA = Cfg::BM + (F64 ? 16 : 4);
  // FP64 B: k row stride of the LDS-direct path.  BN + 8 puts adjacent k
  // rows 16 banks apart: the K loop unrolled by two steps reads fragments of
  // adjacent k rows in one ds_read2_b64, which at BN + 16 (rows in the same
  // banks) cost 64 conflict cycles per K step and workgroup.  The register-
  // staged path keeps BN + 16 (at BN + 8 its loop ran 8% slower: n = 1037
  // classical, 0.220 against 0.203 ms).  A tile fills and reads its buffers
  // in one loop, so the two layouts never meet.
  static constexpr int SB = Cfg::BN + 8;
  static constexpr int SBR = Cfg::BN + 16;
  static constexpr int PAIR = 2 * Cfg::BN + 8;  // FP32 B: stride of a pair of k rows
  static constexpr int LDS_A = Cfg::BK * SA;
  static constexpr int LDS_B = F64 ? Cfg::BK * SBR : Cfg::BK / 2 * PAIR;
  static constexpr int ELEMS = 2 * (LDS_A + LDS_B);
  static_assert(Cfg::BM * Cfg::BK <= LDS_A, "the row-major A tile fits an A buffer");
  static __device__ __forceinline__ int b_row(int k) { return F64 ? k * SB : (k >> 1) * PAIR + (k & 1) * Cfg::BN; }
  static __device__ __forceinline__ int b_row_r(int k) {
    return F64 ? k * SBR : (k >> 1) * PAIR + (k & 1) * Cfg::BN;
  }
};

// Element pair idx of the A tile -> (row, kp): the pair A[row][kp..kp+1].
// LDS has 32 four-byte banks and serves 128 bytes per cycle (16 lanes of a
// 64-bit store, 32 lanes of a 32-bit one); RUN consecutive lanes take RUN
// consecutive rows of the same k-row pair, so the transposed stores of those
// lanes cover every bank once.  Mapping consecutive lanes along k instead
// would put all k-row pairs of a row in the same banks.
template <class T, class Cfg>
__device__ __forceinline__ void a_slot(int idx, int& row, int& kp) {
  constexpr int RUN = 128 / sizeof(T), BK = Cfg::BK;
  static_assert(Cfg::BM % RUN == 0, "A tile rows must split into runs");
  row = idx % RUN + RUN * (idx / (RUN * (BK / 2)));
  kp = 2 * ((idx / RUN) % (BK / 2));
}

// Element pair idx of the B tile -> (k row, column pair).
template <class T, class Cfg>
__device__ __forceinline__ void b_slot(int idx, int& kr, int& cp) {
  kr = idx / (Cfg::BN / 2);
  cp = (idx % (Cfg::BN / 2)) * 2;
}

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v2 __attribute__((ext_vector_type(2)));
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef float v2 __attribute__((ext_vector_type(2)));
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

// Global -> register prefetch of one BM x BK tile of an A view and one
// BK x BN tile of a B view, two consecutive elements per load (the fused-
// operand path and edge tiles).
//
// Interior tiles (every element valid, rows 16-byte aligned): raw buffer loads
// whose descriptors (tile origin at the current k0) live in scalar registers,
// so each lane keeps only two 32-bit byte offsets per operand across the K loop
// (row * ld + column, fixed for the whole loop).  Edge tiles: plain loads with
// per-element masks; entries outside the view's valid rows/columns are zero
// and only valid elements are read.
template <class Cfg>
struct LaneOffsets {
  int a[Cfg::LPT_A], b[Cfg::LPT_B];
};

template <class T, class Cfg>
__device__ __forceinline__ LaneOffsets<Cfg> lane_offsets(int lda, int ldb, int t) {
  LaneOffsets<Cfg> o;
#pragma unroll
  for (int q = 0; q < Cfg::LPT_A; ++q) {
    int row, kp;
    a_slot<T, Cfg>(t + Cfg::NTHREADS * q, row, kp);
    // row < 256 and ld <= 2^21: every offset is below 2^31 bytes.
    o.a[q] = (row * lda + kp) * (int)sizeof(T);
  }
#pragma unroll
  for (int q = 0; q < Cfg::LPT_B; ++q) {
    int kr, cp;
    b_slot<T, Cfg>(t + Cfg::NTHREADS * q, kr, cp);
    o.b[q] = (kr * ldb + cp) * (int)sizeof(T);
  }
  return o;
}

// Descriptor word 3 for raw (untyped) buffer access on gfx9-family parts:
// 32-bit data format, no swizzle, no index stride.  The record count only
// bounds offsets, which are below 2^31 here.  The base is the same in every
// lane (a tile origin); taking it from the first lane tells the compiler so,
// which keeps the descriptor in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(lo | hi << 32), (short)0, 0x7fffffff,
                                           0x00020000);
}

template <class T>
__device__ __forceinline__ typename Mfma<T>::v2 buffer_pair(__amdgpu_buffer_rsrc_t r, int off) {
  typedef typename Mfma<T>::v2 v2;
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  else
    return __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

template <class T, class Cfg>
__device__ __forceinline__ void load_a_masked(const T* __restrict__ pa, int lda, int a_vr, int a_vc, int i0, int k0,
                                              int t, typename Mfma<T>::v2 (&ra)[Cfg::LPT_A]) {
  typedef typename Mfma<T>::v2 v2;
#pragma unroll
  for (int q = 0; q < Cfg::LPT_A; ++q) {
    int row, kp;
    a_slot<T, Cfg>(t + Cfg::NTHREADS * q, row, kp);
    const int gi = i0 + row, gk = k0 + kp;
    v2 v = {T(0), T(0)};
    if (gi < a_vr) {
      if (gk < a_vc) v.x = pa[(size_t)gi * lda + gk];
      if (gk + 1 < a_vc) v.y = pa[(size_t)gi * lda + gk + 1];
    }
    ra[q] = v;
  }
}

template <class T, class Cfg>
__device__ __forceinline__ void load_b_masked(const T* __restrict__ pb, int ldb, int b_vr, int b_vc, int j0, int k0,
                                              int t, typename Mfma<T>::v2 (&rb)[Cfg::LPT_B]) {
  typedef typename Mfma<T>::v2 v2;
#pragma unroll
  for (int q = 0; q < Cfg::LPT_B; ++q) {
    int kr, cp;
    b_slot<T, Cfg>(t + Cfg::NTHREADS * q, kr, cp);
    const int gk = k0 + kr, gj = j0 + cp;
    v2 v = {T(0), T(0)};
    if (gk < b_vr) {
      if (gj < b_vc) v.x = pb[(size_t)gk * ldb + gj];
      if (gj + 1 < b_vc) v.y = pb[(size_t)gk * ldb + gj + 1];
    }
    rb[q] = v;
  }
}

template <class T, class Cfg>
__device__ __forceinline__ void load_tiles_masked(const T* __restrict__ pa, int lda, int a_vr, int a_vc,
                                                  const T* __restrict__ pb, int ldb, int b_vr, int b_vc, int i0,
                                                  int j0, int k0, int t, typename Mfma<T>::v2 (&ra)[Cfg::LPT_A],
                                                  typename Mfma<T>::v2 (&rb)[Cfg::LPT_B]) {
  load_a_masked<T, Cfg>(pa, lda, a_vr, a_vc, i0, k0, t, ra);
  load_b_masked<T, Cfg>(pb, ldb, b_vr, b_vc, j0, k0, t, rb);
}

template <class T, class Cfg>
__device__ __forceinline__ void store_tiles(T* As, T* Bs, int t, const typename Mfma<T>::v2 (&ra)[Cfg::LPT_A],
                                            const typename Mfma<T>::v2 (&rb)[Cfg::LPT_B]) {
  typedef typename Mfma<T>::v2 v2;
#pragma unroll
  for (int q = 0; q < Cfg::LPT_A; ++q) {
    int row, kp;
    a_slot<T, Cfg>(t + Cfg::NTHREADS * q, row, kp);
    As[kp * Geom<T, Cfg>::SA + row] = ra[q].x;
    As[(kp + 1) * Geom<T, Cfg>::SA + row] = ra[q].y;
  }
#pragma unroll
  for (int q = 0; q < Cfg::LPT_B; ++q) {
    int kr, cp;
    b_slot<T, Cfg>(t + Cfg::NTHREADS * q, kr, cp);
    *reinterpret_cast<v2*>(Bs + Geom<T, Cfg>::b_row_r(kr) + cp) = rb[q];
  }
}

// Wait until at most N of this thread's vector memory operations (loads into
// LDS included) are outstanding: s_waitcnt vmcnt(N), LDS and export counters
// left alone.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}

// k of MFMA k-step s (of the 4 in a K step of 16) in the lanes of row group
// lk = l / 16.  With P elements per 16-byte piece (2 in FP64, 4 in FP32),
// step s takes element s % P of piece 4 (s / P) + lk of the k range, so the
// elements of a piece feed consecutive k-steps and one 16-byte LDS read
// serves P steps.  Every path (LDS-direct, register-staged, fused) uses this
// order, so products agree bit for bit whichever path loaded their operands.
template <class T>
__device__ __forceinline__ int kslot(int s, int lk) {
  constexpr int P = 16 / sizeof(T);
  return P * (4 * (s / P) + lk) + s % P;
}

template <class T, class Cfg>
__device__ __forceinline__ void load_frags(const T* As, const T* Bs, int s, int wm, int wn, int lr, int lk,
                                           T (&fa)[Cfg::WM_T], T (&fb)[Cfg::WN_T]) {
  const int k = kslot<T>(s, lk);
#pragma unroll
  for (int mi = 0; mi < Cfg::WM_T; ++mi) fa[mi] = As[k * Geom<T, Cfg>::SA + wm + 16 * mi + lr];
#pragma unroll
  for (int ni = 0; ni < Cfg::WN_T; ++ni) fb[ni] = Bs[Geom<T, Cfg>::b_row_r(k) + wn + 16 * ni + lr];
}

// LDS-direct geometry of one element type: P elements per 16-byte piece,
// RA rows of A and RB k rows of B per wave instruction (64 pieces), and the
// swizzle of A pieces within a row: piece c of row r sits at position
// c ^ swz(r), so that the 8 lanes one LDS cycle serves in a 16-byte fragment
// read (rows r..r+7, one piece index) hit every bank once.
template <class T, class Cfg>
struct Dma {
  static constexpr int P = 16 / sizeof(T);
  static constexpr int NW = Cfg::NTHREADS / 64;
  static constexpr int PPR = Cfg::BK / P;  // pieces per A row
  static constexpr int RA = 64 / PPR, RB = 64 * P / Cfg::BN;
  static constexpr int A_INSTR = Cfg::BM / (NW * RA), B_INSTR = Cfg::BK / (NW * RB);
  static_assert(A_INSTR * NW * RA == Cfg::BM && B_INSTR * NW * RB == Cfg::BK && 4 % P == 0 && RA % 8 == 0,
                "whole A rows and whole B k rows per wave instruction");
  // FP64: a row is 128 bytes (all 32 banks) of 8 pieces, so 8 rows need 8
  // distinct positions.  FP32: a row is 64 bytes of 4 pieces; rows r and
  // r + 2 start in the same bank, so the position follows r / 2.
  static __device__ __forceinline__ int swz(int r) { return P == 2 ? (r & 7) : ((r >> 1) & 3); }
};

// One K step's A and B tiles of a wave, memory -> LDS (see k_loop_dma).
// Kept out of the loop's lambdas: those are host-device functions, and the
// builtin exists only on the device.
// Lane byte offsets oa, ob address instruction 0; instruction q adds
// q * sa_step (sb_step) bytes, a wave-uniform value passed as the scalar
// offset, so each lane holds one offset per operand.
template <class T, class Cfg>
__device__ __forceinline__ void dma_tiles(T* As, T* Bs, const T* a0, const T* b0, int oa, int ob, int sa_step,
                                          int sb_step, int w) {
  typedef Dma<T, Cfg> D;
  const __amdgpu_buffer_rsrc_t sa = raw_rsrc(a0);
  const __amdgpu_buffer_rsrc_t sb = raw_rsrc(b0);
#pragma unroll
  for (int q = 0; q < D::A_INSTR; ++q)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(sa, As + D::RA * (w + D::NW * q) * Cfg::BK, 16, oa, q * sa_step, 0, 0);
#pragma unroll
  for (int q = 0; q < D::B_INSTR; ++q)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(sb, Bs + Geom<T, Cfg>::b_row(D::RB * (w + D::NW * q)), 16, ob,
                                             q * sb_step, 0, 0);
}

// Interior tiles with both operands moved straight from memory to LDS
// (buffer_load ... lds, 16 bytes per lane, lane l of a wave landing at the
// instruction's LDS base + 16 l), so no registers hold the next tile and no
// LDS store instructions run.
//   A tile: row-major, BM rows of BK / P pieces, swizzled (Dma::swz).  A
//     fragment read (ds_read_b128) of rows r..r+7 for one piece index hits
//     every bank once; one read gives a lane the A values of P k-steps.
//   B tile: k-major rows (Geom::b_row), RB rows per wave instruction.
// Each K step issues the next tile's loads first (into the buffer every wave
// finished reading before the previous barrier) and ends with the wait for
// them and the barrier, placed before the last k-step's MFMAs so that the
// wait and the next step's first fragment reads overlap MFMAs.
template <class T, class Cfg>
__device__ __forceinline__ void k_loop_dma(T* lds, const T* __restrict__ pa, int lda, const T* __restrict__ pb,
                                           int ldb, int i0, int j0, int KT, int t, int wm, int wn, int lr, int lk,
                                           typename Mfma<T>::v4 (&acc)[Cfg::WM_T][Cfg::WN_T]) {
  typedef Dma<T, Cfg> D;
  typedef Geom<T, Cfg> G;
  constexpr int P = D::P, WM_T = Cfg::WM_T, WN_T = Cfg::WN_T, BK = Cfg::BK;
  typedef T vp __attribute__((ext_vector_type(P)));
  static_assert(BK == 16, "4 MFMA k-steps per K step");
  const int lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int rl = lane / D::PPR;  // A row within an instruction (whose first row is a multiple of 8)
  const int oa = ((D::RA * w + rl) * lda + P * ((lane % D::PPR) ^ D::swz(rl))) * (int)sizeof(T);
  const int ob = ((D::RB * w + lane / (64 / D::RB)) * ldb + P * (lane % (64 / D::RB))) * (int)sizeof(T);
  const int sa_step = D::RA * D::NW * lda * (int)sizeof(T), sb_step = D::RB * D::NW * ldb * (int)sizeof(T);
  auto a_buf = [&](int b) { return lds + b * G::LDS_A; };
  auto b_buf = [&](int b) { return lds + 2 * G::LDS_A + b * G::LDS_B; };
  auto issue = [&](int k0, int buf) {
    dma_tiles<T, Cfg>(a_buf(buf), b_buf(buf), pa + (size_t)i0 * lda + k0, pb + (size_t)k0 * ldb + j0, oa, ob, sa_step,
                      sb_step, w);
  };
  // the A values of k-steps P p .. P p + P - 1: piece 4 p + lk of each row
  auto read_a = [&](const T* As, int p, vp (&f)[WM_T]) {
    const int pos = (4 * p + lk) ^ D::swz(lr);
#pragma unroll
    for (int mi = 0; mi < WM_T; ++mi) f[mi] = *reinterpret_cast<const vp*>(As + (wm + 16 * mi + lr) * BK + P * pos);
  };
  auto read_b = [&](const T* Bs, int s, T (&f)[WN_T]) {
    const int row = G::b_row(kslot<T>(s, lk));
#pragma unroll
    for (int ni = 0; ni < WN_T; ++ni) f[ni] = Bs[row + wn + 16 * ni + lr];
  };
  auto mma = [&](const vp (&a)[WM_T], int e, const T (&b)[WN_T]) {
#pragma unroll
    for (int mi = 0; mi < WM_T; ++mi)
#pragma unroll
      for (int ni = 0; ni < WN_T; ++ni) acc[mi][ni] = Mfma<T>::op(a[mi][e], b[ni], acc[mi][ni]);
  };
  issue(0, 0);
  wait_vmcnt<0>();
  __syncthreads();
  T fb[2][WN_T];
  if constexpr (P == 2) {
    // FP64: two A reads per K step (k-steps 0-1 and 2-3)
    vp fa[2][WM_T];
    read_a(a_buf(0), 0, fa[0]);
    read_b(b_buf(0), 0, fb[0]);
    auto step = [&](int kt, int cur) {
      const bool more = kt + 1 < KT;
      if (more) issue((kt + 1) * BK, cur ^ 1);
      const T* As = a_buf(cur);
      const T* Bs = b_buf(cur);
      read_b(Bs, 1, fb[1]);
      mma(fa[0], 0, fb[0]);
      read_a(As, 1, fa[1]);
      read_b(Bs, 2, fb[0]);
      mma(fa[0], 1, fb[1]);
      read_b(Bs, 3, fb[1]);
      mma(fa[1], 0, fb[0]);
      wait_vmcnt<0>();
      __syncthreads();
      if (more) {
        read_a(a_buf(cur ^ 1), 0, fa[0]);
        read_b(b_buf(cur ^ 1), 0, fb[0]);
      }
      mma(fa[1], 1, fb[1]);
    };
    // two K steps per iteration, so that the buffer of each is a constant
    // (FP64 n = 8192: depth-3 GEMM 10.23 -> 10.03 ms, classical 14.92 ->
    // 14.50 ms; issuing the next tile's loads after the first MFMAs instead
    // measured slower)
    int kt = 0;
    for (; kt + 1 < KT; kt += 2) {
      step(kt, 0);
      step(kt + 1, 1);
    }
    if (kt < KT) step(kt, 0);
  } else {
    // FP32: one A read per K step serves all four k-steps; the next step's
    // is read after the barrier into the other set.  At four waves per SIMD
    // two K steps run per iteration, so that each step's buffer and A set are
    // constants; the six-wave budget (80 VGPRs) keeps one step per iteration,
    // since unrolled it spills 21 VGPRs.
    vp fa[WM_T], fn[WM_T];
    read_a(a_buf(0), 0, fa);
    read_b(b_buf(0), 0, fb[0]);
    if constexpr (Cfg::WAVES_PER_SIMD > 4) {
      for (int kt = 0; kt < KT; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < KT;
        if (more) issue((kt + 1) * BK, cur ^ 1);
        const T* Bs = b_buf(cur);
        read_b(Bs, 1, fb[1]);
        mma(fa, 0, fb[0]);
        read_b(Bs, 2, fb[0]);
        mma(fa, 1, fb[1]);
        read_b(Bs, 3, fb[1]);
        mma(fa, 2, fb[0]);
        wait_vmcnt<0>();
        __syncthreads();
        if (more) {
          read_a(a_buf(cur ^ 1), 0, fn);
          read_b(b_buf(cur ^ 1), 0, fb[0]);
        }
        mma(fa, 3, fb[1]);
#pragma unroll
        for (int mi = 0; mi < WM_T; ++mi) fa[mi] = fn[mi];
      }
      return;
    }
    auto step = [&](int kt, int cur, vp(&fx)[WM_T], vp(&fy)[WM_T]) {
      const bool more = kt + 1 < KT;
      if (more) issue((kt + 1) * BK, cur ^ 1);
      const T* Bs = b_buf(cur);
      read_b(Bs, 1, fb[1]);
      mma(fx, 0, fb[0]);
      read_b(Bs, 2, fb[0]);
      mma(fx, 1, fb[1]);
      read_b(Bs, 3, fb[1]);
      mma(fx, 2, fb[0]);
      wait_vmcnt<0>();
      __syncthreads();
      if (more) {
        read_a(a_buf(cur ^ 1), 0, fy);
        read_b(b_buf(cur ^ 1), 0, fb[0]);
      }
      mma(fx, 3, fb[1]);
    };
    int kt = 0;
    for (; kt + 1 < KT; kt += 2) {
      step(kt, 0, fa, fn);
      step(kt + 1, 1, fn, fa);
    }
    if (kt < KT) step(kt, 0, fa, fn);
  }
}

template <class T, class Cfg>
__device__ __forceinline__ void mfma_step(const T (&fa)[Cfg::WM_T], const T (&fb)[Cfg::WN_T],
                                          typename Mfma<T>::v4 (&acc)[Cfg::WM_T][Cfg::WN_T]) {
#pragma unroll
  for (int mi = 0; mi < Cfg::WM_T; ++mi)
#pragma unroll
    for (int ni = 0; ni < Cfg::WN_T; ++ni) acc[mi][ni] = Mfma<T>::op(fa[mi], fb[ni], acc[mi][ni]);
}

// Edge tiles: acc += A_view(i0.., k) * B_view(k, j0..) over K steps kt0 ..
// KT - 1 with masked loads through registers (entries outside the views are
// zero).  lds holds the two A buffers (k-major), then the two B buffers.
template <class T, class Cfg>
__device__ __forceinline__ void k_loop_masked(T* lds, const T* __restrict__ pa, int lda, int a_vr, int a_vc,
                                              const T* __restrict__ pb, int ldb, int b_vr, int b_vc, int i0, int j0,
                                              int kt0, int KT, int t, int wm, int wn, int lr, int lk,
                                              typename Mfma<T>::v4 (&acc)[Cfg::WM_T][Cfg::WN_T]) {
  constexpr int WM_T = Cfg::WM_T, WN_T = Cfg::WN_T, BK = Cfg::BK;
  typename Mfma<T>::v2 ra[Cfg::LPT_A], rb[Cfg::LPT_B];
  auto load = [&](int k0) { load_tiles_masked<T, Cfg>(pa, lda, a_vr, a_vc, pb, ldb, b_vr, b_vc, i0, j0, k0, t, ra, rb); };
  auto a_buf = [&](int b) { return lds + b * Geom<T, Cfg>::LDS_A; };
  auto b_buf = [&](int b) { return lds + 2 * Geom<T, Cfg>::LDS_A + b * Geom<T, Cfg>::LDS_B; };
  constexpr int S = BK / 4;  // MFMA k-steps per K step
  load(kt0 * BK);
  store_tiles<T, Cfg>(a_buf(0), b_buf(0), t, ra, rb);
  __syncthreads();
  // fragments double-buffered: the reads of k-step s + 1 are issued before
  // the MFMAs of k-step s
  T fa[2][WM_T], fb[2][WN_T];
  load_frags<T, Cfg>(a_buf(0), b_buf(0), 0, wm, wn, lr, lk, fa[0], fb[0]);
  for (int kt = kt0; kt < KT; ++kt) {
    const int cur = (kt - kt0) & 1;
    const bool more = kt + 1 < KT;
    if (more) load((kt + 1) * BK);
    const T* As = a_buf(cur);
    const T* Bs = b_buf(cur);
#pragma unroll
    for (int s = 0; s < S - 1; ++s) {
      load_frags<T, Cfg>(As, Bs, s + 1, wm, wn, lr, lk, fa[(s + 1) & 1], fb[(s + 1) & 1]);
      mfma_step<T, Cfg>(fa[s & 1], fb[s & 1], acc);
    }
    // The last k-step's fragments are already in registers: store the next
    // tile and pass the barrier while the MFMAs issued above run, then issue
    // the next K step's first fragment reads ahead of the last MFMAs, so the
    // barrier and the LDS latency after it overlap work in the MFMA pipe.
    // (Every read of buffer cur completed before the barrier, so the next
    // step may overwrite it; buffer cur ^ 1 was last read before the previous
    // barrier.)
    if (more) store_tiles<T, Cfg>(a_buf(cur ^ 1), b_buf(cur ^ 1), t, ra, rb);
    __syncthreads();
    if (more) load_frags<T, Cfg>(a_buf(cur ^ 1), b_buf(cur ^ 1), 0, wm, wn, lr, lk, fa[S & 1], fb[S & 1]);
    mfma_step<T, Cfg>(fa[(S - 1) & 1], fb[(S - 1) & 1], acc);
  }
}

// Epilogue of one product: post-addition of the accumulator tile into every
// output block the product feeds (first feeder stores, later ones add).
// acc holds the tile whose origin is (s0, t0); only rows >= i0 and columns
// >= j0 of it are written (an edge tile moved back into the views, see
// gemm_tile, leaves the rows and columns before its own origin to the tiles
// that own them).
template <class T, class Cfg, bool FULL>
__device__ __forceinline__ void product_epilogue(const GemmArgs<T>& g, const ProdDesc& pd, int s0, int t0, int i0,
                                                 int j0, int wm, int wn, int lr, int lk,
                                                 const typename Mfma<T>::v4 (&acc)[Cfg::WM_T][Cfg::WN_T]) {
  constexpr int BM = Cfg::BM, BN = Cfg::BN, WM_T = Cfg::WM_T, WN_T = Cfg::WN_T;
  for (int e = pd.epi_beg; e < pd.epi_end; ++e) {
    const EpiDesc ed = load_uniform(g.epis + e);
    T* pc = dst_ptr(g, ed.c_src) + ed.c_off;
    const bool full = FULL || (s0 == i0 && t0 == j0 && i0 + BM <= ed.c_vr && j0 + BN <= ed.c_vc);
    const bool to_c = g.scale_c && ed.c_src == SRC_C;
    const T coef = to_c ? (T)ed.coef * g.alpha : (T)ed.coef;
    const T beta = to_c ? g.beta : T(0);
#pragma unroll
    for (int mi = 0; mi < WM_T; ++mi)
#pragma unroll
      for (int ni = 0; ni < WN_T; ++ni)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = s0 + wm + 16 * mi + Mfma<T>::row(lk, v);
          const int col = t0 + wn + 16 * ni + lr;
          if (full || (row >= i0 && col >= j0 && row < ed.c_vr && col < ed.c_vc))
            epi_apply<T>(pc + (size_t)row * ed.ldc + col, ed.first, coef, acc[mi][ni][v], beta);
        }
  }
}

// One work item of the grouped GEMM: tile (ti, tj) of every product of group
// grp, in product order, each followed by its epilogue post-additions.
// FULL: the host has checked that every operand view and every epilogue
// output of the plan covers its whole m x m block with 16-byte aligned rows,
// so no tile needs the masked load path or a masked store.
template <class T, class Cfg, bool FULL = false>
__device__ __forceinline__ void gemm_tile(const GemmArgs<T>& g, int grp, int ti, int tj, T* lds) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int BM = Cfg::BM, BN = Cfg::BN, WM_T = Cfg::WM_T, WN_T = Cfg::WN_T, WAVES_N = Cfg::WAVES_N, BK = Cfg::BK;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = (wave / WAVES_N) * (16 * WM_T), wn = (wave % WAVES_N) * (16 * WN_T);
  const int lr = lane & 15, lk = lane >> 4;
  const int i0 = ti * BM, j0 = tj * BN;
  const int r_beg = load_uniform(g.group_beg + grp), r_end = load_uniform(g.group_beg + grp + 1);

  for (int r = r_beg; r < r_end; ++r) {
    const ProdDesc pd = load_uniform(g.prods + r);
    const T* pa = src_ptr(g, pd.a_src) + pd.a_off;
    const T* pb = src_ptr(g, pd.b_src) + pd.b_off;
    const bool vec_a = pd.a_src == SRC_WS || g.vec_in;
    const bool vec_b = pd.b_src == SRC_WS || g.vec_in;
    // The K loop stops at the product's valid inner size: past the A view's
    // valid columns or the B view's valid rows every term is zero.  (The leaf
    // K is padded, and a product of zero-padded views is valid over less of
    // it; only a valid size of whole K steps takes the LDS-direct path.)
    const int k_eff = FULL ? g.k : min(g.k, min(pd.a_vc, pd.b_vr));
    const int KT = FULL ? g.k / BK : (k_eff + BK - 1) / BK;

    v4 acc[WM_T][WN_T];
#pragma unroll
    for (int mi = 0; mi < WM_T; ++mi)
#pragma unroll
      for (int ni = 0; ni < WN_T; ++ni) acc[mi][ni] = v4{T(0), T(0), T(0), T(0)};

    // An edge tile of a view at least one tile wide is computed as the whole
    // tile that ends at the view's last row (column), so that it takes the
    // LDS-direct path; its epilogue writes only the rows (columns) from i0
    // (j0) on.  A moved B tile keeps 16-byte aligned rows.  Only where every
    // output of the product ends inside the moved tile: an output larger
    // than the operand views (a stored product of zero-padded views) takes
    // zeros past them, which the masked path writes.
    int s0 = i0, t0 = j0;
    if constexpr (!FULL) {
      if (i0 + BM > pd.a_vr && pd.a_vr >= BM) s0 = pd.a_vr - BM;
      if (j0 + BN > pd.b_vc && pd.b_vc >= BN && (pd.b_vc * (int)sizeof(T)) % 16 == 0) t0 = pd.b_vc - BN;
      // (a moved dimension must cover the outputs up to their end; the other
      // one is covered by the tile itself)
      if (s0 != i0 || t0 != j0)
        for (int e = pd.epi_beg; e < pd.epi_end; ++e) {
          const EpiDesc ed = load_uniform(g.epis + e);
          if (s0 != i0 && ed.c_vr > s0 + BM) s0 = i0;
          if (t0 != j0 && ed.c_vc > t0 + BN) t0 = j0;
        }
    }
    // whole K steps take the LDS-direct path and a last partial one the
    // masked loop (every LDS read of the first loop ends before its last
    // barrier, so the second may refill the buffers in its own layout; both
    // feed the MFMAs in the same k order)
    const int KTf = FULL ? KT : k_eff / BK;
    const bool interior = FULL || (vec_a && vec_b && s0 + BM <= pd.a_vr && t0 + BN <= pd.b_vc && KTf >= 1);
    int kt0 = 0;  // first K step of the masked loop
    if (interior) {
      k_loop_dma<T, Cfg>(lds, pa, pd.lda, pb, pd.ldb, s0, t0, KTf, t, wm, wn, lr, lk, acc);
      kt0 = KTf;
    } else {
      s0 = i0;
      t0 = j0;
    }
    if constexpr (!FULL)
      if (kt0 < KT)
        k_loop_masked<T, Cfg>(lds, pa, pd.lda, pd.a_vr, pd.a_vc, pb, pd.ldb, pd.b_vr, pd.b_vc, s0, t0, kt0, KT, t, wm,
                              wn, lr, lk, acc);

    product_epilogue<T, Cfg, FULL>(g, pd, s0, t0, i0, j0, wm, wn, lr, lk, acc);
  }
}

// ---------------------------------------------------------------------------
// Fused operands: one level's pre-addition done in the operand load.  The A
// operand tile of a product is sum_t c_t X_t over its terms (views of
// quarters of A); every term's tile of the next K step is loaded into
// registers while the current step's MFMAs run, and the terms are summed just
// before the LDS store, in term order (the first term scaled, or copied for
// a coefficient of 1, then fused multiply-adds) as the combination kernels
// do, so the operand equals the materialised one bit for bit.  So for B.
// ---------------------------------------------------------------------------

template <class T, int NT>
struct FusedOperand {
  int n;            // terms, 1..NT
  int64_t off[NT];  // view origins (elements from the source base)
  T coef[NT];
  int vr[NT], vc[NT];
};

template <class T, int NT>
__device__ __forceinline__ FusedOperand<T, NT> fused_operand(const TermDesc* terms, int beg, int n) {
  FusedOperand<T, NT> f;
  f.n = n;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    f.off[u] = 0;
    f.coef[u] = T(0);
    f.vr[u] = f.vc[u] = 0;
    if (u < n) {
      const TermDesc td = load_uniform(terms + beg + u);
      f.off[u] = td.off;
      f.coef[u] = (T)td.coef;
      f.vr[u] = td.vr;
      f.vc[u] = td.vc;
    }
  }
  return f;
}

template <class T, int NT, int L>
__device__ __forceinline__ void sum_terms(const FusedOperand<T, NT>& f, const typename Mfma<T>::v2 (&x)[NT][L],
                                          typename Mfma<T>::v2 (&r)[L]) {
#pragma unroll
  for (int q = 0; q < L; ++q) {
    r[q] = f.coef[0] == T(1) ? x[0][q] : f.coef[0] * x[0][q];
#pragma unroll
    for (int u = 1; u < NT; ++u)
      if (u < f.n) {
        r[q].x = fma_t(f.coef[u], x[u][q].x, r[q].x);
        r[q].y = fma_t(f.coef[u], x[u][q].y, r[q].y);
      }
  }
}

template <class T, class Cfg, int NT, bool MASKED>
__device__ __forceinline__ void k_loop_fused(T* lds, const T* __restrict__ pa, int lda, const FusedOperand<T, NT>& fa,
                                             const T* __restrict__ pb, int ldb, const FusedOperand<T, NT>& fb, int i0,
                                             int j0, int KT, int t, int wm, int wn, int lr, int lk,
                                             typename Mfma<T>::v4 (&acc)[Cfg::WM_T][Cfg::WN_T]) {
  typedef typename Mfma<T>::v2 v2;
  constexpr int WM_T = Cfg::WM_T, WN_T = Cfg::WN_T, BK = Cfg::BK;
  v2 xa[NT][Cfg::LPT_A], xb[NT][Cfg::LPT_B];
  v2 ra[Cfg::LPT_A], rb[Cfg::LPT_B];
  LaneOffsets<Cfg> o;
  if constexpr (!MASKED) o = lane_offsets<T, Cfg>(lda, ldb, t);
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      if (u < fa.n) {
        if constexpr (MASKED) {
          load_a_masked<T, Cfg>(pa + fa.off[u], lda, fa.vr[u], fa.vc[u], i0, k0, t, xa[u]);
        } else {
          const __amdgpu_buffer_rsrc_t sa = raw_rsrc(pa + fa.off[u] + (size_t)i0 * lda + k0);
#pragma unroll
          for (int q = 0; q < Cfg::LPT_A; ++q) xa[u][q] = buffer_pair<T>(sa, o.a[q]);
        }
      }
      if (u < fb.n) {
        if constexpr (MASKED) {
          load_b_masked<T, Cfg>(pb + fb.off[u], ldb, fb.vr[u], fb.vc[u], j0, k0, t, xb[u]);
        } else {
          const __amdgpu_buffer_rsrc_t sb = raw_rsrc(pb + fb.off[u] + (size_t)k0 * ldb + j0);
#pragma unroll
          for (int q = 0; q < Cfg::LPT_B; ++q) xb[u][q] = buffer_pair<T>(sb, o.b[q]);
        }
      }
    }
  };
  auto a_buf = [&](int b) { return lds + b * Geom<T, Cfg>::LDS_A; };
  auto b_buf = [&](int b) { return lds + 2 * Geom<T, Cfg>::LDS_A + b * Geom<T, Cfg>::LDS_B; };
  constexpr int S = BK / 4;
  load(0);
  sum_terms<T, NT, Cfg::LPT_A>(fa, xa, ra);
  sum_terms<T, NT, Cfg::LPT_B>(fb, xb, rb);
  store_tiles<T, Cfg>(a_buf(0), b_buf(0), t, ra, rb);
  __syncthreads();
  T f_a[2][WM_T], f_b[2][WN_T];
  load_frags<T, Cfg>(a_buf(0), b_buf(0), 0, wm, wn, lr, lk, f_a[0], f_b[0]);
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < KT;
    if (more) load((kt + 1) * BK);
    const T* As = a_buf(cur);
    const T* Bs = b_buf(cur);
#pragma unroll
    for (int s = 0; s < S - 1; ++s) {
      load_frags<T, Cfg>(As, Bs, s + 1, wm, wn, lr, lk, f_a[(s + 1) & 1], f_b[(s + 1) & 1]);
      mfma_step<T, Cfg>(f_a[s & 1], f_b[s & 1], acc);
    }
    // the barrier in the shadow of the last k-step's MFMAs, as in k_loop
    if (more) {
      sum_terms<T, NT, Cfg::LPT_A>(fa, xa, ra);
      sum_terms<T, NT, Cfg::LPT_B>(fb, xb, rb);
      store_tiles<T, Cfg>(a_buf(cur ^ 1), b_buf(cur ^ 1), t, ra, rb);
    }
    __syncthreads();
    if (more) load_frags<T, Cfg>(a_buf(cur ^ 1), b_buf(cur ^ 1), 0, wm, wn, lr, lk, f_a[S & 1], f_b[S & 1]);
    mfma_step<T, Cfg>(f_a[(S - 1) & 1], f_b[(S - 1) & 1], acc);
  }
}

// A work item of a fused-operand plan (one group: all products of the level
// at one tile position of every C block, in product order).  FULL: every
// term covers its whole block with 16-byte aligned rows (host-checked).
template <class T, class Cfg, int NT, bool FULL>
__device__ __forceinline__ void gemm_tile_fused(const GemmArgs<T>& g, int grp, int ti, int tj, T* lds) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int BM = Cfg::BM, BN = Cfg::BN, WM_T = Cfg::WM_T, WN_T = Cfg::WN_T, WAVES_N = Cfg::WAVES_N;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = (wave / WAVES_N) * (16 * WM_T), wn = (wave % WAVES_N) * (16 * WN_T);
  const int lr = lane & 15, lk = lane >> 4;
  const int i0 = ti * BM, j0 = tj * BN;
  const int KT = g.k / Cfg::BK;
  const int r_beg = load_uniform(g.group_beg + grp), r_end = load_uniform(g.group_beg + grp + 1);
  for (int r = r_beg; r < r_end; ++r) {
    const ProdDesc pd = load_uniform(g.prods + r);
    const FusedOperand<T, NT> fa = fused_operand<T, NT>(g.terms, pd.a_term0, pd.a_terms);
    const FusedOperand<T, NT> fb = fused_operand<T, NT>(g.terms, pd.b_term0, pd.b_terms);
    v4 acc[WM_T][WN_T];
#pragma unroll
    for (int mi = 0; mi < WM_T; ++mi)
#pragma unroll
      for (int ni = 0; ni < WN_T; ++ni) acc[mi][ni] = v4{T(0), T(0), T(0), T(0)};
    bool interior = FULL || g.vec_in;
    if (!FULL)
      for (int u = 0; u < NT; ++u) {
        if (u < fa.n) interior = interior && i0 + BM <= fa.vr[u] && fa.vc[u] >= g.k;
        if (u < fb.n) interior = interior && fb.vr[u] >= g.k && j0 + BN <= fb.vc[u];
      }
    if (interior)
      k_loop_fused<T, Cfg, NT, false>(lds, g.A, pd.lda, fa, g.B, pd.ldb, fb, i0, j0, KT, t, wm, wn, lr, lk, acc);
    else if constexpr (!FULL)
      k_loop_fused<T, Cfg, NT, true>(lds, g.A, pd.lda, fa, g.B, pd.ldb, fb, i0, j0, KT, t, wm, wn, lr, lk, acc);
    product_epilogue<T, Cfg, FULL>(g, pd, i0, j0, i0, j0, wm, wn, lr, lk, acc);
  }
}

}  // namespace mf
