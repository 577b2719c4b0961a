// Device-side pieces shared by the grouped GEMM kernels (FP64 / FP32 MFMA
// leaves and BF16 MFMA leaves): kernel arguments, the workgroup -> (group,
// tile) map, and the epilogue post-addition of one output element.
#pragma once

#include "mf_internal.h"

namespace mf {


template <class T>
struct GemmArgs {
  const T* A;
  const T* B;
  T* C;
  T* ws;
  const ProdDesc* prods;
  const EpiDesc* epis;
  const int32_t* group_beg;  // products of group g: [group_beg[g], group_beg[g+1])
  const TermDesc* terms;     // fused-operand plans: operand terms
  int groups;
  int m;        // rows M of every leaf product
  int n, k;     // its columns N and inner size K (both m for square plans)
  int tiles_m;  // output tiles along rows (m / BM) and columns (n / BN)
  int tiles_n;
  int vec_in;   // A and B rows are 16-byte aligned
  int scale_c;  // outputs into C are alpha (sum) + beta C (beta = 0: C is not read)
  T alpha, beta;
};

// Load a descriptor that every lane of the wave reads at the same address and
// mark each word as wave-uniform, so address arithmetic on it runs on the
// scalar unit and buffer descriptors built from it stay in scalar registers.
// Descriptors are written before the kernel starts and never during it, so
// they are read through the constant address space: with a wave-uniform
// address that is one scalar load instead of a vector load in every lane.
template <class S>
__device__ __forceinline__ S load_uniform(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "descriptor must be a whole number of words");
  int w[sizeof(S) / 4];
#if defined(__HIP_DEVICE_COMPILE__)
  typedef const __attribute__((address_space(4))) int cint;
  cint* q = (cint*)p;
#pragma unroll
  for (unsigned i = 0; i < sizeof(S) / 4; ++i) w[i] = __builtin_amdgcn_readfirstlane(q[i]);
#else
  __builtin_memcpy(w, p, sizeof(S));
#endif
  S v;
  __builtin_memcpy(&v, w, sizeof(S));
  return v;
}

// The base of an operand source or output destination.  Selected with
// integer masks: a chain of selects over the fields is turned by the
// compiler into a load at a computed offset, which forces a GemmArgs built
// in a kernel (the batched kernels build one per task) into scratch memory.
template <class T>
__device__ __forceinline__ const T* src_ptr(const GemmArgs<T>& g, int src) {
  const uint64_t m_a = 0 - (uint64_t)(src == SRC_A), m_b = 0 - (uint64_t)(src == SRC_B);
  const uint64_t m_c = 0 - (uint64_t)(src == SRC_C), m_w = ~(m_a | m_b | m_c);
  return reinterpret_cast<const T*>((reinterpret_cast<uint64_t>(g.A) & m_a) | (reinterpret_cast<uint64_t>(g.B) & m_b) |
                                    (reinterpret_cast<uint64_t>(g.C) & m_c) | (reinterpret_cast<uint64_t>(g.ws) & m_w));
}

template <class T>
__device__ __forceinline__ T* dst_ptr(const GemmArgs<T>& g, int dst) {
  const uint64_t m_c = 0 - (uint64_t)(dst == SRC_C);
  return reinterpret_cast<T*>((reinterpret_cast<uint64_t>(g.C) & m_c) | (reinterpret_cast<uint64_t>(g.ws) & ~m_c));
}

// Map a workgroup id to (group, tile position).  Workgroups are dealt
// round-robin to the 8 XCDs; regroup so that each XCD works on a contiguous
// range of (group, position) pairs, and walk positions in bands of BAND tile
// rows so that concurrently running tiles share operand panels in the XCD's
// L2 (8 for the FP64/FP32 tiles; the BF16 kernel passes its own).
template <int BAND = 8>
__device__ __forceinline__ void work_of(int b, int tiles_m, int tiles_n, int groups, int* grp, int* ti, int* tj) {
  const int G = tiles_m * tiles_n;
  const int total = G * groups;
  int L = b;
  if ((total & 7) == 0) L = (b & 7) * (total >> 3) + (b >> 3);
  *grp = L / G;
  L -= *grp * G;
  const int per_band = BAND * tiles_n;
  const int band = L / per_band;
  const int first = band * BAND;
  const int rows = min(BAND, tiles_m - first);
  const int in = L - band * per_band;
  *ti = first + in % rows;
  *tj = in / rows;
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Post-addition of one output element: first == 1 stores coef * v, 0 adds
// coef * v (fused multiply-add), 2 stores zero.  beta != 0 (an output into C
// under scaling, with alpha already in coef): the first store and the zero
// store also add beta times the old value.
template <class T>
__device__ __forceinline__ void epi_apply(T* p, int first, T coef, T v, T beta = T(0)) {
  if (first == 1)
    *p = beta != T(0) ? fma_t(coef, v, beta * *p) : coef * v;
  else if (first == 2)
    *p = beta != T(0) ? beta * *p : T(0);
  else
    *p = fma_t(coef, v, *p);
}

}  // namespace mf
