// Device code of the linear combination of matrix blocks (GEMA), shared by
// the combination kernel and the persistent batched kernel: one thread
// computes VEC consecutive elements at position (i, j) of every output of a
// set from the same position of the set's input views.
#pragma once

#include <type_traits>

#include "gemm_common.h"

namespace mf {

template <class T>
struct CombArgs {
  const T* A;
  const T* B;
  T* C;
  T* ws;
  const CombSet* sets;   // one per blockIdx.y
  const CombIn* ins;     // NIN per set
  const CombOut* outs;
  const double* coef;    // NIN per output
  int m;                 // block size of a square stage (Kronecker-factored and batched stages)
  int vec_in;            // input views with src A/B/C have 16-byte aligned rows
  int vec_out;           // output views with dst C have 16-byte aligned rows
  int scale_c;           // outputs into C are alpha (sum) + beta C
  T alpha, beta;         // (beta = 0: C is not read)
};

template <class T>
__device__ __forceinline__ const T* comb_src(const CombArgs<T>& g, int src) {
  const T* p = g.ws;
  p = src == SRC_A ? g.A : p;
  p = src == SRC_B ? g.B : p;
  p = src == SRC_C ? g.C : p;
  return p;
}

template <class T>
__device__ __forceinline__ T* comb_dst(const CombArgs<T>& g, int dst) {
  return dst == SRC_C ? g.C : g.ws;
}

// Store of a whole output vector.  (Non-temporal stores measured slower on
// the pre-addition of <4,4,4;49>.)
template <class V>
__device__ __forceinline__ void store_out(V* p, const V& v) {
  *p = v;
}

// An output into C under scaling: acc becomes alpha acc + beta C for the
// `valid` leading elements at p (C is read only when beta != 0; vec: the
// VEC elements at p can be read as one vector).
template <class T, int VEC, class TV>
__device__ __forceinline__ void scale_into_c(const CombArgs<T>& g, const T* p, bool vec, int valid, TV& acc) {
  if (g.beta == T(0)) {
#pragma unroll
    for (int q = 0; q < VEC; ++q) acc[q] = g.alpha * acc[q];
    return;
  }
  TV old;
  if (vec && valid >= VEC) {
    old = *reinterpret_cast<const TV*>(p);
  } else {
#pragma unroll
    for (int q = 0; q < VEC; ++q) old[q] = q < valid ? p[q] : T(0);
  }
#pragma unroll
  for (int q = 0; q < VEC; ++q) acc[q] = fma_t(g.beta, old[q], g.alpha * acc[q]);
}

template <class T, int NIN, int VEC, bool FULL>
__device__ __forceinline__ void combine_body(const CombArgs<T>& g, const CombSet& set, int i, int j) {
  typedef T tv __attribute__((ext_vector_type(VEC)));
  const CombIn* ins = g.ins + set.in_beg;
  tv in[NIN];
#pragma unroll
  for (int k = 0; k < NIN; ++k) {
    const CombIn v = load_uniform(ins + k);
    const T* p = comb_src(g, v.src) + v.off + (int64_t)i * v.ld + j;
    if (FULL) {
      in[k] = *reinterpret_cast<const tv*>(p);
    } else {
      const bool vec = v.src == SRC_WS || g.vec_in;
      if (vec && i < v.vr && j + VEC <= v.vc) {
        in[k] = *reinterpret_cast<const tv*>(p);
      } else {
        tv x;
#pragma unroll
        for (int q = 0; q < VEC; ++q) x[q] = (i < v.vr && j + q < v.vc) ? p[q] : T(0);
        in[k] = x;
      }
    }
  }
  for (int o = set.out_beg; o < set.out_end; ++o) {
    const CombOut po = load_uniform(g.outs + o);
    const double* c = g.coef + po.coef_off;
    tv acc;
    bool started = false;
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      const T ck = (T)load_uniform(c + k);
      if (ck != T(0)) {
        if (!started) {
          acc = ck == T(1) ? in[k] : ck * in[k];
          started = true;
        } else {
#pragma unroll
          for (int q = 0; q < VEC; ++q) acc[q] = fma_t(ck, in[k][q], acc[q]);
        }
      }
    }
    if (!started) acc = (tv)(T(0));
    T* p = comb_dst(g, po.dst) + po.off + (int64_t)i * po.ld + j;
    if (g.scale_c && po.dst == SRC_C) {
      if (i >= po.vr) continue;
      scale_into_c<T, VEC>(g, p, FULL || g.vec_out, po.vc - j, acc);
    }
    if (FULL) {
      store_out(reinterpret_cast<tv*>(p), acc);
    } else {
      if (i >= po.vr) continue;
      const bool vec = po.dst == SRC_WS || g.vec_out;
      if (vec && j + VEC <= po.vc) {
        store_out(reinterpret_cast<tv*>(p), acc);
      } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q)
          if (j + q < po.vc) p[q] = acc[q];
      }
    }
  }
}

// The same combination with the outputs held in registers and the inputs
// streamed through them, for sets with many inputs and few outputs (the
// post-addition of a composed algorithm: 49 inputs, 16 outputs).  Each output
// is formed exactly as above: its first nonzero term c_k * in_k, then
// fused multiply-adds in ascending k, so both bodies give identical bits.
template <class T, int NIN, int NOUT, int VEC, bool FULL>
__device__ __forceinline__ void combine_acc_body(const CombArgs<T>& g, const CombSet& set, int i, int j) {
  typedef T tv __attribute__((ext_vector_type(VEC)));
  // inputs are read CHUNK at a time (all loads of a chunk issued before any
  // is used), so every wave keeps several HBM reads in flight
  constexpr int CHUNK = NIN % 8 == 0 ? 8 : NIN % 7 == 0 ? 7 : NIN % 9 == 0 ? 9 : 1;
  const CombIn* ins = g.ins + set.in_beg;
  const int nout = set.out_end - set.out_beg;
  int coef_off[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) coef_off[o] = o < nout ? load_uniform(g.outs + set.out_beg + o).coef_off : 0;
  tv acc[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) acc[o] = (tv)(T(0));
  uint32_t started = 0;  // bit o: output o has its first term (wave-uniform)
  for (int k0 = 0; k0 < NIN; k0 += CHUNK) {
    tv x[CHUNK];
#pragma unroll
    for (int u = 0; u < CHUNK; ++u) {
      const CombIn v = load_uniform(ins + k0 + u);
      const T* p = comb_src(g, v.src) + v.off + (int64_t)i * v.ld + j;
      if (FULL) {
        x[u] = *reinterpret_cast<const tv*>(p);
      } else {
        const bool vec = v.src == SRC_WS || g.vec_in;
        if (vec && i < v.vr && j + VEC <= v.vc) {
          x[u] = *reinterpret_cast<const tv*>(p);
        } else {
#pragma unroll
          for (int q = 0; q < VEC; ++q) x[u][q] = (i < v.vr && j + q < v.vc) ? p[q] : T(0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < CHUNK; ++u) {
      const int k = k0 + u;
#pragma unroll
      for (int o = 0; o < NOUT; ++o) {
        const T ck = o < nout ? (T)load_uniform(g.coef + coef_off[o] + k) : T(0);
        if (ck != T(0)) {
          if (!(started >> o & 1u)) {
            acc[o] = ck == T(1) ? x[u] : ck * x[u];
            started |= 1u << o;
          } else {
#pragma unroll
            for (int q = 0; q < VEC; ++q) acc[o][q] = fma_t(ck, x[u][q], acc[o][q]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    if (o >= nout) continue;
    const CombOut po = load_uniform(g.outs + set.out_beg + o);
    T* p = comb_dst(g, po.dst) + po.off + (int64_t)i * po.ld + j;
    if (g.scale_c && po.dst == SRC_C) {
      if (i >= po.vr) continue;
      scale_into_c<T, VEC>(g, p, FULL || g.vec_out, po.vc - j, acc[o]);
    }
    if (FULL) {
      store_out(reinterpret_cast<tv*>(p), acc[o]);
    } else {
      if (i >= po.vr) continue;
      const bool vec = po.dst == SRC_WS || g.vec_out;
      if (vec && j + VEC <= po.vc) {
        store_out(reinterpret_cast<tv*>(p), acc[o]);
      } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q)
          if (j + q < po.vc) p[q] = acc[o][q];
      }
    }
  }
}

// Number of inputs of a set, as a compile-time dispatch: calls
// f(std::integral_constant<int, NIN>) for the supported counts.
template <class F>
__device__ __forceinline__ void with_nin(int nin, F&& f) {
  switch (nin) {
    case 1: f(std::integral_constant<int, 1>()); break;
    case 4: f(std::integral_constant<int, 4>()); break;
    case 7: f(std::integral_constant<int, 7>()); break;
    case 8: f(std::integral_constant<int, 8>()); break;
    case 9: f(std::integral_constant<int, 9>()); break;
    case 16: f(std::integral_constant<int, 16>()); break;
    default: break;
  }
}

}  // namespace mf
