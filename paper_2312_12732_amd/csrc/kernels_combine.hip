// Linear combination of matrix blocks (GEMA) for gfx950, in FP64 or FP32:
// the pre-additions T_r = sum_k U[k,r] A_k, S_r = sum_l V[l,r] B_l of a fused
// level and its outer post-addition C_c = sum_g W_outer[c,g] P_g (equation
// "strassen", Section 2 of the paper).  HBM-bound: every input element is
// read once and every output element written once.
#include "combine_body.h"

namespace mf {

// Every thread owns VEC consecutive elements at one position (i, j) of the
// m x m blocks, reads that position of all NIN input views of its set
// (blockIdx.y) once and writes it to every output of the set.  Inputs
// outside a view's valid extent are zero; outputs outside a view's valid
// extent are not written.  Sets whose views all have full extent and aligned
// rows take a branch-free path.
template <class T, int NIN, int VEC>
__global__ void __launch_bounds__(256) combine(CombArgs<T> g) {
  const CombSet set = load_uniform(g.sets + blockIdx.y);
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  if (e >= (int64_t)set.rows * set.cols) return;
  const int i = (int)(e / set.cols), j = (int)(e % set.cols);
  if (set.full && g.vec_in && g.vec_out)
    combine_body<T, NIN, VEC, true>(g, set, i, j);
  else
    combine_body<T, NIN, VEC, false>(g, set, i, j);
}

// Outputs in registers, inputs streamed (many inputs, at most NOUT outputs
// per set).
template <class T, int NIN, int NOUT, int VEC>
__global__ void __launch_bounds__(256) combine_acc(CombArgs<T> g) {
  const CombSet set = load_uniform(g.sets + blockIdx.y);
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  if (e >= (int64_t)set.rows * set.cols) return;
  const int i = (int)(e / set.cols), j = (int)(e % set.cols);
  if (set.full && g.vec_in && g.vec_out)
    combine_acc_body<T, NIN, NOUT, VEC, true>(g, set, i, j);
  else
    combine_acc_body<T, NIN, NOUT, VEC, false>(g, set, i, j);
}

// ---------------------------------------------------------------------------
// Kronecker-factored combinations: one level of <8,8,8;343>, the
// three-factor composition of <2,2,2;7> algorithms (U = U1 (x) U2 (x) U3, and
// so for V and W; Section 2, the Kronecker construction).  A set has 64
// blocks on one side and 343 on the other, too many for coefficients per
// output, so the sums run factor by factor in registers:
//   pre:  T[r1 r2 r3] = sum_t1 U1[t1,r1] sum_t2 U2[t2,r2] sum_t3 U3[t3,r3] X[t1 t2 t3]
//   post: C[c1 c2 c3] = sum_r1 W1[c1,r1] sum_r2 W2[c2,r2] sum_r3 W3[c3,r3] P[r1 r2 r3]
// The same sums as the composed coefficients give, associated factor by
// factor (so not bitwise those of the generic kernels; integers stay exact).
// Every input element is read once and every stored output written once.
// ---------------------------------------------------------------------------

template <class T, int VEC>
__device__ __forceinline__ void kron_load(const CombArgs<T>& g, const CombIn& v, int i, int j,
                                          T (&x)[VEC]) {
  typedef T tv __attribute__((ext_vector_type(VEC)));
  const T* p = comb_src(g, v.src) + v.off + (int64_t)i * v.ld + j;
  const bool vec = v.src == SRC_WS || g.vec_in;
  if (vec && i < v.vr && j + VEC <= v.vc) {
    const tv y = *reinterpret_cast<const tv*>(p);
#pragma unroll
    for (int q = 0; q < VEC; ++q) x[q] = y[q];
  } else {
#pragma unroll
    for (int q = 0; q < VEC; ++q) x[q] = (i < v.vr && j + q < v.vc) ? p[q] : T(0);
  }
}

template <class T, int VEC>
__device__ __forceinline__ void kron_store(const CombArgs<T>& g, const CombOut& po, int i, int j,
                                           const T (&x)[VEC]) {
  typedef T tv __attribute__((ext_vector_type(VEC)));
  if (i >= po.vr) return;  // also every output that is not stored (empty extent)
  T* p = comb_dst(g, po.dst) + po.off + (int64_t)i * po.ld + j;
  const bool vec = po.dst == SRC_WS || g.vec_out;
  tv y;
#pragma unroll
  for (int q = 0; q < VEC; ++q) y[q] = x[q];
  if (g.scale_c && po.dst == SRC_C) scale_into_c<T, VEC>(g, p, vec, po.vc - j, y);
  if (vec && j + VEC <= po.vc) {
    *reinterpret_cast<tv*>(p) = y;
  } else {
#pragma unroll
    for (int q = 0; q < VEC; ++q)
      if (j + q < po.vc) p[q] = y[q];
  }
}

// c * x + acc on VEC lanes, skipped for c = 0 (c is wave-uniform)
template <class T, int VEC>
__device__ __forceinline__ void kron_axpy(T c, const T (&x)[VEC], T (&acc)[VEC]) {
  if (c == T(0)) return;
#pragma unroll
  for (int q = 0; q < VEC; ++q) acc[q] = fma_t(c, x[q], acc[q]);
}

// Register budget: the pre-addition holds the 64 inputs, 195 VGPRs, so it
// runs at two waves per SIMD (asking for three spills).  The post-addition
// holds the 64 outputs; its r2 loop stays rolled (unrolled it hoists up to 49
// loads and drops to one wave per SIMD: FP64 n = 8192, 1.41 ms against 1.00).
template <class T, int VEC>
__global__ void __launch_bounds__(256, 2) kron3_pre(CombArgs<T> g) {
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int64_t mm = (int64_t)g.m * g.m;
  if (e >= mm) return;
  const int i = (int)(e / g.m), j = (int)(e % g.m);
  const CombSet set = load_uniform(g.sets + blockIdx.y);
  // U1 | U2 | U3 (each 4 x 7), then the 343 output offsets
  const double* cf = g.coef + load_uniform(g.outs + set.out_beg).coef_off;
  T x[64][VEC];
#pragma unroll
  for (int t = 0; t < 64; ++t) kron_load<T, VEC>(g, load_uniform(g.ins + set.in_beg + t), i, j, x[t]);
  for (int r1 = 0; r1 < 7; ++r1) {
    T y[16][VEC] = {};
#pragma unroll
    for (int t1 = 0; t1 < 4; ++t1) {
      const T c = (T)load_uniform(cf + t1 * 7 + r1);
#pragma unroll
      for (int t = 0; t < 16; ++t) kron_axpy<T, VEC>(c, x[16 * t1 + t], y[t]);
    }
#pragma unroll
    for (int r2 = 0; r2 < 7; ++r2) {
      T z[4][VEC] = {};
#pragma unroll
      for (int t2 = 0; t2 < 4; ++t2) {
        const T c = (T)load_uniform(cf + 28 + t2 * 7 + r2);
#pragma unroll
        for (int t3 = 0; t3 < 4; ++t3) kron_axpy<T, VEC>(c, y[4 * t2 + t3], z[t3]);
      }
#pragma unroll
      for (int r3 = 0; r3 < 7; ++r3) {
        T o[VEC] = {};
#pragma unroll
        for (int t3 = 0; t3 < 4; ++t3) kron_axpy<T, VEC>((T)load_uniform(cf + 56 + t3 * 7 + r3), z[t3], o);
        // stored operands are whole m x m workspace blocks (offset -1: not stored)
        const double off = load_uniform(cf + 84 + 49 * r1 + 7 * r2 + r3);
        if (off >= 0.0) {
          T* p = g.ws + (int64_t)off + (int64_t)i * g.m + j;
          if (VEC == 1) {
            p[0] = o[0];
          } else {
            typedef T tv __attribute__((ext_vector_type(VEC)));
            tv y;
#pragma unroll
            for (int q = 0; q < VEC; ++q) y[q] = o[q];
            *reinterpret_cast<tv*>(p) = y;
          }
        }
      }
    }
  }
}

template <class T, int VEC>
__global__ void __launch_bounds__(256) kron3_post(CombArgs<T> g) {
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int64_t mm = (int64_t)g.m * g.m;
  if (e >= mm) return;
  const int i = (int)(e / g.m), j = (int)(e % g.m);
  const CombSet set = load_uniform(g.sets + blockIdx.y);
  // W1 | W2 | W3 (each 4 x 7), then the 343 input offsets
  const double* cf = g.coef + load_uniform(g.outs + set.out_beg).coef_off;
  T out[64][VEC] = {};
  // products are whole m x m workspace blocks (offset -1: an empty group,
  // zero), each read unconditionally (block 0 for an empty group) and then
  // selected, which measured faster than a conditional load (FP64 n = 8192:
  // 0.75 against 0.86 ms).  (Issuing the 7 loads of the next (r1, r2) before
  // the current 7 are used measured slower: 0.91 ms.)
  auto load7 = [&](int k, T (&P)[7][VEC]) {
#pragma unroll
    for (int r3 = 0; r3 < 7; ++r3) {
      const double off = load_uniform(cf + 84 + 7 * k + r3);
      const T* p = g.ws + (int64_t)(off >= 0.0 ? off : 0.0) + (int64_t)i * g.m + j;
      typedef T tv __attribute__((ext_vector_type(VEC)));
      const tv y = *reinterpret_cast<const tv*>(p);
#pragma unroll
      for (int q = 0; q < VEC; ++q) P[r3][q] = off >= 0.0 ? y[q] : T(0);
    }
  };
  for (int r1 = 0; r1 < 7; ++r1) {
    T t[16][VEC] = {};
#pragma unroll 1
    for (int r2 = 0; r2 < 7; ++r2) {
      T P[7][VEC];
      load7(7 * r1 + r2, P);
      T u[4][VEC] = {};
#pragma unroll
      for (int c3 = 0; c3 < 4; ++c3)
#pragma unroll
        for (int r3 = 0; r3 < 7; ++r3) kron_axpy<T, VEC>((T)load_uniform(cf + 56 + c3 * 7 + r3), P[r3], u[c3]);
#pragma unroll
      for (int c2 = 0; c2 < 4; ++c2) {
        const T c = (T)load_uniform(cf + 28 + c2 * 7 + r2);
#pragma unroll
        for (int c3 = 0; c3 < 4; ++c3) kron_axpy<T, VEC>(c, u[c3], t[4 * c2 + c3]);
      }
    }
#pragma unroll
    for (int c1 = 0; c1 < 4; ++c1) {
      const T c = (T)load_uniform(cf + c1 * 7 + r1);
#pragma unroll
      for (int k = 0; k < 16; ++k) kron_axpy<T, VEC>(c, t[k], out[16 * c1 + k]);
    }
  }
#pragma unroll
  for (int c = 0; c < 64; ++c) kron_store<T, VEC>(g, load_uniform(g.outs + set.out_beg + c), i, j, out[c]);
}


template <class T>
static hipError_t launch_combine_t(const CombineStage& cs, const char* desc, const void* A, const void* B, void* C,
                                   void* ws, bool vec_in, bool vec_out, const CScale& sc, hipStream_t s) {
  if (cs.sets.empty()) return hipSuccess;
  CombArgs<T> g;
  g.A = static_cast<const T*>(A);
  g.B = static_cast<const T*>(B);
  g.C = static_cast<T*>(C);
  g.ws = static_cast<T*>(ws);
  g.sets = img_at<CombSet>(desc, cs.img_sets);
  g.ins = img_at<CombIn>(desc, cs.img_ins);
  g.outs = img_at<CombOut>(desc, cs.img_outs);
  g.coef = img_at<double>(desc, cs.img_coef);
  g.m = (int)cs.m;
  g.vec_in = vec_in ? 1 : 0;
  g.vec_out = vec_out ? 1 : 0;
  g.scale_c = sc.plain() ? 0 : 1;
  g.alpha = (T)sc.alpha;
  g.beta = (T)sc.beta;
  // every set's block size is a multiple of the leaf step (16), so of every VEC
  const int64_t mm = cs.kron3 ? cs.m * cs.m : cs.elems_max;
  auto grid = [&](int vec) { return dim3((unsigned)((mm / vec + 255) / 256), (unsigned)cs.sets.size(), 1); };
  if (cs.kron3) {
    constexpr int V = sizeof(T) == 8 ? 1 : 2;
    if (cs.kpost)
      hipLaunchKernelGGL((kron3_post<T, V>), grid(V), dim3(256), 0, s, g);
    else
      hipLaunchKernelGGL((kron3_pre<T, V>), grid(V), dim3(256), 0, s, g);
    return hipGetLastError();
  }
  // many inputs, few outputs: outputs in registers, inputs streamed with wide loads
  if (cs.nin >= 27 && cs.nout_max <= 16) {
    switch (cs.nin) {
#define MF_COMB_ACC_CASE(N, NO)                                                                   \
  case N:                                                                                         \
    if (cs.nout_max <= NO) {                                                                      \
      hipLaunchKernelGGL((combine_acc<T, N, NO, 4>), grid(4), dim3(256), 0, s, g);                \
      return hipGetLastError();                                                                   \
    }                                                                                             \
    break;
      MF_COMB_ACC_CASE(27, 9)
      MF_COMB_ACC_CASE(36, 9)
      MF_COMB_ACC_CASE(49, 16)
      MF_COMB_ACC_CASE(64, 16)
      MF_COMB_ACC_CASE(81, 9)
#undef MF_COMB_ACC_CASE
      default:
        break;
    }
  }
  switch (cs.nin) {
#define MF_COMB_CASE(N, V) \
  case N: hipLaunchKernelGGL((combine<T, N, V>), grid(V), dim3(256), 0, s, g); break;
    MF_COMB_CASE(1, 4)
    MF_COMB_CASE(4, 4)
    MF_COMB_CASE(6, 4)
    MF_COMB_CASE(7, 4)
    MF_COMB_CASE(8, 4)
    MF_COMB_CASE(9, 4)
    MF_COMB_CASE(11, 4)
    MF_COMB_CASE(12, 4)
    MF_COMB_CASE(16, 4)
    MF_COMB_CASE(17, 2)
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
    case 1: case 4: case 6: case 7: case 8: case 9: case 11: case 12: case 16: case 17: case 27: case 36: case 49:
    case 64:
    case 81:
      return true;
    default: return false;
  }
}

hipError_t launch_combine(const CombineStage& cs, const char* desc, int elem, const void* A, const void* B, void* C,
                          void* ws, bool vec_in, bool vec_out, const CScale& sc, hipStream_t s) {
  return elem == 8 ? launch_combine_t<double>(cs, desc, A, B, C, ws, vec_in, vec_out, sc, s)
                   : launch_combine_t<float>(cs, desc, A, B, C, ws, vec_in, vec_out, sc, s);
}

}  // namespace mf
