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
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int64_t mm = (int64_t)g.m * g.m;
  if (e >= mm) return;
  const int i = (int)(e / g.m), j = (int)(e % g.m);
  const CombSet set = load_uniform(g.sets + blockIdx.y);
  if (set.full && g.vec_in && g.vec_out)
    combine_body<T, NIN, VEC, true>(g, set, i, j);
  else
    combine_body<T, NIN, VEC, false>(g, set, i, j);
}

// Outputs in registers, inputs streamed (many inputs, at most NOUT outputs
// per set).
template <class T, int NIN, int NOUT, int VEC>
__global__ void __launch_bounds__(256) combine_acc(CombArgs<T> g) {
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int64_t mm = (int64_t)g.m * g.m;
  if (e >= mm) return;
  const int i = (int)(e / g.m), j = (int)(e % g.m);
  const CombSet set = load_uniform(g.sets + blockIdx.y);
  if (set.full && g.vec_in && g.vec_out)
    combine_acc_body<T, NIN, NOUT, VEC, true>(g, set, i, j);
  else
    combine_acc_body<T, NIN, NOUT, VEC, false>(g, set, i, j);
}

#ifndef MF_COMB_VEC_SMALL
#define MF_COMB_VEC_SMALL 4
#endif

template <class T>
static hipError_t launch_combine_t(const CombineStage& cs, const void* A, const void* B, void* C, void* ws,
                                   bool vec_in, bool vec_out, hipStream_t s) {
  if (cs.sets.empty()) return hipSuccess;
  CombArgs<T> g;
  g.A = static_cast<const T*>(A);
  g.B = static_cast<const T*>(B);
  g.C = static_cast<T*>(C);
  g.ws = static_cast<T*>(ws);
  g.sets = cs.d_sets;
  g.ins = cs.d_ins;
  g.outs = cs.d_outs;
  g.coef = cs.d_coef;
  g.m = (int)cs.m;
  g.vec_in = vec_in ? 1 : 0;
  g.vec_out = vec_out ? 1 : 0;
  const int64_t mm = cs.m * cs.m;
  auto grid = [&](int vec) { return dim3((unsigned)((mm / vec + 255) / 256), (unsigned)cs.sets.size(), 1); };
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
    MF_COMB_CASE(4, MF_COMB_VEC_SMALL)
    MF_COMB_CASE(7, MF_COMB_VEC_SMALL)
    MF_COMB_CASE(8, MF_COMB_VEC_SMALL)
    MF_COMB_CASE(9, MF_COMB_VEC_SMALL)
    MF_COMB_CASE(16, MF_COMB_VEC_SMALL)
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
    case 4: case 7: case 8: case 9: case 16: case 27: case 36: case 49: case 64: case 81: return true;
    default: return false;
  }
}

hipError_t launch_combine(const CombineStage& cs, int elem, const void* A, const void* B, void* C, void* ws,
                          bool vec_in, bool vec_out, hipStream_t s) {
  return elem == 8 ? launch_combine_t<double>(cs, A, B, C, ws, vec_in, vec_out, s)
                   : launch_combine_t<float>(cs, A, B, C, ws, vec_in, vec_out, s);
}

}  // namespace mf
