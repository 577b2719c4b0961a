// Counter-based operand generator for the serving runtime: element i of a
// request's operand is a function of (seed, i) only, so a request's inputs
// are identical whether it runs alone or among others.
//
// Generator: the SplitMix64 output function (Steele, Lea and Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014) applied to
// the counter state seed + (i + 1) * 0x9e3779b97f4a7c15; the top 53 bits give
// u in [0, 1) and the element is 2u - 1 (uniform in [-1, 1)), rounded to the
// storage type.
#include "mf_internal.h"

namespace mf {

namespace {

__device__ __forceinline__ uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <class T>
__global__ void fill_uniform(T* p, int64_t count, uint64_t seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const uint64_t z = splitmix_out(seed + (uint64_t)(i + 1) * 0x9e3779b97f4a7c15ull);
    const double u = (double)(z >> 11) * 0x1.0p-53;
    p[i] = (T)(2.0 * u - 1.0);
  }
}

}  // namespace

hipError_t launch_fill_uniform(void* p, int64_t count, int elem, uint64_t seed, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 8192);
  if (elem == 8)
    hipLaunchKernelGGL(fill_uniform<double>, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<double*>(p), count,
                       seed);
  else
    hipLaunchKernelGGL(fill_uniform<float>, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<float*>(p), count,
                       seed);
  return hipGetLastError();
}

}  // namespace mf
