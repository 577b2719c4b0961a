// The fast product for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): mf_fastmm with the plan's descriptor image and its workspace
// placed in one fixed device array per GPU instead of the library's pool and
// the plan's own device copy.
#include <mutex>
#include <string>

#include "mf_internal.h"

namespace mf {
namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // MF_NOALLOC_SCRATCH_BYTES

// Every GPU the library runs on holds its own copy of this array until the
// process ends.  In host code its name is only a stand-in: the device address
// of the copy on the current GPU comes from hipGetSymbolAddress (scratch_base).
static __device__ __align__(256) char scratch[kScratchBytes];

struct ScratchAddr {
  std::once_flag once;
  hipError_t err = hipSuccess;
  char* ptr = nullptr;
};
ScratchAddr g_scratch[kMaxDevices];

// Device address of the array on the current device, looked up once per
// device (with that device current) on its first call.
mf_status scratch_base(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MF_ERR_HIP, "hipGetDevice failed");
  }
  if (dev < 0 || dev >= kMaxDevices) return fail(MF_ERR_UNSUPPORTED, "device index beyond the supported range");
  ScratchAddr& s = g_scratch[dev];
  std::call_once(s.once, [&]() {
    void* p = nullptr;
    s.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (s.err != hipSuccess)
      (void)hipGetLastError();
    else
      s.ptr = static_cast<char*>(p);
  });
  if (s.err != hipSuccess || !s.ptr)
    return fail(MF_ERR_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(s.err));
  *out = s.ptr;
  return MF_OK;
}

}  // namespace
}  // namespace mf

using namespace mf;

extern "C" mf_status mf_fastmm_noalloc(const mf_algo* algo, int depth, int cutoff, const void* A, const void* B,
                                       void* C, int64_t n, int dtype, mf_stream stream) {
  clear_error();
  mf_status st = check_request(algo, true, depth, cutoff, A, B, C, n, dtype);
  if (st != MF_OK || n == 0) return st;
  std::shared_ptr<const Plan> pl;
  st = plan_for(algo, depth, cutoff, n, dtype, &pl,
                ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) != 0);
  if (st != MF_OK) return st;
  // [descriptor image | workspace], the workspace 256-byte aligned
  size_t img = (pl->image.size() + 255) / 256 * 256;
  size_t need = img + pl->ws_bytes;
  if (need > kScratchBytes) {
    // rows that are not 16-byte aligned: the plan that reads them in place
    // takes no workspace blocks for copies of them
    Shape sh = Shape::sq(n);
    sh.no_copy = true;
    st = get_plan(depth > 0 ? algo : nullptr, depth, cutoff, sh, dtype, kStandaloneMinWorkgroups, &pl);
    if (st != MF_OK) return st;
    img = (pl->image.size() + 255) / 256 * 256;
    need = img + pl->ws_bytes;
  }
  if (need > kScratchBytes)
    return fail(MF_ERR_SHAPE, "request needs " + std::to_string(need) + " bytes of scratch (descriptors " +
                                  std::to_string(pl->image.size()) + ", workspace " + std::to_string(pl->ws_bytes) +
                                  "), beyond the fixed limit of " + std::to_string(kScratchBytes) + " bytes");
  char* base = nullptr;
  st = scratch_base(&base);
  if (st != MF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(base, pl->image.data(), pl->image.size(), hipMemcpyHostToDevice, s) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MF_ERR_HIP, "copy of the plan descriptors into the scratch array failed");
  }
  return run_at(*pl, base, A, B, C, pl->ws_bytes > 0 ? base + img : nullptr, s, /*may_time=*/false);
}
