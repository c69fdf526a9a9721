// chase_filter_noalloc: the Chebyshev filter of chase_filter (Alg. 4 with
// per-vector degrees) for callers that cannot allocate device memory.  Its
// step buffers and the GEMM remainder split's partial tiles live in one
// static device array per GPU, `scratch`; nothing is allocated per call.
#include <mutex>

#include "kernels.hpp"
#include "solver.hpp"

namespace chase {

constexpr size_t kNoallocScratchBytes = CHASE_FILTER_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

// Device address of `scratch` on each GPU, looked up once per device with
// that device current (the host symbol is only a stand-in for it).
constexpr int kNoallocMaxDevices = 64;
static void *g_scratch_addr[kNoallocMaxDevices];
static hipError_t g_scratch_status[kNoallocMaxDevices];
static std::once_flag g_scratch_once[kNoallocMaxDevices];

static void *scratch_address(int dev) {
  std::call_once(g_scratch_once[dev], [dev] {
    void *p = nullptr;
    g_scratch_status[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_addr[dev] = g_scratch_status[dev] == hipSuccess ? p : nullptr;
  });
  if (g_scratch_status[dev] != hipSuccess) {
    set_error(std::string("hipGetSymbolAddress(scratch): ") +
              hipGetErrorString(g_scratch_status[dev]));
    return nullptr;
  }
  return g_scratch_addr[dev];
}

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace chase

using namespace chase;

extern "C" chase_status chase_filter_noalloc(chase_dtype dtype, const void *H, int64_t N,
                                             int64_t ldh, const void *V, int64_t ldv,
                                             int32_t ncols, const int32_t *deg, double c,
                                             double e, double gamma, void *out, int64_t ldo,
                                             void *stream) {
  if (dtype != CHASE_REAL64 && dtype != CHASE_COMPLEX128) {
    set_error("unknown dtype");
    return CHASE_EINVAL;
  }
  if (N < 1 || N > 2147483647LL || ncols < 0 || ncols > N || ldh < N || ldv < N || ldo < N) {
    set_error("invalid sizes");
    return CHASE_EINVAL;
  }
  if (ncols == 0) return CHASE_OK;  // nothing is read or written
  if (!H || !V || !out || !deg) {
    set_error("NULL argument");
    return CHASE_EINVAL;
  }
  if (!(e > 0.0)) {
    set_error("half-width e must be > 0");
    return CHASE_EINVAL;
  }
  for (int a = 0; a < ncols; ++a)
    if (deg[a] < 1 || (a > 0 && deg[a] < deg[a - 1])) {
      set_error("degrees must be >= 1 and ascending");
      return CHASE_EINVAL;
    }
  const bool cplx = dtype == CHASE_COMPLEX128;
  const size_t es = cplx ? 16 : 8;
  const size_t buf = align256(es * (size_t)N * (size_t)ncols);
  if (3 * buf > kNoallocScratchBytes) {
    set_error("chase_filter_noalloc: 3 N ncols x " + std::to_string(es) + " bytes = " +
              std::to_string(3 * buf) + " exceed the scratch of " +
              std::to_string(kNoallocScratchBytes) + " bytes (use chase_filter)");
    return CHASE_EINVAL;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoallocMaxDevices) {
    (void)hipGetLastError();
    set_error("chase_filter_noalloc: no usable current device");
    return CHASE_EDEVICE;
  }
  char *base = (char *)scratch_address(dev);
  if (base == nullptr) return CHASE_EDEVICE;
  // three step buffers (N x ncols, leading dimension N); what is left over
  // holds the remainder split's partial tiles (the launcher does not split
  // when they would not fit)
  void *const bufs[3] = {base, base + buf, base + 2 * buf};
  void *tail = base + 3 * buf;
  const size_t tail_bytes = kNoallocScratchBytes - 3 * buf;
  try {
    filter_enqueue((hipStream_t)stream, tail_bytes ? tail : nullptr, tail_bytes, cplx, false, H,
                   ldh, N, V, ldv, bufs, N, ncols, deg, c, e, gamma, out, ldo);
  } catch (const DeviceError &) {
    return CHASE_EDEVICE;
  } catch (...) {
    set_error("chase_filter_noalloc: internal error");
    return CHASE_EINTERNAL;
  }
  return CHASE_OK;
}
