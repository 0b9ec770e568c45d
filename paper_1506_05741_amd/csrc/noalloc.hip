// Entry point for callers that cannot allocate device memory: the stopping
// errors of Section 3.3 for caller-held moments, with the reduction partials
// in a file-scope device array instead of a workspace.
#include <math.h>
#include <stdarg.h>

#include <mutex>

#include "../../include/diam.h"
#include "kernels.h"

int diam_fail_v(int code, const char* fmt, va_list ap);

namespace {

int nfail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  diam_fail_v(code, fmt, ap);
  va_end(ap);
  return code;
}

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_scratch[MAX_DEVICES];  // device address of `scratch` on each device (null until looked up)

}  // namespace

// The partials and the two results of dk::moment_error (24.6 KB; every GPU
// the library runs on holds its own copy until the process ends).  In host
// code this name is not a device address: kernels and copies get the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[dk::MERR_SCRATCH_DOUBLES];

// Device address of `scratch` on the current device, looked up once per device.
static int scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return nfail(DIAM_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) return nfail(DIAM_E_ARG, "device %d beyond the %d supported", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return nfail(DIAM_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return DIAM_OK;
}

extern "C" int diam_moment_error_noalloc(const double* S, const double* m, int32_t d, const double* Sigma,
                                         const double* mu, double* cov_rel, double* mean_abs, void* hip_stream) {
  if (!S || !m || !Sigma || !cov_rel) return nfail(DIAM_E_ARG, "null argument");
  if (d < 1) return nfail(DIAM_E_ARG, "d = %d: must be >= 1", (int)d);
  // the grid is capped at MERR_BLOCKS workgroups whatever d is, so the
  // partials of any d fit the array; the check guards the layout itself
  const long nb = ((long)d * d + 255) / 256 < dk::MERR_BLOCKS ? ((long)d * d + 255) / 256 : dk::MERR_BLOCKS;
  if (2 + 3 * (size_t)nb > dk::MERR_SCRATCH_DOUBLES)
    return nfail(DIAM_E_ARG, "d = %d needs %ld partial sums, beyond the %d the static buffer holds", (int)d, nb,
                 dk::MERR_BLOCKS);
  double* ptr = nullptr;
  int r = scratch_on_current_device(&ptr);
  if (r) return r;
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = dk::moment_error(S, m, Sigma, mu, d, ptr, s);
  if (e != hipSuccess) return nfail(DIAM_E_HIP, "moment_error: %s", hipGetErrorString(e));
  double h[2];
  e = hipMemcpyAsync(h, ptr, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return nfail(DIAM_E_HIP, "reading the stopping errors: %s", hipGetErrorString(e));
  *cov_rel = h[0];
  if (mean_abs) *mean_abs = mu ? h[1] : NAN;
  return DIAM_OK;
}
