// bkwd_true_residual_noalloc: the true residual of Sec. 4.3 with no device
// allocation and no caller workspace, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).
//
// The residual kernel computes ||b_i - D x_i||^2 and ||b_i||^2 per column
// without storing b - D x; its per-workgroup partial sums and the two-stage
// reduction live in `scratch`, a file-scope device array of fixed size that
// each GPU holds until the process ends.  Its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is handed to kernels and copies.  Every call on a GPU uses
// the same array: each call overwrites all of the partial sums it reads, so
// nothing has to be cleared, and calls that overlap on one GPU race.
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/bkwd.h"
#include "bkwd_internal.h"
#include "blas.h"

namespace {

// partial sums [kResidualBlocks][2 L], reduction staging, reduced [2 L]
constexpr size_t kPartDoubles = (size_t)kResidualBlocks * 2 * BKWD_MAX_RHS;
constexpr size_t kStageHalf = 8 * 2 * BKWD_MAX_RHS;
constexpr size_t kOutDoubles = 2 * BKWD_MAX_RHS;
constexpr size_t kScratchDoubles = kPartDoubles + 2 * kStageHalf + kOutDoubles;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_dev_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first
// call there), or nullptr with *err set
double* scratch_ptr(std::string* err) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *err = std::string("hipGetDevice: ") + (e != hipSuccess ? hipGetErrorString(e) : "device index out of range");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_dev_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_dev_ptr[dev] = static_cast<double*>(p);
  }
  return g_dev_ptr[dev];
}

}  // namespace

static_assert(kScratchDoubles * sizeof(double) == BKWD_NOALLOC_SCRATCH_BYTES,
              "the header states the size of the static scratch");

int true_residual_noalloc(LatticeImpl& lat, int L, const cpx<double>* B, const cpx<double>* X, double* per_col,
                          hipStream_t s, std::string* err) {
  const int grid = residual_grid(lat.g.vol, L);
  const size_t nv = 2 * (size_t)L;
  const long long nsplit = (grid + 255) / 256;
  if ((size_t)grid * nv > kPartDoubles || (size_t)nsplit * nv > kStageHalf || nv > kOutDoubles) {
    *err = "L or the lattice exceeds the static scratch of bkwd_true_residual_noalloc";
    return BKWD_EINVAL;
  }
  double* base = scratch_ptr(err);
  if (base == nullptr) return BKWD_EDEVICE;
  double* part = base;
  double* stage = base + kPartDoubles;
  double* out = stage + 2 * kStageHalf;
  int nblk = 0;
  hipError_t e = launch_residual_norms64(lat, 0, L, B, X, part, &nblk, s);
  if (e == hipSuccess) e = launch_reduce(part, nblk, (int)nv, stage, kStageHalf, out, s);
  double* host = reinterpret_cast<double*>(lat.host_scratch);
  if (e == hipSuccess) e = hipMemcpyAsync(host, out, nv * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    *err = std::string("true residual (no allocation): ") + hipGetErrorString(e);
    return BKWD_EDEVICE;
  }
  for (int i = 0; i < L; ++i) per_col[i] = host[L + i] > 0.0 ? std::sqrt(host[i] / host[L + i]) : INFINITY;
  return BKWD_OK;
}
