// diag.hip -- deterministic on-device reductions for diagnostics: volume
// integrals of operator results (the divergence and curl of Section 4.7
// integrate to zero because every edge flux enters its two end nodes with
// opposite signs) and error norms against a reference.
//
// Determinism: rows are split into a fixed number of contiguous parts; each
// part is reduced in row order (a fixed tree inside a workgroup for the
// norms), the parts are then summed in part order.  All sums are FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "atlas_diag.h"
#include "internal.h"

namespace atlasx {
namespace {

constexpr int kParts = 1024;  // row partition of both reductions
constexpr int kBlock = 256;

// Partials of the volume integral that allocates nothing: one static array
// per GPU, held until the process ends (4 MiB).  Host code never names it
// in a launch: its device address is looked up once per device below.
static __device__ __align__(256) double scratch[kParts * ATLAS_DIAG_NOALLOC_MAX_COLS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with that device current).
atlas_status scratch_on_current_device(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ATLAS_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return ATLAS_OK;
}

// max that keeps a NaN (fmax would drop it)
__device__ __forceinline__ double nanmax(double a, double b) {
  return (a != a) ? a : (b != b) ? b : fmax(a, b);
}

// partial[b][j] = sum over positions p of part b (in order) of
// vol[p] * field[perm[p]][j], for the cols = nlev * ncomp columns.
template <class T>
__global__ void __launch_bounds__(kBlock) k_vol_partial(const int32_t *__restrict__ perm,
                                                         const double *__restrict__ vol,
                                                         const T *__restrict__ field, int V,
                                                         int cols, double *__restrict__ partial) {
  const int b = blockIdx.x;
  const int j = blockIdx.y * kBlock + threadIdx.x;
  if (j >= cols) return;
  const int p0 = (int)((int64_t)V * b / kParts), p1 = (int)((int64_t)V * (b + 1) / kParts);
  double acc = 0.0;
  for (int p = p0; p < p1; ++p) {
    const size_t row = (size_t)perm[p] * (size_t)cols;
    acc = acc + vol[p] * (double)field[row + j];
  }
  partial[(size_t)b * cols + j] = acc;
}

__global__ void __launch_bounds__(kBlock) k_parts_sum(const double *__restrict__ partial,
                                                       int cols, double *__restrict__ out) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int b = 0; b < kParts; ++b) s = s + partial[(size_t)b * cols + j];
  out[j] = s;
}

// Per part and component: max|d|, sum d^2, max|r|, sum r^2 with d = g - r.
template <class TG, class TR>
__global__ void __launch_bounds__(kBlock) k_norm_partial(const TG *__restrict__ got,
                                                          const TR *__restrict__ ref, int64_t n,
                                                          int ncomp, double *__restrict__ partial) {
  __shared__ double sh[4][2][kBlock];
  const int b = blockIdx.x, t = threadIdx.x;
  const int64_t r0 = n * b / kParts, r1 = n * (b + 1) / kParts;
  double a[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  for (int64_t r = r0 + t; r < r1; r += kBlock) {
    for (int c = 0; c < ncomp; ++c) {
      const double rv = (double)ref[r * ncomp + c];
      const double d = (double)got[r * ncomp + c] - rv;
      a[c][0] = nanmax(a[c][0], fabs(d));
      a[c][1] = a[c][1] + d * d;
      a[c][2] = nanmax(a[c][2], fabs(rv));
      a[c][3] = a[c][3] + rv * rv;
    }
  }
  for (int c = 0; c < 2; ++c)
    for (int q = 0; q < 4; ++q) sh[q][c][t] = a[c][q];
  __syncthreads();
  // fixed pairwise tree
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (t < w) {
      for (int c = 0; c < 2; ++c) {
        sh[0][c][t] = nanmax(sh[0][c][t], sh[0][c][t + w]);
        sh[1][c][t] = sh[1][c][t] + sh[1][c][t + w];
        sh[2][c][t] = nanmax(sh[2][c][t], sh[2][c][t + w]);
        sh[3][c][t] = sh[3][c][t] + sh[3][c][t + w];
      }
    }
    __syncthreads();
  }
  if (t < 4 * ncomp) {
    const int c = t / 4, q = t % 4;
    partial[(size_t)b * 4 * ncomp + t] = sh[q][c][0];
  }
}

__global__ void __launch_bounds__(kBlock) k_norm_final(const double *__restrict__ partial,
                                                        int ncomp, double *__restrict__ out) {
  const int t = threadIdx.x;
  if (t >= 4 * ncomp) return;
  const int q = t % 4;
  double s = 0.0;
  for (int b = 0; b < kParts; ++b) {
    const double v = partial[(size_t)b * 4 * ncomp + t];
    s = (q == 0 || q == 2) ? nanmax(s, v) : s + v;
  }
  out[t] = s;
}

template <class TG, class TR>
atlas_status launch_norms(const void *got, const void *ref, int64_t n, int ncomp, double *part,
                          double *out, hipStream_t st) {
  hipLaunchKernelGGL((k_norm_partial<TG, TR>), dim3(kParts), dim3(kBlock), 0, st,
                     static_cast<const TG *>(got), static_cast<const TR *>(ref), n, ncomp, part);
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kBlock), 0, st, (const double *)part, ncomp, out);
  ATLASX_HIP(hipGetLastError());
  return ATLAS_OK;
}

atlas_status check_volume_args(atlas_mesh_t mesh, const void *field, int32_t nlev,
                               int32_t ncomp, atlas_dtype dtype, const double *out) {
  if (!mesh || !mesh->store || !field || !out) return fail(ATLAS_EINVAL, "NULL argument");
  if (nlev < 1) return fail(ATLAS_EINVAL, "nlev must be >= 1");
  if (ncomp != 1 && ncomp != 2) return fail(ATLAS_EINVAL, "ncomp must be 1 or 2");
  if (dtype != ATLAS_F32 && dtype != ATLAS_F64) return fail(ATLAS_EINVAL, "unknown dtype");
  const size_t w = dtype == ATLAS_F64 ? 8 : 4;
  if ((uintptr_t)field % w || (uintptr_t)out % 8)
    return fail(ATLAS_EINVAL, "pointer not aligned to its element size");
  if ((int64_t)mesh->store->d.V * nlev * ncomp >= ((int64_t)1 << 40))
    return fail(ATLAS_EINVAL, "field too large");
  return ATLAS_OK;
}

// Partials into part[kParts][cols], then their sum in part order into out.
hipError_t launch_volume(const DevMesh &m, const void *field, int cols, atlas_dtype dtype,
                         double *part, double *out, hipStream_t stream) {
  const dim3 grid(kParts, (cols + kBlock - 1) / kBlock);
  if (dtype == ATLAS_F64)
    hipLaunchKernelGGL(k_vol_partial<double>, grid, dim3(kBlock), 0, stream, m.perm, m.vol,
                       static_cast<const double *>(field), m.V, cols, part);
  else
    hipLaunchKernelGGL(k_vol_partial<float>, grid, dim3(kBlock), 0, stream, m.perm, m.vol,
                       static_cast<const float *>(field), m.V, cols, part);
  hipLaunchKernelGGL(k_parts_sum, dim3((cols + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                     (const double *)part, cols, out);
  return hipGetLastError();
}

}  // namespace
}  // namespace atlasx

using namespace atlasx;

extern "C" {

atlas_status atlas_diag_volume_integral(atlas_mesh_t mesh, const void *field, int32_t nlev,
                                        int32_t ncomp, atlas_dtype dtype, double *out,
                                        hipStream_t stream) {
  const atlas_status c = check_volume_args(mesh, field, nlev, ncomp, dtype, out);
  if (c != ATLAS_OK) return c;
  const int cols = nlev * ncomp;
  double *part = nullptr;
  if (hipMallocAsync((void **)&part, sizeof(double) * kParts * (size_t)cols, stream) != hipSuccess)
    return fail(ATLAS_ENOMEM, "diagnostics temporary");
  const hipError_t e = launch_volume(mesh->store->d, field, cols, dtype, part, out, stream);
  (void)hipFreeAsync(part, stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics launch");
  return ATLAS_OK;
}

atlas_status atlas_diag_volume_integral_noalloc(atlas_mesh_t mesh, const void *field,
                                                int32_t nlev, int32_t ncomp, atlas_dtype dtype,
                                                double *out, hipStream_t stream) {
  const atlas_status c = check_volume_args(mesh, field, nlev, ncomp, dtype, out);
  if (c != ATLAS_OK) return c;
  const int64_t cols = (int64_t)nlev * ncomp;
  if (cols > ATLAS_DIAG_NOALLOC_MAX_COLS)
    return fail(ATLAS_EINVAL, "nlev * ncomp = " + std::to_string(cols) +
                                  " exceeds the static workspace's " +
                                  std::to_string(ATLAS_DIAG_NOALLOC_MAX_COLS) + " columns");
  int dev = -1;
  ATLASX_HIP(hipGetDevice(&dev));
  if (dev != mesh->store->device) return fail(ATLAS_EINVAL, "mesh lives on another device");
  double *part = nullptr;
  const atlas_status sp = scratch_on_current_device(dev, &part);
  if (sp != ATLAS_OK) return sp;
  // every partial the sum reads is written by the partial kernel first:
  // nothing to clear
  const hipError_t e = launch_volume(mesh->store->d, field, (int)cols, dtype, part, out, stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics launch");
  return ATLAS_OK;
}

atlas_status atlas_diag_error_norms(const void *got, atlas_dtype got_dtype, const void *ref,
                                    atlas_dtype ref_dtype, int64_t n, int32_t ncomp,
                                    double *out, hipStream_t stream) {
  if (!got || !ref || !out) return fail(ATLAS_EINVAL, "NULL argument");
  if (n < 1) return fail(ATLAS_EINVAL, "n must be >= 1");
  if (ncomp != 1 && ncomp != 2) return fail(ATLAS_EINVAL, "ncomp must be 1 or 2");
  if ((got_dtype != ATLAS_F32 && got_dtype != ATLAS_F64) ||
      (ref_dtype != ATLAS_F32 && ref_dtype != ATLAS_F64))
    return fail(ATLAS_EINVAL, "unknown dtype");
  if ((uintptr_t)got % (got_dtype == ATLAS_F64 ? 8 : 4) ||
      (uintptr_t)ref % (ref_dtype == ATLAS_F64 ? 8 : 4) || (uintptr_t)out % 8)
    return fail(ATLAS_EINVAL, "pointer not aligned to its element size");
  double *part = nullptr;
  if (hipMallocAsync((void **)&part, sizeof(double) * kParts * 4 * (size_t)ncomp, stream) !=
      hipSuccess)
    return fail(ATLAS_ENOMEM, "diagnostics temporary");
  atlas_status s;
  if (got_dtype == ATLAS_F64 && ref_dtype == ATLAS_F64)
    s = launch_norms<double, double>(got, ref, n, ncomp, part, out, stream);
  else if (got_dtype == ATLAS_F32 && ref_dtype == ATLAS_F64)
    s = launch_norms<float, double>(got, ref, n, ncomp, part, out, stream);
  else if (got_dtype == ATLAS_F64 && ref_dtype == ATLAS_F32)
    s = launch_norms<double, float>(got, ref, n, ncomp, part, out, stream);
  else
    s = launch_norms<float, float>(got, ref, n, ncomp, part, out, stream);
  (void)hipFreeAsync(part, stream);
  return s;
}

}  // extern "C"
