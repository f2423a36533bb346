// remap.hip -- interpolation of nodal fields from a source mesh to other
// points (Section 1: remapping / interpolation between grids).  Method: the
// piecewise-linear interpolant on the source triangles in the (lon, lat)
// plane; targets poleward of a polar parallel interpolate along it (the
// header atlas_remap.h states the method in full).
//
// Two kernels:
//  * location (setup, once per remap): one thread per target finds its strip
//    by a binary search over the parallels' latitudes, then walks the few
//    triangles of the strip's triangulation that can hold it and keeps the
//    one whose smallest barycentric coordinate is largest (the first such
//    in strip order), giving one 48-byte record per target;
//  * apply (the hot path): an HBM-bound gather, three source rows per
//    target row; short rows (under 64 columns) take one thread per (target,
//    column) element so every lane is busy, long rows one wavefront per row;
//    workgroups are mapped to XCDs in contiguous runs of targets so
//    neighbouring targets, which share source rows, share an L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "atlas_remap.h"
#include "internal.h"

namespace atlasx {

static_assert(sizeof(RemapRec) == 48, "remap record is 48 bytes");

namespace {

constexpr double kTwoPi = 6.283185307179586476925;
constexpr int kLocBlock = 256;
constexpr int kApplyBlock = 256;
constexpr int kXcds = 8;

// z-component of (q - p) x (r - p): twice the signed area of (p, q, r)
__device__ __forceinline__ double area2(double px, double py, double qx, double qy, double rx,
                                        double ry) {
  return (qx - px) * (ry - py) - (qy - py) * (rx - px);
}

// largest i in [0, n) with lon[o + i] <= x (lon[o] = 0 <= x)
__device__ __forceinline__ int32_t bracket(const double *__restrict__ lon, int64_t o, int32_t n,
                                           double x) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (lon[o + mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The walk between parallels of nu (upper) and nl (lower) points: at state
// (a, b) the next triangle takes the upper parallel's next point iff
// (a+1)/nu < (b+1)/nl, ties to the parallel with more points, the lower one
// if counts are equal.  States run from (0, 0) to (nu, nl) (unwrapped).
__device__ __forceinline__ bool takes_upper(int64_t a, int64_t b, int64_t nu, int64_t nl) {
  if (a == nu) return false;
  if (b == nl) return true;
  const int64_t lhs = (a + 1) * nl, rhs = (b + 1) * nu;
  return lhs < rhs || (lhs == rhs && nu > nl);
}
// b at the first state with a == A (the walk's b when it first reaches A)
__device__ __forceinline__ int64_t b_enter(int64_t A, int64_t nu, int64_t nl) {
  if (A == 0) return 0;
  const int64_t q = A * nl;
  return q / nu - ((q % nu == 0 && nu > nl) ? 1 : 0);
}
// a at the first state with b == B
__device__ __forceinline__ int64_t a_enter(int64_t B, int64_t nu, int64_t nl) {
  if (B == 0) return 0;
  const int64_t q = B * nu;
  return q / nl - ((q % nl == 0 && nu <= nl) ? 1 : 0);
}

__global__ void __launch_bounds__(kLocBlock)
    k_remap_locate(int32_t nr, const int64_t *__restrict__ off, const double *__restrict__ rlat,
                   const double *__restrict__ lon, const double *__restrict__ tlon,
                   const double *__restrict__ tlat, int64_t nt, RemapRec *__restrict__ rec,
                   int32_t *__restrict__ polar_flag) {
  const int64_t t = (int64_t)blockIdx.x * kLocBlock + threadIdx.x;
  if (t >= nt) return;
  double x = fmod(tlon[t], kTwoPi);
  if (x < 0.0) x += kTwoPi;
  if (x >= kTwoPi) x = 0.0;
  const double y = tlat[t];
  RemapRec r;
  r.w[3] = 0.0;
  if (y > rlat[0] || y < rlat[nr - 1]) {
    // polar cap: linear along the polar parallel
    const int32_t j = y > rlat[0] ? 0 : nr - 1;
    const int64_t o = off[j];
    const int32_t n = (int32_t)(off[j + 1] - o);
    const int32_t i = bracket(lon, o, n, x);
    const double x0 = lon[o + i];
    const double x1 = i + 1 < n ? lon[o + i + 1] : lon[o] + kTwoPi;
    const double s = (x - x0) / (x1 - x0);
    r.i[0] = (int32_t)(o + i);
    r.i[1] = (int32_t)(o + (i + 1) % n);
    r.i[2] = r.i[0];
    r.i[3] = r.i[0];
    r.w[0] = 1.0 - s;
    r.w[1] = s;
    r.w[2] = 0.0;
    rec[t] = r;
    polar_flag[t] = 1;
    return;
  }
  // strip j: the first whose lower parallel is at or below y
  int32_t lo = 0, hi = nr - 2;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (rlat[mid + 1] <= y) hi = mid; else lo = mid + 1;
  }
  const int32_t j = lo;
  const int64_t ou = off[j], nu = off[j + 1] - ou;
  const int64_t ol = off[j + 1], nl = off[j + 2] - ol;
  const int64_t a0 = bracket(lon, ou, (int32_t)nu, x), b0 = bracket(lon, ol, (int32_t)nl, x);
  // A triangle of state (a, b) spans longitudes [min(U_a, L_b),
  // min(U_{a+1}, L_{b+1})], so one holding x has a >= a0 - 1, b >= b0 - 1 and
  // (a <= a0 or b <= b0): a run of consecutive states, walked here with one
  // state of margin on each side.
  const int64_t A1 = a0 >= 2 ? a0 - 2 : 0, B1 = b0 >= 2 ? b0 - 2 : 0;
  int64_t a = A1, b = b_enter(A1, nu, nl);
  {
    const int64_t ab = a_enter(B1, nu, nl);
    if (ab + B1 > a + b) { a = ab; b = B1; }
  }
  double best = -HUGE_VAL;
  int32_t bi[3] = {0, 0, 0};
  double bw[3] = {0.0, 0.0, 0.0};
  while (a + b < nu + nl && (a <= a0 + 1 || b <= b0 + 1)) {
    const bool up = takes_upper(a, b, nu, nl);
    int64_t node[3];
    double X[3], Y[3];
    node[0] = ou + a % nu;
    X[0] = lon[node[0]] + (a == nu ? kTwoPi : 0.0);
    Y[0] = rlat[j];
    node[1] = ol + b % nl;
    X[1] = lon[node[1]] + (b == nl ? kTwoPi : 0.0);
    Y[1] = rlat[j + 1];
    if (up) {
      node[2] = ou + (a + 1) % nu;
      X[2] = lon[node[2]] + (a + 1 >= nu ? kTwoPi : 0.0);
      Y[2] = rlat[j];
    } else {
      node[2] = ol + (b + 1) % nl;
      X[2] = lon[node[2]] + (b + 1 >= nl ? kTwoPi : 0.0);
      Y[2] = rlat[j + 1];
    }
    // barycentric coordinate k: area of the sub-triangle opposite vertex k
    // over the whole, the whole measured from vertex k itself (so a target
    // on vertex k gets exactly 1 there)
    double w[3];
    for (int k = 0; k < 3; ++k) {
      const int k1 = k == 2 ? 0 : k + 1, k2 = k == 0 ? 2 : k - 1;
      const double whole = area2(X[k], Y[k], X[k1], Y[k1], X[k2], Y[k2]);
      const double part = area2(x, y, X[k1], Y[k1], X[k2], Y[k2]);
      w[k] = part / whole;
    }
    const double mn = fmin(w[0], fmin(w[1], w[2]));
    if (mn > best) {
      best = mn;
      for (int k = 0; k < 3; ++k) {
        bi[k] = (int32_t)node[k];
        bw[k] = w[k];
      }
    }
    if (up) ++a; else ++b;
  }
  for (int k = 0; k < 3; ++k) {
    r.i[k] = bi[k];
    r.w[k] = bw[k];
  }
  r.i[3] = bi[0];
  rec[t] = r;
  polar_flag[t] = 0;
}

// out[t][c] = (w0 in[i0][c] + w1 in[i1][c]) + w2 in[i2][c], in FP64.
// Workgroup g of the launch runs on XCD g % 8; it takes logical block
// (g % 8) * per_xcd + g / 8, so each XCD walks one contiguous run of targets.
// The element's target row comes from a floating-point quotient (e < 2^40
// is exact in FP64; the quotient is off by at most one and corrected): a
// 64-bit integer division per element would cost more than its loads.
template <class T>
__global__ void __launch_bounds__(kApplyBlock)
    k_remap_apply(const RemapRec *__restrict__ rec, const T *__restrict__ in, int32_t ncol,
                  double inv_ncol, int64_t nelem, int64_t per_xcd, T *__restrict__ out) {
  const int64_t g = blockIdx.x;
  const int64_t lb = (g % kXcds) * per_xcd + g / kXcds;
  const int64_t e = lb * kApplyBlock + threadIdx.x;
  if (e >= nelem) return;
  int64_t t = (int64_t)((double)e * inv_ncol);
  int64_t c = e - t * ncol;
  if (c < 0) {
    --t;
    c += ncol;
  } else if (c >= ncol) {
    ++t;
    c -= ncol;
  }
  const RemapRec &r = rec[t];
  const double v0 = (double)in[(int64_t)r.i[0] * ncol + c];
  const double v1 = (double)in[(int64_t)r.i[1] * ncol + c];
  const double v2 = (double)in[(int64_t)r.i[2] * ncol + c];
  const double s = r.w[0] * v0 + r.w[1] * v1 + r.w[2] * v2;
  out[e] = (T)s;
}

// Long rows (ncol >= 64): one wavefront per target row, lanes over its
// columns, four column blocks of 64 in flight per lane; the record is read
// once per row with scalar loads.  Same arithmetic per element as the flat
// form, so the same bits.
#define ATLASX_RCST __attribute__((address_space(4)))
template <class T>
__global__ void __launch_bounds__(kApplyBlock)
    k_remap_rows(const RemapRec *__restrict__ rec, const T *__restrict__ in, int32_t ncol,
                 int64_t nt, int64_t per_xcd, T *__restrict__ out) {
  constexpr int kWaves = kApplyBlock / 64, kU = 4;
  const int64_t g = blockIdx.x;
  const int64_t lb = (g % kXcds) * per_xcd + g / kXcds;
  const int64_t t = lb * kWaves + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (t >= nt) return;
  const int lane = threadIdx.x & 63;
  const ATLASX_RCST RemapRec *r = (const ATLASX_RCST RemapRec *)(rec + t);
  const int32_t i0 = r->i[0], i1 = r->i[1], i2 = r->i[2];
  const double w0 = r->w[0], w1 = r->w[1], w2 = r->w[2];
  const T *a = in + (int64_t)i0 * ncol, *b = in + (int64_t)i1 * ncol, *c = in + (int64_t)i2 * ncol;
  T *o = out + t * ncol;
  for (int c0 = 0; c0 < ncol; c0 += 64 * kU) {
    double va[kU], vb[kU], vc[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = c0 + 64 * u + lane;
      const bool on = k < ncol;
      va[u] = on ? (double)a[k] : 0.0;
      vb[u] = on ? (double)b[k] : 0.0;
      vc[u] = on ? (double)c[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = c0 + 64 * u + lane;
      if (k < ncol) o[k] = (T)(w0 * va[u] + w1 * vb[u] + w2 * vc[u]);
    }
  }
}

atlas_status check_targets(int64_t nt, const double *lon, const double *lat) {
  for (int64_t t = 0; t < nt; ++t) {
    if (!std::isfinite(lon[t]) || !std::isfinite(lat[t]))
      return fail(ATLAS_EINVAL, "non-finite target coordinate at " + std::to_string(t));
    if (lat[t] > 0.25 * kTwoPi || lat[t] < -0.25 * kTwoPi)
      return fail(ATLAS_EINVAL, "target latitude outside [-pi/2, pi/2] at " + std::to_string(t));
  }
  return ATLAS_OK;
}

// Locate the targets (device arrays) on the source; fills the plan.
atlas_status build_plan(const MeshStore &src, const double *tlon, const double *tlat,
                        int64_t nt, RemapPlan &plan) {
  int dev = -1;
  ATLASX_HIP(hipGetDevice(&dev));
  if (dev != src.device) return fail(ATLAS_EINVAL, "source mesh lives on another device");
  plan.device = dev;
  plan.nsrc = src.d.V;
  plan.nt = nt;
  ATLASX_HIP(hipMalloc((void **)&plan.rec, sizeof(RemapRec) * (size_t)nt));
  plan.bytes = sizeof(RemapRec) * (size_t)nt;
  int32_t *flag = nullptr;
  ATLASX_HIP(hipMalloc((void **)&flag, sizeof(int32_t) * (size_t)nt));
  const unsigned nblk = (unsigned)((nt + kLocBlock - 1) / kLocBlock);
  hipLaunchKernelGGL(k_remap_locate, dim3(nblk), dim3(kLocBlock), 0, 0, src.rs.nrings,
                     src.rs.ring_off, src.rs.ring_lat, src.node_lon, tlon, tlat, nt, plan.rec,
                     flag);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  std::vector<RemapRec> h;
  std::vector<int32_t> hf;
  if (e == hipSuccess) {
    try {
      h.resize((size_t)nt);
      hf.resize((size_t)nt);
    } catch (const std::bad_alloc &) {
      (void)hipFree(flag);
      return fail(ATLAS_ENOMEM, "out of host memory");
    }
    e = hipMemcpy(h.data(), plan.rec, sizeof(RemapRec) * (size_t)nt, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
      e = hipMemcpy(hf.data(), flag, sizeof(int32_t) * (size_t)nt, hipMemcpyDeviceToHost);
  }
  (void)hipFree(flag);
  if (e != hipSuccess) return hip_fail(e, "remap location");
  // source nodes the weights touch (for the byte model)
  std::vector<uint8_t> seen((size_t)plan.nsrc, 0);
  for (int64_t t = 0; t < nt; ++t) {
    for (int k = 0; k < 3; ++k) {
      const int32_t i = h[t].i[k];
      if (i < 0 || i >= plan.nsrc) return fail(ATLAS_EDEVICE, "remap location out of range");
      if (h[t].w[k] != 0.0) seen[i] = 1;
    }
    plan.npolar += hf[t];
  }
  for (uint8_t s : seen) plan.touched += s;
  return ATLAS_OK;
}

}  // namespace

atlas_status remap_launch(const RemapPlan &p, const void *in, int32_t ncol, atlas_dtype dt,
                          void *out, hipStream_t st) {
  if (ncol >= 64) {
    const int64_t nblk = (p.nt + kApplyBlock / 64 - 1) / (kApplyBlock / 64);
    const int64_t per_xcd = (nblk + kXcds - 1) / kXcds;
    const int64_t grid = per_xcd * kXcds;
    if (grid >= ((int64_t)1 << 31)) return fail(ATLAS_EINVAL, "field too large");
    if (dt == ATLAS_F64)
      hipLaunchKernelGGL(k_remap_rows<double>, dim3((unsigned)grid), dim3(kApplyBlock), 0, st,
                         p.rec, static_cast<const double *>(in), ncol, p.nt, per_xcd,
                         static_cast<double *>(out));
    else
      hipLaunchKernelGGL(k_remap_rows<float>, dim3((unsigned)grid), dim3(kApplyBlock), 0, st,
                         p.rec, static_cast<const float *>(in), ncol, p.nt, per_xcd,
                         static_cast<float *>(out));
    ATLASX_HIP(hipGetLastError());
    return ATLAS_OK;
  }
  const int64_t nelem = p.nt * (int64_t)ncol;
  const int64_t nblk = (nelem + kApplyBlock - 1) / kApplyBlock;
  const int64_t per_xcd = (nblk + kXcds - 1) / kXcds;
  const int64_t grid = per_xcd * kXcds;
  if (grid >= ((int64_t)1 << 31)) return fail(ATLAS_EINVAL, "field too large");
  if (dt == ATLAS_F64)
    hipLaunchKernelGGL(k_remap_apply<double>, dim3((unsigned)grid), dim3(kApplyBlock), 0, st,
                       p.rec, static_cast<const double *>(in), ncol, 1.0 / ncol, nelem, per_xcd,
                       static_cast<double *>(out));
  else
    hipLaunchKernelGGL(k_remap_apply<float>, dim3((unsigned)grid), dim3(kApplyBlock), 0, st,
                       p.rec, static_cast<const float *>(in), ncol, 1.0 / ncol, nelem, per_xcd,
                       static_cast<float *>(out));
  ATLASX_HIP(hipGetLastError());
  return ATLAS_OK;
}

}  // namespace atlasx

using namespace atlasx;

namespace {

atlas_status finish_create(atlasx::RemapPlan *plan, atlas_status st, atlas_remap_t *out) {
  if (st != ATLAS_OK) {
    delete plan;
    return st;
  }
  atlas_remap_t r = new (std::nothrow) atlas_remap_s{plan};
  if (!r) {
    delete plan;
    return fail(ATLAS_ENOMEM, "out of host memory");
  }
  *out = r;
  return ATLAS_OK;
}

atlas_status check_source(atlas_mesh_t source) {
  if (!source || !source->store) return fail(ATLAS_EINVAL, "NULL source mesh");
  if (!source->store->rs.ok)
    return fail(ATLAS_EINVAL,
                "source mesh is not triangulated strip by strip between parallels "
                "(atlas_remap.h describes the meshes a remap starts from)");
  return ATLAS_OK;
}

}  // namespace

extern "C" {

atlas_status atlas_remap_create(atlas_mesh_t source, int64_t ntarget, const double *lon,
                                const double *lat, atlas_remap_t *out) {
  if (!out || !lon || !lat) return fail(ATLAS_EINVAL, "NULL argument");
  atlas_status st = check_source(source);
  if (st != ATLAS_OK) return st;
  if (ntarget < 1 || ntarget >= ((int64_t)1 << 31))
    return fail(ATLAS_EINVAL, "ntarget must be in [1, 2^31)");
  if ((st = check_targets(ntarget, lon, lat)) != ATLAS_OK) return st;
  RemapPlan *plan = new (std::nothrow) RemapPlan();
  if (!plan) return fail(ATLAS_ENOMEM, "out of host memory");
  double *d = nullptr;
  if (hipMalloc((void **)&d, sizeof(double) * 2 * (size_t)ntarget) != hipSuccess) {
    delete plan;
    return fail(ATLAS_ENOMEM, "remap target coordinates");
  }
  hipError_t e = hipMemcpy(d, lon, sizeof(double) * ntarget, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(d + ntarget, lat, sizeof(double) * ntarget, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    delete plan;
    return hip_fail(e, "remap target upload");
  }
  st = build_plan(*source->store, d, d + ntarget, ntarget, *plan);
  (void)hipFree(d);
  return finish_create(plan, st, out);
}

atlas_status atlas_remap_create_to_mesh(atlas_mesh_t source, atlas_mesh_t target,
                                        atlas_remap_t *out) {
  if (!out || !target || !target->store) return fail(ATLAS_EINVAL, "NULL argument");
  atlas_status st = check_source(source);
  if (st != ATLAS_OK) return st;
  if (target->store->device != source->store->device)
    return fail(ATLAS_EINVAL, "source and target meshes live on different devices");
  RemapPlan *plan = new (std::nothrow) RemapPlan();
  if (!plan) return fail(ATLAS_ENOMEM, "out of host memory");
  st = build_plan(*source->store, target->store->node_lon, target->store->node_lat,
                  target->store->d.V, *plan);
  return finish_create(plan, st, out);
}

atlas_status atlas_remap_apply(atlas_remap_t remap, const void *in, int32_t ncol,
                               atlas_dtype dtype, void *out, hipStream_t stream) {
  if (!remap || !remap->plan || !in || !out) return fail(ATLAS_EINVAL, "NULL argument");
  if (ncol < 1) return fail(ATLAS_EINVAL, "ncol must be >= 1");
  if (dtype != ATLAS_F32 && dtype != ATLAS_F64) return fail(ATLAS_EINVAL, "unknown dtype");
  const RemapPlan &p = *remap->plan;
  const size_t w = dtype == ATLAS_F64 ? 8 : 4;
  if ((uintptr_t)in % w || (uintptr_t)out % w)
    return fail(ATLAS_EINVAL, "pointer not aligned to its element size");
  const int64_t nelem = p.nt * (int64_t)ncol;
  if (nelem >= ((int64_t)1 << 40) || p.nsrc * (int64_t)ncol >= ((int64_t)1 << 40))
    return fail(ATLAS_EINVAL, "field too large");
  const uintptr_t i0 = (uintptr_t)in, i1 = i0 + (uintptr_t)(p.nsrc * ncol) * w;
  const uintptr_t o0 = (uintptr_t)out, o1 = o0 + (uintptr_t)nelem * w;
  if (i0 < o1 && o0 < i1) return fail(ATLAS_EINVAL, "input and output overlap");
  return remap_launch(p, in, ncol, dtype, out, stream);
}

atlas_status atlas_remap_get_weights(atlas_remap_t remap, int32_t *idx, double *w) {
  if (!remap || !remap->plan || !idx || !w) return fail(ATLAS_EINVAL, "NULL argument");
  const RemapPlan &p = *remap->plan;
  std::vector<RemapRec> h;
  try {
    h.resize((size_t)p.nt);
  } catch (const std::bad_alloc &) {
    return fail(ATLAS_ENOMEM, "out of host memory");
  }
  ATLASX_HIP(hipMemcpy(h.data(), p.rec, sizeof(RemapRec) * (size_t)p.nt, hipMemcpyDeviceToHost));
  for (int64_t t = 0; t < p.nt; ++t)
    for (int k = 0; k < 3; ++k) {
      idx[3 * t + k] = h[t].i[k];
      w[3 * t + k] = h[t].w[k];
    }
  return ATLAS_OK;
}

atlas_status atlas_remap_get_info(atlas_remap_t remap, atlas_remap_info *info) {
  if (!remap || !remap->plan || !info) return fail(ATLAS_EINVAL, "NULL argument");
  const RemapPlan &p = *remap->plan;
  info->nsource = p.nsrc;
  info->ntarget = p.nt;
  info->nsource_touched = p.touched;
  info->npolar = p.npolar;
  info->device_bytes = p.bytes;
  info->values_per_column = (double)(p.touched + p.nt);
  info->table_bytes = (double)p.nt * 36.0;
  return ATLAS_OK;
}

atlas_status atlas_remap_free(atlas_remap_t remap) {
  if (!remap) return fail(ATLAS_EINVAL, "NULL remap");
  if (remap->plan && remap->plan->serve_refs > 0)
    return fail(ATLAS_EBUSY, "remap is registered with a server");
  delete remap->plan;
  delete remap;
  return ATLAS_OK;
}

}  // extern "C"
