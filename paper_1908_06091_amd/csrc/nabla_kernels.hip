// nabla_kernels.hip -- gfx950 kernels of the edge-based median-dual
// finite-volume nabla operators (Section 4.7, Figure 33: gradient,
// divergence, curl; the Laplacian is the divergence of the gradient).
//
// Field layout follows the NodeColumns function space (Section 4.5,
// Figure 31): a node's vertical column is contiguous, [node][level];
// vectors are [node][level][2].  Wavefront lanes run over levels, so every
// load and store of a column is coalesced.
//
// Per node i and level k the operators are signed sums over the node's own
// edges in a fixed order (ascending edge id, pole edge last):
//   gradient   G_i = sum_r sS_r (x_i + x_n)/2        (pole edge: lat only)
//   divergence D_i = sum_r sS_lon (u_i+u_n)/2 + sS_lat (W_i+W_n)/2, W = v cos
//   curl       C_i = sum_r sS_lon (v_i+v_n)/2 - sS_lat (Z_i+Z_n)/2, Z = u cos
// scaled by alpha_i = R/V_i (beta_i = R cos/V_i for the meridional gradient).
// Pole edges enter the gradient only (W and Z vanish on the pole line).
// No atomics: every output element has exactly one writer, so results are
// bitwise reproducible and independent of the launch shape.
//
// FP32 fields: the same sums in difference form, sum_r sS_r (x_n - x_i)/2 +
// x_i sum_r sS_r (equal in exact arithmetic), with FP32 edge terms, a
// compensated (Kahan) FP32 node sum, the closure term and the final scaling
// in FP64.  Differences of neighbouring values are small and nearly exact in
// FP32, which keeps the error relative to the result instead of the field.
//
// Compiled with -ffp-contract=off: no operation is fused, so the separate
// edge-flux form (flux buffer, then gather) and the fused forms produce the
// same bits.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace atlasx {

enum { OP_GRAD = 0, OP_DIV = 1, OP_CURL = 2 };

// Tiles are numbered so that each XCD (workgroups are dealt round-robin to
// the 8 XCDs) receives a contiguous run of the processing order and keeps
// neighbouring columns in its own L2.
__device__ __forceinline__ int xcd_tile(int b, int per_xcd) {
  return (b & 7) * per_xcd + (b >> 3);
}

struct PosInfo {
  int node, r0, r1;
};

// Chunked tiles: either the mesh's tiles or fixed blocks of positions.
__device__ __forceinline__ bool tile_range(const DevMesh &m, int tile, int npb,
                                           int &p0, int &p1) {
  if (npb > 0) {
    p0 = tile * npb;
    if (p0 >= m.V) return false;
    p1 = min(m.V, p0 + npb);
    return true;
  }
  if (tile >= m.ntiles) return false;
  p0 = m.tile_ptr[tile];
  p1 = m.tile_ptr[tile + 1];
  return true;
}

// ---------------------------------------------------------------------------
// One output element (position p, level k) -- FP64 sum form.
// ---------------------------------------------------------------------------
template <int OP>
__device__ __forceinline__ void element_f64(const DevMesh &m, const double *__restrict__ in,
                                            double *__restrict__ out, int nlev, int p,
                                            int node, int r0, int r1, int k) {
  const size_t L = (size_t)nlev;
  if (OP == OP_GRAD) {
    const double xi = in[(size_t)node * L + k];
    double gl = 0.0, gt = 0.0;
    int r = r0;
    for (; r + 4 <= r1; r += 4) {
      uint32_t nb[4];
      double2 s[4];
      double xn[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        nb[j] = (uint32_t)m.nbr[r + j];
        s[j] = m.S[r + j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) xn[j] = in[(size_t)(nb[j] & ~kPoleBit) * L + k];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double xe = 0.5 * (xi + xn[j]);
        if (!(nb[j] & kPoleBit)) gl = gl + s[j].x * xe;
        gt = gt + s[j].y * xe;
      }
    }
    for (; r < r1; ++r) {
      const uint32_t nb = (uint32_t)m.nbr[r];
      const double2 s = m.S[r];
      const double xe = 0.5 * (xi + in[(size_t)(nb & ~kPoleBit) * L + k]);
      if (!(nb & kPoleBit)) gl = gl + s.x * xe;
      gt = gt + s.y * xe;
    }
    double2 o;
    o.x = m.alpha[p] * gl;
    o.y = m.beta[p] * gt;
    reinterpret_cast<double2 *>(out)[(size_t)node * L + k] = o;
  } else {
    const double2 *vin = reinterpret_cast<const double2 *>(in);
    const double2 ui = vin[(size_t)node * L + k];
    const double ci = m.coslat[node];
    // divergence: (a, b) = (u, v cos); curl: (a, b) = (v, u cos), minus sign
    const double ai = (OP == OP_DIV) ? ui.x : ui.y;
    const double bi = ((OP == OP_DIV) ? ui.y : ui.x) * ci;
    double acc = 0.0;
    int r = r0;
    for (; r + 4 <= r1; r += 4) {
      uint32_t nb[4];
      double2 s[4], un[4];
      double cn[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        nb[j] = (uint32_t)m.nbr[r + j];
        s[j] = m.S[r + j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t n = nb[j] & ~kPoleBit;
        un[j] = vin[(size_t)n * L + k];
        cn[j] = m.coslat[n];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (nb[j] & kPoleBit) continue;
        const double an = (OP == OP_DIV) ? un[j].x : un[j].y;
        const double bn = ((OP == OP_DIV) ? un[j].y : un[j].x) * cn[j];
        const double ae = 0.5 * (ai + an), be = 0.5 * (bi + bn);
        const double f = (OP == OP_DIV) ? s[j].x * ae + s[j].y * be : s[j].x * ae - s[j].y * be;
        acc = acc + f;
      }
    }
    for (; r < r1; ++r) {
      const uint32_t nb = (uint32_t)m.nbr[r];
      if (nb & kPoleBit) continue;
      const double2 s = m.S[r];
      const double2 un = vin[(size_t)nb * L + k];
      const double an = (OP == OP_DIV) ? un.x : un.y;
      const double bn = ((OP == OP_DIV) ? un.y : un.x) * m.coslat[nb];
      const double ae = 0.5 * (ai + an), be = 0.5 * (bi + bn);
      const double f = (OP == OP_DIV) ? s.x * ae + s.y * be : s.x * ae - s.y * be;
      acc = acc + f;
    }
    out[(size_t)node * L + k] = m.alpha[p] * acc;
  }
}

// ---------------------------------------------------------------------------
// One output element -- FP32 fields, difference form, Kahan node sums.
// ---------------------------------------------------------------------------
struct Kahan {
  float s = 0.0f, c = 0.0f;
  __device__ __forceinline__ void add(float t) {
    const float y = t - c;
    const float u = s + y;
    c = (u - s) - y;
    s = u;
  }
  __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// Edge term of the FP32 difference form (identical for both endpoints of a
// mesh edge, negated for the two ends of a pole edge).
template <int OP>
__device__ __forceinline__ void diff_terms_f32(const double2 &s, float xi, float xn,
                                               float2 ui, float2 un, double ci, double cn,
                                               float &tx, float &ty, float &t) {
  if (OP == OP_GRAD) {
    const float h = 0.5f * (xn - xi);
    tx = (float)s.x * h;
    ty = (float)s.y * h;
  } else {
    const float csum = (float)(cn + ci), cdif = (float)(cn - ci);
    // divergence: a = u, b = v cos;  curl: a = v, b = u cos
    const float ai = (OP == OP_DIV) ? ui.x : ui.y, an = (OP == OP_DIV) ? un.x : un.y;
    const float qi = (OP == OP_DIV) ? ui.y : ui.x, qn = (OP == OP_DIV) ? un.y : un.x;
    // b_n - b_i = ((q_n - q_i)(c_n + c_i) + (q_n + q_i)(c_n - c_i)) / 2
    const float db = 0.5f * ((qn - qi) * csum + (qn + qi) * cdif);
    const float da = an - ai;
    const float ta = (float)s.x * (0.5f * da), tb = (float)s.y * (0.5f * db);
    t = (OP == OP_DIV) ? ta + tb : ta - tb;
  }
}

template <int OP>
__device__ __forceinline__ void element_f32(const DevMesh &m, const float *__restrict__ in,
                                            float *__restrict__ out, int nlev, int p,
                                            int node, int r0, int r1, int k) {
  const size_t L = (size_t)nlev;
  if (OP == OP_GRAD) {
    const float xi = in[(size_t)node * L + k];
    Kahan kx, ky;
    double cx = 0.0, cy = 0.0;
    int r = r0;
    for (; r + 4 <= r1; r += 4) {
      uint32_t nb[4];
      double2 s[4];
      float xn[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        nb[j] = (uint32_t)m.nbr[r + j];
        s[j] = m.S[r + j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) xn[j] = in[(size_t)(nb[j] & ~kPoleBit) * L + k];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float tx, ty, t;
        diff_terms_f32<OP_GRAD>(s[j], xi, xn[j], float2{}, float2{}, 0.0, 0.0, tx, ty, t);
        if (!(nb[j] & kPoleBit)) { kx.add(tx); cx = cx + s[j].x; }
        ky.add(ty);
        cy = cy + s[j].y;
      }
    }
    for (; r < r1; ++r) {
      const uint32_t nb = (uint32_t)m.nbr[r];
      const double2 s = m.S[r];
      const float xn = in[(size_t)(nb & ~kPoleBit) * L + k];
      float tx, ty, t;
      diff_terms_f32<OP_GRAD>(s, xi, xn, float2{}, float2{}, 0.0, 0.0, tx, ty, t);
      if (!(nb & kPoleBit)) { kx.add(tx); cx = cx + s.x; }
      ky.add(ty);
      cy = cy + s.y;
    }
    float2 o;
    o.x = (float)(m.alpha[p] * (kx.value() + cx * (double)xi));
    o.y = (float)(m.beta[p] * (ky.value() + cy * (double)xi));
    reinterpret_cast<float2 *>(out)[(size_t)node * L + k] = o;
  } else {
    const float2 *vin = reinterpret_cast<const float2 *>(in);
    const float2 ui = vin[(size_t)node * L + k];
    const double ci = m.coslat[node];
    Kahan ka;
    double cx = 0.0, cy = 0.0;
    int r = r0;
    for (; r + 4 <= r1; r += 4) {
      uint32_t nb[4];
      double2 s[4];
      float2 un[4];
      double cn[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        nb[j] = (uint32_t)m.nbr[r + j];
        s[j] = m.S[r + j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t n = nb[j] & ~kPoleBit;
        un[j] = vin[(size_t)n * L + k];
        cn[j] = m.coslat[n];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (nb[j] & kPoleBit) continue;
        float tx, ty, t;
        diff_terms_f32<OP>(s[j], 0.0f, 0.0f, ui, un[j], ci, cn[j], tx, ty, t);
        ka.add(t);
        cx = cx + s[j].x;
        cy = cy + s[j].y;
      }
    }
    for (; r < r1; ++r) {
      const uint32_t nb = (uint32_t)m.nbr[r];
      if (nb & kPoleBit) continue;
      const double2 s = m.S[r];
      float tx, ty, t;
      diff_terms_f32<OP>(s, 0.0f, 0.0f, ui, vin[(size_t)nb * L + k], ci, m.coslat[nb], tx, ty, t);
      ka.add(t);
      cx = cx + s.x;
      cy = cy + s.y;
    }
    const double a_i = (OP == OP_DIV) ? (double)ui.x : (double)ui.y;
    const double b_i = ((OP == OP_DIV) ? (double)ui.y : (double)ui.x) * ci;
    const double closure = (OP == OP_DIV) ? cx * a_i + cy * b_i : cx * a_i - cy * b_i;
    out[(size_t)node * L + k] = (float)(m.alpha[p] * (ka.value() + closure));
  }
}

template <class T, int OP>
__device__ __forceinline__ void element(const DevMesh &m, const T *__restrict__ in,
                                        T *__restrict__ out, int nlev, int p, int node,
                                        int r0, int r1, int k) {
  if constexpr (sizeof(T) == 8)
    element_f64<OP>(m, in, out, nlev, p, node, r0, r1, k);
  else
    element_f32<OP>(m, in, out, nlev, p, node, r0, r1, k);
}

// ---------------------------------------------------------------------------
// Column form: one wavefront per position, lanes over levels.  The node's
// incidence range is wavefront-uniform.
// ---------------------------------------------------------------------------
template <class T, int OP>
__global__ void __launch_bounds__(1024) k_column(DevMesh m, const T *__restrict__ in,
                                                 T *__restrict__ out, int nlev, int npb,
                                                 int per_xcd) {
  int p0, p1;
  if (!tile_range(m, xcd_tile(blockIdx.x, per_xcd), npb, p0, p1)) return;
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  for (int p = p0 + wave; p < p1; p += nw) {
    const int node = __builtin_amdgcn_readfirstlane(m.perm[p]);
    const int r0 = __builtin_amdgcn_readfirstlane(m.rowp[p]);
    const int r1 = __builtin_amdgcn_readfirstlane(m.rowp[p + 1]);
    for (int k = lane; k < nlev; k += 64) element<T, OP>(m, in, out, nlev, p, node, r0, r1, k);
  }
}

// ---------------------------------------------------------------------------
// Flat form: lanes over flattened (position, level) pairs of the tile --
// full lanes for short columns (nlev = 1 .. 40).
// ---------------------------------------------------------------------------
template <class T, int OP>
__global__ void __launch_bounds__(1024) k_flat(DevMesh m, const T *__restrict__ in,
                                               T *__restrict__ out, int nlev, int npb,
                                               int per_xcd) {
  int p0, p1;
  if (!tile_range(m, xcd_tile(blockIdx.x, per_xcd), npb, p0, p1)) return;
  const int nel = (p1 - p0) * nlev;
  for (int e = threadIdx.x; e < nel; e += blockDim.x) {
    const int pl = e / nlev;
    const int k = e - pl * nlev;
    const int p = p0 + pl;
    element<T, OP>(m, in, out, nlev, p, m.perm[p], m.rowp[p], m.rowp[p + 1], k);
  }
}

// ---------------------------------------------------------------------------
// Flux form, kernel 1 of 2: one value per (edge slot, level) into an
// EdgeColumns-like buffer [E + npole][nlev] (x2 for the gradient).  Slots
// E.. are the pole edges (gradient only).
// ---------------------------------------------------------------------------
template <class T, int OP>
__global__ void __launch_bounds__(256) k_edge_flux(DevMesh m, const T *__restrict__ in,
                                                   T *__restrict__ flux, int nlev) {
  const int nslot = (OP == OP_GRAD) ? m.E + m.npole : m.E;
  const size_t L = (size_t)nlev;
  const size_t total = (size_t)nslot * L;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (size_t)gridDim.x * blockDim.x) {
    const int e = (int)(g / L);
    const int k = (int)(g - (size_t)e * L);
    const int a = m.e2n[2 * e], b = m.e2n[2 * e + 1];
    const double2 S = m.eS[e];
    if constexpr (sizeof(T) == 8) {
      if (OP == OP_GRAD) {
        const double xe = 0.5 * (in[(size_t)a * L + k] + in[(size_t)b * L + k]);
        double2 f;
        f.x = S.x * xe;
        f.y = S.y * xe;
        reinterpret_cast<double2 *>(flux)[g] = f;
      } else {
        const double2 *vin = reinterpret_cast<const double2 *>(in);
        const double2 ua = vin[(size_t)a * L + k], ub = vin[(size_t)b * L + k];
        const double ca = m.coslat[a], cb = m.coslat[b];
        const double aa = (OP == OP_DIV) ? ua.x : ua.y, ab = (OP == OP_DIV) ? ub.x : ub.y;
        const double ba = ((OP == OP_DIV) ? ua.y : ua.x) * ca;
        const double bb = ((OP == OP_DIV) ? ub.y : ub.x) * cb;
        const double ae = 0.5 * (aa + ab), be = 0.5 * (ba + bb);
        flux[g] = (OP == OP_DIV) ? S.x * ae + S.y * be : S.x * ae - S.y * be;
      }
    } else {
      // difference form seen from endpoint a (neighbour b)
      float tx, ty, t;
      if (OP == OP_GRAD) {
        diff_terms_f32<OP_GRAD>(S, in[(size_t)a * L + k], in[(size_t)b * L + k], float2{},
                                float2{}, 0.0, 0.0, tx, ty, t);
        float2 f;
        f.x = tx;
        f.y = ty;
        reinterpret_cast<float2 *>(flux)[g] = f;
      } else {
        const float2 *vin = reinterpret_cast<const float2 *>(in);
        diff_terms_f32<OP>(S, 0.0f, 0.0f, vin[(size_t)a * L + k], vin[(size_t)b * L + k],
                           m.coslat[a], m.coslat[b], tx, ty, t);
        flux[g] = t;
      }
    }
  }
}

// Flux form, kernel 2 of 2: each node gathers its slots in the same order
// and with the same signs as the fused forms.
template <class T, int OP>
__global__ void __launch_bounds__(1024) k_gather_flux(DevMesh m, const T *__restrict__ in,
                                                      const T *__restrict__ flux,
                                                      T *__restrict__ out, int nlev,
                                                      int per_xcd) {
  int p0, p1;
  if (!tile_range(m, xcd_tile(blockIdx.x, per_xcd), 0, p0, p1)) return;
  const size_t L = (size_t)nlev;
  const int nel = (p1 - p0) * nlev;
  for (int e = threadIdx.x; e < nel; e += blockDim.x) {
    const int pl = e / nlev;
    const int k = e - pl * nlev;
    const int p = p0 + pl;
    const int node = m.perm[p], r0 = m.rowp[p], r1 = m.rowp[p + 1];
    if constexpr (sizeof(T) == 8) {
      if (OP == OP_GRAD) {
        double gl = 0.0, gt = 0.0;
        for (int r = r0; r < r1; ++r) {
          const uint32_t slot = (uint32_t)m.inc_edge[r];
          const bool pole = ((uint32_t)m.nbr[r] & kPoleBit) != 0;
          const double2 f = reinterpret_cast<const double2 *>(flux)[(size_t)(slot & ~kPoleBit) * L + k];
          const bool neg = (slot & kPoleBit) != 0;
          if (!pole) gl = gl + (neg ? -f.x : f.x);
          gt = gt + (neg ? -f.y : f.y);
        }
        double2 o;
        o.x = m.alpha[p] * gl;
        o.y = m.beta[p] * gt;
        reinterpret_cast<double2 *>(out)[(size_t)node * L + k] = o;
      } else {
        double acc = 0.0;
        for (int r = r0; r < r1; ++r) {
          if ((uint32_t)m.nbr[r] & kPoleBit) continue;
          const uint32_t slot = (uint32_t)m.inc_edge[r];
          const double f = flux[(size_t)(slot & ~kPoleBit) * L + k];
          acc = acc + ((slot & kPoleBit) ? -f : f);
        }
        out[(size_t)node * L + k] = m.alpha[p] * acc;
      }
    } else {
      if (OP == OP_GRAD) {
        const float xi = in[(size_t)node * L + k];
        Kahan kx, ky;
        double cx = 0.0, cy = 0.0;
        for (int r = r0; r < r1; ++r) {
          const uint32_t slot = (uint32_t)m.inc_edge[r] & ~kPoleBit;
          const bool pole = ((uint32_t)m.nbr[r] & kPoleBit) != 0;
          float2 f = reinterpret_cast<const float2 *>(flux)[(size_t)slot * L + k];
          const double2 s = m.S[r];
          // the pole term changes sign at the pole edge's second node
          if (pole && m.e2n[2 * slot] != node) f.y = -f.y;
          if (!pole) { kx.add(f.x); cx = cx + s.x; }
          ky.add(f.y);
          cy = cy + s.y;
        }
        float2 o;
        o.x = (float)(m.alpha[p] * (kx.value() + cx * (double)xi));
        o.y = (float)(m.beta[p] * (ky.value() + cy * (double)xi));
        reinterpret_cast<float2 *>(out)[(size_t)node * L + k] = o;
      } else {
        const float2 ui = reinterpret_cast<const float2 *>(in)[(size_t)node * L + k];
        const double ci = m.coslat[node];
        Kahan ka;
        double cx = 0.0, cy = 0.0;
        for (int r = r0; r < r1; ++r) {
          if ((uint32_t)m.nbr[r] & kPoleBit) continue;
          const uint32_t slot = (uint32_t)m.inc_edge[r] & ~kPoleBit;
          const double2 s = m.S[r];
          ka.add(flux[(size_t)slot * L + k]);
          cx = cx + s.x;
          cy = cy + s.y;
        }
        const double a_i = (OP == OP_DIV) ? (double)ui.x : (double)ui.y;
        const double b_i = ((OP == OP_DIV) ? (double)ui.y : (double)ui.x) * ci;
        const double closure = (OP == OP_DIV) ? cx * a_i + cy * b_i : cx * a_i - cy * b_i;
        out[(size_t)node * L + k] = (float)(m.alpha[p] * (ka.value() + closure));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Per-node scales, derived once at upload: alpha = R/V, beta = R cos/V.
// ---------------------------------------------------------------------------
__global__ void k_derive_scales(int V, const double *__restrict__ vol,
                                const double *__restrict__ cosl, double R,
                                double *__restrict__ alpha, double *__restrict__ beta) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < V) {
    alpha[p] = R / vol[p];
    beta[p] = (R * cosl[p]) / vol[p];
  }
}

atlas_status derive_scales(MeshStore &m, const double *vol_by_pos, const double *cos_by_pos,
                           double radius) {
  const int V = m.d.V;
  hipLaunchKernelGGL(k_derive_scales, dim3((V + 255) / 256), dim3(256), 0, 0, V, vol_by_pos,
                     cos_by_pos, radius, const_cast<double *>(m.d.alpha),
                     const_cast<double *>(m.d.beta));
  ATLASX_HIP(hipGetLastError());
  return ATLAS_OK;
}

// ---------------------------------------------------------------------------
// Host-side dispatch
// ---------------------------------------------------------------------------
size_t flux_ws_bytes(const MeshStore &m, atlas_op op, int nlev, atlas_dtype dt) {
  const size_t w = dt == ATLAS_F64 ? 8 : 4;
  const bool grad = op == ATLAS_OP_GRADIENT || op == ATLAS_OP_LAPLACIAN;
  const size_t slots = (size_t)m.d.E + (grad ? (size_t)m.d.npole : 0);
  return slots * (size_t)nlev * w * (grad ? 2 : 1);
}

LaunchShape default_shape(const MeshStore &m, atlas_op op, int nlev, atlas_dtype dt) {
  (void)m;
  (void)op;
  (void)dt;
  LaunchShape s;
  s.variant = nlev >= 48 ? ATLAS_VARIANT_COLUMN : ATLAS_VARIANT_FLAT;
  s.block = 256;
  s.nodes_per_block = 0;
  return s;
}

template <class T, int OP>
static atlas_status launch_typed(const MeshStore &ms, const T *in, int nlev, T *out, void *ws,
                                 const LaunchShape &sh, hipStream_t st) {
  const DevMesh &m = ms.d;
  const int ntiles = sh.nodes_per_block > 0 ? (m.V + sh.nodes_per_block - 1) / sh.nodes_per_block
                                            : m.ntiles;
  const int per_xcd = (ntiles + 7) / 8;
  const dim3 grid(per_xcd * 8), block(sh.block);
  switch (sh.variant) {
    case ATLAS_VARIANT_COLUMN:
      hipLaunchKernelGGL((k_column<T, OP>), grid, block, 0, st, m, in, out, nlev,
                         sh.nodes_per_block, per_xcd);
      break;
    case ATLAS_VARIANT_FLAT:
      hipLaunchKernelGGL((k_flat<T, OP>), grid, block, 0, st, m, in, out, nlev,
                         sh.nodes_per_block, per_xcd);
      break;
    case ATLAS_VARIANT_FLUX: {
      T *flux = static_cast<T *>(ws);
      const size_t nslot = (size_t)m.E + (OP == OP_GRAD ? m.npole : 0);
      const size_t total = nslot * (size_t)nlev;
      const unsigned nb = (unsigned)std::min<size_t>((total + 255) / 256, 256 * 1024);
      hipLaunchKernelGGL((k_edge_flux<T, OP>), dim3(nb), dim3(256), 0, st, m, in, flux, nlev);
      const int per = (m.ntiles + 7) / 8;
      hipLaunchKernelGGL((k_gather_flux<T, OP>), dim3(per * 8), block, 0, st, m, in,
                         (const T *)flux, out, nlev, per);
      break;
    }
    default:
      return fail(ATLAS_EINVAL, "unknown launch variant");
  }
  ATLASX_HIP(hipGetLastError());
  return ATLAS_OK;
}

template <class T>
static atlas_status launch_dtype(const MeshStore &ms, atlas_op op, const void *in, int nlev,
                                 void *out, void *ws, const LaunchShape &sh, hipStream_t st) {
  const T *i = static_cast<const T *>(in);
  T *o = static_cast<T *>(out);
  switch (op) {
    case ATLAS_OP_GRADIENT: return launch_typed<T, OP_GRAD>(ms, i, nlev, o, ws, sh, st);
    case ATLAS_OP_DIVERGENCE: return launch_typed<T, OP_DIV>(ms, i, nlev, o, ws, sh, st);
    case ATLAS_OP_CURL: return launch_typed<T, OP_CURL>(ms, i, nlev, o, ws, sh, st);
    default: return fail(ATLAS_EINVAL, "unknown operator");
  }
}

// Laplacian: gradient into the workspace [V][nlev][2], then its divergence;
// the flux form needs its flux buffer behind the gradient.
atlas_status launch_op(const MeshStore &ms, atlas_op op, atlas_dtype dt, const void *in,
                       int nlev, void *out, void *ws, const LaunchShape &sh, hipStream_t st) {
  if (op == ATLAS_OP_LAPLACIAN) {
    const size_t w = dt == ATLAS_F64 ? 8 : 4;
    char *grad = static_cast<char *>(ws);
    void *flux = grad + (size_t)ms.d.V * nlev * 2 * w;
    atlas_status s = launch_op(ms, ATLAS_OP_GRADIENT, dt, in, nlev, grad, flux, sh, st);
    if (s != ATLAS_OK) return s;
    return launch_op(ms, ATLAS_OP_DIVERGENCE, dt, grad, nlev, out, flux, sh, st);
  }
  if (dt == ATLAS_F64) return launch_dtype<double>(ms, op, in, nlev, out, ws, sh, st);
  return launch_dtype<float>(ms, op, in, nlev, out, ws, sh, st);
}

}  // namespace atlasx
