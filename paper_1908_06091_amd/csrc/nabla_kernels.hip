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

// native 2-vectors (kept in registers; also the [node][level][2] element)
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

// Tiles are numbered so that each XCD (workgroups are dealt round-robin to
// the 8 XCDs) receives a contiguous run of the processing order and keeps
// neighbouring columns in its own L2.
__device__ __forceinline__ int xcd_tile(int b, int per_xcd) {
  return (b & 7) * per_xcd + (b >> 3);
}

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
// Per-element arithmetic.  A policy holds the running state of one output
// element (one node, one level) and is fed the node's incidences in CSR
// order; every launch form drives the same policy, so all forms produce the
// same bits.
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
                                               v2f ui, v2f un, double ci, double cn,
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

// Output stores are non-temporal (streamed past the caches, so they do not
// evict input columns that neighbours still need); ATLASX_CACHED_STORE
// selects ordinary stores.
__device__ __forceinline__ void st_out(double *p, double v) {
#ifndef ATLASX_CACHED_STORE
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}
__device__ __forceinline__ void st_out(float *p, float v) {
#ifndef ATLASX_CACHED_STORE
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}
__device__ __forceinline__ void st_out2(double *p, double x, double y) {
  v2d v = {x, y};
#ifndef ATLASX_CACHED_STORE
  __builtin_nontemporal_store(v, reinterpret_cast<v2d *>(p));
#else
  *reinterpret_cast<v2d *>(p) = v;
#endif
}
__device__ __forceinline__ void st_out2(float *p, float x, float y) {
  v2f v = {x, y};
#ifndef ATLASX_CACHED_STORE
  __builtin_nontemporal_store(v, reinterpret_cast<v2f *>(p));
#else
  *reinterpret_cast<v2f *>(p) = v;
#endif
}

template <class T, int OP> struct Pol;

// FP64 gradient: G += sS (x_i + x_n)/2; the pole edge feeds the lat part.
template <> struct Pol<double, OP_GRAD> {
  static constexpr int kOp = OP_GRAD;
  using V = double;
  static constexpr bool kVecIn = false, kVecOut = true;
  struct St { double xi, gl, gt; };
  static __device__ __forceinline__ void init(St &s, V xi, double) { s.xi = xi; s.gl = 0.0; s.gt = 0.0; }
  static __device__ __forceinline__ void add(St &s, V xn, const double2 &S, bool pole, double) {
    const double xe = 0.5 * (s.xi + xn);
    if (!pole) s.gl = s.gl + S.x * xe;
    s.gt = s.gt + S.y * xe;
  }
  using Out = v2d;
  static __device__ __forceinline__ Out result(const St &s, double al, double be, double, double,
                                               double) {
    return Out{al * s.gl, be * s.gt};
  }
  static __device__ __forceinline__ void store(double *out, size_t idx, const St &s, double al,
                                               double be, double cx, double cy, double ci) {
    const Out r = result(s, al, be, cx, cy, ci);
    st_out2(out + 2 * idx, r.x, r.y);
  }
  static __device__ __forceinline__ void keep(St &s, const St &t, bool use) {
    s.gl = use ? t.gl : s.gl;
    s.gt = use ? t.gt : s.gt;
  }
};

// FP64 divergence / curl: sum of sS_lon a_e +- sS_lat b_e with edge
// averages of a = u (v) and b = v cos (u cos); pole edges do not enter.
template <int OP> struct PolDC64 {
  static constexpr int kOp = OP;
  using V = v2d;
  static constexpr bool kVecIn = true, kVecOut = false;
  struct St { double ai, bi, acc; };
  static __device__ __forceinline__ void init(St &s, V ui, double ci) {
    s.ai = (OP == OP_DIV) ? ui.x : ui.y;
    s.bi = ((OP == OP_DIV) ? ui.y : ui.x) * ci;
    s.acc = 0.0;
  }
  static __device__ __forceinline__ void add(St &s, V un, const double2 &S, bool, double cn) {
    const double an = (OP == OP_DIV) ? un.x : un.y;
    const double bn = ((OP == OP_DIV) ? un.y : un.x) * cn;
    const double ae = 0.5 * (s.ai + an), be = 0.5 * (s.bi + bn);
    const double f = (OP == OP_DIV) ? S.x * ae + S.y * be : S.x * ae - S.y * be;
    s.acc = s.acc + f;
  }
  using Out = double;
  static __device__ __forceinline__ Out result(const St &s, double al, double, double, double,
                                               double) {
    return al * s.acc;
  }
  static __device__ __forceinline__ void store(double *out, size_t idx, const St &s, double al,
                                               double be, double cx, double cy, double ci) {
    st_out(out + idx, result(s, al, be, cx, cy, ci));
  }
  static __device__ __forceinline__ void keep(St &s, const St &t, bool use) {
    s.acc = use ? t.acc : s.acc;
  }
};
template <> struct Pol<double, OP_DIV> : PolDC64<OP_DIV> {};
template <> struct Pol<double, OP_CURL> : PolDC64<OP_CURL> {};

// FP32 gradient, difference form with Kahan sums; the closure sums
// (cx, cy) = sum sS are formed in FP64 by the caller.
template <> struct Pol<float, OP_GRAD> {
  static constexpr int kOp = OP_GRAD;
  using V = float;
  static constexpr bool kVecIn = false, kVecOut = true;
  struct St { float xi; Kahan kx, ky; };
  static __device__ __forceinline__ void init(St &s, V xi, double) { s.xi = xi; s.kx = Kahan(); s.ky = Kahan(); }
  static __device__ __forceinline__ void add(St &s, V xn, const double2 &S, bool pole, double) {
    float tx, ty, t;
    diff_terms_f32<OP_GRAD>(S, s.xi, xn, v2f{}, v2f{}, 0.0, 0.0, tx, ty, t);
    if (!pole) s.kx.add(tx);
    s.ky.add(ty);
  }
  using Out = v2f;
  static __device__ __forceinline__ Out result(const St &s, double al, double be, double cx,
                                               double cy, double) {
    return Out{(float)(al * (s.kx.value() + cx * (double)s.xi)),
               (float)(be * (s.ky.value() + cy * (double)s.xi))};
  }
  static __device__ __forceinline__ void store(float *out, size_t idx, const St &s, double al,
                                               double be, double cx, double cy, double ci) {
    const Out r = result(s, al, be, cx, cy, ci);
    st_out2(out + 2 * idx, r.x, r.y);
  }
  static __device__ __forceinline__ void keep(St &s, const St &t, bool use) {
    s.kx.s = use ? t.kx.s : s.kx.s;
    s.kx.c = use ? t.kx.c : s.kx.c;
    s.ky.s = use ? t.ky.s : s.ky.s;
    s.ky.c = use ? t.ky.c : s.ky.c;
  }
};

template <int OP> struct PolDC32 {
  static constexpr int kOp = OP;
  using V = v2f;
  static constexpr bool kVecIn = true, kVecOut = false;
  struct St { v2f ui; double ci; Kahan ka; };
  static __device__ __forceinline__ void init(St &s, V ui, double ci) { s.ui = ui; s.ci = ci; s.ka = Kahan(); }
  static __device__ __forceinline__ void add(St &s, V un, const double2 &S, bool, double cn) {
    float tx, ty, t;
    diff_terms_f32<OP>(S, 0.0f, 0.0f, s.ui, un, s.ci, cn, tx, ty, t);
    s.ka.add(t);
  }
  using Out = float;
  static __device__ __forceinline__ Out result(const St &s, double al, double, double cx,
                                               double cy, double) {
    const double a_i = (OP == OP_DIV) ? (double)s.ui.x : (double)s.ui.y;
    const double b_i = ((OP == OP_DIV) ? (double)s.ui.y : (double)s.ui.x) * s.ci;
    const double closure = (OP == OP_DIV) ? cx * a_i + cy * b_i : cx * a_i - cy * b_i;
    return (float)(al * (s.ka.value() + closure));
  }
  static __device__ __forceinline__ void store(float *out, size_t idx, const St &s, double al,
                                               double be, double cx, double cy, double ci) {
    st_out(out + idx, result(s, al, be, cx, cy, ci));
  }
  static __device__ __forceinline__ void keep(St &s, const St &t, bool use) {
    s.ka.s = use ? t.ka.s : s.ka.s;
    s.ka.c = use ? t.ka.c : s.ka.c;
  }
};
template <> struct Pol<float, OP_DIV> : PolDC32<OP_DIV> {};
template <> struct Pol<float, OP_CURL> : PolDC32<OP_CURL> {};

// Closure sums of a node (FP32 forms): sum over the incidences that enter
// the operator of the signed normals.
template <int OP>
__device__ __forceinline__ void closure_add(double &cx, double &cy, const double2 &S, bool pole) {
  if (OP == OP_GRAD) {
    if (!pole) cx = cx + S.x;
    cy = cy + S.y;
  } else if (!pole) {
    cx = cx + S.x;
    cy = cy + S.y;
  }
}

// One element at level k (any nlev); used by the generic column loop and
// by the flat form.
template <class T, int OP>
__device__ __forceinline__ void element(const DevMesh &m, const T *__restrict__ in,
                                        T *__restrict__ out, int nlev, int p, int node, int r0,
                                        int r1, int k) {
  using P = Pol<T, OP>;
  using V = typename P::V;
  const V *vin = reinterpret_cast<const V *>(in);
  const size_t L = (size_t)nlev;
  const double ci = P::kVecIn ? m.coslat[node] : 0.0;
  typename P::St st;
  P::init(st, vin[(size_t)node * L + k], ci);
  double cx = 0.0, cy = 0.0;
  for (int r = r0; r < r1; ++r) {
    const uint32_t nb = (uint32_t)m.nbr[r];
    const bool pole = (nb & kPoleBit) != 0;
    if (P::kVecIn && pole) continue;
    const double2 S = m.S[r];
    const size_t n = nb & ~kPoleBit;
    const double cn = P::kVecIn ? m.coslat[n] : 0.0;
    closure_add<OP>(cx, cy, S, pole);
    P::add(st, vin[n * L + k], S, pole, cn);
  }
  const double al = m.alpha[p], be = P::kVecOut ? m.beta[p] : 0.0;
  P::store(out, (size_t)node * L + k, st, al, be, cx, cy, ci);
}

// Chunked column form: work units are (level chunk, tile), chunk-major, so
// the whole mesh is swept once per chunk and consecutive parallels of one
// chunk meet in the XCD's L2.  One wavefront per position; lanes over the
// chunk's levels.
template <class T, int OP>
__global__ void __launch_bounds__(1024) k_column_chunked(DevMesh m, const T *__restrict__ in,
                                                         T *__restrict__ out, int nlev, int npb,
                                                         int kc, int ntiles, int per_xcd) {
  const int u = xcd_tile(blockIdx.x, per_xcd);
  const int c = u / ntiles;
  int p0, p1;
  if (!tile_range(m, u - c * ntiles, npb, p0, p1)) return;
  const int k0 = c * kc;
  if (k0 >= nlev) return;
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int k = k0 + lane;
  const bool active = lane < kc && k < nlev;
  for (int p = p0 + wave; p < p1; p += nw) {
    const int node = __builtin_amdgcn_readfirstlane(m.perm[p]);
    const int r0 = __builtin_amdgcn_readfirstlane(m.rowp[p]);
    const int r1 = __builtin_amdgcn_readfirstlane(m.rowp[p + 1]);
    if (active) element<T, OP>(m, in, out, nlev, p, node, r0, r1, k);
  }
}

// ---------------------------------------------------------------------------
// Column form: one wavefront per position, lanes over levels.  NCH chunks
// of 64 levels are processed together and all of a node's incidences (up to
// G) are fetched in one round trip, so up to G*NCH column loads are in
// flight per wavefront.  The position record and the incidence rows are
// wavefront-uniform (scalar loads); the next position's record is fetched
// while the current one is computed.
// ---------------------------------------------------------------------------
// One group of up to G incidences starting at rb: every load first (the
// incidence arrays are padded, so entries past the row name valid nodes and
// need no branch), then the accumulation in row order.
template <class P, int NCH, int G>
__device__ __forceinline__ void column_group(const DevMesh &m, const typename P::V *__restrict__ vin,
                                             size_t L, const int (&kk)[NCH], int rb, int n,
                                             typename P::St (&st)[NCH], double &cx, double &cy) {
  using V = typename P::V;
  uint32_t nb[G];
  double2 S[G];
  double cn[G];
  V xn[G][NCH];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    nb[j] = (uint32_t)m.nbr[rb + j];
    S[j] = m.S[rb + j];
    cn[j] = P::kVecIn ? m.ncos[rb + j] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const size_t q = nb[j] & ~kPoleBit;
#pragma unroll
    for (int c = 0; c < NCH; ++c) xn[j][c] = vin[q * L + kk[c]];
  }
#pragma unroll
  for (int j = 0; j < G; ++j) {
    if (j < n) {
      const bool pole = (nb[j] & kPoleBit) != 0;
      if (!(P::kVecIn && pole)) {
        closure_add<P::kOp>(cx, cy, S[j], pole);
#pragma unroll
        for (int c = 0; c < NCH; ++c) P::add(st[c], xn[j][c], S[j], pole, cn[j]);
      }
    }
  }
}

// ONE_GROUP: every row has at most G incidences and is handled by a single
// group without a loop (a loop back-edge makes the compiler wait for every
// outstanding memory operation, stores included, before the next loads).
template <class T, int OP, int NCH, int G, bool ONE_GROUP>
__device__ __forceinline__ void column_node(const DevMesh &m, const T *__restrict__ in,
                                            T *__restrict__ out, int nlev, const PosRec &pr,
                                            int lane) {
  using P = Pol<T, OP>;
  using V = typename P::V;
  const V *vin = reinterpret_cast<const V *>(in);
  const size_t L = (size_t)nlev;
  const int node = pr.node, r0 = pr.r0, r1 = pr.r1;
  int kk[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) kk[c] = min(lane + 64 * c, nlev - 1);  // clamped, in bounds
  const double ci = P::kVecIn ? m.coslat[node] : 0.0;
  typename P::St st[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) P::init(st[c], vin[(size_t)node * L + kk[c]], ci);
  double cx = 0.0, cy = 0.0;
  if (ONE_GROUP) {
    column_group<P, NCH, G>(m, vin, L, kk, r0, r1 - r0, st, cx, cy);
  } else {
    for (int rb = r0; rb < r1; rb += G) column_group<P, NCH, G>(m, vin, L, kk, rb, min(G, r1 - rb), st, cx, cy);
  }
  const double al = pr.alpha, be = P::kVecOut ? pr.beta : 0.0;
#pragma unroll
  for (int c = 0; c < NCH; ++c)
    if (lane + 64 * c < nlev) P::store(out, (size_t)node * L + lane + 64 * c, st[c], al, be, cx, cy, ci);
}

template <class T, int OP, int NCH, int G>
__device__ __forceinline__ void column_pos(const DevMesh &m, const T *__restrict__ in,
                                           T *__restrict__ out, int nlev, int p,
                                           const PosRec &pr, int lane) {
  if (NCH > 0) {
    // G = 6: one load group covers every row of a mesh of degree <= 6 (the
    // octahedral mesh, pole edge included); G = 8: rows in groups
    column_node<T, OP, (NCH > 0 ? NCH : 1), G, G == 6>(m, in, out, nlev, pr, lane);
  } else {
    // any nlev: chunks of 64 levels one after another
    for (int k = lane; k < nlev; k += 64) element<T, OP>(m, in, out, nlev, p, pr.node, pr.r0, pr.r1, k);
  }
}

// Tiled schedule (cyc == 0): one workgroup per tile / block of positions.
// Persistent schedule (cyc > 0 workgroups per XCD): the wavefronts of XCD x
// take positions of its share [V x/8, V (x+1)/8) cyclically, wavefront g at
// step t computing position lo + g + t * (cyc * waves per block).
template <class T, int OP, int NCH, int G>
__global__ void __launch_bounds__(512) k_column(DevMesh m, const T *__restrict__ in,
                                                 T *__restrict__ out, int nlev, int npb,
                                                 int per_xcd, int cyc) {
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int p, p1, stride;
  if (cyc > 0) {
    const int x = blockIdx.x & 7, i = blockIdx.x >> 3;
    const int lo = (int)((int64_t)m.V * x / 8);
    p1 = (int)((int64_t)m.V * (x + 1) / 8);
    p = lo + i * nw + wave;
    stride = cyc * nw;
  } else {
    int p0;
    if (!tile_range(m, xcd_tile(blockIdx.x, per_xcd), npb, p0, p1)) return;
    p = p0 + wave;
    stride = nw;
  }
  if (p >= p1) return;
  PosRec cur = m.pos[p];
  for (; p < p1; p += stride) {
    const PosRec nxt = m.pos[min(p + stride, p1 - 1)];  // prefetch
    column_pos<T, OP, NCH, G>(m, in, out, nlev, p, cur, lane);
    cur = nxt;
  }
}

// ---------------------------------------------------------------------------
// Level-vector column form: as the column form, but every lane owns NV
// consecutive levels of the column and moves them with one 16-byte access
// (FP64 scalar columns: 2 levels per lane; FP32 scalar: 4; FP32 vector: 2).
// A wavefront load instruction then carries 1 KiB instead of 256-512 B, so a
// node needs 2-3x fewer vector memory instructions -- the address path, not
// the bytes, is what limits the one-level-per-lane form.  Column starts are
// only element-aligned (a column of 137 FP64 levels is 1096 B), so these are
// unaligned 16-byte accesses.  A lane's first level is clamped to
// nlev - NV: every access stays inside the column, and the lanes at the end
// recompute and store levels that a neighbouring lane also owns -- the same
// operation sequence, so the same bits are written twice.
// ---------------------------------------------------------------------------
// Buffer accesses.  A column (or a node's output run) is described by a
// buffer resource whose range is exactly that column; a lane whose offset is
// out of range makes no memory access at all (loads return 0, stores are
// dropped).  Lanes past the last lane vector therefore cost no cache
// traffic, unlike clamped duplicate accesses.
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
__device__ i32x4 buf_load16(i32x4 rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.v4i32");
__device__ i32x2 buf_load8(i32x4 rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.v2i32");
__device__ void buf_store16(i32x4 v, i32x4 rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.store.v4i32");
__device__ void buf_store8(i32x2 v, i32x4 rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.store.v2i32");
__device__ void buf_store4(int v, i32x4 rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.store.i32");

constexpr int kBufOff = 0x7fffff00;  // an offset outside every range used here
#ifndef ATLASX_CACHED_STORE
constexpr int kStoreAux = 2;         // non-temporal (streamed past the caches)
#else
constexpr int kStoreAux = 0;
#endif

// Raw buffer resource (stride 0) over [base, base + bytes); wavefront-uniform.
__device__ __forceinline__ i32x4 make_rsrc(const void *base, uint32_t bytes) {
  const uint64_t a = (uint64_t)base;
  i32x4 r;
  r.x = __builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  r.y = __builtin_amdgcn_readfirstlane((int)((uint32_t)(a >> 32) & 0xffffu));
  r.z = __builtin_amdgcn_readfirstlane((int)bytes);
  r.w = 0x00020000;
  return r;
}

// Read-only mesh data seen through the constant address space: the compiler
// may then serve wavefront-uniform reads with scalar loads even where the
// kernel also writes through buffer stores (which it cannot prove disjoint
// from a generic pointer).
#define ATLASX_CST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const ATLASX_CST T *cst(const T *p) {
  return (const ATLASX_CST T *)p;
}

// Structures read field by field through the constant address space.
__device__ __forceinline__ double2 cst_double2(const double2 *p, size_t i) {
  const ATLASX_CST double *d = cst(reinterpret_cast<const double *>(p));
  double2 r;
  r.x = d[2 * i];
  r.y = d[2 * i + 1];
  return r;
}
__device__ __forceinline__ PosRec cst_pos(const PosRec *p, size_t i) {
  const ATLASX_CST PosRec *q = cst(p) + i;
  PosRec r;
  r.node = q->node;
  r.r0 = q->r0;
  r.r1 = q->r1;
  r.selfslot = q->selfslot;
  r.alpha = q->alpha;
  r.beta = q->beta;
  return r;
}

typedef int i32x3 __attribute__((ext_vector_type(3)));
__device__ int buf_load4(i32x4 rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.i32");
__device__ i32x3 buf_load12(i32x4 rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.v3i32");
__device__ void buf_store12(i32x3 v, i32x4 rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.store.v3i32");

// A lane vector of 4..32 bytes, in 16-, 8- and 4-byte pieces.
template <class R>
__device__ __forceinline__ R buf_load(const i32x4 &rsrc, int voff) {
  constexpr int B = (int)sizeof(R);
  static_assert(B % 4 == 0 && B <= 32, "lane vectors are 4..32 bytes");
  int w[B / 4];
  int at = 0;
#pragma unroll
  for (; at + 16 <= B; at += 16) {
    const i32x4 v = buf_load16(rsrc, voff + at, 0, 0);
    w[at / 4] = v.x; w[at / 4 + 1] = v.y; w[at / 4 + 2] = v.z; w[at / 4 + 3] = v.w;
  }
  if constexpr (B % 16 == 12) {
    const i32x3 v = buf_load12(rsrc, voff + (B / 16) * 16, 0, 0);
    w[(B / 16) * 4] = v.x;
    w[(B / 16) * 4 + 1] = v.y;
    w[(B / 16) * 4 + 2] = v.z;
  } else {
    if constexpr (B % 16 >= 8) {
      const i32x2 v = buf_load8(rsrc, voff + (B / 16) * 16, 0, 0);
      w[(B / 16) * 4] = v.x;
      w[(B / 16) * 4 + 1] = v.y;
    }
    if constexpr (B % 8 == 4) w[B / 4 - 1] = buf_load4(rsrc, voff + B - 4, 0, 0);
  }
  R r;
  __builtin_memcpy(&r, w, B);
  return r;
}

// Stores `W` 32-bit words of one lane at byte offset `ob`, in 16-, 8- and
// 4-byte pieces (non-temporal).
template <int W>
__device__ __forceinline__ void buf_store_words(const int (&w)[W], const i32x4 &rsrc, int ob) {
#pragma unroll
  for (int k = 0; k + 4 <= W; k += 4)
    buf_store16(i32x4{w[k], w[k + 1], w[k + 2], w[k + 3]}, rsrc, ob + 4 * k, 0, kStoreAux);
  if constexpr (W % 4 == 3) {
    buf_store12(i32x3{w[W - 3], w[W - 2], w[W - 1]}, rsrc, ob + 4 * (W - 3), 0, kStoreAux);
  } else {
    if constexpr (W % 4 >= 2)
      buf_store8(i32x2{w[(W / 4) * 4], w[(W / 4) * 4 + 1]}, rsrc, ob + 16 * (W / 4), 0, kStoreAux);
    if constexpr (W % 2 == 1) buf_store4(w[W - 1], rsrc, ob + 4 * (W - 1), 0, kStoreAux);
  }
}

// A lane vector: NV consecutive levels of one column, NV * sizeof(V) bytes.
template <class V> struct ElemOf { using E = V; static constexpr int C = 1; };
template <> struct ElemOf<v2d> { using E = double; static constexpr int C = 2; };
template <> struct ElemOf<v2f> { using E = float; static constexpr int C = 2; };

template <class V, int NV> struct LaneVec {
  using E = typename ElemOf<V>::E;
  static constexpr int C = ElemOf<V>::C;
  struct raw {
    E e[NV * C];
  };
  static __device__ __forceinline__ V get(const raw &r, int v) {
    if constexpr (C == 1) {
      return r.e[v];
    } else {
      return V{r.e[2 * v], r.e[2 * v + 1]};
    }
  }
};

// The level-vector form exists for this element type and width: NV levels
// of at most 32 bytes per lane.
template <class T, int OP, int NV>
constexpr bool lane_vec_ok() {
  return NV >= 1 && NV <= 4 && NV * sizeof(typename Pol<T, OP>::V) <= 32;
}

// Incidences every row of a mesh has besides its pole edge (the octahedral
// meshes: at least 4); below it the level-vector kernels need no select.
constexpr int kMinRow = 4;

// One node (rows of at most 6 incidences, one load group), NCH chunks of
// 64 lanes x NV levels.
template <class T, int OP, int NV, int NCH>
__device__ __forceinline__ void colv_node(const DevMesh &m, const T *__restrict__ in,
                                          T *__restrict__ out, int nlev, const PosRec &pr,
                                          int lane) {
  using P = Pol<T, OP>;
  using V = typename P::V;
  using LV = LaneVec<V, NV>;
  using R = typename LV::raw;
  using Out = typename P::Out;
  const V *vin = reinterpret_cast<const V *>(in);
  const size_t L = (size_t)nlev;
  const uint32_t col_bytes = (uint32_t)(L * sizeof(V));
  const int node = pr.node, r0 = pr.r0, n = pr.r1 - pr.r0;
  // lane vector c of this lane starts at level s[c]; the last vector is
  // clamped inside the column, lanes past it get an out-of-range offset
  const int nvec = (nlev + NV - 1) / NV;
  int s[NCH], off[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int idx = lane + 64 * c;
    s[c] = min(NV * idx, nlev - NV);
    off[c] = idx < nvec ? s[c] * (int)sizeof(V) : kBufOff;
  }
  const double ci = P::kVecIn ? cst(m.coslat)[node] : 0.0;
  typename P::St st[NCH][NV];
  {
    const i32x4 rs = make_rsrc(vin + (size_t)node * L, col_bytes);
    R xi[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) xi[c] = buf_load<R>(rs, off[c]);
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < NV; ++v) P::init(st[c][v], LV::get(xi[c], v), ci);
  }
  constexpr int G = 6;
  uint32_t nb[G];
  double2 S[G];
  double cn[G];
  R xn[G][NCH];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    nb[j] = (uint32_t)cst(m.nbr)[r0 + j];
    S[j] = cst_double2(m.S, r0 + j);
    cn[j] = P::kVecIn ? cst(m.ncos)[r0 + j] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const size_t q = nb[j] & ~kPoleBit;
    const i32x4 rs = make_rsrc(vin + q * L, col_bytes);
#pragma unroll
    for (int c = 0; c < NCH; ++c) xn[j][c] = buf_load<R>(rs, off[c]);
  }
  // Every incidence of the group is accumulated into a candidate state and
  // kept by a select (not a branch): the loads above then have unconditional
  // uses and stay one burst, instead of being moved into a branch per
  // incidence and waited for one at a time.  Padding entries (j >= n) and
  // pole edges of div/curl leave the state as it was.
  double cx = 0.0, cy = 0.0;
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const bool pole = (nb[j] & kPoleBit) != 0;
    if (j < kMinRow) {  // present in every row, never the pole edge
      closure_add<P::kOp>(cx, cy, S[j], false);
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < NV; ++v) P::add(st[c][v], LV::get(xn[j][c], v), S[j], false, cn[j]);
      continue;
    }
    const bool use = j < n && !(P::kVecIn && pole);
    double tx = cx, ty = cy;
    closure_add<P::kOp>(tx, ty, S[j], pole);
    cx = use ? tx : cx;
    cy = use ? ty : cy;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        typename P::St t = st[c][v];
        P::add(t, LV::get(xn[j][c], v), S[j], pole, cn[j]);
        P::keep(st[c][v], t, use);
      }
  }
  // A lane's NV results are contiguous in the output run of the node:
  // written in 16-byte pieces (8 / 4 bytes for a shorter run).
  const double al = pr.alpha, be = P::kVecOut ? pr.beta : 0.0;
  const i32x4 ro = make_rsrc(out + (size_t)node * L * (sizeof(Out) / sizeof(T)),
                             (uint32_t)(L * sizeof(Out)));
  constexpr int W = NV * (int)sizeof(Out) / 4;  // 32-bit words per lane vector
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    int w[W];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const Out r = P::result(st[c][v], al, be, cx, cy, ci);
      __builtin_memcpy(&w[v * (int)sizeof(Out) / 4], &r, sizeof(Out));
    }
    const int ob = off[c] == kBufOff ? kBufOff : s[c] * (int)sizeof(Out);
    buf_store_words<W>(w, ro, ob);
  }
}

// Same schedules as k_column (tiled, or persistent wave-cyclic).  The
// occupancy hint lets the register allocator keep a node's whole load burst
// in flight (at the default target it delays part of the burst to save
// registers, and each delayed load is then waited for on its own).  The
// most waves per SIMD at which the burst fits without spilling: five for
// FP32 in one chunk (the FP32 divergence at 137 levels: 85 registers and
// 4.55 ms, against 97 and 4.75 ms at four); four up to two chunks, and for
// FP64 lanes of at most 16 bytes (the FP64 divergence: 97 registers and
// 7.31 ms, against 169 and 7.73 ms at two); otherwise two.
template <class T, int LB, int NCH> constexpr int colv_waves() {
  return sizeof(T) == 4 && NCH == 1 ? 5 : NCH <= 2 || (sizeof(T) == 8 && LB <= 16) ? 4 : 2;
}
// The same for the one-pass divergence + curl (two states per level).
template <class T, int NV, int NCH> constexpr int colv_dc_waves() {
  return sizeof(T) == 4 && NCH == 1 && NV <= 3 ? 5
         : NCH <= 2 || (sizeof(T) == 8 && NV == 1 && NCH == 3) ? 4 : 2;
}

template <class T, int OP, int NV, int NCH>
__global__ void __launch_bounds__(512)
    __attribute__((amdgpu_waves_per_eu(
        colv_waves<T, NV * (int)sizeof(typename Pol<T, OP>::V), NCH>(),
        colv_waves<T, NV * (int)sizeof(typename Pol<T, OP>::V), NCH>())))
    k_colv(DevMesh m, const T *__restrict__ in,
                                               T *__restrict__ out, int nlev, int npb,
                                               int per_xcd, int cyc) {
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int p, p1, stride;
  if (cyc > 0) {
    const int x = blockIdx.x & 7, i = blockIdx.x >> 3;
    const int lo = (int)((int64_t)m.V * x / 8);
    p1 = (int)((int64_t)m.V * (x + 1) / 8);
    p = lo + i * nw + wave;
    stride = cyc * nw;
  } else {
    int p0;
    if (!tile_range(m, xcd_tile(blockIdx.x, per_xcd), npb, p0, p1)) return;
    p = p0 + wave;
    stride = nw;
  }
  if (p >= p1) return;
  PosRec cur = cst_pos(m.pos, p);
  for (; p < p1; p += stride) {
    const PosRec nxt = cst_pos(m.pos, min(p + stride, p1 - 1));  // prefetch
    colv_node<T, OP, NV, NCH>(m, in, out, nlev, cur, lane);
    cur = nxt;
  }
}

// Divergence and curl of one vector field in one pass: the column form of
// colv_node with both operators' states fed from the same loads, so (u, v)
// is read once and each output gets exactly the operation sequence of its
// own operator (bitwise equal to the two separate calls).
template <class T, int NV, int NCH>
__device__ __forceinline__ void colv_node_dc(const DevMesh &m, const T *__restrict__ in,
                                             T *__restrict__ out_d, T *__restrict__ out_c,
                                             int nlev, const PosRec &pr, int lane) {
  using PD = Pol<T, OP_DIV>;
  using PC = Pol<T, OP_CURL>;
  using V = typename PD::V;
  using LV = LaneVec<V, NV>;
  using R = typename LV::raw;
  const V *vin = reinterpret_cast<const V *>(in);
  const size_t L = (size_t)nlev;
  const uint32_t col_bytes = (uint32_t)(L * sizeof(V));
  const int node = pr.node, r0 = pr.r0, n = pr.r1 - pr.r0;
  const int nvec = (nlev + NV - 1) / NV;
  int s[NCH], off[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int idx = lane + 64 * c;
    s[c] = min(NV * idx, nlev - NV);
    off[c] = idx < nvec ? s[c] * (int)sizeof(V) : kBufOff;
  }
  const double ci = cst(m.coslat)[node];
  typename PD::St sd[NCH][NV];
  typename PC::St sc[NCH][NV];
  {
    const i32x4 rs = make_rsrc(vin + (size_t)node * L, col_bytes);
    R xi[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) xi[c] = buf_load<R>(rs, off[c]);
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        PD::init(sd[c][v], LV::get(xi[c], v), ci);
        PC::init(sc[c][v], LV::get(xi[c], v), ci);
      }
  }
  constexpr int G = 6;
  uint32_t nb[G];
  double2 S[G];
  double cn[G];
  R xn[G][NCH];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    nb[j] = (uint32_t)cst(m.nbr)[r0 + j];
    S[j] = cst_double2(m.S, r0 + j);
    cn[j] = cst(m.ncos)[r0 + j];
  }
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const size_t q = nb[j] & ~kPoleBit;
    const i32x4 rs = make_rsrc(vin + q * L, col_bytes);
#pragma unroll
    for (int c = 0; c < NCH; ++c) xn[j][c] = buf_load<R>(rs, off[c]);
  }
  double cx = 0.0, cy = 0.0;  // the same closure sums serve both operators
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const bool pole = (nb[j] & kPoleBit) != 0;
    if (j < kMinRow) {
      closure_add<OP_DIV>(cx, cy, S[j], false);
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          PD::add(sd[c][v], LV::get(xn[j][c], v), S[j], false, cn[j]);
          PC::add(sc[c][v], LV::get(xn[j][c], v), S[j], false, cn[j]);
        }
      continue;
    }
    const bool use = j < n && !pole;
    double tx = cx, ty = cy;
    closure_add<OP_DIV>(tx, ty, S[j], pole);
    cx = use ? tx : cx;
    cy = use ? ty : cy;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        typename PD::St td = sd[c][v];
        PD::add(td, LV::get(xn[j][c], v), S[j], pole, cn[j]);
        PD::keep(sd[c][v], td, use);
        typename PC::St tc = sc[c][v];
        PC::add(tc, LV::get(xn[j][c], v), S[j], pole, cn[j]);
        PC::keep(sc[c][v], tc, use);
      }
  }
  const double al = pr.alpha;
  const i32x4 rd = make_rsrc(out_d + (size_t)node * L, (uint32_t)(L * sizeof(T)));
  const i32x4 rc = make_rsrc(out_c + (size_t)node * L, (uint32_t)(L * sizeof(T)));
  constexpr int W = NV * (int)sizeof(T) / 4;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    int wd[W], wc[W];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T a = PD::result(sd[c][v], al, 0.0, cx, cy, ci);
      const T b = PC::result(sc[c][v], al, 0.0, cx, cy, ci);
      __builtin_memcpy(&wd[v * (int)sizeof(T) / 4], &a, sizeof(T));
      __builtin_memcpy(&wc[v * (int)sizeof(T) / 4], &b, sizeof(T));
    }
    const int ob = off[c] == kBufOff ? kBufOff : s[c] * (int)sizeof(T);
    buf_store_words<W>(wd, rd, ob);
    buf_store_words<W>(wc, rc, ob);
  }
}

template <class T, int NV, int NCH>
__global__ void __launch_bounds__(512)
    __attribute__((amdgpu_waves_per_eu(colv_dc_waves<T, NV, NCH>(), colv_dc_waves<T, NV, NCH>())))
    k_colv_dc(DevMesh m, const T *__restrict__ in, T *__restrict__ out_d,
              T *__restrict__ out_c, int nlev, int npb, int per_xcd) {
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int p0, p1;
  if (!tile_range(m, xcd_tile(blockIdx.x, per_xcd), npb, p0, p1)) return;
  for (int p = p0 + wave; p < p1; p += nw) {
    const PosRec pr = cst_pos(m.pos, p);
    colv_node_dc<T, NV, NCH>(m, in, out_d, out_c, nlev, pr, lane);
  }
}

// Levels per lane of the level-vector form for (T, OP, nlev).  FP64 (bound
// by memory traffic): 16-byte lanes.  FP32 (its compensated sums make the
// arithmetic the larger cost): the width (1..4 levels, at most 32 bytes per
// lane) that needs the fewest level slots per lane (NV x chunks of 64
// lanes; the arithmetic runs once per slot), then the fewest load
// instructions per column.  `want` > 0 forces a width.  0 when the form
// does not apply (mesh degree above 6 or a row shorter than kMinRow, no
// width fitting the column, more than 4 chunks) and the one-level-per-lane
// column kernel runs instead.
template <class T, int OP>
__host__ __device__ inline int auto_level_vec(int nlev, int maxdeg, int mindeg, int want = 0) {
  if (maxdeg > 6 || mindeg < kMinRow) return 0;
  const int vb = (int)sizeof(typename Pol<T, OP>::V);
  if (want == 0 && sizeof(T) == 8) want = 16 / vb;
  int best = 0, best_slots = 1 << 30, best_loads = 1 << 30;
  for (int nv = 1; nv <= 4; ++nv) {
    if (nv * vb > 32 || nlev < nv || (want > 0 && nv != want)) continue;
    const int nch = ((nlev + nv - 1) / nv + 63) / 64;
    if (nch > 4) continue;
    const int bytes = nv * vb;
    const int pieces = bytes / 16 + ((bytes % 16) ? 1 : 0);  // 16/12/8/4-byte accesses
    const int slots = nv * nch, loads = nch * pieces;
    if (slots < best_slots || (slots == best_slots && loads < best_loads)) {
      best = nv;
      best_slots = slots;
      best_loads = loads;
    }
  }
  return best;
}

// ---------------------------------------------------------------------------
// Parallel-sweep form.  A workgroup owns one tile (a longitude sector of a
// band of parallels) and one chunk of levels.  It walks down the band one
// parallel at a time, keeping the runs of the parallels above, at and below
// the current one in a 4-slot LDS ring buffer; while it computes parallel q
// it has the loads of parallel q+2 in flight (staged through registers).
// Every column is read from memory once per chunk plus a thin halo; every
// neighbour comes from LDS.  One wavefront per position, lanes over levels.
// ---------------------------------------------------------------------------
template <class T, int OP, int EPT>
__global__ void __launch_bounds__(1024) k_sweep(DevMesh m, const T *__restrict__ in,
                                               T *__restrict__ out, int nlev, int kcmax,
                                               int ntiles, int per_xcd) {
  using P = Pol<T, OP>;
  using V = typename P::V;
  constexpr int G = 8;  // incidences fetched together
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *buf = reinterpret_cast<V *>(smem_raw);
  const int u = xcd_tile(blockIdx.x, per_xcd);
  const int c = u / ntiles;
  const int tile = u - c * ntiles;
  const int k0 = c * kcmax;
  if (k0 >= nlev) return;
  const int kc = min(kcmax, nlev - k0);
  const int s0 = m.tile_seg[tile];
  const int nseg = m.tile_seg[tile + 1] - s0;
  const int slot_stride = m.segmax * kc;  // elements per LDS slot
  const V *vin = reinterpret_cast<const V *>(in);
  const size_t L = (size_t)nlev;
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const bool lane_on = lane < kc;

  // staging: wavefront w moves nodes w, w+nw, ... of a run; lanes = levels
  V regs[EPT];
  const int lane_c = min(lane, kc - 1);
  auto fetch = [&](int q) {
    const int4 sg = m.seg[s0 + q];  // ring offset, ring size, first index, length
    // no branches around the loads: slots past the run re-read its last node
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int t = max(0, min(wave + i * nw, sg.w - 1));
      int ii = sg.z + t;
      if (ii >= sg.y) ii -= sg.y;
      regs[i] = vin[(size_t)(sg.x + ii) * L + k0 + lane_c];
    }
  };
  auto deposit = [&](int q) {
    const int len = m.seg[s0 + q].w;
    V *b = buf + (q & 3) * slot_stride;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int t = wave + i * nw;
      if (t < len && lane_on) b[t * kc + lane] = regs[i];
    }
  };

  // first and last parallel with positions of this tile
  int qa = nseg, qb = -1;
  for (int q = 0; q < nseg; ++q) {
    const int2 pr = m.seg_pos[s0 + q];
    if (pr.y > pr.x) {
      qa = min(qa, q);
      qb = q;
    }
  }
  if (qb < 0) return;
  for (int q = 0; q <= min(nseg - 1, qa + 1); ++q) {
    fetch(q);
    deposit(q);
  }
  __syncthreads();
  for (int q = qa; q <= qb; ++q) {
    const bool pf = q + 2 < nseg;
    if (pf) fetch(q + 2);
    const int2 pr = m.seg_pos[s0 + q];
    if (lane_on) {
      const V *bq = buf + (q & 3) * slot_stride;
      for (int p = pr.x + wave; p < pr.y; p += nw) {
        const PosRec rec = m.pos[p];
        const int node = rec.node, r0 = rec.r0, r1 = rec.r1, ts = rec.selfslot;
        const double ci = P::kVecIn ? m.coslat[node] : 0.0;
        typename P::St st;
        P::init(st, bq[ts * kc + lane], ci);
        double cx = 0.0, cy = 0.0;
        for (int rb = r0; rb < r1; rb += G) {
          // all loads of the group first (indices clamped into the row),
          // then the accumulation in row order
          int lr[G];
          double2 S[G];
          V xn[G];
          double cn[G];
#pragma unroll
          for (int j = 0; j < G; ++j) {  // whole group, contiguous (arrays padded)
            lr[j] = m.lref[rb + j];
            S[j] = m.S[rb + j];
            cn[j] = P::kVecIn ? m.ncos[rb + j] : 0.0;
          }
#pragma unroll
          for (int j = 0; j < G; ++j) {
            const int l = lr[j] & ~kLrefPole;
            xn[j] = buf[((q + (l >> 16) - 1) & 3) * slot_stride + (l & 0xffff) * kc + lane];
          }
#pragma unroll
          for (int j = 0; j < G; ++j) {
            if (rb + j >= r1) break;
            const bool pole = (lr[j] & kLrefPole) != 0;
            if (P::kVecIn && pole) continue;
            closure_add<OP>(cx, cy, S[j], pole);
            P::add(st, xn[j], S[j], pole, cn[j]);
          }
        }
        const double al = rec.alpha, be = P::kVecOut ? rec.beta : 0.0;
        P::store(out, (size_t)node * L + k0 + lane, st, al, be, cx, cy, ci);
      }
    }
    if (pf) deposit(q + 2);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Flat form: lanes over flattened (position, level) pairs of the tile --
// full lanes for short columns (nlev = 1 .. 40).
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Level-vector sweep form.  As the parallel sweep above, but every LDS entry
// and every lane holds a lane vector of NV levels (16 bytes), a workgroup
// covers `vpc` lane vectors of every column (a level chunk), columns are
// staged into LDS with range-checked buffer loads (one pass over each
// column per chunk, coalesced over the run), and each position's result is
// written with buffer stores (lanes past the chunk make no access).  The
// geometry of the positions is staged into LDS as well, one step ahead (the
// position records of run q+2 and the incidence rows of run q+1 while run
// q is computed), so a position needs no dependent scalar loads: per step
// the chain is one LDS read of its record and rows, one of its neighbours.
// ---------------------------------------------------------------------------
constexpr int kSweepEpt = 4;   // staged lane vectors per thread and run
constexpr int kGeoWords = 11;  // 16-byte words of staged rows per position:
                               // S[6] (6), lref[8] (2), ncos[6] (3)
constexpr int kSweepMinTiles = 1024;  // tiles below which the default stays
                                      // with the column form

template <class T, int OP, int NV, int EPT>
__global__ void __launch_bounds__(1024) k_sweepv(DevMesh m, const T *__restrict__ in,
                                                 T *__restrict__ out, int nlev, int vpc,
                                                 int ntiles, int per_xcd) {
  using P = Pol<T, OP>;
  using V = typename P::V;
  using LV = LaneVec<V, NV>;
  using R = typename LV::raw;
  using Out = typename P::Out;
  constexpr int WPP = P::kVecIn ? kGeoWords : 8;  // rows words staged per position
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int segmax = m.segmax;
  R *buf = reinterpret_cast<R *>(smem_raw);                        // [4][segmax][vpc]
  i32x4 *gpos = reinterpret_cast<i32x4 *>(buf + 4 * segmax * vpc);  // [4][segmax][2]
  i32x4 *grow = gpos + 4 * segmax * 2;                              // [4][segmax][kGeoWords]
  // chunk-minor order: the chunks of a tile run next to each other on one
  // XCD, so the geometry and the cache lines a chunk boundary splits are
  // fetched once into its L2
  const int u = xcd_tile(blockIdx.x, per_xcd);
  const int nvec = (nlev + NV - 1) / NV;
  const int nchunk = (nvec + vpc - 1) / vpc;
  const int tile = u / nchunk;
  const int c = u - tile * nchunk;
  if (tile >= ntiles) return;
  const int v0 = c * vpc;
  if (v0 >= nvec) return;
  const int nvc = min(vpc, nvec - v0);  // lane vectors in this chunk
  const int s0 = cst(m.tile_seg)[tile];
  const int nseg = cst(m.tile_seg)[tile + 1] - s0;
  const int slot_stride = segmax * vpc;  // lane vectors per LDS slot
  const V *vin = reinterpret_cast<const V *>(in);
  const size_t L = (size_t)nlev;
  const uint32_t col_bytes = (uint32_t)(L * sizeof(V));
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int *segi = reinterpret_cast<const int *>(m.seg);
  const int *segp = reinterpret_cast<const int *>(m.seg_pos);
  auto first = [&](int k) { return min(NV * (v0 + k), nlev - NV); };
  auto run_lo = [&](int q) { return cst(segp)[2 * (s0 + q)]; };
  auto run_hi = [&](int q) { return cst(segp)[2 * (s0 + q) + 1]; };

  // ---- columns: item = (node t of the segment, lane vector k); a thread's
  // items are the same every step (computed once)
  R regs[EPT];
  int it_t[EPT], it_off[EPT], it_lds[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = threadIdx.x + e * (int)blockDim.x;
    const int t = i / nvc, k = i - t * nvc;
    it_t[e] = t;
    it_off[e] = first(k) * (int)sizeof(V);
    it_lds[e] = t * vpc + k;
  }
  int seg_len = 0;
  auto fetch = [&](int q) {
    const int rb = cst(segi)[4 * (s0 + q)], nx = cst(segi)[4 * (s0 + q) + 1];
    const int lo = cst(segi)[4 * (s0 + q) + 2];
    seg_len = cst(segi)[4 * (s0 + q) + 3];
    const i32x4 rs = make_rsrc(vin + (size_t)rb * L, (uint32_t)nx * col_bytes);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      int ii = lo + it_t[e];
      if (ii >= nx) ii -= nx;
      const int off = it_t[e] < seg_len ? ii * (int)col_bytes + it_off[e] : kBufOff;
      regs[e] = buf_load<R>(rs, off);
    }
  };
  auto deposit = [&](int q) {
    R *b = buf + (q & 3) * slot_stride;
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (it_t[e] < seg_len) b[it_lds[e]] = regs[e];
  };
  // ---- position records of run q (2 words each) and rows of run q (WPP
  // words each, at the record's first incidence); a thread moves at most one
  // word of each kind per step (the dispatch guarantees the block is large
  // enough)
  i32x4 preg = {0, 0, 0, 0}, rreg = {0, 0, 0, 0};
  int pitem = -1, ritem = -1;
  auto fetch_pos = [&](int q) {
    const int plo = run_lo(q), n = run_hi(q) - plo;
    pitem = (int)threadIdx.x < 2 * n ? (int)threadIdx.x : -1;
    if (pitem >= 0) {
      const i32x4 *src = reinterpret_cast<const i32x4 *>(m.pos + plo + (pitem >> 1)) + (pitem & 1);
      preg = *src;
    }
  };
  auto deposit_pos = [&](int q) {
    if (pitem >= 0) gpos[((q & 3) * segmax) * 2 + pitem] = preg;
  };
  auto fetch_rows = [&](int q) {
    const int n = run_hi(q) - run_lo(q);
    ritem = (int)threadIdx.x < WPP * n ? (int)threadIdx.x : -1;
    if (ritem >= 0) {
      const int t = ritem / WPP, w = ritem - t * WPP;
      const int r0 = gpos[((q & 3) * segmax + t) * 2].y;  // staged record: node, r0, r1, slot
      const unsigned char *src;
      if (w < 6) src = reinterpret_cast<const unsigned char *>(m.S + r0 + w);
      else if (w < 8) src = reinterpret_cast<const unsigned char *>(m.lref + r0) + 16 * (w - 6);
      else src = reinterpret_cast<const unsigned char *>(m.ncos + r0) + 16 * (w - 8);
      i32x4 v;
      __builtin_memcpy(&v, src, 16);
      rreg = v;
    }
  };
  auto deposit_rows = [&](int q) {
    if (ritem >= 0) {
      const int t = ritem / WPP, w = ritem - t * WPP;
      grow[((q & 3) * segmax + t) * kGeoWords + w] = rreg;
    }
  };

  // first and last parallel with positions of this tile
  int qa = nseg, qb = -1;
  for (int q = 0; q < nseg; ++q) {
    if (run_hi(q) > run_lo(q)) {
      qa = min(qa, q);
      qb = q;
    }
  }
  if (qb < 0) return;
  for (int q = 0; q <= min(nseg - 1, qa + 1); ++q) {
    fetch(q);
    deposit(q);
  }
  fetch_pos(qa);
  deposit_pos(qa);
  if (qa + 1 < nseg) {
    fetch_pos(qa + 1);
    deposit_pos(qa + 1);
  }
  __syncthreads();
  fetch_rows(qa);
  deposit_rows(qa);
  __syncthreads();

  const int kc = min(lane, nvc - 1);  // lanes past the chunk read a valid entry
  const int s_l = first(kc);
  const bool lane_on = lane < nvc;
  for (int q = qa; q <= qb; ++q) {
    const bool pf = q + 2 < nseg;
    if (pf) {
      fetch(q + 2);
      fetch_pos(q + 2);
    }
    const bool rf = q + 1 < nseg;
    if (rf) fetch_rows(q + 1);
    const int plo = run_lo(q), phi = run_hi(q);
    const R *bq = buf + (q & 3) * slot_stride;
    const i32x4 *gp = gpos + (q & 3) * segmax * 2;
    const i32x4 *gr = grow + (q & 3) * segmax * kGeoWords;
    for (int p = plo + wave; p < phi; p += nw) {
      const int t = p - plo;
      const i32x4 w0 = gp[2 * t], w1 = gp[2 * t + 1];
      const int node = w0.x, n = w0.z - w0.y, selfslot = w0.w;
      double al, be;
      {
        const int a2[2] = {w1.x, w1.y}, b2[2] = {w1.z, w1.w};
        __builtin_memcpy(&al, a2, 8);
        __builtin_memcpy(&be, b2, 8);
      }
      if (!P::kVecOut) be = 0.0;
      const double ci = P::kVecIn ? cst(m.coslat)[node] : 0.0;
      constexpr int G = 6;
      double2 S[G];
      int lr[8];
      double cn[G];
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const i32x4 v = gr[t * kGeoWords + j];
        __builtin_memcpy(&S[j], &v, 16);
      }
      {
        const i32x4 a = gr[t * kGeoWords + 6], b = gr[t * kGeoWords + 7];
        lr[0] = a.x; lr[1] = a.y; lr[2] = a.z; lr[3] = a.w;
        lr[4] = b.x; lr[5] = b.y; lr[6] = b.z; lr[7] = b.w;
      }
      if (P::kVecIn) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const i32x4 v = gr[t * kGeoWords + 8 + k];
          __builtin_memcpy(&cn[2 * k], &v, 16);
        }
      } else {
#pragma unroll
        for (int j = 0; j < G; ++j) cn[j] = 0.0;
      }
      typename P::St st[NV];
      {
        const R xi = bq[selfslot * vpc + kc];
#pragma unroll
        for (int v = 0; v < NV; ++v) P::init(st[v], LV::get(xi, v), ci);
      }
      R xn[G];
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const int l = lr[j] & ~kLrefPole;
        xn[j] = buf[((q + ((l >> 16) & 3) - 1) & 3) * slot_stride + (l & 0xffff) * vpc + kc];
      }
      double cx = 0.0, cy = 0.0;
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const bool pole = (lr[j] & kLrefPole) != 0;
        if (j < kMinRow) {  // present in every row, never the pole edge
          closure_add<P::kOp>(cx, cy, S[j], false);
#pragma unroll
          for (int v = 0; v < NV; ++v) P::add(st[v], LV::get(xn[j], v), S[j], false, cn[j]);
          continue;
        }
        const bool use = j < n && !(P::kVecIn && pole);
        double tx = cx, ty = cy;
        closure_add<P::kOp>(tx, ty, S[j], pole);
        cx = use ? tx : cx;
        cy = use ? ty : cy;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          typename P::St tt = st[v];
          P::add(tt, LV::get(xn[j], v), S[j], pole, cn[j]);
          P::keep(st[v], tt, use);
        }
      }
      const i32x4 ro = make_rsrc(out + (size_t)node * L * (sizeof(Out) / sizeof(T)),
                                 (uint32_t)(L * sizeof(Out)));
      constexpr int W = NV * (int)sizeof(Out) / 4;
      int w[W];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const Out r = P::result(st[v], al, be, cx, cy, ci);
        __builtin_memcpy(&w[v * (int)sizeof(Out) / 4], &r, sizeof(Out));
      }
      const int ob = lane_on ? s_l * (int)sizeof(Out) : kBufOff;
      buf_store_words<W>(w, ro, ob);
    }
    if (pf) {
      deposit(q + 2);
      deposit_pos(q + 2);
    }
    if (rf) deposit_rows(q + 1);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Wave-specialised sweep.  The same walk down a tile's band as k_sweepv, but
// the waves of a workgroup split the work: producer waves only move data
// into LDS, with buffer loads that write LDS directly (no registers, no
// deposit pass), and consumer waves only compute from LDS and store
// results.  One vector-memory counter per wave counts loads and stores
// alike and retires them in order; so a wave that both stored results and
// later waited for its next loads would wait for those stores too.  Here the
// consumers never wait on memory (their stores drain while the next
// parallels are computed) and the producers wait only for their own loads.
// The producers form two groups that take alternate runs: at step q the
// group of run q+3 loads its columns and packed geometry into ring slot
// (q+3) mod 5, and at the end of step q the other group waits for run q+2,
// which it issued one step earlier -- so every load has two steps to land.
// The consumers compute the own positions of run q from slots q-1, q, q+1.
// The roles run separate loops that meet at one workgroup barrier per step.
// Lane vectors are 16 bytes (FP64: 2 levels of a scalar, 1 of a vector;
// FP32: 4 of a scalar, 2 of a vector).  Items of a slot are numbered (node
// of the run) x (lane vector of the chunk), so each load instruction fills
// 64 consecutive 16-byte LDS words.  The packed normals are halved (exact):
// the FP64 edge term sS (x_i + x_n)/2 is formed as (sS/2)(x_i + x_n) with the
// same bits and one multiplication less.
// ---------------------------------------------------------------------------
constexpr int kSgeoWords = 14;  // packed sweep geometry per position (16-byte
                                // words): {node, n, selfslot, 0}, (alpha,
                                // beta), S[6] / 2, lref[8], ncos[6],
                                // (cos lat, 0)
// Positions per wavefront: as many as 64 lanes hold chunks of (at most 8)
// 8 lane vectors: eight, 12: five, 16: four, 21: three, 32: two; wider
// chunks one.
constexpr int kSweepwNpn8 = 8;
constexpr int kSweepwGroups = 2;     // producer groups (runs taken in turn)
constexpr int kSweepwLead = kSweepwGroups + 1;  // run q + lead issued at step q
constexpr int kSweepwSlots = kSweepwLead + 2;   // field ring: runs q-1 .. q+lead
constexpr int kSweepwGeoSlots = kSweepwLead + 1;  // geometry ring: runs q ..
                                                  // q+lead (the consumers read
                                                  // only run q's records)
// Waves per producer group: two for every operator (with the item indices
// advanced incrementally, a second producer wave made the FP64 divergence
// sweep faster too: 7.84 -> 7.62 ms at O1280, 137 levels; 2.08 -> 1.97 ms
// at 37 levels).
template <int OP> constexpr int sweepw_group_waves() { return 2; }

__device__ __forceinline__ void lds_dma16(const i32x4 &rsrc, void *lds_wave_base, int voff) {
  __amdgpu_buffer_rsrc_t r;
  __builtin_memcpy(&r, &rsrc, 16);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(
      r, (__attribute__((address_space(3))) void *)lds_wave_base, 16, voff, 0, 0, 0);
}

// The FP64 edge terms with halved normals (bits of Pol<double, *>::add).
__device__ __forceinline__ void sweep_add_half(Pol<double, OP_GRAD>::St &s, double xn,
                                               const double2 &Sh, bool pole, double) {
  const double xe = s.xi + xn;
  if (!pole) s.gl = s.gl + Sh.x * xe;
  s.gt = s.gt + Sh.y * xe;
}
template <int OP>
__device__ __forceinline__ void sweep_add_half(typename PolDC64<OP>::St &s, v2d un,
                                               const double2 &Sh, bool, double cn) {
  const double an = (OP == OP_DIV) ? un.x : un.y;
  const double bn = ((OP == OP_DIV) ? un.y : un.x) * cn;
  const double ae = s.ai + an, be = s.bi + bn;
  const double f = (OP == OP_DIV) ? Sh.x * ae + Sh.y * be : Sh.x * ae - Sh.y * be;
  s.acc = s.acc + f;
}

template <class T, int OP>
__device__ __forceinline__ void sweep_term(typename Pol<T, OP>::St &s,
                                           typename Pol<T, OP>::V xn, const double2 &Sh,
                                           bool pole, double cn) {
  if constexpr (sizeof(T) == 8) {
    if constexpr (OP == OP_GRAD) sweep_add_half(s, xn, Sh, pole, cn);
    else sweep_add_half<OP>(s, xn, Sh, pole, cn);
  } else {
    Pol<T, OP>::add(s, xn, make_double2(Sh.x + Sh.x, Sh.y + Sh.y), pole, cn);
  }
}

// DC (OP = OP_DIV only): the curl of the same field as well, into out2,
// from the same loads; each output bitwise that of its own operator.
template <class T, int OP, int NV, int NPN, bool DC = false>
__global__ void __launch_bounds__(1024) k_sweepw(DevMesh m, const T *__restrict__ in,
                                                 T *__restrict__ out, T *__restrict__ out2,
                                                 int nlev, int vpc, int ntiles, int per_xcd,
                                                 int fcap, int gcap) {
  static_assert(!DC || OP == OP_DIV, "the one-pass curl rides on the divergence");
  using P = Pol<T, OP>;
  using PC = Pol<T, OP_CURL>;
  using V = typename P::V;
  using LV = LaneVec<V, NV>;
  using R = typename LV::raw;
  using Out = typename P::Out;
  static_assert(sizeof(R) == 16, "wave-specialised sweep: 16-byte lane vectors");
  constexpr int GW = P::kVecIn ? kSgeoWords : 10;  // geometry words read per position
  constexpr int kSweepwGroupWaves = sweepw_group_waves<OP>();
  constexpr int NPW = kSweepwGroups * kSweepwGroupWaves;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R *fbuf = reinterpret_cast<R *>(smem_raw);                           // [field slots][fcap]
  i32x4 *gbuf = reinterpret_cast<i32x4 *>(fbuf + kSweepwSlots * fcap);  // [geometry slots][gcap]
  const int u = xcd_tile(blockIdx.x, per_xcd);
  const int nvec = (nlev + NV - 1) / NV;
  const int nchunk = (nvec + vpc - 1) / vpc;
  const int tile = u / nchunk;
  const int c = u - tile * nchunk;
  if (tile >= ntiles) return;
  const int v0 = c * vpc;
  if (v0 >= nvec) return;
  const int nvc = min(vpc, nvec - v0);  // lane vectors in this chunk
  const int s0 = cst(m.tile_seg)[tile];
  const int nseg = cst(m.tile_seg)[tile + 1] - s0;
  const size_t L = (size_t)nlev;
  const uint32_t col_bytes = (uint32_t)(L * sizeof(V));
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int lane = threadIdx.x & 63;
  const int *segi = reinterpret_cast<const int *>(m.seg);
  const int *segp = reinterpret_cast<const int *>(m.seg_pos);
  auto run_lo = [&](int q) { return cst(segp)[2 * (s0 + q)]; };
  auto run_hi = [&](int q) { return cst(segp)[2 * (s0 + q) + 1]; };
  // first and last parallel with positions of this tile
  int qa = nseg, qb = -1;
  for (int q = 0; q < nseg; ++q) {
    if (run_hi(q) > run_lo(q)) {
      qa = min(qa, q);
      qb = q;
    }
  }
  if (qb < 0) return;

  if (wave < NPW) {
    // ---- producers: group grp loads the runs r with r mod groups = grp ----
    const int grp = wave / kSweepwGroupWaves, gwave = wave - grp * kSweepwGroupWaves;
    const V *vin = reinterpret_cast<const V *>(in);
    // columns and geometry of run q into the ring slots of q, the waves of
    // the calling group (or, with nwv = NPW, all producers) sharing the
    // load instructions
    auto load = [&](int q, int w, int nwv) {
      const int sl = q % kSweepwSlots;
      {
        const int rb = cst(segi)[4 * (s0 + q)], nx = cst(segi)[4 * (s0 + q) + 1];
        const int lo = cst(segi)[4 * (s0 + q) + 2], len = cst(segi)[4 * (s0 + q) + 3];
        const i32x4 rs = make_rsrc(vin + (size_t)rb * L, (uint32_t)nx * col_bytes);
        const int nitems = len * nvc;
        R *slot = fbuf + sl * fcap;
        // item i = (node t of the run) x (lane vector k); t and k advance
        // by whole strides of the calling waves' load instructions
        const int i0 = w * 64 + lane, di = nwv * 64;
        int t = i0 / nvc, k = i0 - t * nvc;
        const int dt = di / nvc, dk = di - dt * nvc;
        for (int b = w; b * 64 < nitems; b += nwv) {
          int off = kBufOff;
          if (b * 64 + lane < nitems) {
            int ii = lo + t;
            if (ii >= nx) ii -= nx;
            off = ii * (int)col_bytes + min(NV * (v0 + k), nlev - NV) * (int)sizeof(V);
          }
          lds_dma16(rs, slot + b * 64, off);
          t += dt;
          k += dk;
          if (k >= nvc) {
            k -= nvc;
            ++t;
          }
        }
      }
      {
        const int plo = run_lo(q), n = run_hi(q) - plo;
        const i32x4 rs = make_rsrc(m.sgeo + (size_t)plo * kSgeoWords,
                                   (uint32_t)n * kSgeoWords * 16u);
        const int nitems = n * GW;
        i32x4 *slot = gbuf + (q % kSweepwGeoSlots) * gcap;
        for (int b = w; b * 64 < nitems; b += nwv) {
          const int i = b * 64 + lane;
          int off = kBufOff;
          if (i < nitems) {
            const int t = i / GW, wd = i - t * GW;
            off = (t * kSgeoWords + wd) * 16;
          }
          lds_dma16(rs, slot + b * 64, off);
        }
      }
    };
    // prologue: runs qa-1 .. qa+1 by every producer (waited), runs qa+2 ..
    // qa+lead-1 by their groups (run r waited at the end of step r-2)
    for (int q = max(0, qa - 1); q <= min(nseg - 1, qa + 1); ++q) load(q, wave, NPW);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    for (int r = qa + 2; r < min(nseg, qa + kSweepwLead); ++r)
      if (r % kSweepwGroups == grp) load(r, gwave, kSweepwGroupWaves);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    for (int q = qa; q <= qb; ++q) {
      if (q + kSweepwLead < nseg && (q + kSweepwLead) % kSweepwGroups == grp)
        load(q + kSweepwLead, gwave, kSweepwGroupWaves);
      // run q+2 (issued lead-2 steps ago by its group, which has issued
      // nothing since) is in LDS before step q+1 reads it
      if ((q + 2) % kSweepwGroups == grp) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
    }
    // loads of runs past qb + 2 are never read; let them land before exit
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    return;
  }

  // ---- consumers ----------------------------------------------------------
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
  const int cw = wave - NPW, ncw = nw - NPW;
  // NPN positions per wavefront, 64 / NPN lanes each (chunks of at most
  // 64 / NPN lane vectors); where NPN does not divide 64 the lanes left over
  // repeat the last position's first lanes and store nothing
  constexpr int LPN = 64 / NPN;
  const int sub_raw = NPN > 1 ? lane / LPN : 0;
  const int sub = min(sub_raw, NPN - 1);
  const int hl = lane - sub_raw * LPN;
  const int kc = min(hl, nvc - 1);  // lanes past the chunk read a valid entry
  const bool lane_on = sub_raw < NPN && hl < nvc;
  // Lanes whose results exceed 16 bytes (the gradient: two components at
  // NV levels) would make every store instruction strided, each lane
  // writing part of its own piece of the row.  Such a lane takes NG groups
  // of GS adjacent levels (16 bytes of output each), one from each of the
  // chunk's NG equal parts: group g holds level slots g GS nvc + GS kc + e,
  // so the g-th store of the lanes covers one contiguous run of the row.
  // Every level goes through the same arithmetic: the bits are unchanged.
  constexpr bool kSplit = NV * sizeof(Out) > 16;
  constexpr int GS = kSplit ? (int)(16 / sizeof(Out)) : NV;  // levels per group
  constexpr int NG = NV / GS;
  static_assert(!kSplit || (ElemOf<V>::C == 1 && NV % GS == 0), "split lanes: scalar inputs");
  int s_g[NG];  // first output level of each group
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int p = kSplit ? g * GS * nvc + GS * kc : NV * kc;  // slot in the chunk
    s_g[g] = min(NV * (v0 + p / NV), nlev - NV) + p % NV;
  }
  // the lane's NV levels of the chunk row starting at lane vector `base`
  auto ldrow = [&](int base) {
    if constexpr (kSplit) {
      struct Grp { typename ElemOf<V>::E e[GS]; };
      const Grp *fv = reinterpret_cast<const Grp *>(fbuf + base);
      R r;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const Grp x = fv[g * nvc + kc];
        __builtin_memcpy(&r.e[g * GS], x.e, sizeof(Grp));
      }
      return r;
    } else {
      return fbuf[base + kc];
    }
  };
  int sq = qa % kSweepwSlots;           // slot of run q
  for (int q = qa; q <= qb; ++q) {
    const int plo = run_lo(q), phi = run_hi(q);
    const int sm = sq == 0 ? kSweepwSlots - 1 : sq - 1;  // slot of run q-1
    const int sp = sq == kSweepwSlots - 1 ? 0 : sq + 1;  // slot of run q+1
    const i32x4 *gq = gbuf + (q % kSweepwGeoSlots) * gcap;
    for (int p = plo + NPN * cw + sub; p < phi; p += NPN * ncw) {
      const i32x4 *g = gq + (p - plo) * GW;
      const i32x4 w0 = g[0], w1 = g[1];
      const int node = w0.x, n = w0.y, selfslot = w0.z;
      double al, be;
      {
        const int a2[2] = {w1.x, w1.y}, b2[2] = {w1.z, w1.w};
        __builtin_memcpy(&al, a2, 8);
        __builtin_memcpy(&be, b2, 8);
      }
      if (!P::kVecOut) be = 0.0;
      constexpr int G = 6;
      double2 Sh[G];
      int lr[8];
      double cn[G];
      double ci = 0.0;
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const i32x4 v = g[2 + j];
        __builtin_memcpy(&Sh[j], &v, 16);
      }
      {
        const i32x4 a = g[8], b = g[9];
        lr[0] = a.x; lr[1] = a.y; lr[2] = a.z; lr[3] = a.w;
        lr[4] = b.x; lr[5] = b.y; lr[6] = b.z; lr[7] = b.w;
      }
      if constexpr (P::kVecIn) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const i32x4 v = g[10 + k];
          __builtin_memcpy(&cn[2 * k], &v, 16);
        }
        const i32x4 v = g[13];
        const int cc[2] = {v.x, v.y};
        __builtin_memcpy(&ci, cc, 8);
      } else {
#pragma unroll
        for (int j = 0; j < G; ++j) cn[j] = 0.0;
      }
      typename P::St st[NV];
      typename PC::St stc[DC ? NV : 1];
      {
        const R xi = ldrow(sq * fcap + selfslot * nvc);
#pragma unroll
        for (int v = 0; v < NV; ++v) P::init(st[v], LV::get(xi, v), ci);
        if constexpr (DC) {
#pragma unroll
          for (int v = 0; v < NV; ++v) PC::init(stc[v], LV::get(xi, v), ci);
        }
      }
      R xn[G];
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const int l = lr[j] & ~kLrefPole;
        const int dq = (l >> 16) & 3;  // 0: run q-1, 1: run q, 2: run q+1
        const int sl = dq == 0 ? sm : (dq == 1 ? sq : sp);
        xn[j] = ldrow(sl * fcap + (l & 0xffff) * nvc);
      }
      double cx = 0.0, cy = 0.0;  // closure sums (FP32 forms): full normals
      double ccx = 0.0, ccy = 0.0;  // the curl's (DC)
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const bool pole = (lr[j] & kLrefPole) != 0;
        const double2 S2 = make_double2(Sh[j].x + Sh[j].x, Sh[j].y + Sh[j].y);
        if (j < kMinRow) {  // present in every row, never the pole edge
          if constexpr (sizeof(T) == 4) closure_add<P::kOp>(cx, cy, S2, false);
          if constexpr (sizeof(T) == 4 && DC) closure_add<OP_CURL>(ccx, ccy, S2, false);
#pragma unroll
          for (int v = 0; v < NV; ++v) sweep_term<T, OP>(st[v], LV::get(xn[j], v), Sh[j], false, cn[j]);
          if constexpr (DC) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
              sweep_term<T, OP_CURL>(stc[v], LV::get(xn[j], v), Sh[j], false, cn[j]);
          }
          continue;
        }
        const bool use = j < n && !(P::kVecIn && pole);
        if constexpr (sizeof(T) == 4) {
          double tx = cx, ty = cy;
          closure_add<P::kOp>(tx, ty, S2, pole);
          cx = use ? tx : cx;
          cy = use ? ty : cy;
          if constexpr (DC) {
            double ux = ccx, uy = ccy;
            closure_add<OP_CURL>(ux, uy, S2, pole);
            ccx = use ? ux : ccx;
            ccy = use ? uy : ccy;
          }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          typename P::St tt = st[v];
          sweep_term<T, OP>(tt, LV::get(xn[j], v), Sh[j], pole, cn[j]);
          P::keep(st[v], tt, use);
        }
        if constexpr (DC) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            typename PC::St tt = stc[v];
            sweep_term<T, OP_CURL>(tt, LV::get(xn[j], v), Sh[j], pole, cn[j]);
            PC::keep(stc[v], tt, use);
          }
        }
      }
      constexpr int W = NV * (int)sizeof(Out) / 4;
      int wd[W];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const Out r = P::result(st[v], al, be, cx, cy, ci);
        __builtin_memcpy(&wd[v * (int)sizeof(Out) / 4], &r, sizeof(Out));
      }
      auto store_row = [&](T *dst, const int (&w)[W]) {
        if constexpr (kSplit) {
          // one contiguous run per group (16 bytes per lane)
          const size_t ew = sizeof(Out) / sizeof(T);
          const i32x4 ro = make_rsrc(dst + (size_t)node * L * ew, (uint32_t)(L * sizeof(Out)));
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            const i32x4 v4 = {w[4 * g], w[4 * g + 1], w[4 * g + 2], w[4 * g + 3]};
            if constexpr (NPN == 1) {
              buf_store16(v4, ro, lane_on ? s_g[g] * (int)sizeof(Out) : kBufOff, 0, kStoreAux);
            } else if (lane_on) {
              *reinterpret_cast<i32x4 *>(dst + ((size_t)node * L + s_g[g]) * ew) = v4;
            }
          }
        } else if constexpr (NPN == 1) {
          // one position per wavefront: a buffer store over its row (the
          // resource is wavefront-uniform)
          const i32x4 ro = make_rsrc(dst + (size_t)node * L * (sizeof(Out) / sizeof(T)),
                                     (uint32_t)(L * sizeof(Out)));
          const int ob = lane_on ? s_g[0] * (int)sizeof(Out) : kBufOff;
          buf_store_words<W>(w, ro, ob);
        } else if (lane_on) {
          // several positions per wavefront: a store through each lane's
          // own address
          struct Words { int v[W]; } o;
          __builtin_memcpy(o.v, w, sizeof(o));
          *reinterpret_cast<Words *>(dst + ((size_t)node * L + s_g[0]) * (sizeof(Out) / sizeof(T))) = o;
        }
      };
      store_row(out, wd);
      if constexpr (DC) {
        static_assert(sizeof(typename PC::Out) == sizeof(Out), "curl output type");
        int wc[W];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const typename PC::Out r = PC::result(stc[v], al, be, ccx, ccy, ci);
          __builtin_memcpy(&wc[v * (int)sizeof(Out) / 4], &r, sizeof(Out));
        }
        store_row(out2, wc);
      }
    }
    // this step's LDS reads are done before the producers refill a slot
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    sq = sp;
  }
}

// ---------------------------------------------------------------------------
// Fused Laplacian: one pass over the two-ring plan.  A workgroup owns one
// tile and one chunk of lane vectors and walks the tile's window of
// parallels.  At step q it forms the gradient at every node of the g-run of
// parallel q from the field runs q-1, q, q+1 (LDS) into a 4-slot LDS ring,
// and the divergence of those gradients at the tile's own positions of
// parallel q-2 from the g-runs q-3, q-2, q-1 (the ring slot written at step
// q held the g-run of q-4, last read at step q-1).  Meanwhile it loads the
// field run of parallel q+2 and the packed geometry of step q+1 (records of
// the g-run q+1 and of the own positions of parallel q-1) into registers
// and deposits them in LDS after the compute, so the compute reads nothing
// but LDS.  Every gradient goes through the gradient policy and is rounded
// to its output type exactly as the two-pass form stores it, and every
// divergence through the divergence policy: the result is bitwise that of
// the two passes.
// ---------------------------------------------------------------------------
constexpr int kGGeoWords = 10;  // packed gradient-node record (16-byte words):
                                // S[6] / 2, refs[8], (alpha, beta),
                                // (f self, n, cos lat)
constexpr int kLGeoWords = 13;  // packed own-position record: S[6] / 2,
                                // refs[8], (alpha, cos lat), (node, n, g self),
                                // ncos[6] (FP32 only: the FP64 kernel stages
                                // the first kLGeoWords64 words)
constexpr int kLGeoWords64 = 10;
constexpr int kGeoEpt = 2;      // geometry words a thread stages per step
constexpr int kLsweepEpt = 2;   // field lane vectors a thread stages per step

// FP64 steps of the fused Laplacian with halved normals Sh = S / 2 (exact):
// (xi + xn) Sh rounds like S (0.5 (xi + xn)), so these give the bits of
// Pol<double, OP_GRAD>::add and PolDC64<OP_DIV>::add (operands not
// subnormal).  For the divergence the second component arrives as
// w = v cos(lat), the product PolDC64 forms from v and the node's cos(lat).
__device__ __forceinline__ void grad_add_half(Pol<double, OP_GRAD>::St &s, double xn,
                                              const double2 &Sh, bool pole) {
  const double xe = s.xi + xn;
  if (!pole) s.gl = s.gl + Sh.x * xe;
  s.gt = s.gt + Sh.y * xe;
}
__device__ __forceinline__ void div_init_w(PolDC64<OP_DIV>::St &s, const v2d &uw) {
  s.ai = uw.x;
  s.bi = uw.y;
  s.acc = 0.0;
}
__device__ __forceinline__ void div_add_half_w(PolDC64<OP_DIV>::St &s, const v2d &uw,
                                               const double2 &Sh) {
  const double ae = s.ai + uw.x, be = s.bi + uw.y;
  s.acc = s.acc + (Sh.x * ae + Sh.y * be);
}
// (overloads for the FP32 instantiation, never called)
__device__ __forceinline__ void grad_add_half(Pol<float, OP_GRAD>::St &, float, const double2 &,
                                              bool) {}
__device__ __forceinline__ void div_init_w(PolDC32<OP_DIV>::St &, const v2f &) {}
__device__ __forceinline__ void div_add_half_w(PolDC32<OP_DIV>::St &, const v2f &,
                                               const double2 &) {}

__device__ __forceinline__ int4 cst_int4(const int4 *p, size_t i) {
  const ATLASX_CST int *d = cst(reinterpret_cast<const int *>(p));
  return make_int4(d[4 * i], d[4 * i + 1], d[4 * i + 2], d[4 * i + 3]);
}
__device__ __forceinline__ int2 cst_int2(const int2 *p, size_t i) {
  const ATLASX_CST int *d = cst(reinterpret_cast<const int *>(p));
  return make_int2(d[2 * i], d[2 * i + 1]);
}

template <class T, int NV, int EPT, int NL>
__global__ void __launch_bounds__(1024) k_lsweep(DevMesh m, const T *__restrict__ in,
                                                 T *__restrict__ out, int nlev, int vpc,
                                                 int ntiles, int per_xcd, int lpn) {
  using PG = Pol<T, OP_GRAD>;
  using PD = Pol<T, OP_DIV>;
  using LF = LaneVec<T, NV>;
  using RF = typename LF::raw;         // NV levels of the field
  using GV = typename PD::V;           // gradient (zonal, meridional) of one level
  using LG = LaneVec<GV, NV>;
  using RG = typename LG::raw;         // NV levels of the gradient
  static_assert(sizeof(typename PG::Out) == sizeof(GV), "gradient output type");
  constexpr int G = 6;
  // FP64 keeps the second gradient component multiplied by cos(lat) in the
  // ring (the divergence's b = v cos(lat), formed once per node instead of
  // once per incidence) and uses the halved normals as they are
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int LGW = F64 ? kLGeoWords64 : kLGeoWords;  // own-position words staged
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int fmax = m.l2_fmax, gmax = m.l2_gmax;
  const int gw = gmax * kGGeoWords;                          // g part of a geometry slot
  const int geo_stride = gw + m.l2_pmax * LGW;               // words per geometry slot
  // the gradient ring holds each lane vector as two planes of its first
  // and second half (consecutive lanes then read consecutive 16-byte words)
  static_assert(sizeof(RG) == 2 * sizeof(RF), "gradient lane vector = two field lane vectors");
  RF *fbuf = reinterpret_cast<RF *>(smem_raw);               // [4][fmax][vpc]
  RF *gbuf = fbuf + 4 * fmax * vpc;                          // [4][gmax][2][vpc]
  i32x4 *geo = reinterpret_cast<i32x4 *>(gbuf + 8 * gmax * vpc);  // [2][geo_stride]
  const int fstride = fmax * vpc, gstride = 2 * gmax * vpc;
  auto gload = [&](int at) {  // at: ring slot offset + node * 2 * vpc + lane vector
    RG r;
    __builtin_memcpy(&r, &gbuf[at], sizeof(RF));
    __builtin_memcpy(reinterpret_cast<char *>(&r) + sizeof(RF), &gbuf[at + vpc], sizeof(RF));
    return r;
  };
  // chunk-minor order (as in k_sweepv): a tile's chunks share its geometry
  // and boundary lines through one XCD's L2
  const int u = xcd_tile(blockIdx.x, per_xcd);
  const int nvec = (nlev + NV - 1) / NV;
  const int nchunk = (nvec + vpc - 1) / vpc;
  const int tile = u / nchunk;
  const int c = u - tile * nchunk;
  if (tile >= ntiles) return;
  const int v0 = c * vpc;
  if (v0 >= nvec) return;
  const int nvc = min(vpc, nvec - v0);
  const int k0 = cst(m.l2_tile_seg)[tile];
  const int W = cst(m.l2_tile_seg)[tile + 1] - k0;
  const size_t L = (size_t)nlev;
  const uint32_t col_bytes = (uint32_t)(L * sizeof(T));
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  auto first = [&](int k) { return min(NV * (v0 + k), nlev - NV); };

  // ---- field runs: item = (node t of the run, lane vector k); a thread's
  // items are the same every step
  RF regs[EPT];
  int it_t[EPT], it_off[EPT], it_lds[EPT];  // it_off: byte offset of (t, k) from the run start
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = threadIdx.x + e * (int)blockDim.x;
    const int t = i / nvc, k = i - t * nvc;
    it_t[e] = t;
    it_off[e] = t * (int)col_bytes + first(k) * (int)sizeof(T);
    it_lds[e] = t * vpc + k;
  }
  int run_len = 0;
  auto fetch = [&](int q) {
    const int4 f = cst_int4(m.l2_fseg, k0 + q);  // {ring offset, ring size, first, length}
    run_len = f.w;
    const i32x4 rs = make_rsrc(in + (size_t)f.x * L, (uint32_t)f.y * col_bytes);
    const int start = f.z * (int)col_bytes, wrap = f.y * (int)col_bytes;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      int off = start + it_off[e];
      if (off >= wrap) off -= wrap;  // the run wraps round the parallel
      regs[e] = buf_load<RF>(rs, it_t[e] < run_len ? off : kBufOff);
    }
  };
  auto deposit = [&](int q) {
    RF *b = fbuf + (q & 3) * fstride;
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (it_t[e] < run_len) b[it_lds[e]] = regs[e];
  };
  // ---- packed geometry of step q: the g-run records of parallel q (words
  // [0, glen * kGGeoWords)) and the own-position records of parallel q - 2
  // (from word gw on), into slot q & 1
  // On deposit, the references of a record become LDS element offsets for
  // the step it serves (ring slot and run slot resolved, the pole flag
  // kept), and the self slots likewise, so the compute adds only the lane.
  // A thread's geometry items are fixed: item i < gw is word i % kGGeoWords
  // of g record i / kGGeoWords; item gw + j is word j % kLGeoWords of own
  // position record j / kLGeoWords.
  i32x4 greg[kGeoEpt];
  int gdst[kGeoEpt], gkind[kGeoEpt];  // kind: 0 plain, 1 f-refs, 2 f-self, 3 g-refs, 4 g-self
  int grec[kGeoEpt], gword[kGeoEpt];  // record index (-1: none) and word
  bool gisg[kGeoEpt], gon[kGeoEpt];
#pragma unroll
  for (int e = 0; e < kGeoEpt; ++e) {
    const int i = threadIdx.x + e * (int)blockDim.x;
    gdst[e] = i;
    gisg[e] = i < gw;
    if (i < gw) {
      grec[e] = i / kGGeoWords;
      gword[e] = i - grec[e] * kGGeoWords;
      gkind[e] = (gword[e] == 6 || gword[e] == 7) ? 1 : (gword[e] == 9) ? 2 : 0;
    } else if (i < geo_stride) {
      grec[e] = (i - gw) / LGW;
      gword[e] = (i - gw) - grec[e] * LGW;
      gkind[e] = (gword[e] == 6 || gword[e] == 7) ? 3 : (gword[e] == 9) ? 4 : 0;
    } else {
      grec[e] = -1;
      gword[e] = 0;
      gkind[e] = 0;
    }
    gon[e] = false;
  }
  auto fref = [&](int r, int qq) {
    const int l = r & ~kLrefPole;
    return (r & kLrefPole) | (((qq + ((l >> 16) & 3) - 1) & 3) * fstride + (l & 0xffff) * vpc);
  };
  auto gref = [&](int r, int qq) {
    const int l = r & ~kLrefPole;
    return (r & kLrefPole) | (((qq + ((l >> 16) & 3) - 1) & 3) * gstride + (l & 0xffff) * 2 * vpc);
  };
  auto fetch_geo = [&](int q) {
    int ng = 0, gb = 0, p0 = 0, np = 0;  // records of each kind this step
    if (q < W) {
      const int4 gs = cst_int4(m.l2_gseg, k0 + q);
      ng = gs.y;
      gb = gs.z;
    }
    if (q >= 2 && q - 2 < W) {
      const int2 sp = cst_int2(m.l2_seg_pos, k0 + q - 2);
      p0 = sp.x;
      np = sp.y - sp.x;
    }
#pragma unroll
    for (int e = 0; e < kGeoEpt; ++e) {
      gon[e] = grec[e] >= 0 && grec[e] < (gisg[e] ? ng : np);
      if (gon[e]) {
        const int4 *src = gisg[e] ? m.l2_ggeo + (size_t)(gb + grec[e]) * kGGeoWords
                                  : m.l2_lgeo + (size_t)(p0 + grec[e]) * kLGeoWords;
        greg[e] = *reinterpret_cast<const i32x4 *>(src + gword[e]);
      }
    }
  };
  auto deposit_geo = [&](int q) {  // records of step q: g-run q, own positions of q - 2
    i32x4 *g = geo + (q & 1) * geo_stride;
#pragma unroll
    for (int e = 0; e < kGeoEpt; ++e) {
      if (!gon[e]) continue;
      i32x4 v = greg[e];
      if (gkind[e] == 1) {
        v.x = fref(v.x, q); v.y = fref(v.y, q); v.z = fref(v.z, q); v.w = fref(v.w, q);
      } else if (gkind[e] == 2) {
        v.x = (q & 3) * fstride + v.x * vpc;
      } else if (gkind[e] == 3) {
        v.x = gref(v.x, q - 2); v.y = gref(v.y, q - 2); v.z = gref(v.z, q - 2); v.w = gref(v.w, q - 2);
      } else if (gkind[e] == 4) {
        v.z = ((q - 2) & 3) * gstride + v.z * 2 * vpc;
      }
      g[gdst[e]] = v;
    }
  };

  for (int q = 0; q < min(W, 2); ++q) {
    fetch(q);
    deposit(q);
  }
  fetch_geo(0);
  deposit_geo(0);
  __syncthreads();

  // lpn lanes per node, 64 / lpn nodes per wavefront (lanes past the last
  // whole group idle); lane hl of a group walks the chunk's lane vectors
  // hl, hl + lpn, ... (NL of them, lpn * NL >= nvc) with the node's
  // geometry in registers, so one broadcast read of a record serves
  // 64 / lpn nodes and NL lane vectors
  const int npw = 64 / lpn;
  const int sub = lane / lpn;
  const int hl = lane - sub * lpn;
  const bool sub_on = sub < npw;
  for (int q = 0; q < W + 2; ++q) {
    const bool pf = q + 2 < W;
    if (pf) fetch(q + 2);
    const bool gf = q + 1 < W + 2;
    if (gf) fetch_geo(q + 1);
    const i32x4 *gq = geo + (q & 1) * geo_stride;
    // ---- gradients at the g-run of parallel q
    if (q < W) {
      const int glen = sub_on ? cst_int4(m.l2_gseg, k0 + q).y : 0;
      for (int s = npw * wave + sub; s < glen; s += npw * nw) {
        const i32x4 *r = gq + s * kGGeoWords;
        double2 S[G];  // halved normals (FP64), the normals (FP32)
        int lr[8];
#pragma unroll
        for (int j = 0; j < G; ++j) {
          __builtin_memcpy(&S[j], &r[j], 16);
          if constexpr (!F64) S[j] = make_double2(S[j].x + S[j].x, S[j].y + S[j].y);
        }
        {
          const i32x4 a = r[6], b = r[7];
          lr[0] = a.x; lr[1] = a.y; lr[2] = a.z; lr[3] = a.w;
          lr[4] = b.x; lr[5] = b.y; lr[6] = b.z; lr[7] = b.w;
        }
        double al, be;
        {
          const i32x4 w8 = r[8];
          const int a2[2] = {w8.x, w8.y}, b2[2] = {w8.z, w8.w};
          __builtin_memcpy(&al, a2, 8);
          __builtin_memcpy(&be, b2, 8);
        }
        const i32x4 w9 = r[9];
        const int fself = w9.x, n = w9.y;  // fself: LDS offset
        double cosg;
        {
          const int c2[2] = {w9.z, w9.w};
          __builtin_memcpy(&cosg, c2, 8);
        }
        // closure of the node's normals (level independent)
        double cx = 0.0, cy = 0.0;
#pragma unroll
        for (int j = 0; j < G; ++j) {
          const bool pole = (lr[j] & kLrefPole) != 0;
          if (j < kMinRow) {
            closure_add<OP_GRAD>(cx, cy, S[j], false);
            continue;
          }
          double tx = cx, ty = cy;
          closure_add<OP_GRAD>(tx, ty, S[j], pole);
          cx = j < n ? tx : cx;
          cy = j < n ? ty : cy;
        }
#pragma unroll 1
        for (int i = 0; i < NL; ++i) {
          const int k = hl + lpn * i;
          const int kc = min(k, nvc - 1);  // lanes past the chunk read a valid entry
          typename PG::St st[NV];
          {
            const RF xi = fbuf[fself + kc];
#pragma unroll
            for (int v = 0; v < NV; ++v) PG::init(st[v], LF::get(xi, v), 0.0);
          }
          RF xn[G];
#pragma unroll
          for (int j = 0; j < G; ++j) xn[j] = fbuf[(lr[j] & ~kLrefPole) + kc];
#pragma unroll
          for (int j = 0; j < G; ++j) {
            const bool pole = (lr[j] & kLrefPole) != 0;
            if (j < kMinRow) {  // present in every row, never the pole edge
#pragma unroll
              for (int v = 0; v < NV; ++v) {
                if constexpr (F64) grad_add_half(st[v], LF::get(xn[j], v), S[j], false);
                else PG::add(st[v], LF::get(xn[j], v), S[j], false, 0.0);
              }
              continue;
            }
            const bool use = j < n;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              typename PG::St tt = st[v];
              if constexpr (F64) grad_add_half(tt, LF::get(xn[j], v), S[j], pole);
              else PG::add(tt, LF::get(xn[j], v), S[j], pole, 0.0);
              PG::keep(st[v], tt, use);
            }
          }
          RG g;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const typename PG::Out o = PG::result(st[v], al, be, cx, cy, 0.0);
            g.e[2 * v] = o.x;
            if constexpr (F64) g.e[2 * v + 1] = o.y * cosg;  // v cos(lat), as the divergence forms it
            else g.e[2 * v + 1] = o.y;
          }
          if (k < nvc) {
            RF *d = gbuf + (q & 3) * gstride + s * 2 * vpc + kc;
            __builtin_memcpy(d, &g, sizeof(RF));
            __builtin_memcpy(d + vpc, reinterpret_cast<const char *>(&g) + sizeof(RF), sizeof(RF));
          }
        }
      }
    }
    // The staged loads go to LDS here, between the two phases: the slots
    // they fill (field ring (q + 2) mod 4, geometry slot (q + 1) mod 2) are
    // read by neither phase of this step, the gradient phase has hidden
    // their latency, and the wait for them comes before this step's output
    // stores (vector memory operations retire in issue order).
    if (pf) deposit(q + 2);
    if (gf) deposit_geo(q + 1);
    // ---- Laplacian at the own positions of parallel q - 2
    if (q >= 2) {
      const int q2 = q - 2;
      const int2 sp = cst_int2(m.l2_seg_pos, k0 + q2);
      const int nown = sub_on ? sp.y - sp.x : 0;
      for (int t = npw * wave + sub; t < nown; t += npw * nw) {
        const i32x4 *r = gq + gw + t * LGW;
        double2 S[G];  // halved normals (FP64), the normals (FP32)
        int lr[8];
        double cn[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
          __builtin_memcpy(&S[j], &r[j], 16);
          if constexpr (!F64) S[j] = make_double2(S[j].x + S[j].x, S[j].y + S[j].y);
        }
        {
          const i32x4 a = r[6], b = r[7];
          lr[0] = a.x; lr[1] = a.y; lr[2] = a.z; lr[3] = a.w;
          lr[4] = b.x; lr[5] = b.y; lr[6] = b.z; lr[7] = b.w;
        }
        if constexpr (!F64) {
#pragma unroll
          for (int k = 0; k < 3; ++k) __builtin_memcpy(&cn[2 * k], &r[10 + k], 16);
        } else {
#pragma unroll
          for (int j = 0; j < G; ++j) cn[j] = 0.0;
        }
        double al, ci;
        {
          const i32x4 w8 = r[8];
          const int a2[2] = {w8.x, w8.y}, c2[2] = {w8.z, w8.w};
          __builtin_memcpy(&al, a2, 8);
          __builtin_memcpy(&ci, c2, 8);
        }
        const i32x4 w9 = r[9];
        const int node = w9.x, n = w9.y, self = w9.z;  // self: LDS offset
        double cx = 0.0, cy = 0.0;
#pragma unroll
        for (int j = 0; j < G; ++j) {
          const bool pole = (lr[j] & kLrefPole) != 0;
          if (j < kMinRow) {
            closure_add<OP_DIV>(cx, cy, S[j], false);
            continue;
          }
          double tx = cx, ty = cy;
          closure_add<OP_DIV>(tx, ty, S[j], pole);
          const bool use = j < n && !pole;
          cx = use ? tx : cx;
          cy = use ? ty : cy;
        }
#pragma unroll 1
        for (int i = 0; i < NL; ++i) {
          const int k = hl + lpn * i;
          const int kc = min(k, nvc - 1);
          typename PD::St st[NV];
          {
            const RG gi = gload(self + kc);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              if constexpr (F64) div_init_w(st[v], LG::get(gi, v));
              else PD::init(st[v], LG::get(gi, v), ci);
            }
          }
          RG gn[G];
#pragma unroll
          for (int j = 0; j < G; ++j) gn[j] = gload((lr[j] & ~kLrefPole) + kc);
#pragma unroll
          for (int j = 0; j < G; ++j) {
            const bool pole = (lr[j] & kLrefPole) != 0;
            if (j < kMinRow) {
#pragma unroll
              for (int v = 0; v < NV; ++v) {
                if constexpr (F64) div_add_half_w(st[v], LG::get(gn[j], v), S[j]);
                else PD::add(st[v], LG::get(gn[j], v), S[j], false, cn[j]);
              }
              continue;
            }
            const bool use = j < n && !pole;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              typename PD::St tt = st[v];
              if constexpr (F64) div_add_half_w(tt, LG::get(gn[j], v), S[j]);
              else PD::add(tt, LG::get(gn[j], v), S[j], pole, cn[j]);
              PD::keep(st[v], tt, use);
            }
          }
          constexpr int WD = NV * (int)sizeof(T) / 4;
          struct Words { int v[WD]; } o;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const T x = PD::result(st[v], al, 0.0, cx, cy, ci);
            __builtin_memcpy(&o.v[v * (int)sizeof(T) / 4], &x, sizeof(T));
          }
          if (k < nvc) *reinterpret_cast<Words *>(out + (size_t)node * L + first(kc)) = o;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Fused Laplacian, wave-specialised: the register-staged kernel above waits
// at every parallel for the loads it issued one parallel earlier, one
// memory round trip per step.  Here two producer groups of two wavefronts
// load the field runs and packed geometry straight into LDS (16-byte DMA
// loads, as in the wave-specialised sweep) two steps ahead, and never
// store, so each waits for exactly its own loads; the consumer wavefronts
// only compute and store.
//
// Step q forms the gradients of the g-run of parallel q (field runs q-1,
// q, q+1) into gradient slot q mod 3, then -- after a workgroup barrier --
// the Laplacian of the own positions of parallel q-1 from the gradients of
// parallels q-2, q-1, q.  Load set k = {field run k+1, geometry of step k
// (g records of parallel k, own records of parallel k-1)} is issued at step
// k-2 by group k mod 2 and waited for by that group at the end of step
// k-1: field ring 5 slots, geometry ring 3, gradient ring 3.  With FS = 4
// field slots the field run of set k is issued after the mid-step barrier
// of step k-2 instead (the gradients of that step have then finished
// reading the slot it takes), one step before it is read rather than one
// and a half: the ring holds one parallel of columns less, so a longer
// level chunk fits in LDS.  References in the packed records are resolved
// once the set has landed, into LDS offsets.
// ---------------------------------------------------------------------------
constexpr int kLswFSlots = 5, kLswGSlots = 3, kLswGeoSlots = 3;
constexpr int kLswProducers = 4;  // two groups of two wavefronts

template <class T, int NV, int FS = kLswFSlots>
__global__ void __launch_bounds__(1024) k_lsweepw(DevMesh m, const T *__restrict__ in,
                                                  T *__restrict__ out, int nlev, int vpc,
                                                  int ntiles, int per_xcd, int lpn, int fcap,
                                                  int gcap, int ocap) {
  using PG = Pol<T, OP_GRAD>;
  using PD = Pol<T, OP_DIV>;
  using LF = LaneVec<T, NV>;
  using RF = typename LF::raw;
  using GV = typename PD::V;
  using LG = LaneVec<GV, NV>;
  using RG = typename LG::raw;
  static_assert(sizeof(RF) == 16, "wave-specialised fused Laplacian: 16-byte lane vectors");
  static_assert(sizeof(RG) == 2 * sizeof(RF), "gradient lane vector = two field lane vectors");
  static_assert(FS == 4 || FS == 5, "field ring of four or five slots");
  constexpr int G = 6;
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int LGW = F64 ? kLGeoWords64 : kLGeoWords;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int gmax = m.l2_gmax;
  const int gstride = 2 * gmax * vpc;   // gradient slot (field lane vectors)
  const int geo_stride = gcap + ocap;   // geometry slot (16-byte words)
  RF *fbuf = reinterpret_cast<RF *>(smem_raw);                         // [FS][fcap]
  RF *gbuf = fbuf + FS * fcap;                                         // [3][gmax][2][vpc]
  i32x4 *geo = reinterpret_cast<i32x4 *>(gbuf + kLswGSlots * gstride);  // [3][gcap + ocap]
  const int u = xcd_tile(blockIdx.x, per_xcd);
  const int nvec = (nlev + NV - 1) / NV;
  const int nchunk = (nvec + vpc - 1) / vpc;
  const int tile = u / nchunk;
  const int c = u - tile * nchunk;
  if (tile >= ntiles) return;
  const int v0 = c * vpc;
  if (v0 >= nvec) return;
  const int nvc = min(vpc, nvec - v0);
  const int k0 = cst(m.l2_tile_seg)[tile];
  const int W = cst(m.l2_tile_seg)[tile + 1] - k0;
  const size_t L = (size_t)nlev;
  const uint32_t col_bytes = (uint32_t)(L * sizeof(T));
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  auto first = [&](int k) { return min(NV * (v0 + k), nlev - NV); };

  if (wave < kLswProducers) {
    // ---- producers: waves 0, 1 form group 0 and waves 2, 3 group 1; the
    // even wave of a group loads and resolves geometry, the odd one loads
    // field runs, so every wave waits only for the loads it issued ---------
    const int grp = wave >> 1;
    const bool geo_wave = (wave & 1) == 0;
    // field run q into slot q mod FS: item i = (node t of the run) x (lane
    // vector kk); t and kk advance by whole load instructions
    auto load_f = [&](int q) {
      if (q < 0 || q >= W) return;
      const int4 f = cst_int4(m.l2_fseg, k0 + q);  // {ring offset, ring size, first, length}
      const i32x4 rs = make_rsrc(in + (size_t)f.x * L, (uint32_t)f.y * col_bytes);
      const int nitems = f.w * nvc;
      RF *slot = fbuf + (q % FS) * fcap;
      int t = lane / nvc, kk = lane - t * nvc;
      const int dt = 64 / nvc, dk = 64 - dt * nvc;
      for (int b = 0; b * 64 < nitems; ++b) {
        int off = kBufOff;
        if (b * 64 + lane < nitems) {
          int ii = f.z + t;
          if (ii >= f.y) ii -= f.y;  // the run wraps round the parallel
          off = ii * (int)col_bytes + first(kk) * (int)sizeof(T);
        }
        lds_dma16(rs, slot + b * 64, off);
        t += dt;
        kk += dk;
        if (kk >= nvc) {
          kk -= nvc;
          ++t;
        }
      }
    };
    // geometry of step k: g records of parallel k, own records of k - 1
    auto load_g = [&](int k) {
      if (k < 0 || k > W) return;
      i32x4 *gs = geo + (k % kLswGeoSlots) * geo_stride;
      if (k < W) {
        const int4 g = cst_int4(m.l2_gseg, k0 + k);  // {g first, g length, first g record, 0}
        const i32x4 rs = make_rsrc(m.l2_ggeo + (size_t)g.z * kGGeoWords,
                                   (uint32_t)g.y * kGGeoWords * 16u);
        const int nitems = g.y * kGGeoWords;
        for (int b = 0; b * 64 < nitems; ++b) {
          const int i = b * 64 + lane;
          lds_dma16(rs, gs + b * 64, i < nitems ? i * 16 : kBufOff);
        }
      }
      if (k >= 1) {
        const int2 sp = cst_int2(m.l2_seg_pos, k0 + k - 1);
        const int np = sp.y - sp.x;
        const i32x4 rs = make_rsrc(m.l2_lgeo + (size_t)sp.x * kLGeoWords,
                                   (uint32_t)np * kLGeoWords * 16u);
        const int nitems = np * LGW;
        int t = lane / LGW, wd = lane - t * LGW;
        constexpr int dt = 64 / LGW, dw = 64 - dt * LGW;
        for (int b = 0; b * 64 < nitems; ++b) {
          lds_dma16(rs, gs + gcap + b * 64,
                    b * 64 + lane < nitems ? (t * kLGeoWords + wd) * 16 : kBufOff);
          t += dt;
          wd += dw;
          if (wd >= LGW) {
            wd -= LGW;
            ++t;
          }
        }
      }
    };
    // The reference words of geometry set k (words 6, 7, 9 of each record:
    // one g record and one own record per lane) also go to registers with
    // the set's loads; once the set has landed they become LDS element
    // offsets for the step that reads them (field-run references of the g
    // records of parallel k: runs k-1, k, k+1; gradient-run references of
    // the own records of parallel k-1: runs k-2, k-1, k; pole flags kept)
    // and overwrite the copied words.
    i32x4 gr6 = {}, gr7 = {}, gr9 = {}, or6 = {}, or7 = {}, or9 = {};
    auto load_refs = [&](int k) {
      if (k < 0 || k > W) return;
      if (k < W) {
        const int4 g = cst_int4(m.l2_gseg, k0 + k);
        const i32x4 rs = make_rsrc(m.l2_ggeo + (size_t)g.z * kGGeoWords,
                                   (uint32_t)g.y * kGGeoWords * 16u);
        const int o = lane < g.y ? lane * kGGeoWords * 16 : kBufOff;
        gr6 = buf_load<i32x4>(rs, o + 6 * 16);
        gr7 = buf_load<i32x4>(rs, o + 7 * 16);
        gr9 = buf_load<i32x4>(rs, o + 9 * 16);
      }
      if (k >= 1) {
        const int2 sp = cst_int2(m.l2_seg_pos, k0 + k - 1);
        const i32x4 rs = make_rsrc(m.l2_lgeo + (size_t)sp.x * kLGeoWords,
                                   (uint32_t)(sp.y - sp.x) * kLGeoWords * 16u);
        const int o = lane < sp.y - sp.x ? lane * kLGeoWords * 16 : kBufOff;
        or6 = buf_load<i32x4>(rs, o + 6 * 16);
        or7 = buf_load<i32x4>(rs, o + 7 * 16);
        or9 = buf_load<i32x4>(rs, o + 9 * 16);
      }
    };
    auto resolve = [&](int k) {
      // the loaded words are used from here on only: no computation on them
      // may move up to the loads, where it would wait for the whole set
      asm volatile("" : "+v"(gr6), "+v"(gr7), "+v"(gr9), "+v"(or6), "+v"(or7), "+v"(or9));
      if (k < 0 || k > W) return;
      i32x4 *gs = geo + (k % kLswGeoSlots) * geo_stride;
      if (k < W) {
        const int b0 = ((k + FS - 1) % FS) * fcap;
        const int b1 = (k % FS) * fcap, b2 = ((k + 1) % FS) * fcap;
        auto rf = [&](int v) {
          const int l = v & ~kLrefPole, dq = (l >> 16) & 3;
          return (v & kLrefPole) | ((dq == 0 ? b0 : dq == 1 ? b1 : b2) + (l & 0xffff) * nvc);
        };
        if (lane < cst_int4(m.l2_gseg, k0 + k).y) {
          i32x4 *r = gs + lane * kGGeoWords;
          i32x4 a = gr6, b = gr7, c = gr9;
          a.x = rf(a.x); a.y = rf(a.y); a.z = rf(a.z); a.w = rf(a.w);
          b.x = rf(b.x); b.y = rf(b.y); b.z = rf(b.z); b.w = rf(b.w);
          c.x = b1 + c.x * nvc;
          r[6] = a; r[7] = b; r[9] = c;
        }
      }
      if (k >= 1) {
        const int b0 = ((k + 1) % kLswGSlots) * gstride;
        const int b1 = ((k + 2) % kLswGSlots) * gstride, b2 = (k % kLswGSlots) * gstride;
        auto rg = [&](int v) {
          const int l = v & ~kLrefPole, dq = (l >> 16) & 3;
          return (v & kLrefPole) | ((dq == 0 ? b0 : dq == 1 ? b1 : b2) + (l & 0xffff) * 2 * vpc);
        };
        const int2 sp = cst_int2(m.l2_seg_pos, k0 + k - 1);
        if (lane < sp.y - sp.x) {
          i32x4 *r = gs + gcap + lane * LGW;
          i32x4 a = or6, b = or7, c = or9;
          a.x = rg(a.x); a.y = rg(a.y); a.z = rg(a.z); a.w = rg(a.w);
          b.x = rg(b.x); b.y = rg(b.y); b.z = rg(b.z); b.w = rg(b.w);
          c.z = b1 + c.z * 2 * vpc;
          r[6] = a; r[7] = b; r[9] = c;
        }
      }
    };
    // prologue: group 0 takes geometry 0 and field runs 0, 1; group 1
    // geometry 1 and field run 2; each geometry wave resolves its own set
    if (geo_wave) {
      load_refs(grp);  // first: no DMA of the set may wait on these registers
      load_g(grp);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      resolve(grp);
    } else {
      if (grp == 0) {
        load_f(0);
        load_f(1);
      } else {
        load_f(2);
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    // the resolved words are in LDS before the consumers pass the barrier
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    for (int q = 0; q <= W; ++q) {
      // set q + 2 (field run q + 3, geometry q + 2) by group q mod 2
      if ((q & 1) == grp) {
        if (geo_wave) {
          load_refs(q + 2);
          load_g(q + 2);
        } else if (FS == 5) {
          load_f(q + 3);
        }
      }
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();  // between the consumers' two phases
      asm volatile("" ::: "memory");
      // four slots: field run q + 3 takes the slot of run q - 1, which the
      // gradients of step q (runs q - 1 .. q + 1) have finished reading
      if (FS == 4 && (q & 1) == grp && !geo_wave) load_f(q + 3);
      // set q + 1 (issued at step q - 1 by this group; sets 0 and 1 came
      // with the prologue) lands, and is resolved, before step q + 1
      if (((q + 1) & 1) == grp && q >= 1) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if (geo_wave) resolve(q + 1);
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    return;
  }

  // ---- consumers ------------------------------------------------------------
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
  const int cw = wave - kLswProducers, ncw = nw - kLswProducers;
  const int npw = 64 / lpn;  // nodes per wavefront, lpn lanes each
  const int sub = lane / lpn;
  const int hl = lane - sub * lpn;
  const bool sub_on = sub < npw;
  const int kc = min(hl, nvc - 1);  // lanes past the chunk read a valid entry
  const bool lane_on = sub_on && hl < nvc;
  auto gload = [&](int at) {
    RG r;
    __builtin_memcpy(&r, &gbuf[at], sizeof(RF));
    __builtin_memcpy(reinterpret_cast<char *>(&r) + sizeof(RF), &gbuf[at + vpc], sizeof(RF));
    return r;
  };
  for (int q = 0; q <= W; ++q) {
    const i32x4 *gq = geo + (q % kLswGeoSlots) * geo_stride;
    // ---- gradients at the g-run of parallel q
    if (q < W) {
      RF *gout = gbuf + (q % kLswGSlots) * gstride;
      const int glen = sub_on ? cst_int4(m.l2_gseg, k0 + q).y : 0;
      for (int s = npw * cw + sub; s < glen; s += npw * ncw) {
        const i32x4 *r = gq + s * kGGeoWords;
        double2 S[G];  // halved normals (FP64), the normals (FP32)
        int lr[8];
#pragma unroll
        for (int j = 0; j < G; ++j) {
          __builtin_memcpy(&S[j], &r[j], 16);
          if constexpr (!F64) S[j] = make_double2(S[j].x + S[j].x, S[j].y + S[j].y);
        }
        {
          const i32x4 a = r[6], b = r[7];
          lr[0] = a.x; lr[1] = a.y; lr[2] = a.z; lr[3] = a.w;
          lr[4] = b.x; lr[5] = b.y; lr[6] = b.z; lr[7] = b.w;
        }
        double al, be;
        {
          const i32x4 w8 = r[8];
          const int a2[2] = {w8.x, w8.y}, b2[2] = {w8.z, w8.w};
          __builtin_memcpy(&al, a2, 8);
          __builtin_memcpy(&be, b2, 8);
        }
        const i32x4 w9 = r[9];
        const int fself = w9.x, n = w9.y;
        double cosg;
        {
          const int c2[2] = {w9.z, w9.w};
          __builtin_memcpy(&cosg, c2, 8);
        }
        typename PG::St st[NV];
        {
          const RF xi = fbuf[fself + kc];
#pragma unroll
          for (int v = 0; v < NV; ++v) PG::init(st[v], LF::get(xi, v), 0.0);
        }
        RF xn[G];
#pragma unroll
        for (int j = 0; j < G; ++j) xn[j] = fbuf[(lr[j] & ~kLrefPole) + kc];
        double cx = 0.0, cy = 0.0;
#pragma unroll
        for (int j = 0; j < G; ++j) {
          const bool pole = (lr[j] & kLrefPole) != 0;
          if (j < kMinRow) {  // present in every row, never the pole edge
            closure_add<OP_GRAD>(cx, cy, S[j], false);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              if constexpr (F64) grad_add_half(st[v], LF::get(xn[j], v), S[j], false);
              else PG::add(st[v], LF::get(xn[j], v), S[j], false, 0.0);
            }
            continue;
          }
          const bool use = j < n;
          double tx = cx, ty = cy;
          closure_add<OP_GRAD>(tx, ty, S[j], pole);
          cx = use ? tx : cx;
          cy = use ? ty : cy;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            typename PG::St tt = st[v];
            if constexpr (F64) grad_add_half(tt, LF::get(xn[j], v), S[j], pole);
            else PG::add(tt, LF::get(xn[j], v), S[j], pole, 0.0);
            PG::keep(st[v], tt, use);
          }
        }
        RG g;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const typename PG::Out o = PG::result(st[v], al, be, cx, cy, 0.0);
          g.e[2 * v] = o.x;
          if constexpr (F64) g.e[2 * v + 1] = o.y * cosg;  // v cos(lat), as the divergence forms it
          else g.e[2 * v + 1] = o.y;
        }
        if (lane_on) {
          RF *d = gout + s * 2 * vpc + kc;
          __builtin_memcpy(d, &g, sizeof(RF));
          __builtin_memcpy(d + vpc, reinterpret_cast<const char *>(&g) + sizeof(RF), sizeof(RF));
        }
      }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();  // the gradients of parallel q are in LDS
    asm volatile("" ::: "memory");
    // ---- Laplacian at the own positions of parallel q - 1
    if (q >= 1) {
      const int q1 = q - 1;
      const int2 sp = cst_int2(m.l2_seg_pos, k0 + q1);
      const int nown = sub_on ? sp.y - sp.x : 0;
      for (int t = npw * cw + sub; t < nown; t += npw * ncw) {
        const i32x4 *r = gq + gcap + t * LGW;
        double2 S[G];
        int lr[8];
        double cn[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
          __builtin_memcpy(&S[j], &r[j], 16);
          if constexpr (!F64) S[j] = make_double2(S[j].x + S[j].x, S[j].y + S[j].y);
        }
        {
          const i32x4 a = r[6], b = r[7];
          lr[0] = a.x; lr[1] = a.y; lr[2] = a.z; lr[3] = a.w;
          lr[4] = b.x; lr[5] = b.y; lr[6] = b.z; lr[7] = b.w;
        }
        if constexpr (!F64) {
#pragma unroll
          for (int k = 0; k < 3; ++k) __builtin_memcpy(&cn[2 * k], &r[10 + k], 16);
        } else {
#pragma unroll
          for (int j = 0; j < G; ++j) cn[j] = 0.0;
        }
        double al, ci;
        {
          const i32x4 w8 = r[8];
          const int a2[2] = {w8.x, w8.y}, c2[2] = {w8.z, w8.w};
          __builtin_memcpy(&al, a2, 8);
          __builtin_memcpy(&ci, c2, 8);
        }
        const i32x4 w9 = r[9];
        const int node = w9.x, n = w9.y, self = w9.z;
        typename PD::St st[NV];
        {
          const RG gi = gload(self + kc);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            if constexpr (F64) div_init_w(st[v], LG::get(gi, v));
            else PD::init(st[v], LG::get(gi, v), ci);
          }
        }
        RG gn[G];
#pragma unroll
        for (int j = 0; j < G; ++j) gn[j] = gload((lr[j] & ~kLrefPole) + kc);
        double cx = 0.0, cy = 0.0;
#pragma unroll
        for (int j = 0; j < G; ++j) {
          const bool pole = (lr[j] & kLrefPole) != 0;
          if (j < kMinRow) {
            closure_add<OP_DIV>(cx, cy, S[j], false);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              if constexpr (F64) div_add_half_w(st[v], LG::get(gn[j], v), S[j]);
              else PD::add(st[v], LG::get(gn[j], v), S[j], false, cn[j]);
            }
            continue;
          }
          const bool use = j < n && !pole;
          double tx = cx, ty = cy;
          closure_add<OP_DIV>(tx, ty, S[j], pole);
          cx = use ? tx : cx;
          cy = use ? ty : cy;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            typename PD::St tt = st[v];
            if constexpr (F64) div_add_half_w(tt, LG::get(gn[j], v), S[j]);
            else PD::add(tt, LG::get(gn[j], v), S[j], pole, cn[j]);
            PD::keep(st[v], tt, use);
          }
        }
        constexpr int WD = NV * (int)sizeof(T) / 4;
        struct Words { int v[WD]; } o;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const T x = PD::result(st[v], al, 0.0, cx, cy, ci);
          __builtin_memcpy(&o.v[v * (int)sizeof(T) / 4], &x, sizeof(T));
        }
        if (lane_on) *reinterpret_cast<Words *>(out + (size_t)node * L + first(kc)) = o;
      }
    }
    // this step's LDS reads are done before the producers refill a slot
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  }
}

// Packs the fused Laplacian's per-record geometry (after the scales are
// derived): gradient-node records in g-record order, own-position records
// in position order.
__global__ void k_pack_ggeo(DevMesh m, int ng, i32x4 *__restrict__ dst) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const int4 gn = m.l2_gnode[g];  // {row start, row length, f self, position}
  i32x4 *o = dst + (size_t)g * kGGeoWords;
  for (int j = 0; j < 6; ++j) {  // halved normals (exact)
    const double2 h = make_double2(0.5 * m.S[gn.x + j].x, 0.5 * m.S[gn.x + j].y);
    __builtin_memcpy(&o[j], &h, 16);
  }
  __builtin_memcpy(&o[6], m.l2_glref + (size_t)g * kGRefs, 32);
  const PosRec pr = m.pos[gn.w];
  const double ab[2] = {pr.alpha, pr.beta};
  __builtin_memcpy(&o[8], ab, 16);
  const double c = m.coslat[pr.node];
  int cw[2];
  __builtin_memcpy(cw, &c, 8);
  o[9] = i32x4{gn.z, gn.y, cw[0], cw[1]};
}
__global__ void k_pack_lgeo(DevMesh m, i32x4 *__restrict__ dst) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m.V) return;
  const PosRec pr = m.pos[p];
  i32x4 *o = dst + (size_t)p * kLGeoWords;
  for (int j = 0; j < 6; ++j) {  // halved normals (exact)
    const double2 h = make_double2(0.5 * m.S[pr.r0 + j].x, 0.5 * m.S[pr.r0 + j].y);
    __builtin_memcpy(&o[j], &h, 16);
  }
  __builtin_memcpy(&o[6], m.l2_lref + pr.r0, 32);
  const double ac[2] = {pr.alpha, m.coslat[pr.node]};
  __builtin_memcpy(&o[8], ac, 16);
  o[9] = i32x4{pr.node, pr.r1 - pr.r0, m.l2_lself[p], 0};
  __builtin_memcpy(&o[10], m.ncos + pr.r0, 48);
}

// Packs the wave-specialised sweep's per-position geometry (after the
// scales are derived): kSgeoWords 16-byte words per position, in position
// order, normals halved.  Entries past a row are neutral: zero normals, the
// position's own LDS slot as reference, cos(lat) 1.
__global__ void k_pack_sgeo(DevMesh m, i32x4 *__restrict__ dst) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m.V) return;
  const PosRec pr = m.pos[p];
  const int n = pr.r1 - pr.r0;
  i32x4 *o = dst + (size_t)p * kSgeoWords;
  o[0] = i32x4{pr.node, n, pr.selfslot, 0};
  const double ab[2] = {pr.alpha, pr.beta};
  __builtin_memcpy(&o[1], ab, 16);
  for (int j = 0; j < 6; ++j) {  // halved normals (exact)
    const double2 v = j < n ? make_double2(0.5 * m.S[pr.r0 + j].x, 0.5 * m.S[pr.r0 + j].y)
                            : make_double2(0.0, 0.0);
    __builtin_memcpy(&o[2 + j], &v, 16);
  }
  int lr[8];
  for (int j = 0; j < 8; ++j) lr[j] = j < n ? m.lref[pr.r0 + j] : ((1 << 16) | pr.selfslot);
  __builtin_memcpy(&o[8], lr, 32);
  double cn[6];
  for (int j = 0; j < 6; ++j) cn[j] = j < n ? m.ncos[pr.r0 + j] : 1.0;
  __builtin_memcpy(&o[10], cn, 48);
  const double c2[2] = {m.coslat[pr.node], 0.0};
  __builtin_memcpy(&o[13], c2, 16);
}

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
        diff_terms_f32<OP_GRAD>(S, in[(size_t)a * L + k], in[(size_t)b * L + k], v2f{},
                                v2f{}, 0.0, 0.0, tx, ty, t);
        float2 f;
        f.x = tx;
        f.y = ty;
        reinterpret_cast<float2 *>(flux)[g] = f;
      } else {
        const v2f *vin = reinterpret_cast<const v2f *>(in);
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
// Batched persistent form.  Workgroup b serves work queue b mod 8 (one per
// XCD); units are (item, block of positions, phase).  One launch runs one
// pass: phase 0 (every single operator, and the gradient of every
// Laplacian into its workspace), then, if any item is a Laplacian, a second
// launch runs phase 1 (the divergence of that gradient) -- the dependency is
// the launch order.  A workgroup never waits for another: it takes units
// from its queue until the queue is drained, then exits.  heads[x] is queue
// x's next unit.
// ---------------------------------------------------------------------------
// Lane vectors wider than 16 bytes: the batch kernel takes them one per
// lane only (two would not fit its register budget).
template <class T, int OP, int NV>
__host__ __device__ constexpr bool batch_wide() {
  return NV * sizeof(typename Pol<T, OP>::V) > 16;
}

// Column-form positions p0 + wave, p0 + wave + nw, ... below p1 with lane
// vectors of NV levels and nchv (1 or 2; 1 if wide) vectors per lane; false
// if that width does not exist for this dtype and operator.
template <class T, int OP, int NV>
__device__ __forceinline__ bool batch_colv(const DevMesh &m, const T *in, T *out, int nlev,
                                           int nchv, int p0, int p1, int wave, int nw, int lane) {
  if constexpr (lane_vec_ok<T, OP, NV>()) {
    for (int p = p0 + wave; p < p1; p += nw) {
      const PosRec pr = m.pos[p];
      if (batch_wide<T, OP, NV>() || nchv == 1) colv_node<T, OP, NV, 1>(m, in, out, nlev, pr, lane);
      else colv_node<T, OP, NV, 2>(m, in, out, nlev, pr, lane);
    }
    return true;
  }
  return false;
}

template <class T, int OP>
__device__ __forceinline__ void batch_unit_op(const DevMesh &m, int form, int level_vec,
                                              const T *in, T *out, int nlev, int p0, int p1) {
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (form == FORM_COLUMN) {
    // lane vectors as in the single-launch column form, up to two per lane
    // (one if wider than 16 bytes: the batch kernel's registers are sized
    // for that); wider columns and level_vec 1 take one level per lane
    const int nv = level_vec == 1 ? 0 : auto_level_vec<T, OP>(nlev, m.maxdeg, m.mindeg, level_vec);
    if (nv > 0) {
      const int nchv = ((nlev + nv - 1) / nv + 63) / 64;
      const bool wide = nv * (int)sizeof(typename Pol<T, OP>::V) > 16;
      bool done = false;
      if (nchv <= (wide ? 1 : 2)) {
        if (nv == 1) done = batch_colv<T, OP, 1>(m, in, out, nlev, nchv, p0, p1, wave, nw, lane);
        else if (nv == 2) done = batch_colv<T, OP, 2>(m, in, out, nlev, nchv, p0, p1, wave, nw, lane);
        else if (nv == 3) done = batch_colv<T, OP, 3>(m, in, out, nlev, nchv, p0, p1, wave, nw, lane);
        else done = batch_colv<T, OP, 4>(m, in, out, nlev, nchv, p0, p1, wave, nw, lane);
      }
      if (done) return;
    }
    const int nch = (nlev + 63) / 64;
    for (int p = p0 + wave; p < p1; p += nw) {
      const PosRec pr = m.pos[p];
      if (m.maxdeg <= 6 && nch == 1) column_node<T, OP, 1, 6, true>(m, in, out, nlev, pr, lane);
      else if (m.maxdeg <= 6 && nch == 2) column_node<T, OP, 2, 6, true>(m, in, out, nlev, pr, lane);
      else if (m.maxdeg <= 6 && nch == 3) column_node<T, OP, 3, 6, true>(m, in, out, nlev, pr, lane);
      else
        for (int k = lane; k < nlev; k += 64) element<T, OP>(m, in, out, nlev, p, pr.node, pr.r0, pr.r1, k);
    }
  } else {
    const int nel = (p1 - p0) * nlev;
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
      const int pl = e / nlev;
      const int k = e - pl * nlev;
      const int p = p0 + pl;
      element<T, OP>(m, in, out, nlev, p, m.perm[p], m.rowp[p], m.rowp[p + 1], k);
    }
  }
}

// waves per SIMD the batch kernel is compiled for (FP64: three, so the
// one-level-per-lane column paths keep their registers)
template <class T>
constexpr int batch_waves() { return sizeof(T) == 8 ? 3 : 4; }

template <class T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(batch_waves<T>()))) k_batch(const BatchItem *__restrict__ items,
                                               const BatchUnit *__restrict__ units,
                                               const int *__restrict__ qbeg, int *heads) {
  // Unit indices pass through two LDS slots: while the workgroup runs unit
  // s_u[k], thread 0 already takes the next one into s_u[k ^ 1], so the
  // atomic's latency hides behind the unit and one barrier per unit
  // suffices (s_u[k] is rewritten only after every thread has passed the
  // barrier that follows its read).
  __shared__ int s_u[2];
  const int x = blockIdx.x & 7;
  const int qend = qbeg[x + 1];
  if (threadIdx.x == 0) s_u[0] = qbeg[x] + atomicAdd(&heads[x], 1);
  __syncthreads();
  for (int k = 0;; k ^= 1) {
    const int u = s_u[k];
    if (u >= qend) break;  // this queue is drained: every wave exits
    if (threadIdx.x == 0) s_u[k ^ 1] = qbeg[x] + atomicAdd(&heads[x], 1);
    const BatchUnit un = units[u];
    const BatchItem &it = items[un.item];
    const int op = it.lapl ? (un.phase ? OP_DIV : OP_GRAD) : it.op;
    const T *src = static_cast<const T *>(un.phase ? it.ws : it.in);
    T *dst = static_cast<T *>((it.lapl && un.phase == 0) ? it.ws : it.out);
    const int lv = un.phase ? it.level_vec1 : it.level_vec;
    if (op == OP_GRAD)
      batch_unit_op<T, OP_GRAD>(it.m, it.form, lv, src, dst, it.nlev, un.p0, un.p1);
    else if (op == OP_DIV)
      batch_unit_op<T, OP_DIV>(it.m, it.form, lv, src, dst, it.nlev, un.p0, un.p1);
    else
      batch_unit_op<T, OP_CURL>(it.m, it.form, lv, src, dst, it.nlev, un.p0, un.p1);
    __syncthreads();
  }
}

__global__ void k_fill(int *p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

atlas_status launch_fill(int *p, int n, int value, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, st, p, n, value);
  ATLASX_HIP(hipGetLastError());
  return ATLAS_OK;
}

int batch_blocks_per_cu(atlas_dtype dt, int block) {
  int n = 0;
  hipError_t e = dt == ATLAS_F64
                     ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<double>, block, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<float>, block, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

// One batch = counter reset (a kernel, not a memset, so it can live in a
// captured graph) + the phase-0 pass + (if any) the phase-1 pass.
atlas_status launch_batch(atlas_dtype dt, const BatchItem *items, const BatchUnit *units,
                          const int *qbeg0, const int *qbeg1, bool two_pass, int *heads,
                          int grid, int block, hipStream_t st) {
  atlas_status s = launch_fill(heads, 16, 0, st);
  if (s != ATLAS_OK) return s;
  for (int pass = 0; pass < (two_pass ? 2 : 1); ++pass) {
    const int *qb = pass ? qbeg1 : qbeg0;
    int *hd = heads + 8 * pass;
    if (dt == ATLAS_F64)
      hipLaunchKernelGGL(k_batch<double>, dim3(grid), dim3(block), 0, st, items, units, qb, hd);
    else
      hipLaunchKernelGGL(k_batch<float>, dim3(grid), dim3(block), 0, st, items, units, qb, hd);
    ATLASX_HIP(hipGetLastError());
  }
  return ATLAS_OK;
}

// ---------------------------------------------------------------------------
// Streaming reference: read n, write 2n (the gradient's byte pattern).  One
// element per thread and a grid that covers the array (a grid-stride loop
// over fewer blocks reached only ~75 % of this rate on MI355X), each store
// instruction one contiguous run of 64 lane pairs.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_stream_r1w2(const T *__restrict__ x, T *__restrict__ y,
                                                     int64_t n) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 *yv = reinterpret_cast<v2 *>(y);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T v = x[i];
    yv[i] = v2{v, v};
  }
}

atlas_status bandwidth_probe(const void *in, void *out, int64_t n, int elem, hipStream_t st) {
  // one thread per element up to 2^22 blocks (2^30 elements), then a loop
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, (int64_t)1 << 22);
  if (elem == 8)
    hipLaunchKernelGGL(k_stream_r1w2<double>, dim3(grid), dim3(256), 0, st,
                       static_cast<const double *>(in), static_cast<double *>(out), n);
  else
    hipLaunchKernelGGL(k_stream_r1w2<float>, dim3(grid), dim3(256), 0, st,
                       static_cast<const float *>(in), static_cast<float *>(out), n);
  ATLASX_HIP(hipGetLastError());
  return ATLAS_OK;
}

// ---------------------------------------------------------------------------
// Per-node scales, derived once at upload: alpha = R/V, beta = R cos/V.
// ---------------------------------------------------------------------------
__global__ void k_derive_scales(int V, const double *__restrict__ vol,
                                const double *__restrict__ cosl, double R,
                                double *__restrict__ alpha, double *__restrict__ beta,
                                PosRec *__restrict__ pos) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < V) {
    const double a = R / vol[p], b = (R * cosl[p]) / vol[p];
    alpha[p] = a;
    beta[p] = b;
    pos[p].alpha = a;
    pos[p].beta = b;
  }
}

atlas_status pack_lapl_geometry(MeshStore &m, int64_t ngrec) {
  void *g = nullptr, *l = nullptr;
  const size_t gb = std::max<size_t>(16, (size_t)ngrec * kGGeoWords * 16);
  const size_t lb = std::max<size_t>(16, (size_t)m.d.V * kLGeoWords * 16);
  if (hipMalloc(&g, gb) != hipSuccess) return fail(ATLAS_ENOMEM, "hipMalloc of mesh store failed");
  m.allocations.push_back(g);
  if (hipMalloc(&l, lb) != hipSuccess) return fail(ATLAS_ENOMEM, "hipMalloc of mesh store failed");
  m.allocations.push_back(l);
  m.bytes += gb + lb;
  if (ngrec > 0)
    hipLaunchKernelGGL(k_pack_ggeo, dim3((unsigned)((ngrec + 255) / 256)), dim3(256), 0, 0, m.d,
                       (int)ngrec, static_cast<i32x4 *>(g));
  if (m.d.V > 0)
    hipLaunchKernelGGL(k_pack_lgeo, dim3((m.d.V + 255) / 256), dim3(256), 0, 0, m.d,
                       static_cast<i32x4 *>(l));
  ATLASX_HIP(hipGetLastError());
  m.d.l2_ggeo = static_cast<const int4 *>(g);
  m.d.l2_lgeo = static_cast<const int4 *>(l);
  return ATLAS_OK;
}

atlas_status pack_sweep_geometry(MeshStore &m) {
  void *g = nullptr;
  const size_t gb = std::max<size_t>(16, (size_t)m.d.V * kSgeoWords * 16);
  if (hipMalloc(&g, gb) != hipSuccess) return fail(ATLAS_ENOMEM, "hipMalloc of mesh store failed");
  m.allocations.push_back(g);
  m.bytes += gb;
  if (m.d.V > 0)
    hipLaunchKernelGGL(k_pack_sgeo, dim3((m.d.V + 255) / 256), dim3(256), 0, 0, m.d,
                       static_cast<i32x4 *>(g));
  ATLASX_HIP(hipGetLastError());
  m.d.sgeo = static_cast<const int4 *>(g);
  return ATLAS_OK;
}

atlas_status derive_scales(MeshStore &m, const double *vol_by_pos, const double *cos_by_pos,
                           double radius) {
  const int V = m.d.V;
  hipLaunchKernelGGL(k_derive_scales, dim3((V + 255) / 256), dim3(256), 0, 0, V, vol_by_pos,
                     cos_by_pos, radius, const_cast<double *>(m.d.alpha),
                     const_cast<double *>(m.d.beta), const_cast<PosRec *>(m.d.pos));
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

// Built-in shape (the autotuner can replace it per mesh and class), from
// measurements at O1280, 137 levels.  Long columns: the column form over
// blocks of 16 consecutive positions (a run of one parallel, so the
// neighbour columns of consecutive blocks overlap in L2) with the automatic
// lane-vector width, except: the FP64 gradient runs the wave-specialised
// sweep (1024 threads), the FP32 gradient one level per lane (its
// compensated sums keep every lane busy that way).  The Laplacian takes each
// pass's own shape.  Short columns (measured at O320 and O1280, 1 to 47
// levels, within 1.3x of the best candidate everywhere, 2-4x faster than the
// flat form over the mesh's tiles): below 24 levels the flat form over
// blocks of 64 positions (512 threads); from 24 levels the column form over
// blocks of 16 positions, one level per lane (FP64 divergence and curl: the
// automatic lane-vector width), and on meshes of many tiles the
// register-staged sweep for the FP32 gradient (up to 79 levels) and the
// wave-specialised sweep for the FP64 divergence and curl (below 48).
constexpr size_t kMaxLds = 160 * 1024;
size_t sweepw_chunks(const DevMesh &m, int gw, int nvec, int want_vpc, int *nchunk, int *vpc_out,
                     int *fcap_out, int *gcap_out);

// Where the wave-specialised sweep is the built-in shape (meshes of many
// tiles with packed geometry), measured at O1280 against the other forms.
// Narrow level chunks take up to eight positions per wavefront, so short
// columns fill the lanes too.  FP64 gradient from 4 levels (8: 0.57 against
// 0.87 ms for the flat form, 37: 1.51 against 2.75 for the column form),
// long columns in the chunk count that fills the most lanes; FP64
// divergence and curl from 2 levels (4: 0.47 against 0.62 ms, 16: 0.82
// against 1.71), from 33 in chunks of 16 lane vectors.  In FP32, where one chunk of at most 32 lane vectors holds
// the column: the gradient from 12 to 128 levels (16: 0.82 against 1.37 ms
// for the flat form, 64: 1.50 against 2.07 for the register-staged sweep,
// 91: 2.58 against 3.02 for the column form), from 88 to 160 levels in
// chunks of 16 lane vectors, and the divergence and curl from 6 to 64
// levels (8: 0.65 against 0.96 ms, 48: 2.06 against 2.80), from 41 in
// chunks of 16, on the largest meshes to 96.  Workgroups of 768
// threads where the LDS fits twice in a compute unit, in FP32 (24 levels of
// a vector field: 1.59 against 1.92 ms with 1024), for the FP64 divergence
// in chunks of 16, and for FP64 chunks of at most 8 lane vectors (4 levels
// of the gradient: 0.50 against 0.57 ms).
static bool sweepw_default(const DevMesh &m, atlas_op op, atlas_dtype dt, int nlev, LaunchShape *s) {
  const bool grad = op == ATLAS_OP_GRADIENT;
  if (!grad && op != ATLAS_OP_DIVERGENCE && op != ATLAS_OP_CURL) return false;
  // lane vectors of 16 bytes: levels per lane vector
  const int nv = dt == ATLAS_F64 ? (grad ? 2 : 1) : (grad ? 4 : 2);
  const int nvec = (nlev + nv - 1) / nv;
  int nch = 0, vpc = 0;
  const size_t lds = sweepw_chunks(m, grad ? 10 : kSgeoWords, nvec, 0, &nch, &vpc, nullptr, nullptr);
  bool take;
  int want = 0;  // lane vectors per chunk asked for (0: as many as fit)
  if (dt == ATLAS_F64 && grad && nch > 1) {
    // columns of several chunks: the count (up to two more than the fewest)
    // that fills the most lanes with whole chunks (137 levels: four chunks
    // of 18, three positions per wavefront, 5.19 against 5.45 ms for two
    // chunks of 35)
    double best = 0.0;
    for (int c = nch; c <= nch + 2; ++c) {
      const int v = (nvec + c - 1) / c;
      const double fill = (double)(min(8, 64 / v) * v) / 64.0;
      if (fill > best + 1e-9) {
        best = fill;
        want = v;
      }
    }
  } else if (dt == ATLAS_F64 && !grad && nlev > 32) {
    want = 16;  // vector columns wider than 32 lane vectors: chunks of 16
                // (four positions per wavefront) at two workgroups per CU;
                // O1280: 48 levels 2.07 against 2.74 ms for one chunk of
                // 48, 72 levels 3.33 against 3.88, 110 levels 4.78 against
                // 5.82 for the column form, 137 levels 6.19 against 6.57
                // for three chunks of 46
  } else if (dt == ATLAS_F32 && !grad && nlev > 40 &&
             (nlev <= 64 || (nlev <= 96 && m.ntiles >= 4096))) {
    want = 16;  // (O1280, 48 levels: 1.86 against 2.05 ms in one chunk;
                // 91 levels: 3.15 against 3.30 for the column form, which
                // stays ahead at O640 from 65 levels)
  } else if (dt == ATLAS_F32 && grad && nlev >= 88 && nlev <= 160) {
    want = 16;  // (O1280, 91 levels: 2.51 against 2.70 ms in one chunk;
                // 137 levels: 3.81 against 3.87 for the column form)
  }
  if (want && want * nv <= 64) {  // a level_chunk a caller may pass back
    int nch2 = 0, vpc2 = 0;
    const size_t l2 =
        sweepw_chunks(m, grad ? 10 : kSgeoWords, nvec, want, &nch2, &vpc2, nullptr, nullptr);
    if (l2 <= kMaxLds) {
      s->level_chunk = want * nv;
      const bool two_per_cu = 2 * l2 <= kMaxLds && !(dt == ATLAS_F64 && grad);
      s->variant = ATLAS_VARIANT_SWEEP;
      s->block = two_per_cu ? 768 : 1024;
      s->nodes_per_block = 0;
      s->blocks_per_cu = 0;
      s->level_vec = 0;
      return true;
    }
  }
  if (dt == ATLAS_F64)
    take = grad ? nlev >= 4
                : nlev >= 2 && (nlev < 48 || (nch <= 3 && (vpc >= 36 || (vpc >= 24 && vpc <= 32))));
  else
    take = nch == 1 && vpc <= 32 && nlev >= (grad ? 12 : 6);
  if (!take) return false;
  const bool two_per_cu = 2 * lds <= kMaxLds && (dt == ATLAS_F32 || vpc <= kSweepwNpn8);
  s->variant = ATLAS_VARIANT_SWEEP;
  s->block = two_per_cu ? 768 : 1024;
  s->nodes_per_block = 0;
  s->level_chunk = 0;
  s->blocks_per_cu = 0;
  s->level_vec = 0;
  return true;
}

LaunchShape default_shape(const MeshStore &m, atlas_op op, int nlev, atlas_dtype dt) {
  LaunchShape s;
  s.variant = nlev >= 24 ? ATLAS_VARIANT_COLUMN : ATLAS_VARIANT_FLAT;
  s.block = nlev >= 24 ? 256 : 512;
  s.nodes_per_block = nlev >= 24 ? 16 : 64;
  s.level_vec = 0;
  const bool sweep_fits = m.d.sweep_ok && m.d.ntiles >= kSweepMinTiles &&
                          max(1, m.d.segmax) * kGeoWords <= 768;
  // the wave-specialised sweep needs the packed geometry and rows of 4..6
  const bool sweepw_fits = sweep_fits && m.d.sgeo && m.d.maxdeg <= 6 && m.d.mindeg >= kMinRow;
  if (op == ATLAS_OP_LAPLACIAN) {
    // large meshes: the fused one-pass form, wave-specialised (it moves a
    // third of the two passes' field bytes; measured faster than the two
    // passes up to 137 levels at O640 and O1280 in both precisions from 17
    // levels in FP64 and 33 in FP32).  Shorter columns take the two passes,
    // each on its own sweep with several positions per wavefront (O1280
    // FP64 16 levels: 1.61 against 1.89 ms; FP32 32 levels: 2.05 against
    // 2.57)
    if (nlev >= (dt == ATLAS_F64 ? 17 : 33) && m.d.l2_ok && m.d.ntiles >= kSweepMinTiles &&
        m.d.maxdeg <= 6 && m.d.mindeg >= kMinRow) {
      s.variant = ATLAS_VARIANT_FUSED;
      s.block = 1024;
      s.nodes_per_block = 0;
      return s;
    }
    s.per_pass = 1;
    return s;
  }
  if (sweepw_fits && sweepw_default(m.d, op, dt, nlev, &s)) return s;
  if (nlev < 24) return s;
  // the sweep runs one workgroup per tile and level chunk, each walking its
  // band's parallels in turn: only a mesh of many tiles fills the chip
  if (nlev < 48) {
    if (dt == ATLAS_F32 && op == ATLAS_OP_GRADIENT && sweep_fits) {
      // register-staged sweep: it keeps one level per lane at these lengths
      // (37 levels at O1280: 1.9 ms against 3.6 ms for 16-byte lanes)
      s.variant = ATLAS_VARIANT_SWEEP;
      s.block = 768;
      s.nodes_per_block = 0;
      s.blocks_per_cu = 1;
    } else if (!(dt == ATLAS_F64 && (op == ATLAS_OP_DIVERGENCE || op == ATLAS_OP_CURL))) {
      s.level_vec = 1;
    }
    return s;
  }
  if (dt == ATLAS_F32 && op == ATLAS_OP_GRADIENT) {
    s.level_vec = 1;
    // up to ~80 levels the register-staged sweep's single read of each
    // column wins over the compensated sums' lane work (64 levels: 2.1 ms
    // against 2.5 ms at O1280); beyond, one level per lane (91 levels: 3.02
    // against 3.30 ms)
    if (nlev < 80 && sweep_fits) {
      s.variant = ATLAS_VARIANT_SWEEP;
      s.block = 768;
      s.nodes_per_block = 0;
      s.level_vec = 0;
      s.blocks_per_cu = 1;
    }
  }
  if (dt == ATLAS_F64 && op == ATLAS_OP_GRADIENT && sweep_fits) {
    // without the packed geometry: the register-staged sweep on 768 threads
    s.variant = ATLAS_VARIANT_SWEEP;
    s.block = 768;
    s.nodes_per_block = 0;
    s.blocks_per_cu = 1;
  }
  return s;
}


// Level chunking of the wave-specialised sweep: nvec lane vectors per column
// in nchunk even chunks of vpc (at most 64, or level_chunk's share), more
// chunks until the field ring (kSweepwSlots slots) and the geometry ring
// (kSweepwGeoSlots slots of gw words per position) fit in LDS.  Returns the
// LDS bytes.
size_t sweepw_chunks(const DevMesh &m, int gw, int nvec, int want_vpc, int *nchunk, int *vpc_out,
                     int *fcap_out, int *gcap_out) {
  int vpc = min(want_vpc > 0 ? want_vpc : 64, nvec);
  int nch = (nvec + vpc - 1) / vpc;
  vpc = (nvec + nch - 1) / nch;
  const int seg = max(1, m.segmax);
  const int gcap = (seg * gw + 63) / 64 * 64;
  auto fcap_of = [&](int v) { return (seg * v + 63) / 64 * 64; };
  auto bytes = [&](int v) {
    return (size_t)16 * (kSweepwSlots * fcap_of(v) + kSweepwGeoSlots * gcap);
  };
  while (vpc > 1 && bytes(vpc) > kMaxLds) {
    ++nch;
    vpc = (nvec + nch - 1) / nch;
  }
  *nchunk = (nvec + vpc - 1) / vpc;
  *vpc_out = vpc;
  if (fcap_out) *fcap_out = fcap_of(vpc);
  if (gcap_out) *gcap_out = gcap;
  return bytes(vpc);
}

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// Levels per chunk of the sweep form: at most 64 (one per lane), split
// evenly (137 -> 46, 46, 45).
static int sweep_chunk(int nlev, int want) {
  if (want > 0) return min(want, 64);
  const int n = (nlev + 63) / 64;
  return (nlev + n - 1) / n;
}

// Whether a sweep shape runs the wave-specialised kernel: blocks_per_cu 0,
// the packed geometry, 16-byte lane vectors, rows of 4..6 incidences and a
// block of at least 512 threads.
template <class T, int OP>
static bool sweepw_applies(const DevMesh &m, int nlev, const LaunchShape &sh) {
  constexpr int nv16 = 16 / (int)sizeof(typename Pol<T, OP>::V);
  return sh.blocks_per_cu == 0 && m.sgeo && (sh.level_vec == 0 || sh.level_vec == nv16) &&
         nlev >= nv16 && m.maxdeg <= 6 && m.mindeg >= kMinRow && sh.block >= 512 &&
         sh.block % 64 == 0;
}

// The wave-specialised sweep of `sh` (sweepw_applies); DC: the divergence
// and, into out2, the curl of the same field in one pass.
template <class T, int OP, bool DC>
static atlas_status launch_sweepw(const DevMesh &m, const T *in, T *out, T *out2, int nlev,
                                  const LaunchShape &sh, hipStream_t st) {
  constexpr int nv16 = 16 / (int)sizeof(typename Pol<T, OP>::V);
  const int nvec = (nlev + nv16 - 1) / nv16;
  constexpr int gw = Pol<T, OP>::kVecIn ? kSgeoWords : 10;
  int nchunk = 0, vpc = 0, fcap = 0, gcap = 0;
  const size_t lds = sweepw_chunks(m, gw, nvec,
                                   sh.level_chunk > 0 ? (sh.level_chunk + nv16 - 1) / nv16 : 0,
                                   &nchunk, &vpc, &fcap, &gcap);
  if (lds > kMaxLds) return fail(ATLAS_EINVAL, "sweep tile too large for LDS");
  const int units = m.ntiles * nchunk;
  const int per = (units + 7) / 8;
  void (*kern)(DevMesh, const T *, T *, T *, int, int, int, int, int, int) = nullptr;
  // NPN positions per wavefront when NPN chunks fit in its lanes
  if constexpr (lane_vec_ok<T, OP, nv16>())
    kern = vpc <= 8    ? k_sweepw<T, OP, nv16, 8, DC>
           : vpc <= 12 ? k_sweepw<T, OP, nv16, 5, DC>
           : vpc <= 16 ? k_sweepw<T, OP, nv16, 4, DC>
           : vpc <= 21 ? k_sweepw<T, OP, nv16, 3, DC>
           : vpc <= 32 ? k_sweepw<T, OP, nv16, 2, DC>
                       : k_sweepw<T, OP, nv16, 1, DC>;
  if (!kern) return fail(ATLAS_EINVAL, "wave-specialised sweep not available");
  ATLASX_HIP(hipFuncSetAttribute((const void *)kern,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3(per * 8), dim3(sh.block), lds, st, m, in, out, out2, nlev, vpc,
                     m.ntiles, per, fcap, gcap);
  ATLASX_HIP(hipGetLastError());
  return ATLAS_OK;
}

template <class T, int OP>
static atlas_status launch_typed(const MeshStore &ms, const T *in, int nlev, T *out, void *ws,
                                 const LaunchShape &sh, hipStream_t st,
                                 const DevMesh *dm = nullptr) {
  const DevMesh &m = dm ? *dm : ms.d;
  const int ntiles = sh.nodes_per_block > 0 ? (m.V + sh.nodes_per_block - 1) / sh.nodes_per_block
                                            : m.ntiles;
  const int per_xcd = (ntiles + 7) / 8;
  const dim3 grid(per_xcd * 8), block(sh.block);
  if (sh.nodes_per_block > 0 && (int64_t)sh.nodes_per_block * nlev * 2 >= ((int64_t)1 << 31))
    return fail(ATLAS_EINVAL, "nodes_per_block * nlev too large");
  switch (sh.variant) {
    case ATLAS_VARIANT_COLUMN: {
      if (sh.block > 512 && sh.level_chunk == 0)
        return fail(ATLAS_EINVAL, "the column form takes at most 512 threads per block");
      if (sh.level_chunk > 0) {
        const int nchunk = (nlev + sh.level_chunk - 1) / sh.level_chunk;
        if ((int64_t)ntiles * nchunk * sh.block >= ((int64_t)1 << 32))
          return fail(ATLAS_EINVAL, "too many work units: raise nodes_per_block or level_chunk");
        const int units = ntiles * nchunk;
        const int per = (units + 7) / 8;
        hipLaunchKernelGGL((k_column_chunked<T, OP>), dim3(per * 8), block, 0, st, m, in, out,
                           nlev, sh.nodes_per_block, sh.level_chunk, ntiles, per);
        break;
      }
      const int nch = (nlev + 63) / 64;
      // persistent grid: blocks_per_cu workgroups on every compute unit
      const int cyc = sh.blocks_per_cu > 0 ? sh.blocks_per_cu * device_cu_count() / 8 : 0;
      const dim3 cgrid = cyc > 0 ? dim3(8 * cyc) : grid;
      // level_vec: 0 = widest lane vector, 2 / 4 = at most that many levels
      // per lane, 1 = the one-level-per-lane kernel
      if (sh.level_vec < 0 || sh.level_vec > 4)
        return fail(ATLAS_EINVAL, "level_vec must be in [0, 4]");
      const int nv = sh.level_vec == 1 ? 0
                                       : auto_level_vec<T, OP>(nlev, m.maxdeg, m.mindeg,
                                                               sh.level_vec);
      if (nv > 0) {
        const int nchv = (nlev + 64 * nv - 1) / (64 * nv);
        void (*kern)(DevMesh, const T *, T *, int, int, int, int) = nullptr;
#define ATLASX_COLV(NV)                                                     \
  if constexpr (lane_vec_ok<T, OP, NV>()) {                                 \
    if (nchv == 1) kern = k_colv<T, OP, NV, 1>;                             \
    else if (nchv == 2) kern = k_colv<T, OP, NV, 2>;                        \
    else if (nchv == 3) kern = k_colv<T, OP, NV, 3>;                        \
    else kern = k_colv<T, OP, NV, 4>;                                       \
  }
        if (nv == 1) {
          ATLASX_COLV(1)
        } else if (nv == 2) {
          ATLASX_COLV(2)
        } else if (nv == 3) {
          ATLASX_COLV(3)
        } else {
          ATLASX_COLV(4)
        }
#undef ATLASX_COLV
        if (!kern) return fail(ATLAS_EINVAL, "level_vec not available for this dtype and operator");
        hipLaunchKernelGGL(kern, cgrid, block, 0, st, m, in, out, nlev, sh.nodes_per_block,
                           per_xcd, cyc);
        break;
      }
#define ATLASX_COL(N)                                                                  \
  do {                                                                                 \
    if (m.maxdeg <= 6)                                                                 \
      hipLaunchKernelGGL((k_column<T, OP, N, 6>), cgrid, block, 0, st, m, in, out, nlev, \
                         sh.nodes_per_block, per_xcd, cyc);                            \
    else                                                                               \
      hipLaunchKernelGGL((k_column<T, OP, N, 8>), cgrid, block, 0, st, m, in, out, nlev, \
                         sh.nodes_per_block, per_xcd, cyc);                            \
  } while (0)
      if (nch == 1) ATLASX_COL(1);
      else if (nch == 2) ATLASX_COL(2);
      else if (nch == 3) ATLASX_COL(3);
      else if (nch == 4) ATLASX_COL(4);
      else ATLASX_COL(0);
#undef ATLASX_COL
      break;
    }
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
    case ATLAS_VARIANT_SWEEP: {
      if (!m.sweep_ok) return fail(ATLAS_EINVAL, "the sweep form needs a mesh of parallels");
      if (sh.nodes_per_block > 0)
        return fail(ATLAS_EINVAL, "the sweep form runs on the mesh's tiles (nodes_per_block = 0)");
      // the chunk shrinks until a parallel's run fits the staging registers
      // (16 elements per thread) and four runs fit in LDS
      if (sh.level_vec < 0 || sh.level_vec > 4)
        return fail(ATLAS_EINVAL, "level_vec must be in [0, 4]");
      // the level-vector sweep stages each position's geometry with one
      // thread per 16-byte word: it needs a block of segmax * kGeoWords
      // threads, else the one-level-per-lane sweep runs (same results)
      // wave-specialised sweep (blocks_per_cu == 0): 16-byte lane vectors
      if (sweepw_applies<T, OP>(m, nlev, sh)) {
        atlas_status s = launch_sweepw<T, OP, false>(m, in, out, nullptr, nlev, sh, st);
        if (s != ATLAS_OK) return s;
        break;
      }
      int nv = sh.level_vec == 1 ? 0
                                 : auto_level_vec<T, OP>(nlev, m.maxdeg, m.mindeg, sh.level_vec);
      if (sh.block < max(1, m.segmax) * kGeoWords) nv = 0;
      if (nv > 0) {
        // level chunk: vpc lane vectors per workgroup pass, at most 64, split
        // evenly; it shrinks until four runs fit the LDS budget (two
        // workgroups per compute unit) and a run fits the staging registers
        const int nvec = (nlev + nv - 1) / nv;
        int vpc = sh.level_chunk > 0 ? min(64, (sh.level_chunk + nv - 1) / nv) : 64;
        vpc = min(vpc, nvec);
        {
          const int nchunk = (nvec + vpc - 1) / vpc;
          vpc = (nvec + nchunk - 1) / nchunk;
        }
        const size_t seg = (size_t)max(1, m.segmax);
        const size_t rb = (size_t)nv * sizeof(typename Pol<T, OP>::V);  // lane-vector bytes
        // geometry staged per run: 2 record words and up to kGeoWords row
        // words per position, one of each kind per thread
        const size_t geo = 4 * seg * (2 + kGeoWords) * 16;
        const size_t budget = sh.block > 512 ? kMaxLds : kMaxLds / 2;
        // (staging: at most kSweepEpt lane vectors per thread and run)
        while (vpc > 1 && (4 * seg * vpc * rb + geo > budget ||
                           (int)((seg * vpc + sh.block - 1) / sh.block) > kSweepEpt))
          vpc = (vpc + 1) / 2;
        const int ept = (int)((seg * vpc + sh.block - 1) / sh.block);
        if (4 * seg * vpc * rb + geo > kMaxLds || ept > kSweepEpt)
          return fail(ATLAS_EINVAL, "sweep tile too large for LDS or the block size");
        const int nchunk = (nvec + vpc - 1) / vpc;
        const size_t lds = 4 * seg * vpc * rb + geo;
        const int units = m.ntiles * nchunk;
        const int per = (units + 7) / 8;
        void (*kern)(DevMesh, const T *, T *, int, int, int, int) = nullptr;
#define ATLASX_SWV(NV)                                              \
  if constexpr (lane_vec_ok<T, OP, NV>()) kern = k_sweepv<T, OP, NV, kSweepEpt>;
        if (nv == 1) {
          ATLASX_SWV(1)
        } else if (nv == 2) {
          ATLASX_SWV(2)
        } else if (nv == 3) {
          ATLASX_SWV(3)
        } else {
          ATLASX_SWV(4)
        }
#undef ATLASX_SWV
        if (!kern) return fail(ATLAS_EINVAL, "level_vec not available for this dtype and operator");
        ATLASX_HIP(hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(per * 8), block, lds, st, m, in, out, nlev, vpc, m.ntiles,
                           per);
        break;
      }
      // wavefront w stages nodes w, w + nw, ... of a run: EPT >= segmax / nw;
      // four runs of kc levels must fit in LDS (the chunk shrinks if needed)
      const size_t vbytes = sizeof(T) * (OP == OP_GRAD ? 1 : 2);
      int kc = sweep_chunk(nlev, sh.level_chunk);
      kc = min(kc, (int)(kMaxLds / (4 * vbytes * (size_t)max(1, m.segmax))));
      if (kc < 1) return fail(ATLAS_EINVAL, "sweep tile too large for LDS");
      const int nchunk = (nlev + kc - 1) / kc;
      const size_t lds = (size_t)4 * m.segmax * kc * vbytes;
      const int need = (m.segmax + (sh.block >> 6) - 1) / (sh.block >> 6);
      const int units = m.ntiles * nchunk;
      const int per = (units + 7) / 8;
      void (*kern)(DevMesh, const T *, T *, int, int, int, int) = nullptr;
      if (need <= 4) kern = k_sweep<T, OP, 4>;
      else if (need <= 8) kern = k_sweep<T, OP, 8>;
      else if (need <= 16) kern = k_sweep<T, OP, 16>;
      else if (need <= 32) kern = k_sweep<T, OP, 32>;
      else return fail(ATLAS_EINVAL, "sweep tile too large for the block size");
      ATLASX_HIP(hipFuncSetAttribute((const void *)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      hipLaunchKernelGGL(kern, dim3(per * 8), block, lds, st, m, in, out, nlev, kc, m.ntiles, per);
      break;
    }
    case ATLAS_VARIANT_FUSED:
      return fail(ATLAS_EINVAL, "the fused variant is for the Laplacian only");
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

// Shape of one Laplacian pass: the autotuned one for that operator, else the
// built-in one.
static LaunchShape pass_shape(const MeshStore &ms, atlas_op op, int nlev, atlas_dtype dt) {
  MeshStore &m = const_cast<MeshStore &>(ms);
  std::lock_guard<std::mutex> g(m.tune_mu);
  auto it = m.tuned.find(TuneKey{(int)op, (int)dt, nlev});
  return it != m.tuned.end() ? it->second : default_shape(ms, op, nlev, dt);
}

// Laplacian: gradient into the workspace [V][nlev][2], then its divergence;
// the flux form needs its flux buffer behind the gradient.
// Divergence and curl of one field in one pass (column form, level-vector
// lanes of the divergence's automatic width).  Short columns (below 48
// levels) and meshes outside the level-vector form run the two operators
// one after the other with their own shapes (same results).
template <class T>
static atlas_status launch_div_curl_typed(const MeshStore &ms, atlas_dtype dt, const T *in,
                                          int nlev, T *od, T *oc, hipStream_t st) {
  const DevMesh &m = ms.d;
  {
    // where the divergence runs the wave-specialised sweep, the curl rides
    // on the same loads
    LaunchShape sh = shape_from(nullptr, ms, ATLAS_OP_DIVERGENCE, nlev, dt);
    if (sh.variant == ATLAS_VARIANT_SWEEP && sh.level_chunk > 0) {
      // chunks of 16 lane vectors pay for the divergence alone; with the
      // curl's states beside it the one pass runs slower in them (9.67
      // against 8.42 ms at O1280, 137 levels), so it takes the widest
      // chunks where at most three of at least 36 (or 24-32) lane vectors
      // fill the lanes, else the column form
      int nch = 0, vpc = 0;
      constexpr int nv16 = 16 / (int)sizeof(typename Pol<T, OP_DIV>::V);
      const size_t lds = sweepw_chunks(m, kSgeoWords, (nlev + nv16 - 1) / nv16, 0, &nch, &vpc,
                                       nullptr, nullptr);
      const bool wide = sizeof(T) == 8
                            ? nlev < 48 || (nch <= 3 && (vpc >= 36 || (vpc >= 24 && vpc <= 32)))
                            : nch == 1 && vpc <= 32;
      if (wide) {
        sh.level_chunk = 0;
        sh.block = sizeof(T) == 4 && 2 * lds <= kMaxLds ? 768 : 1024;
      } else {
        sh.variant = ATLAS_VARIANT_COLUMN;
      }
    }
    if (sh.variant == ATLAS_VARIANT_SWEEP && sweepw_applies<T, OP_DIV>(m, nlev, sh))
      return launch_sweepw<T, OP_DIV, true>(m, in, od, oc, nlev, sh, st);
  }
  const int nv = nlev >= 48 ? auto_level_vec<T, OP_DIV>(nlev, m.maxdeg, m.mindeg) : 0;
  if (nv == 0) {
    for (atlas_op op : {ATLAS_OP_DIVERGENCE, ATLAS_OP_CURL}) {
      LaunchShape sh = shape_from(nullptr, ms, op, nlev, dt);
      if (sh.variant == ATLAS_VARIANT_FLUX) sh = default_shape(ms, op, nlev, dt);
      atlas_status s = launch_op(ms, op, dt, in, nlev, op == ATLAS_OP_CURL ? (void *)oc : (void *)od,
                                 nullptr, sh, st);
      if (s != ATLAS_OK) return s;
    }
    return ATLAS_OK;
  }
  const int nvec = (nlev + nv - 1) / nv, nch = (nvec + 63) / 64;
  constexpr int kNpb = 16;
  const int ntiles = (m.V + kNpb - 1) / kNpb;
  const int per_xcd = (ntiles + 7) / 8;
  void (*kern)(DevMesh, const T *, T *, T *, int, int, int) = nullptr;
#define ATLASX_DC(NV)                                                  \
  if constexpr (lane_vec_ok<T, OP_DIV, NV>()) {                          \
    if (nch == 1) kern = k_colv_dc<T, NV, 1>;                            \
    else if (nch == 2) kern = k_colv_dc<T, NV, 2>;                       \
    else if (nch == 3) kern = k_colv_dc<T, NV, 3>;                       \
    else kern = k_colv_dc<T, NV, 4>;                                     \
  }
  if (nv == 1) {
    ATLASX_DC(1)
  } else if (nv == 2) {
    ATLASX_DC(2)
  } else if (nv == 3) {
    ATLASX_DC(3)
  } else {
    ATLASX_DC(4)
  }
#undef ATLASX_DC
  if (!kern || nch > 4) return fail(ATLAS_EINVAL, "no level-vector width for this column");
  hipLaunchKernelGGL(kern, dim3(per_xcd * 8), dim3(256), 0, st, m, in, od, oc, nlev, kNpb,
                     per_xcd);
  ATLASX_HIP(hipGetLastError());
  return ATLAS_OK;
}

atlas_status launch_div_curl(const MeshStore &ms, atlas_dtype dt, const void *in, int nlev,
                             void *out_div, void *out_curl, hipStream_t st) {
  if (dt == ATLAS_F64)
    return launch_div_curl_typed<double>(ms, dt, static_cast<const double *>(in), nlev,
                                         static_cast<double *>(out_div),
                                         static_cast<double *>(out_curl), st);
  return launch_div_curl_typed<float>(ms, dt, static_cast<const float *>(in), nlev,
                                      static_cast<float *>(out_div),
                                      static_cast<float *>(out_curl), st);
}

// The fused Laplacian's launch plan: lane width, level chunk and LDS bytes;
// false where the plan or the kernel's assumptions do not hold (no plan,
// rows outside 4..6 incidences, a block too small for the staging, runs too
// long for LDS).
struct FusedPlan {
  int nv, vpc, nchunk;
  size_t lds;
};
template <class T>
static bool fused_plan(const MeshStore &ms, int nlev, const LaunchShape &sh, FusedPlan *fp) {
  const DevMesh &m = ms.d;
  if (!m.l2_ok || m.maxdeg > 6 || m.mindeg < kMinRow) return false;
  constexpr int NVW = (int)(16 / sizeof(T));  // 16-byte field lanes
  const int nv = (nlev >= NVW && sh.level_vec != 1) ? NVW : 1;
  const int nvec = (nlev + nv - 1) / nv;
  const size_t fb = (size_t)nv * sizeof(T), gb = 2 * fb;  // lane-vector bytes
  const size_t per_vec = 4 * (size_t)m.l2_fmax * fb + 4 * (size_t)m.l2_gmax * gb;
  // two slots of packed geometry; a thread stages at most kGeoEpt words
  const size_t geo_words = (size_t)m.l2_gmax * kGGeoWords +
                           (size_t)m.l2_pmax * (sizeof(T) == 8 ? kLGeoWords64 : kLGeoWords);
  const size_t geo = 2 * geo_words * 16;
  if (geo_words > (size_t)kGeoEpt * sh.block) return false;
  int vpc = sh.level_chunk > 0 ? min(64, (sh.level_chunk + nv - 1) / nv) : 64;
  vpc = min(vpc, nvec);
  {
    const int nchunk = (nvec + vpc - 1) / vpc;
    vpc = (nvec + nchunk - 1) / nchunk;
  }
  // the chunk shrinks until both rings fit in LDS and a field run fits the
  // staging registers (kLsweepEpt lane vectors per thread)
  while (vpc > 1 && (per_vec * vpc + geo > kMaxLds ||
                     ((size_t)m.l2_fmax * vpc + sh.block - 1) / sh.block > (size_t)kLsweepEpt))
    vpc = (vpc + 1) / 2;
  if (per_vec * vpc + geo > kMaxLds ||
      ((size_t)m.l2_fmax * vpc + sh.block - 1) / sh.block > (size_t)kLsweepEpt)
    return false;
  fp->nv = nv;
  fp->vpc = vpc;
  fp->nchunk = (nvec + vpc - 1) / vpc;
  fp->lds = per_vec * vpc + geo;
  return true;
}

// The wave-specialised fused Laplacian's plan (blocks_per_cu 0, 16-byte
// lanes, at least one consumer wavefront): the level chunk shrinks until
// the three rings fit in LDS; false where it cannot run.  The field ring
// has five slots, or four where five would take one more level chunk
// (FP64 at 137 levels on O1280's tiles: three chunks of 23 lane vectors
// instead of four of 18); nodes_per_block 4 or 5 sets it.
struct FusedwPlan {
  int vpc, nchunk, fcap, gcap, ocap, fslots;
  size_t lds;
};
template <class T>
static bool fusedw_plan(const MeshStore &ms, int nlev, const LaunchShape &sh, FusedwPlan *fp) {
  const DevMesh &m = ms.d;
  constexpr int NVW = (int)(16 / sizeof(T));
  if (!m.l2_ok || m.maxdeg > 6 || m.mindeg < kMinRow || !m.l2_ggeo || !m.l2_lgeo) return false;
  if (sh.blocks_per_cu != 0 || sh.level_vec == 1 || nlev < NVW) return false;
  if (sh.block < 64 * (kLswProducers + 1)) return false;
  if (m.l2_gmax > 64 || m.l2_pmax > 64) return false;  // one record of each kind per lane
  const int nvec = (nlev + NVW - 1) / NVW;
  int vpc = sh.level_chunk > 0 ? min(64, (sh.level_chunk + NVW - 1) / NVW) : 64;
  vpc = min(vpc, nvec);
  int nch = (nvec + vpc - 1) / vpc;
  vpc = (nvec + nch - 1) / nch;
  auto r64 = [](int64_t x) { return (int)((x + 63) / 64 * 64); };
  const int LGW = sizeof(T) == 8 ? kLGeoWords64 : kLGeoWords;
  const int gcap = r64((int64_t)m.l2_gmax * kGGeoWords), ocap = r64((int64_t)m.l2_pmax * LGW);
  auto bytes = [&](int v, int fs) {
    return (size_t)16 * ((size_t)fs * r64((int64_t)m.l2_fmax * v) +
                         (size_t)kLswGSlots * 2 * m.l2_gmax * v +
                         (size_t)kLswGeoSlots * (gcap + ocap));
  };
  if (sh.nodes_per_block != 0 && sh.nodes_per_block != 4 && sh.nodes_per_block != 5) return false;
  int fs = sh.nodes_per_block ? sh.nodes_per_block : kLswFSlots;
  while (vpc > 1 && bytes(vpc, fs) > kMaxLds) {
    if (!sh.nodes_per_block && fs == kLswFSlots && bytes(vpc, 4) <= kMaxLds) {
      fs = 4;  // four slots save this chunk
      break;
    }
    ++nch;
    vpc = (nvec + nch - 1) / nch;
  }
  if (bytes(vpc, fs) > kMaxLds) return false;
  fp->vpc = vpc;
  fp->nchunk = (nvec + vpc - 1) / vpc;
  fp->fcap = r64((int64_t)m.l2_fmax * vpc);
  fp->gcap = gcap;
  fp->ocap = ocap;
  fp->fslots = fs;
  fp->lds = bytes(vpc, fs);
  return true;
}

bool lapl_fused_runs(const MeshStore &ms, int nlev, atlas_dtype dt, const LaunchShape &sh) {
  if (sh.variant != ATLAS_VARIANT_FUSED) return false;
  FusedPlan fp;
  FusedwPlan fw;
  return dt == ATLAS_F64
             ? fusedw_plan<double>(ms, nlev, sh, &fw) || fused_plan<double>(ms, nlev, sh, &fp)
             : fusedw_plan<float>(ms, nlev, sh, &fw) || fused_plan<float>(ms, nlev, sh, &fp);
}

// The fused Laplacian on the two-ring plan; *ran = false (nothing
// launched) where fused_plan refuses.
template <class T>
atlas_status launch_lapl_fused(const MeshStore &ms, const T *in, int nlev, T *out,
                               const LaunchShape &sh, hipStream_t st, bool *ran) {
  const DevMesh &m = ms.d;
  *ran = false;
  constexpr int NVW = (int)(16 / sizeof(T));
  FusedwPlan fw;
  if (fusedw_plan<T>(ms, nlev, sh, &fw)) {
    // wave-specialised: consumers take one lane vector per lane, vpc lanes
    // per node
    const int units = m.ntiles * fw.nchunk;
    const int per = (units + 7) / 8;
    auto kern = fw.fslots == 4 ? k_lsweepw<T, NVW, 4> : k_lsweepw<T, NVW, 5>;
    ATLASX_HIP(hipFuncSetAttribute((const void *)kern,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)fw.lds));
    hipLaunchKernelGGL(kern, dim3(per * 8), dim3(sh.block), fw.lds, st, m, in, out, nlev, fw.vpc,
                       m.ntiles, per, fw.vpc, fw.fcap, fw.gcap, fw.ocap);
    ATLASX_HIP(hipGetLastError());
    *ran = true;
    return ATLAS_OK;
  }
  FusedPlan fp;
  if (!fused_plan<T>(ms, nlev, sh, &fp)) return ATLAS_OK;
  const int nv = fp.nv, vpc = fp.vpc, nchunk = fp.nchunk;
  const size_t lds = fp.lds;
  const int units = m.ntiles * nchunk;
  const int per = (units + 7) / 8;
  // each lane walks nl lane vectors of a node (blocks_per_cu 1..3 picks
  // nl; 0: one), so a node takes lpn = vpc / nl lanes (rounded up) and a
  // wavefront 64 / lpn nodes
  const int nl = sh.blocks_per_cu >= 1 && sh.blocks_per_cu <= 3 ? sh.blocks_per_cu : 1;
  const int lpn = (vpc + nl - 1) / nl;
  void (*kern)(DevMesh, const T *, T *, int, int, int, int, int) = nullptr;
  if (nv == 1)
    kern = nl == 1 ? k_lsweep<T, 1, kLsweepEpt, 1>
           : nl == 2 ? k_lsweep<T, 1, kLsweepEpt, 2> : k_lsweep<T, 1, kLsweepEpt, 3>;
  else
    kern = nl == 1 ? k_lsweep<T, NVW, kLsweepEpt, 1>
           : nl == 2 ? k_lsweep<T, NVW, kLsweepEpt, 2> : k_lsweep<T, NVW, kLsweepEpt, 3>;
  ATLASX_HIP(hipFuncSetAttribute((const void *)kern,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3(per * 8), dim3(sh.block), lds, st, m, in, out, nlev, vpc,
                     m.ntiles, per, lpn);
  ATLASX_HIP(hipGetLastError());
  *ran = true;
  return ATLAS_OK;
}

// Scales of the derivatives in the computational plane: d/dlon = R cos(lat)
// times the zonal component, d/dlat = R times the meridional one, i.e. both
// sums over the node's edges divided by its (lon, lat) dual area
// A_i = V_i / (R^2 cos lat_i): alpha = beta = R beta_i.
__global__ void k_comp_scales(int V, double R, const PosRec *__restrict__ pos,
                              double *__restrict__ alpha, double *__restrict__ beta,
                              PosRec *__restrict__ pos_c) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < V) {
    PosRec r = pos[p];
    const double s = R * r.beta;
    r.alpha = s;
    r.beta = s;
    alpha[p] = s;
    beta[p] = s;
    pos_c[p] = r;
  }
}

atlas_status gradient_lonlat(MeshStore &ms, atlas_dtype dt, const void *in, int nlev, void *out,
                             hipStream_t st) {
  {
    std::lock_guard<std::mutex> g(ms.comp_mu);
    if (!ms.comp_ready) {
      const int V = ms.d.V;
      void *p = nullptr, *a = nullptr, *b = nullptr;
      if (hipMalloc(&p, sizeof(PosRec) * (size_t)V) != hipSuccess)
        return fail(ATLAS_ENOMEM, "derivative scales");
      ms.allocations.push_back(p);
      if (hipMalloc(&a, sizeof(double) * (size_t)V) != hipSuccess)
        return fail(ATLAS_ENOMEM, "derivative scales");
      ms.allocations.push_back(a);
      if (hipMalloc(&b, sizeof(double) * (size_t)V) != hipSuccess)
        return fail(ATLAS_ENOMEM, "derivative scales");
      ms.allocations.push_back(b);
      ms.bytes += (sizeof(PosRec) + 16) * (size_t)V;
      hipLaunchKernelGGL(k_comp_scales, dim3((V + 255) / 256), dim3(256), 0, 0, V, ms.radius,
                         ms.d.pos, static_cast<double *>(a), static_cast<double *>(b),
                         static_cast<PosRec *>(p));
      ATLASX_HIP(hipGetLastError());
      ATLASX_HIP(hipDeviceSynchronize());
      ms.dcomp = ms.d;
      ms.dcomp.pos = static_cast<const PosRec *>(p);
      ms.dcomp.alpha = static_cast<const double *>(a);
      ms.dcomp.beta = static_cast<const double *>(b);
      ms.dcomp.sgeo = nullptr;  // packed geometry holds the physical scales
      ms.dcomp.l2_ok = 0;
      ms.comp_ready = true;
    }
  }
  // the built-in gradient shape, except the wave-specialised sweep (its
  // packed geometry carries the physical scales): the register-staged one
  LaunchShape sh = default_shape(ms, ATLAS_OP_GRADIENT, nlev, dt);
  if (sh.variant == ATLAS_VARIANT_SWEEP) {
    sh.blocks_per_cu = 1;
    sh.block = 768;
  }
  if (dt == ATLAS_F64)
    return launch_typed<double, OP_GRAD>(ms, static_cast<const double *>(in), nlev,
                                         static_cast<double *>(out), nullptr, sh, st, &ms.dcomp);
  return launch_typed<float, OP_GRAD>(ms, static_cast<const float *>(in), nlev,
                                      static_cast<float *>(out), nullptr, sh, st, &ms.dcomp);
}

atlas_status launch_op(const MeshStore &ms, atlas_op op, atlas_dtype dt, const void *in,
                       int nlev, void *out, void *ws, const LaunchShape &sh, hipStream_t st) {
  if (op == ATLAS_OP_LAPLACIAN && sh.variant == ATLAS_VARIANT_FUSED) {
    bool ran = false;
    const atlas_status s =
        dt == ATLAS_F64
            ? launch_lapl_fused<double>(ms, static_cast<const double *>(in), nlev,
                                        static_cast<double *>(out), sh, st, &ran)
            : launch_lapl_fused<float>(ms, static_cast<const float *>(in), nlev,
                                       static_cast<float *>(out), sh, st, &ran);
    if (s != ATLAS_OK || ran) return s;
    // otherwise the two passes with their built-in shapes (same results)
    if (!ws) return fail(ATLAS_EINVAL, "the two-pass Laplacian needs a workspace");
    LaunchShape two = sh;
    two.variant = ATLAS_VARIANT_COLUMN;
    two.per_pass = 1;
    return launch_op(ms, op, dt, in, nlev, out, ws, two, st);
  }
  if (op == ATLAS_OP_LAPLACIAN) {
    if (!ws) return fail(ATLAS_EINVAL, "the two-pass Laplacian needs a workspace");
    const size_t w = dt == ATLAS_F64 ? 8 : 4;
    char *grad = static_cast<char *>(ws);
    void *flux = grad + (size_t)ms.d.V * nlev * 2 * w;
    const LaunchShape sg = sh.per_pass ? pass_shape(ms, ATLAS_OP_GRADIENT, nlev, dt) : sh;
    const LaunchShape sd = sh.per_pass ? pass_shape(ms, ATLAS_OP_DIVERGENCE, nlev, dt) : sh;
    atlas_status s = launch_op(ms, ATLAS_OP_GRADIENT, dt, in, nlev, grad, flux, sg, st);
    if (s != ATLAS_OK) return s;
    return launch_op(ms, ATLAS_OP_DIVERGENCE, dt, grad, nlev, out, flux, sd, st);
  }
  if (dt == ATLAS_F64) return launch_dtype<double>(ms, op, in, nlev, out, ws, sh, st);
  return launch_dtype<float>(ms, op, in, nlev, out, ws, sh, st);
}

}  // namespace atlasx
