/*
 * nabla_oracle.c -- FP64 CPU oracle for the edge-based median-dual
 * finite-volume nabla operators on the octahedral reduced Gaussian grid.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference against
 * which the GPU library is checked.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or helper with the GPU library, and it never reads anything the GPU
 * library produced: it builds its own grid, its own triangulation, its own
 * edge list and its own dual geometry from (N, R) alone.
 *
 * What it follows:
 *   - Grid: Section 4.2.3.5 (Gaussian latitudes are the roots of a Legendre
 *     polynomial; the first point of every parallel sits at x = 0) and
 *     Section 4.2.3.7 "Octahedral reduced Gaussian grids" (Listing 6: the nx
 *     array is 20 + 4j up to the equator, mirrored about it); Section 4.2
 *     (points are equispaced along each parallel).
 *   - Mesh: Section 4.3 (triangles between the parallels, edges between
 *     nodes; Eq. 1; on request the blocked quadrilaterals of regular grids
 *     between parallels of equal counts, the two element types kept in two
 *     blocks as in Figure 27) and Section 4.3 on vertical extrusion (levels
 *     are independent prisms, so every level is an independent 2-D
 *     problem).  Grids: also the regular longitude-latitude grids of
 *     Section 4.2.3.8 without points on the poles (latitude-shifted and
 *     shifted variants).
 *   - Field layout: Section 4.5, Figure 31 (NodeColumns: one vertical column
 *     contiguous per node, i.e. [node][level]); Listing 12 (gradient output
 *     has two variables, stored [node][level][2]).
 *   - Operators: Section 4.7 and Figure 33 (gradient, divergence, curl,
 *     Laplacian of an edge-based finite-volume method).  The paper names the
 *     operators without formulas; the discretisation implemented here is the
 *     textbook median-dual Green-Gauss scheme in the (lon, lat) plane with a
 *     nodal cos(lat) metric.  Every reading taken where the paper is silent
 *     is listed in the design notes of the repository and repeated at the
 *     function that takes it.
 *
 * Precision: FP64 throughout.  Build: gcc -O2 -ffp-contract=off -fopenmp,
 * no fast-math.  Threads partition the LEVELS into disjoint chunks, so no
 * two threads ever touch the same accumulator and the result does not depend
 * on the thread count.
 *
 * Pins (tests that tie this code to something other than itself):
 *   latitudes      -> numpy leggauss (library routine), symmetry
 *   node counts    -> printed counts (Section 4.4, Figure 28) + Listing 6
 *   triangulation  -> Euler counts, CCW areas, band area, edge multiplicity
 *   dual geometry  -> sum of areas = 2 pi^2; cell closure; brute-force
 *                     median-dual polygons built independently in the tests
 *                     (triangles and quadrilaterals)
 *   gradient       -> exact for linear data (interior), zero for constants,
 *                     Galerkin identity sum_T |T|/3 grad(phi_T) (brute force)
 *   polar nodes    -> pole-face value recovered from the output against
 *                     brute-force polar cells: exact for fields vanishing at
 *                     the pole, the node value for even orders, second-order
 *                     convergence to the analytic pole value
 *   divergence     -> exact special cases, telescoping sum(V div) = 0
 *   curl           -> exact special cases, telescoping sum(V curl) = 0
 *   Laplacian      -> spherical-harmonic eigenvalue convergence
 *   all            -> level independence, second-order convergence on random
 *                     low-degree spherical harmonics away from the poles
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Mesh record (owned by the oracle; opaque to Python except via getters).  */
/* ------------------------------------------------------------------------ */
typedef struct {
  int N;                 /* Gaussian number: parallels per hemisphere      */
  double R;              /* sphere radius                                   */
  int nrings;            /* 2N                                              */
  int32_t *nx;           /* [nrings] points per parallel                    */
  int64_t *ring_off;     /* [nrings+1] first node of each parallel          */
  int64_t V;             /* nodes                                           */
  double *lon, *lat;     /* [V] radians                                     */
  double *coslat;        /* [V] cos(lat)                                    */
  int64_t F;             /* triangles                                       */
  int32_t *tri;          /* [F][3] counter-clockwise in (lon, lat)          */
  int64_t Q;             /* quadrilaterals (second block of elements)       */
  int32_t *quad;         /* [Q][4] counter-clockwise in (lon, lat)          */
  int shift;             /* longitudes shifted by half a spacing            */
  int64_t E;             /* mesh edges                                      */
  int32_t *edge;         /* [E][2], edge[e][0] < edge[e][1]                 */
  double *S;             /* [E][2] dual-face normal (S_lon, S_lat), a -> b  */
  double *A;             /* [V] dual area in the (lon, lat) plane           */
  double *vol;           /* [V] R^2 cos(lat) A                              */
  int npole;             /* pole edges                                      */
  int32_t *pole_edge;    /* [npole][2]                                      */
  double *pole_normal;   /* [npole] lat-component of the pole face normal   */
  /* the oracle's own node -> (edge, sign) lists, ascending edge id; used by
   * the sampled evaluators only                                            */
  int64_t *adj_ptr;      /* [V+1]                                           */
  int32_t *adj_edge;     /* [2E]                                            */
  int32_t *pole_of;      /* [V] pole edge of a node, or -1                  */
} orc_mesh;

/* ------------------------------------------------------------------------ */
/* Gaussian latitudes: the 2N roots of the Legendre polynomial P_{2N}(mu),   */
/* in descending order (north to south).  Section 4.2.3.5.  Newton's method  */
/* on the three-term recurrence, started from the classical asymptotic      */
/* guess cos(pi (j + 3/4) / (n + 1/2)), carried out in extended precision   */
/* (x86 long double, 64-bit significand) and rounded to double once, so     */
/* that each mu is the double nearest the true root.  A root found in       */
/* double is only good to a few ulps, and near the poles an ulp of latitude  */
/* is a relative change of ~2e-13 in cos(lat) and in the polar dual volumes. */
/* ------------------------------------------------------------------------ */
static void legendre_pair(int n, long double x, long double *p_n, long double *p_nm1) {
  long double p0 = 1.0L, p1 = x;
  if (n == 0) { *p_n = 1.0L; *p_nm1 = 0.0L; return; }
  for (int k = 2; k <= n; ++k) {
    long double pk = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / (long double)k;
    p0 = p1;
    p1 = pk;
  }
  *p_n = p1;
  *p_nm1 = p0;
}

int orc_gauss_mu(int N, double *mu) {
  if (N < 1 || !mu) return -1;
  const int n = 2 * N;
  for (int j = 0; j < N; ++j) {
    long double x = cosl(3.14159265358979323846264338327950288L * (j + 0.75L) / (n + 0.5L));
    int converged = 0;
    for (int it = 0; it < 100; ++it) {
      long double p, pm1;
      legendre_pair(n, x, &p, &pm1);
      long double dp = n * (x * p - pm1) / (x * x - 1.0L); /* P_n'(x) */
      long double dx = p / dp;
      x -= dx;
      if (fabsl(dx) <= 1e-18L) {
        if (converged) break; /* one extra step after convergence */
        converged = 1;
      }
    }
    mu[j] = (double)x;          /* northern hemisphere: descending positive roots */
    mu[n - 1 - j] = -(double)x; /* southern mirror                                */
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Small helpers                                                             */
/* ------------------------------------------------------------------------ */
static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

/* Unwrap longitude x so that it lies within pi of the reference xref. */
static double unwrap(double x, double xref) {
  while (x - xref > ORC_PI) x -= 2.0 * ORC_PI;
  while (x - xref < -ORC_PI) x += 2.0 * ORC_PI;
  return x;
}

/* Edge id of the unordered pair (p, q); edges are sorted lexicographically,
 * first[a] is the first edge whose smaller node is a.                       */
static int64_t find_edge(const orc_mesh *m, const int64_t *first, int32_t p,
                         int32_t q) {
  int32_t a = p < q ? p : q, b = p < q ? q : p;
  int64_t lo = first[a], hi = first[a + 1] - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    int32_t bb = m->edge[2 * mid + 1];
    if (bb == b) return mid;
    if (bb < b) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

void orc_mesh_free(orc_mesh *m) {
  if (!m) return;
  free(m->nx); free(m->ring_off); free(m->lon); free(m->lat); free(m->coslat);
  free(m->tri); free(m->quad); free(m->edge); free(m->S); free(m->A); free(m->vol);
  free(m->pole_edge); free(m->pole_normal); free(m->adj_ptr);
  free(m->adj_edge); free(m->pole_of);
  free(m);
}

/* ------------------------------------------------------------------------ */
/* Build a reduced Gaussian grid (Section 4.2.3.7: nrings = 2N parallels at  */
/* the Gaussian latitudes of degree 2N, nx[j] points on parallel j; the      */
/* regular grid F<N> of Section 4.2.3.6 has nx[j] = 4N), its triangulation,  */
/* edges and median-dual geometry.  Needs nrings even, every nx >= 4 and     */
/* the two polar parallels even (their nodes pair up across the pole).       */
/* ------------------------------------------------------------------------ */
/* The general builder.  lat_in: the latitudes of the parallels (strictly
 * decreasing, inside (-pi/2, pi/2)), or NULL for the Gaussian latitudes of
 * degree nrings (nrings even).  shift: every longitude displaced by half its
 * parallel's spacing (the shifted regular grids of Section 4.2.3.8; needs
 * equal counts on all parallels).  quads: a strip between two parallels of
 * equal counts becomes quadrilaterals (U_a, L_a, L_a+1, U_a+1) -- the
 * blocked arrangement of quadrilaterals of Section 4.3 -- instead of
 * triangles; other strips stay triangulated, so a mesh can hold both element
 * types (two blocks, Section 4.3, Figure 27). */
static orc_mesh *build_general(int nrings, const int32_t *nx_in, const double *lat_in,
                               int shift, int quads, double R) {
  if (nrings < 2 || !nx_in || !(R > 0.0)) return NULL;
  if (!lat_in && (nrings & 1)) return NULL;
  for (int j = 0; j < nrings; ++j)
    if (nx_in[j] < 4) return NULL;
  if ((nx_in[0] & 1) || (nx_in[nrings - 1] & 1)) return NULL;
  if (lat_in) {
    for (int j = 0; j < nrings; ++j) {
      if (!isfinite(lat_in[j]) || !(fabs(lat_in[j]) < 0.5 * ORC_PI)) return NULL;
      if (j > 0 && !(lat_in[j] < lat_in[j - 1])) return NULL;
    }
  }
  if (shift)
    for (int j = 1; j < nrings; ++j)
      if (nx_in[j] != nx_in[0]) return NULL;
  orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
  if (!m) return NULL;
  const int N = nrings / 2;
  m->N = N;
  m->shift = shift ? 1 : 0;
  m->R = R;
  m->nrings = nrings;
  const int nr = m->nrings;

  m->nx = (int32_t *)malloc(sizeof(int32_t) * nr);
  m->ring_off = (int64_t *)malloc(sizeof(int64_t) * (nr + 1));
  for (int j = 0; j < nr; ++j) m->nx[j] = nx_in[j];
  m->ring_off[0] = 0;
  for (int j = 0; j < nr; ++j) m->ring_off[j + 1] = m->ring_off[j] + m->nx[j];
  const int64_t V = m->ring_off[nr];
  m->V = V;

  double *mu = (double *)malloc(sizeof(double) * nr);
  if (!lat_in) orc_gauss_mu(N, mu);
  m->lon = (double *)malloc(sizeof(double) * V);
  m->lat = (double *)malloc(sizeof(double) * V);
  m->coslat = (double *)malloc(sizeof(double) * V);
  for (int j = 0; j < nr; ++j) {
    double th = lat_in ? lat_in[j] : asin(mu[j]);
    for (int i = 0; i < m->nx[j]; ++i) {
      int64_t id = m->ring_off[j] + i;
      /* equispaced along the parallel, first point at lon = 0 (Sec 4.2.3.5),
       * or half a spacing east of it on a shifted grid (Sec 4.2.3.8) */
      m->lon[id] = shift ? 2.0 * ORC_PI * ((double)i + 0.5) / (double)m->nx[j]
                         : 2.0 * ORC_PI * (double)i / (double)m->nx[j];
      m->lat[id] = th;
      m->coslat[id] = cos(th);
    }
  }
  free(mu);

  /* --- triangulation between consecutive parallels (zipper rule) --------
   * Upper ring u with nu points, lower ring l with nl points; a, b count the
   * points consumed.  The next upper point lies at lon 2pi(a+1)/nu and the
   * next lower point at 2pi(b+1)/nl; the one further west is consumed first
   * (compared exactly in integers).  On a tie the ring with more points
   * advances; with equal counts the lower ring advances.                   */
  int64_t F = 0, Q = 0;
  for (int j = 0; j + 1 < nr; ++j) {
    if (quads && m->nx[j] == m->nx[j + 1]) Q += m->nx[j];
    else F += m->nx[j] + m->nx[j + 1];
  }
  m->F = F;
  m->Q = Q;
  m->tri = (int32_t *)malloc(sizeof(int32_t) * 3 * (F > 0 ? F : 1));
  m->quad = (int32_t *)malloc(sizeof(int32_t) * 4 * (Q > 0 ? Q : 1));
  int64_t t = 0, qd = 0;
  for (int j = 0; j + 1 < nr; ++j) {
    const int64_t nu = m->nx[j], nl = m->nx[j + 1];
    const int64_t ou = m->ring_off[j], ol = m->ring_off[j + 1];
    if (quads && nu == nl) {
      for (int64_t a = 0; a < nu; ++a) {
        m->quad[4 * qd + 0] = (int32_t)(ou + a);
        m->quad[4 * qd + 1] = (int32_t)(ol + a);
        m->quad[4 * qd + 2] = (int32_t)(ol + (a + 1) % nl);
        m->quad[4 * qd + 3] = (int32_t)(ou + (a + 1) % nu);
        ++qd;
      }
      continue;
    }
    int64_t a = 0, b = 0;
    while (a < nu || b < nl) {
      int64_t up = (a + 1) * nl, lo = (b + 1) * nu;
      int advance_upper;
      if (up < lo) advance_upper = 1;
      else if (up > lo) advance_upper = 0;
      else advance_upper = (nu > nl) ? 1 : 0;
      if (a == nu) advance_upper = 0;
      if (b == nl) advance_upper = 1;
      int32_t Ua = (int32_t)(ou + (a % nu)), Lb = (int32_t)(ol + (b % nl));
      if (advance_upper) {
        m->tri[3 * t + 0] = Ua;
        m->tri[3 * t + 1] = Lb;
        m->tri[3 * t + 2] = (int32_t)(ou + ((a + 1) % nu));
        ++a;
      } else {
        m->tri[3 * t + 0] = Ua;
        m->tri[3 * t + 1] = Lb;
        m->tri[3 * t + 2] = (int32_t)(ol + ((b + 1) % nl));
        ++b;
      }
      ++t;
    }
  }

  /* --- unique edges (a < b), sorted lexicographically; id = rank -------- */
  const int64_t nkeys = 3 * F + 4 * Q;
  int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * nkeys);
  for (int64_t f = 0; f < F; ++f) {
    for (int k = 0; k < 3; ++k) {
      int64_t p = m->tri[3 * f + k], q = m->tri[3 * f + (k + 1) % 3];
      int64_t a = p < q ? p : q, b = p < q ? q : p;
      keys[3 * f + k] = a * V + b;
    }
  }
  for (int64_t f = 0; f < Q; ++f) {
    for (int k = 0; k < 4; ++k) {
      int64_t p = m->quad[4 * f + k], q = m->quad[4 * f + (k + 1) % 4];
      int64_t a = p < q ? p : q, b = p < q ? q : p;
      keys[3 * F + 4 * f + k] = a * V + b;
    }
  }
  qsort(keys, (size_t)nkeys, sizeof(int64_t), cmp_i64);
  int64_t E = 0;
  for (int64_t k = 0; k < nkeys; ++k)
    if (k == 0 || keys[k] != keys[k - 1]) keys[E++] = keys[k];
  m->E = E;
  m->edge = (int32_t *)malloc(sizeof(int32_t) * 2 * E);
  for (int64_t e = 0; e < E; ++e) {
    m->edge[2 * e + 0] = (int32_t)(keys[e] / V);
    m->edge[2 * e + 1] = (int32_t)(keys[e] % V);
  }
  free(keys);
  int64_t *first = (int64_t *)malloc(sizeof(int64_t) * (V + 1));
  {
    int64_t e = 0;
    for (int64_t a = 0; a <= V; ++a) {
      while (e < E && m->edge[2 * e] < a) ++e;
      first[a] = e;
    }
  }

  /* --- median-dual geometry in the (lon, lat) plane ----------------------
   * Per triangle, coordinates unwrapped relative to its first vertex.
   * For every triangle edge the dual-face segment runs from the edge
   * midpoint to the triangle centroid; its normal (d_lat, -d_lon) is
   * oriented from the edge's first node a towards its second node b and
   * added to S_e.  Every node receives one third of the triangle's area.  */
  m->S = (double *)calloc((size_t)(2 * E), sizeof(double));
  m->A = (double *)calloc((size_t)V, sizeof(double));
  for (int64_t f = 0; f < F; ++f) {
    int32_t id[3];
    double x[3], y[3];
    for (int k = 0; k < 3; ++k) {
      id[k] = m->tri[3 * f + k];
      x[k] = m->lon[id[k]];
      y[k] = m->lat[id[k]];
    }
    x[1] = unwrap(x[1], x[0]);
    x[2] = unwrap(x[2], x[0]);
    const double cx = (x[0] + x[1] + x[2]) / 3.0;
    const double cy = (y[0] + y[1] + y[2]) / 3.0;
    const double area =
        0.5 * ((x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]));
    for (int k = 0; k < 3; ++k) m->A[id[k]] += area / 3.0;
    for (int k = 0; k < 3; ++k) {
      const int u = k, v = (k + 1) % 3;
      const int64_t e = find_edge(m, first, id[u], id[v]);
      const double mx = 0.5 * (x[u] + x[v]), my = 0.5 * (y[u] + y[v]);
      const double dx = cx - mx, dy = cy - my;
      double nxv = dy, nyv = -dx;
      /* direction a -> b, a the smaller node id */
      const int ia = (id[u] < id[v]) ? u : v, ib = (ia == u) ? v : u;
      const double ex = x[ib] - x[ia], ey = y[ib] - y[ia];
      if (nxv * ex + nyv * ey < 0.0) { nxv = -nxv; nyv = -nyv; }
      m->S[2 * e + 0] += nxv;
      m->S[2 * e + 1] += nyv;
    }
  }
  /* Quadrilaterals: the same median dual about the element centre c (the
   * mean of its four vertices).  Node k of the element receives the area of
   * the polygon (x_k, m_k,k+1, c, m_k-1,k) (shoelace), and every edge the
   * normal of its segment m_e -> c, oriented from a towards b. */
  for (int64_t f = 0; f < Q; ++f) {
    int32_t id[4];
    double x[4], y[4];
    for (int k = 0; k < 4; ++k) {
      id[k] = m->quad[4 * f + k];
      x[k] = m->lon[id[k]];
      y[k] = m->lat[id[k]];
    }
    for (int k = 1; k < 4; ++k) x[k] = unwrap(x[k], x[0]);
    const double cx = 0.25 * (x[0] + x[1] + x[2] + x[3]);
    const double cy = 0.25 * (y[0] + y[1] + y[2] + y[3]);
    for (int k = 0; k < 4; ++k) {
      const int kn = (k + 1) % 4, kp = (k + 3) % 4;
      const double mnx = 0.5 * (x[k] + x[kn]), mny = 0.5 * (y[k] + y[kn]);
      const double mpx = 0.5 * (x[k] + x[kp]), mpy = 0.5 * (y[k] + y[kp]);
      const double px[4] = {x[k], mnx, cx, mpx}, py[4] = {y[k], mny, cy, mpy};
      double a2 = 0.0;
      for (int s2 = 0; s2 < 4; ++s2) a2 += px[s2] * py[(s2 + 1) % 4] - px[(s2 + 1) % 4] * py[s2];
      m->A[id[k]] += 0.5 * a2;
      /* edge (k, k+1): segment from its midpoint to the centre */
      const int64_t e = find_edge(m, first, id[k], id[kn]);
      double nxv = cy - mny, nyv = -(cx - mnx);
      const int ia = (id[k] < id[kn]) ? k : kn, ib = (ia == k) ? kn : k;
      const double ex = x[ib] - x[ia], ey = y[ib] - y[ia];
      if (nxv * ex + nyv * ey < 0.0) { nxv = -nxv; nyv = -nyv; }
      m->S[2 * e + 0] += nxv;
      m->S[2 * e + 1] += nyv;
    }
  }

  /* --- polar closure -----------------------------------------------------
   * The dual cells of the first and last parallel extend to lat = +-pi/2.
   * Each edge along a polar parallel gains the straight segment from its
   * midpoint to the pole line; each polar node gains the rectangle
   * dlon0 x (pi/2 - |lat0|); its face on the pole line (length dlon0,
   * outward normal (0, sigma dlon0)) is carried by the node's pole edge,
   * which pairs it with the node half-way round the same parallel.  dlon0
   * is the spacing of that polar parallel (2 pi / 20 on O<N>).           */
  m->npole = m->nx[0] / 2 + m->nx[nr - 1] / 2;
  m->pole_edge = (int32_t *)malloc(sizeof(int32_t) * 2 * m->npole);
  m->pole_normal = (double *)malloc(sizeof(double) * m->npole);
  for (int side = 0; side < 2; ++side) {
    const int j = side == 0 ? 0 : nr - 1;
    const double sigma = side == 0 ? 1.0 : -1.0;
    const int64_t off = m->ring_off[j];
    const int n = m->nx[j];
    const double dlon0 = 2.0 * ORC_PI / (double)n;
    const double th = m->lat[off];
    const double ext = 0.5 * ORC_PI - fabs(th);
    for (int i = 0; i < n; ++i) {
      const int32_t p = (int32_t)(off + i), q = (int32_t)(off + (i + 1) % n);
      const int64_t e = find_edge(m, first, p, q);
      const int32_t a = m->edge[2 * e], b = m->edge[2 * e + 1];
      const double ex = unwrap(m->lon[b], m->lon[a]) - m->lon[a];
      /* segment from the midpoint straight to the pole line */
      const double dy = sigma * ext; /* d = (0, dy) */
      double nxv = dy, nyv = 0.0;
      if (nxv * ex < 0.0) nxv = -nxv;
      m->S[2 * e + 0] += nxv;
      m->S[2 * e + 1] += nyv;
      m->A[p] += dlon0 * ext;
    }
    for (int i = 0; i < n / 2; ++i) {
      const int k = side * (m->nx[0] / 2) + i;
      m->pole_edge[2 * k + 0] = (int32_t)(off + i);
      m->pole_edge[2 * k + 1] = (int32_t)(off + i + n / 2);
      m->pole_normal[k] = sigma * dlon0;
    }
  }

  /* physical dual volume with the nodal metric: V_i = R^2 cos(lat_i) A_i */
  m->vol = (double *)malloc(sizeof(double) * V);
  for (int64_t i = 0; i < V; ++i) m->vol[i] = R * R * m->coslat[i] * m->A[i];

  /* --- the oracle's own node -> edge lists (ascending edge id) ---------- */
  m->adj_ptr = (int64_t *)calloc((size_t)(V + 1), sizeof(int64_t));
  m->adj_edge = (int32_t *)malloc(sizeof(int32_t) * 2 * E);
  for (int64_t e = 0; e < E; ++e) {
    m->adj_ptr[m->edge[2 * e] + 1]++;
    m->adj_ptr[m->edge[2 * e + 1] + 1]++;
  }
  for (int64_t i = 0; i < V; ++i) m->adj_ptr[i + 1] += m->adj_ptr[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * V);
  for (int64_t i = 0; i < V; ++i) fill[i] = m->adj_ptr[i];
  for (int64_t e = 0; e < E; ++e) {
    m->adj_edge[fill[m->edge[2 * e]]++] = (int32_t)e;
    m->adj_edge[fill[m->edge[2 * e + 1]]++] = (int32_t)e;
  }
  free(fill);
  m->pole_of = (int32_t *)malloc(sizeof(int32_t) * V);
  for (int64_t i = 0; i < V; ++i) m->pole_of[i] = -1;
  for (int k = 0; k < m->npole; ++k) {
    m->pole_of[m->pole_edge[2 * k]] = k;
    m->pole_of[m->pole_edge[2 * k + 1]] = k;
  }
  free(first);
  return m;
}

orc_mesh *orc_mesh_build_pl(int nrings, const int32_t *nx_in, double R) {
  return build_general(nrings, nx_in, NULL, 0, 0, R);
}

/* Any grid of parallels: explicit latitudes (or NULL: Gaussian), shift,
 * quadrilaterals where two consecutive parallels have equal counts. */
orc_mesh *orc_mesh_build_ex(int nrings, const int32_t *nx_in, const double *lat_in, int shift,
                            int quads, double R) {
  return build_general(nrings, nx_in, lat_in, shift, quads, R);
}

/* Grid O<N>: Section 4.2.3.7, Listing 6 (nx = 20 + 4j up to the equator,
 * mirrored about it). */
orc_mesh *orc_mesh_build(int N, double R) {
  if (N < 1) return NULL;
  int32_t *nx = (int32_t *)malloc(sizeof(int32_t) * 2 * N);
  if (!nx) return NULL;
  for (int j = 0; j < N; ++j) {
    nx[j] = 20 + 4 * j;
    nx[2 * N - 1 - j] = nx[j];
  }
  orc_mesh *m = orc_mesh_build_pl(2 * N, nx, R);
  free(nx);
  return m;
}

/* ------------------------------------------------------------------------ */
/* Getters (copy-out) for the tests                                          */
/* ------------------------------------------------------------------------ */
void orc_mesh_sizes(const orc_mesh *m, int64_t *out) {
  out[0] = m->V; out[1] = m->E; out[2] = m->F; out[3] = m->npole;
  out[4] = m->nrings; out[5] = m->N; out[6] = m->Q;
}
void orc_mesh_copy_quads(const orc_mesh *m, int32_t *quad) {
  if (quad && m->Q > 0) memcpy(quad, m->quad, sizeof(int32_t) * 4 * m->Q);
}

void orc_mesh_copy(const orc_mesh *m, int32_t *nx, int64_t *ring_off,
                   double *lon, double *lat, int32_t *tri, int32_t *edge,
                   double *S, double *A, double *vol, int32_t *pole_edge,
                   double *pole_normal) {
  if (nx) memcpy(nx, m->nx, sizeof(int32_t) * m->nrings);
  if (ring_off) memcpy(ring_off, m->ring_off, sizeof(int64_t) * (m->nrings + 1));
  if (lon) memcpy(lon, m->lon, sizeof(double) * m->V);
  if (lat) memcpy(lat, m->lat, sizeof(double) * m->V);
  if (tri) memcpy(tri, m->tri, sizeof(int32_t) * 3 * m->F);
  if (edge) memcpy(edge, m->edge, sizeof(int32_t) * 2 * m->E);
  if (S) memcpy(S, m->S, sizeof(double) * 2 * m->E);
  if (A) memcpy(A, m->A, sizeof(double) * m->V);
  if (vol) memcpy(vol, m->vol, sizeof(double) * m->V);
  if (pole_edge) memcpy(pole_edge, m->pole_edge, sizeof(int32_t) * 2 * m->npole);
  if (pole_normal) memcpy(pole_normal, m->pole_normal, sizeof(double) * m->npole);
}

/* ------------------------------------------------------------------------ */
/* Level chunking: threads own disjoint level ranges.                        */
/* ------------------------------------------------------------------------ */
static int n_chunks(int nlev) {
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  return nt < nlev ? nt : nlev;
}

int orc_threads_used(int nlev) { return n_chunks(nlev); }

/* Threads later calls may use (results do not depend on it); returns the
 * previous maximum.  Timing aid only. */
int orc_set_threads(int n) {
#ifdef _OPENMP
  const int old = omp_get_max_threads();
  if (n >= 1) omp_set_num_threads(n);
  return old;
#else
  (void)n;
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Gradient.  For every edge e = (a, b) and level k the edge value is        */
/* phi_e = (phi_a + phi_b)/2; the flux S_e phi_e is added to a and taken     */
/* from b.  Pole edges add sigma dlon0 (phi_a + phi_b)/2 to the lat          */
/* component of BOTH their nodes (each node's own face on the pole line).   */
/* Output: physical components (zonal, meridional):                          */
/*   grad_lon = G_lon / (R cos(lat_i) A_i),   grad_lat = G_lat / (R A_i).    */
/* f: [V][nlev];  out: [V][nlev][2].                                         */
/* ------------------------------------------------------------------------ */
/* The same sums as derivatives in the computational (lon, lat) plane: both
 * components divided by the dual area A_i,
 *   (d phi/d lon, d phi/d lat)_i = (G_lon, G_lat) / A_i
 * (= (R cos(lat_i) grad_lon, R grad_lat) of the physical gradient). */
static int gradient_sums(const orc_mesh *m, int nlev, const double *f, double *out,
                         int computational);

int orc_gradient_lonlat(const orc_mesh *m, int nlev, const double *f, double *out) {
  return gradient_sums(m, nlev, f, out, 1);
}

int orc_gradient(const orc_mesh *m, int nlev, const double *f, double *out) {
  return gradient_sums(m, nlev, f, out, 0);
}

static int gradient_sums(const orc_mesh *m, int nlev, const double *f, double *out,
                         int computational) {
  if (!m || nlev < 1 || !f || !out) return -1;
  const int64_t V = m->V, E = m->E;
  const int nc = n_chunks(nlev);
  memset(out, 0, sizeof(double) * (size_t)(V * nlev * 2));
#pragma omp parallel for schedule(static, 1)
  for (int c = 0; c < nc; ++c) {
    const int k0 = (int)((int64_t)c * nlev / nc);
    const int k1 = (int)((int64_t)(c + 1) * nlev / nc);
    for (int64_t e = 0; e < E; ++e) {
      const int64_t a = m->edge[2 * e], b = m->edge[2 * e + 1];
      const double Sx = m->S[2 * e], Sy = m->S[2 * e + 1];
      for (int k = k0; k < k1; ++k) {
        const double fe = 0.5 * (f[a * nlev + k] + f[b * nlev + k]);
        const double Fx = Sx * fe, Fy = Sy * fe;
        out[(a * nlev + k) * 2 + 0] += Fx;
        out[(a * nlev + k) * 2 + 1] += Fy;
        out[(b * nlev + k) * 2 + 0] -= Fx;
        out[(b * nlev + k) * 2 + 1] -= Fy;
      }
    }
    for (int p = 0; p < m->npole; ++p) {
      const int64_t a = m->pole_edge[2 * p], b = m->pole_edge[2 * p + 1];
      const double Sy = m->pole_normal[p];
      for (int k = k0; k < k1; ++k) {
        const double fe = 0.5 * (f[a * nlev + k] + f[b * nlev + k]);
        out[(a * nlev + k) * 2 + 1] += Sy * fe;
        out[(b * nlev + k) * 2 + 1] += Sy * fe;
      }
    }
    for (int64_t i = 0; i < V; ++i) {
      const double sx = computational ? m->A[i] : m->R * m->coslat[i] * m->A[i];
      const double sy = computational ? m->A[i] : m->R * m->A[i];
      for (int k = k0; k < k1; ++k) {
        out[(i * nlev + k) * 2 + 0] /= sx;
        out[(i * nlev + k) * 2 + 1] /= sy;
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Divergence of a physical vector field (u east, v north), [V][nlev][2].   */
/* W = v cos(lat) is formed at the nodes; the edge flux is                  */
/* S_lon u_e + S_lat W_e with edge averages u_e, W_e.  Pole edges carry     */
/* nothing: W vanishes on the pole line.                                     */
/*   div_i = sum_e s_ie flux_e / (R cos(lat_i) A_i).                         */
/* Curl (radial component) is the same with (v, -u cos(lat)).               */
/* ------------------------------------------------------------------------ */
static int div_or_curl(const orc_mesh *m, int nlev, const double *uv,
                       double *out, int curl) {
  if (!m || nlev < 1 || !uv || !out) return -1;
  const int64_t V = m->V, E = m->E;
  const int nc = n_chunks(nlev);
  memset(out, 0, sizeof(double) * (size_t)(V * nlev));
#pragma omp parallel for schedule(static, 1)
  for (int c = 0; c < nc; ++c) {
    const int k0 = (int)((int64_t)c * nlev / nc);
    const int k1 = (int)((int64_t)(c + 1) * nlev / nc);
    for (int64_t e = 0; e < E; ++e) {
      const int64_t a = m->edge[2 * e], b = m->edge[2 * e + 1];
      const double Sx = m->S[2 * e], Sy = m->S[2 * e + 1];
      const double ca = m->coslat[a], cb = m->coslat[b];
      for (int k = k0; k < k1; ++k) {
        const double ua = uv[(a * nlev + k) * 2], va = uv[(a * nlev + k) * 2 + 1];
        const double ub = uv[(b * nlev + k) * 2], vb = uv[(b * nlev + k) * 2 + 1];
        double flux;
        if (!curl) {
          const double ue = 0.5 * (ua + ub);
          const double We = 0.5 * (va * ca + vb * cb);
          flux = Sx * ue + Sy * We;
        } else {
          const double ve = 0.5 * (va + vb);
          const double Ze = 0.5 * (ua * ca + ub * cb);
          flux = Sx * ve - Sy * Ze;
        }
        out[a * nlev + k] += flux;
        out[b * nlev + k] -= flux;
      }
    }
    for (int64_t i = 0; i < V; ++i) {
      const double s = m->R * m->coslat[i] * m->A[i];
      for (int k = k0; k < k1; ++k) out[i * nlev + k] /= s;
    }
  }
  return 0;
}

int orc_divergence(const orc_mesh *m, int nlev, const double *uv, double *out) {
  return div_or_curl(m, nlev, uv, out, 0);
}
int orc_curl(const orc_mesh *m, int nlev, const double *uv, double *out) {
  return div_or_curl(m, nlev, uv, out, 1);
}

/* Laplacian = divergence of the gradient, both discrete (two passes). */
int orc_laplacian(const orc_mesh *m, int nlev, const double *f, double *out) {
  if (!m || nlev < 1 || !f || !out) return -1;
  double *g = (double *)malloc(sizeof(double) * (size_t)(m->V * nlev * 2));
  if (!g) return -2;
  int rc = orc_gradient(m, nlev, f, g);
  if (rc == 0) rc = orc_divergence(m, nlev, g, out);
  free(g);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Sampled evaluation: the same operators at selected nodes only, summing    */
/* over the node's own edges in ascending edge id and the pole edge last --  */
/* the order in which the full edge loop above reaches each accumulator, so  */
/* the sampled values are bitwise equal to the full ones.                     */
/* ------------------------------------------------------------------------ */
static void grad_one(const orc_mesh *m, int nlev, const double *f, int64_t i,
                     double *o /* [nlev][2] */) {
  for (int k = 0; k < nlev; ++k) { o[2 * k] = 0.0; o[2 * k + 1] = 0.0; }
  for (int64_t r = m->adj_ptr[i]; r < m->adj_ptr[i + 1]; ++r) {
    const int64_t e = m->adj_edge[r];
    const int64_t a = m->edge[2 * e], b = m->edge[2 * e + 1];
    const double Sx = m->S[2 * e], Sy = m->S[2 * e + 1];
    for (int k = 0; k < nlev; ++k) {
      const double fe = 0.5 * (f[a * nlev + k] + f[b * nlev + k]);
      const double Fx = Sx * fe, Fy = Sy * fe;
      if (a == i) { o[2 * k] += Fx; o[2 * k + 1] += Fy; }
      else        { o[2 * k] -= Fx; o[2 * k + 1] -= Fy; }
    }
  }
  const int p = m->pole_of[i];
  if (p >= 0) {
    const int64_t a = m->pole_edge[2 * p], b = m->pole_edge[2 * p + 1];
    const double Sy = m->pole_normal[p];
    for (int k = 0; k < nlev; ++k) {
      const double fe = 0.5 * (f[a * nlev + k] + f[b * nlev + k]);
      o[2 * k + 1] += Sy * fe;
    }
  }
  const double sx = m->R * m->coslat[i] * m->A[i], sy = m->R * m->A[i];
  for (int k = 0; k < nlev; ++k) { o[2 * k] /= sx; o[2 * k + 1] /= sy; }
}

/* uvval(n, k, c): vector component c of node n at level k, looked up through
 * an accessor so that the Laplacian can feed sampled gradients.            */
typedef double (*uv_get)(const void *ctx, int64_t n, int k, int c);

static void divcurl_one(const orc_mesh *m, int nlev, uv_get get,
                        const void *ctx, int64_t i, double *o, int curl) {
  for (int k = 0; k < nlev; ++k) o[k] = 0.0;
  for (int64_t r = m->adj_ptr[i]; r < m->adj_ptr[i + 1]; ++r) {
    const int64_t e = m->adj_edge[r];
    const int64_t a = m->edge[2 * e], b = m->edge[2 * e + 1];
    const double Sx = m->S[2 * e], Sy = m->S[2 * e + 1];
    const double ca = m->coslat[a], cb = m->coslat[b];
    for (int k = 0; k < nlev; ++k) {
      const double ua = get(ctx, a, k, 0), va = get(ctx, a, k, 1);
      const double ub = get(ctx, b, k, 0), vb = get(ctx, b, k, 1);
      double flux;
      if (!curl) {
        const double ue = 0.5 * (ua + ub);
        const double We = 0.5 * (va * ca + vb * cb);
        flux = Sx * ue + Sy * We;
      } else {
        const double ve = 0.5 * (va + vb);
        const double Ze = 0.5 * (ua * ca + ub * cb);
        flux = Sx * ve - Sy * Ze;
      }
      if (a == i) o[k] += flux; else o[k] -= flux;
    }
  }
  const double s = m->R * m->coslat[i] * m->A[i];
  for (int k = 0; k < nlev; ++k) o[k] /= s;
}

typedef struct { const double *uv; int nlev; } dense_ctx;
static double dense_get(const void *ctx, int64_t n, int k, int c) {
  const dense_ctx *d = (const dense_ctx *)ctx;
  return d->uv[(n * d->nlev + k) * 2 + c];
}

static int check_sel(const orc_mesh *m, int64_t nsel, const int64_t *sel) {
  for (int64_t s = 0; s < nsel; ++s)
    if (sel[s] < 0 || sel[s] >= m->V) return -1;
  return 0;
}

int orc_gradient_at(const orc_mesh *m, int nlev, const double *f,
                    int64_t nsel, const int64_t *sel, double *out) {
  if (!m || nlev < 1 || !f || !out || (nsel && !sel) || check_sel(m, nsel, sel))
    return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < nsel; ++s)
    grad_one(m, nlev, f, sel[s], out + s * nlev * 2);
  return 0;
}

static int divcurl_at(const orc_mesh *m, int nlev, const double *uv,
                      int64_t nsel, const int64_t *sel, double *out, int curl) {
  if (!m || nlev < 1 || !uv || !out || (nsel && !sel) || check_sel(m, nsel, sel))
    return -1;
  dense_ctx ctx = {uv, nlev};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < nsel; ++s)
    divcurl_one(m, nlev, dense_get, &ctx, sel[s], out + s * nlev, curl);
  return 0;
}
int orc_divergence_at(const orc_mesh *m, int nlev, const double *uv,
                      int64_t nsel, const int64_t *sel, double *out) {
  return divcurl_at(m, nlev, uv, nsel, sel, out, 0);
}
int orc_curl_at(const orc_mesh *m, int nlev, const double *uv, int64_t nsel,
                const int64_t *sel, double *out) {
  return divcurl_at(m, nlev, uv, nsel, sel, out, 1);
}

/* Sampled Laplacian: gradients at every node of the sampled nodes' 1-ring,
 * then the divergence of those gradients at the sampled nodes.            */
typedef struct { const int64_t *slot; const double *g; int nlev; } ring_ctx;
static double ring_get(const void *ctx, int64_t n, int k, int c) {
  const ring_ctx *r = (const ring_ctx *)ctx;
  return r->g[(r->slot[n] * r->nlev + k) * 2 + c];
}

int orc_laplacian_at(const orc_mesh *m, int nlev, const double *f,
                     int64_t nsel, const int64_t *sel, double *out) {
  if (!m || nlev < 1 || !f || !out || (nsel && !sel) || check_sel(m, nsel, sel))
    return -1;
  int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * m->V);
  if (!slot) return -2;
  for (int64_t i = 0; i < m->V; ++i) slot[i] = -1;
  int64_t nring = 0;
  for (int64_t s = 0; s < nsel; ++s) {
    const int64_t i = sel[s];
    if (slot[i] < 0) slot[i] = nring++;
    for (int64_t r = m->adj_ptr[i]; r < m->adj_ptr[i + 1]; ++r) {
      const int64_t e = m->adj_edge[r];
      const int64_t o = m->edge[2 * e] == i ? m->edge[2 * e + 1] : m->edge[2 * e];
      if (slot[o] < 0) slot[o] = nring++;
    }
  }
  int64_t *nodes = (int64_t *)malloc(sizeof(int64_t) * (nring ? nring : 1));
  double *g = (double *)malloc(sizeof(double) * (size_t)((nring ? nring : 1) * nlev * 2));
  if (!nodes || !g) { free(slot); free(nodes); free(g); return -2; }
  for (int64_t i = 0; i < m->V; ++i)
    if (slot[i] >= 0) nodes[slot[i]] = i;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < nring; ++q) grad_one(m, nlev, f, nodes[q], g + q * nlev * 2);
  ring_ctx ctx = {slot, g, nlev};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < nsel; ++s)
    divcurl_one(m, nlev, ring_get, &ctx, sel[s], out + s * nlev, 0);
  free(slot); free(nodes); free(g);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Remap: interpolation of a nodal field of this mesh to other points       */
/* (Section 1 lists remapping / interpolation of fields between different   */
/* grids among the mathematical operations; the paper gives no method).     */
/* Reading taken here: the value at a target point is the piecewise-linear  */
/* (P1) interpolant of the nodal values on this mesh's triangles, in the    */
/* (lon, lat) plane with longitudes unwrapped round the target:             */
/*   out(t) = sum over the three vertices k of the containing triangle of   */
/*            w_k(t) * in(vertex k),                                        */
/* w_k the barycentric coordinates of t.  A target poleward of the first    */
/* (last) parallel takes the linear interpolant along that parallel at its  */
/* longitude (the field continued to the pole unchanged in latitude): the   */
/* two bracketing nodes of the parallel, weights (1 - s, s).  Levels are    */
/* independent (vertical extrusion, Section 4.3), so the same weights serve */
/* every level.                                                              */
/* ------------------------------------------------------------------------ */

/* Twice the signed area of (p, q, r). */
static double cross3(double px, double py, double qx, double qy, double rx, double ry) {
  return (qx - px) * (ry - py) - (qy - py) * (rx - px);
}

/* Barycentric coordinates of (x, y) in the triangle (X[k], Y[k]): each
 * coordinate is the area of the sub-triangle opposite vertex k over the
 * triangle's area, the latter taken from vertex k itself (so a target on a
 * vertex gets exactly 1 there and 0 elsewhere). */
static void barycentric(const double *X, const double *Y, double x, double y, double *w) {
  for (int k = 0; k < 3; ++k) {
    const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
    const double whole = cross3(X[k], Y[k], X[k1], Y[k1], X[k2], Y[k2]);
    const double part = cross3(x, y, X[k1], Y[k1], X[k2], Y[k2]);
    w[k] = part / whole;
  }
}

/* Weights of one target; returns 0, or -1 for a latitude outside
 * [-pi/2, pi/2] or a non-finite coordinate. */
static int remap_one(const orc_mesh *m, const int64_t *toff, double lon, double lat,
                     int32_t *idx, double *w) {
  if (!isfinite(lon) || !isfinite(lat) || lat > 0.5 * ORC_PI || lat < -0.5 * ORC_PI) return -1;
  double x = fmod(lon, 2.0 * ORC_PI);
  if (x < 0.0) x += 2.0 * ORC_PI;
  if (x >= 2.0 * ORC_PI) x = 0.0;
  const int nr = m->nrings;
  const double lat_first = m->lat[m->ring_off[0]];
  const double lat_last = m->lat[m->ring_off[nr - 1]];
  if (lat > lat_first || lat < lat_last) {
    /* polar cap: along the polar parallel */
    const int j = lat > lat_first ? 0 : nr - 1;
    const int64_t o = m->ring_off[j];
    const int n = m->nx[j];
    int i = 0;
    while (i + 1 < n && m->lon[o + i + 1] <= x) ++i;
    const double x0 = m->lon[o + i];
    const double x1 = (i + 1 < n) ? m->lon[o + i + 1] : m->lon[o] + 2.0 * ORC_PI;
    const double s = (x - x0) / (x1 - x0);
    idx[0] = (int32_t)(o + i);
    idx[1] = (int32_t)(o + (i + 1) % n);
    idx[2] = (int32_t)(o + i);
    w[0] = 1.0 - s;
    w[1] = s;
    w[2] = 0.0;
    return 0;
  }
  /* the first strip whose lower parallel is at or below the target */
  int j = 0;
  while (j + 2 < nr && m->lat[m->ring_off[j + 1]] > lat) ++j;
  /* the strip's triangle that contains the target most clearly: the one
   * whose smallest barycentric coordinate is largest (first on ties) */
  double best = -HUGE_VAL;
  for (int64_t t = toff[j]; t < toff[j + 1]; ++t) {
    /* the triangle kept whole: its first vertex unwrapped round the
     * target, the other two round the first vertex */
    double X[3], Y[3], wt[3];
    for (int k = 0; k < 3; ++k) {
      const int32_t v = m->tri[3 * t + k];
      X[k] = k == 0 ? unwrap(m->lon[v], x) : unwrap(m->lon[v], X[0]);
      Y[k] = m->lat[v];
    }
    barycentric(X, Y, x, lat, wt);
    double mn = wt[0];
    if (wt[1] < mn) mn = wt[1];
    if (wt[2] < mn) mn = wt[2];
    if (mn > best) {
      best = mn;
      for (int k = 0; k < 3; ++k) {
        idx[k] = m->tri[3 * t + k];
        w[k] = wt[k];
      }
    }
  }
  return 0;
}

int orc_remap_weights(const orc_mesh *m, int64_t nt, const double *lon, const double *lat,
                      int32_t *idx, double *w) {
  if (m->Q > 0 || m->shift) return -3; /* triangles from lon 0 only */
  const int nr = m->nrings;
  int64_t *toff = (int64_t *)malloc(sizeof(int64_t) * nr);
  if (!toff) return -2;
  toff[0] = 0;
  for (int j = 0; j + 1 < nr; ++j) toff[j + 1] = toff[j] + m->nx[j] + m->nx[j + 1];
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
  for (int64_t t = 0; t < nt; ++t)
    bad |= remap_one(m, toff, lon[t], lat[t], idx + 3 * t, w + 3 * t) != 0;
  free(toff);
  return bad ? -1 : 0;
}

/* out[t][k] = w[t][0] in[idx[t][0]][k] + w[t][1] in[idx[t][1]][k]
 *           + w[t][2] in[idx[t][2]][k], summed in that order.  ncol values
 * per node (levels, or levels x components). */
int orc_remap_apply(int64_t nsrc, int64_t nt, const int32_t *idx, const double *w, int ncol,
                    const double *in, double *out) {
  for (int64_t t = 0; t < 3 * nt; ++t)
    if (idx[t] < 0 || idx[t] >= nsrc) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nt; ++t) {
    const double *a = in + (int64_t)idx[3 * t] * ncol;
    const double *b = in + (int64_t)idx[3 * t + 1] * ncol;
    const double *c = in + (int64_t)idx[3 * t + 2] * ncol;
    double *o = out + t * ncol;
    for (int k = 0; k < ncol; ++k) o[k] = w[3 * t] * a[k] + w[3 * t + 1] * b[k] + w[3 * t + 2] * c[k];
  }
  return 0;
}
