// hlbm_device.h -- device-side data structures and helpers of the gfx950
// HLBM hot path (D3Q19 tables, population storage formats, particle geometry).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlbm {

// ---------------------------------------------------------------------------
// D3Q19 velocity set and weights (Sec. 3.1 velocity-set and weight equations).
// Opposite directions are adjacent: opp(i) = i + 1 for odd i, i - 1 for even i.
// ---------------------------------------------------------------------------
constexpr int Q = 19;
constexpr int kCX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double wgt(int i) {
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Work decomposition of the lattice: a tile is 64 (x) x 4 (y) x 4 (z) cells,
// processed by one 256-thread workgroup (one wave per y-row, a loop over z).
constexpr int TX = 64;
constexpr int TY = 4;
constexpr int TZ = 4;
constexpr int MAXC = 48;        // particles a tile can list
constexpr int MAX_AXIS_TILES = 16;

__device__ inline int wave_id() { return threadIdx.x >> 6; }
__device__ inline int lane_id() { return threadIdx.x & 63; }

// Sums and minima over the 64 lanes of a wavefront (fixed butterfly order).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// Workgroups are dispatched to the 8 XCDs (each with its own L2) round-robin.
// Workgroup b is given work item (b mod 8) (n / 8) + b / 8 of n, so that each
// XCD sweeps one contiguous run of items in order and the data neighbouring
// items share is read through the same L2.  The last n mod 8 items map to
// themselves.
__device__ inline int xcd_chunk(int b, int n) {
  const int per = n >> 3;
  if (b >= per * 8) return b;
  return (b & 7) * per + (b >> 3);
}

__device__ inline int wave_min(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

// Status bits raised by kernels.
constexpr int ST_UNSTABLE = 1;
constexpr int ST_WALL_EXIT = 2;
constexpr int ST_TILE_OVERFLOW = 4;
constexpr int ST_CONTACT_OVERFLOW = 8;

struct Lattice {
  int nx, ny, nz;
  int bc[3];
  int ntx, nty, ntz;
  int ntiles;
  long long N;
  double omega;   // 1 / tau
  double eps;     // indicator width
  double af[3];   // fluid body acceleration
  double rho_f;
  double g[3];
  const float *tables;  // per-particle learned distance tables (NULL: none)
  long long table_cap;  // floats per particle table
  const float4 *mesh;   // triangles of the mesh shape: 3 vertices each (unit scale)
  int mesh_nt;          // number of triangles (0: no mesh)
  int psm;              // coupling: 0 exact-difference source (HLBM), 1 partially saturated collision
  double tau_mh;        // tau - 1/2
};

// Particle record on the device (FP64).  The first block mirrors the public
// record; the rest is derived each time the state changes.
struct DevParticle {
  double X[3], q[4], U[3], W[3];
  double m, V, I[3], prm[3];
  double R[9];     // body -> world rotation, row-major
  double rc;       // circumradius
  double Fh[3];    // hydrodynamic force of the last momentum exchange
  double Th[3];    // hydrodynamic torque of the last momentum exchange
  int shape, flags;
  int lo[3], hi[3];  // cells that can have B > 0 (centre within rc + eps/2), unwrapped
  int learned;       // distance table: 0 none, 1 learned (network), 2 exact (mesh)
};

// Tiles touched by a cell range along one axis (wrapped on periodic axes),
// in increasing cell order; returns the count (<= MAX_AXIS_TILES).  Steps from
// tile to tile (one division per tile, not per cell).
__device__ inline int axis_tiles(int lo, int hi, int n, int periodic, int tsize, int *out) {
  int cnt = 0;
  int c = lo;
  while (c <= hi) {
    int w = c;
    if (periodic) { w %= n; if (w < 0) w += n; }
    if (w < 0) { c = 0; continue; }
    if (w >= n) break;
    const int t = w / tsize;
    bool seen = false;
    for (int k = 0; k < cnt; ++k) seen |= (out[k] == t);
    if (!seen && cnt < MAX_AXIS_TILES) out[cnt++] = t;
    c += min((t + 1) * tsize, n) - w;  // first cell of the next tile
  }
  return cnt;
}

// Offset of a cell inside a particle's coupling box (wrapped on periodic axes);
// the table index is lx + sx (ly + sy lz).
__device__ inline int box_offset(int v, int lo, int n, int periodic) {
  int d = v - lo;
  if (periodic) {
    if (d < 0) d += n;
    else if (d >= n) d -= n;
  }
  return d;
}

// ---------------------------------------------------------------------------
// Population storage.  Every format holds the relative deviation
//   s_i = K (f_i - w_i) / w_i
// (K = 1 for FP64 / FP32, K = 256 for FP16S), so the equilibrium needs no
// per-direction weight:  K (feq_i - w_i) / w_i = K (rho - 1) + K rho (3 c.u +
// 4.5 (c.u)^2 - 1.5 u.u),  and FP16 deviations down to ~2e-7 stay normal.
// T is the arithmetic precision, G the precision of particle geometry.
// ---------------------------------------------------------------------------
struct StoreF64 {
  using S = double;
  using T = double;
  using G = double;
  static constexpr int kind = 0;
  __device__ static constexpr double K() { return 1.0; }
  __device__ static inline T dec(S v) { return v; }
  __device__ static inline S enc(T v) { return v; }
};
struct StoreF32 {
  using S = float;
  using T = float;
  using G = float;
  static constexpr int kind = 1;
  __device__ static constexpr float K() { return 1.0f; }
  __device__ static inline T dec(S v) { return v; }
  __device__ static inline S enc(T v) { return v; }
};
struct StoreF16S {
  using S = _Float16;
  using T = float;
  using G = float;
  static constexpr int kind = 2;
  __device__ static constexpr float K() { return 256.0f; }
  __device__ static inline T dec(S v) { return (float)v; }
  __device__ static inline S enc(T v) { return (_Float16)v; }
};

// Population f_i in FP64 from a stored value.
template <class ST>
__device__ inline double pop_f64(typename ST::S v, int i) {
  return wgt(i) * (1.0 + (double)ST::dec(v) / (double)ST::K());
}

// ---------------------------------------------------------------------------
// Geometry.  Signed distances are negative inside (Sec. 3.2).
// ---------------------------------------------------------------------------
// Reciprocal: exact division in FP64, the hardware reciprocal (1 ulp) in FP32.
__device__ inline double frcp(double v) { return 1.0 / v; }
__device__ inline float frcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ inline double dsqrt(double v) { return sqrt(v); }
__device__ inline float dsqrt(float v) { return sqrtf(v); }
__device__ inline double dcos(double v) { return cos(v); }
__device__ inline float dcos(float v) { return __cosf(v); }
__device__ inline double dabs(double v) { return fabs(v); }
__device__ inline float dabs(float v) { return fabsf(v); }
__device__ inline double dmax(double a, double b) { return fmax(a, b); }
__device__ inline float dmax(float a, float b) { return fmaxf(a, b); }
__device__ inline double dmin(double a, double b) { return fmin(a, b); }
__device__ inline float dmin(float a, float b) { return fminf(a, b); }

// Distance from (y0, y1) >= 0 to the ellipse (u/e0)^2 + (v/e1)^2 = 1, e0 >= e1.
// The nearest point is x_k = e_k^2 y_k / (t + e_k^2) where t is the root of
// G(t) = sum_k (e_k y_k / (t + e_k^2))^2 - 1.  G is convex and decreasing for
// t > -e1^2, so Newton's method started at t0 = e1 y1 - e1^2 (G >= 0 there)
// increases monotonically to the root.
template <typename G>
__device__ inline G ellipse_distance(G e0, G e1, G y0, G y1) {
  const G e0s = e0 * e0, e1s = e1 * e1;
  if (y1 > G(0)) {
    if (y0 > G(0)) {
      const G a = e0 * y0, b = e1 * y1;
      const G lo = b - e1s;  // G(lo) >= 0
      // Newton from t = 0 (the root for a point on the surface).  Outside,
      // G(0) > 0 and the iteration increases monotonically to the root; inside,
      // the first step overshoots to the left of the root (G is convex), is
      // clamped to the bracket, and the iteration then increases monotonically.
      G t = G(0);
      for (int it = 0; it < 100; ++it) {
        const G i0 = frcp(t + e0s), i1 = frcp(t + e1s);
        const G r0 = a * i0, r1 = b * i1;
        const G gv = r0 * r0 + r1 * r1 - G(1);
        const G dg = G(-2) * (r0 * r0 * i0 + r1 * r1 * i1);
        G tn = t - gv * frcp(dg);
        if (tn < lo) tn = lo;
        if (it > 0 && !(tn > t)) break;
        t = tn;
      }
      const G x0 = e0s * y0 / (t + e0s), x1 = e1s * y1 / (t + e1s);
      return dsqrt((x0 - y0) * (x0 - y0) + (x1 - y1) * (x1 - y1));
    }
    return dabs(y1 - e1);
  }
  const G den = e0s - e1s;
  if (e0 * y0 < den) {
    const G x0 = e0s * y0 / den;
    const G s = x0 / e0;
    const G x1 = e1 * dsqrt(dmax(G(0), G(1) - s * s));
    return dsqrt((x0 - y0) * (x0 - y0) + x1 * x1);
  }
  return dabs(y0 - e0);
}

// Body-frame signed distance of a rounded cube or spheroid (shape 1, 2).
template <typename G>
__device__ inline G sdf_body(int shape, G p0, G p1, G b0, G b1, G b2) {
  if (shape == 0) return dsqrt(b0 * b0 + b1 * b1 + b2 * b2) - p0;
  if (shape == 1) {
    const G core = p0 - p1;
    const G q0 = dabs(b0) - core, q1 = dabs(b1) - core, q2 = dabs(b2) - core;
    const G o0 = dmax(q0, G(0)), o1 = dmax(q1, G(0)), o2 = dmax(q2, G(0));
    return dsqrt(o0 * o0 + o1 * o1 + o2 * o2) + dmin(dmax(q0, dmax(q1, q2)), G(0)) - p1;
  }
  // spheroid: symmetry axis body x (semi-axis p0), equal semi-axes p1
  const G y0 = dabs(b0), y1 = dsqrt(b1 * b1 + b2 * b2);
  const G d = (p0 >= p1) ? ellipse_distance<G>(p0, p1, y0, y1) : ellipse_distance<G>(p1, p0, y1, y0);
  const G k = (b0 * b0) / (p0 * p0) + (b1 * b1 + b2 * b2) / (p1 * p1);
  return k <= G(1) ? -d : d;
}

// Signed distance for the indicator, with a cheap classification of cells that
// are certainly farther than eps/2 from the surface: returns +-1e30 there.
// ia2, ib2 = 1/p0^2, 1/p1^2.
template <typename G>
__device__ inline G sdf_for_indicator(int shape, G p0, G p1, G ia2, G ib2, G b0, G b1, G b2, G half_eps) {
  if (shape == 2) {
    // s^2 = implicit value; |d| >= |s - 1| * min(p0, p1) (the scaled spheroids
    // s E and E are at least that far apart), so only a thin shell iterates.
    const G k = b0 * b0 * ia2 + (b1 * b1 + b2 * b2) * ib2;
    const G s = dsqrt(k);
    if (dabs(s - G(1)) * dmin(p0, p1) >= half_eps) return k <= G(1) ? G(-1e30) : G(1e30);
  }
  return sdf_body<G>(shape, p0, p1, b0, b1, b2);
}

// ---------------------------------------------------------------------------
// Triangle-mesh particles (shape 3): a closed mesh at unit scale, triangles
// counter-clockwise seen from outside, scaled by param[0].  The unsigned
// distance is the least distance to a triangle (the foot of the perpendicular
// on the triangle's plane when it falls inside the triangle, else the nearest
// edge); the sign comes from the generalised winding number, the summed solid
// angles of the triangles over 4 pi (Van Oosterom and Strackee's formula for
// the solid angle of a triangle), which is 1 inside and 0 outside.
// ---------------------------------------------------------------------------
__device__ inline double datan2(double y, double x) { return atan2(y, x); }
__device__ inline float datan2(float y, float x) { return atan2f(y, x); }

template <typename G>
struct V3 {
  G x, y, z;
};
template <typename G>
__device__ inline V3<G> v3sub(V3<G> a, V3<G> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename G>
__device__ inline G v3dot(V3<G> a, V3<G> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename G>
__device__ inline V3<G> v3cross(V3<G> a, V3<G> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename G>
__device__ inline V3<G> v3load(const float4 &v) { return {(G)v.x, (G)v.y, (G)v.z}; }

// squared distance from q to the segment [a, b]
template <typename G>
__device__ inline G seg_dist2(V3<G> q, V3<G> a, V3<G> b) {
  const V3<G> ab = v3sub(b, a), aq = v3sub(q, a);
  G t = v3dot(aq, ab) / v3dot(ab, ab);
  t = dmin(dmax(t, G(0)), G(1));
  const V3<G> d = {aq.x - t * ab.x, aq.y - t * ab.y, aq.z - t * ab.z};
  return v3dot(d, d);
}

template <typename G>
__device__ inline G tri_dist2(V3<G> q, V3<G> a, V3<G> b, V3<G> c) {
  const V3<G> e0 = v3sub(b, a), e1 = v3sub(c, a), aq = v3sub(q, a);
  const V3<G> n = v3cross(e0, e1);
  const G nn = v3dot(n, n);
  const G h = v3dot(aq, n) / nn;
  const V3<G> f = {aq.x - h * n.x, aq.y - h * n.y, aq.z - h * n.z};
  const G d00 = v3dot(e0, e0), d01 = v3dot(e0, e1), d11 = v3dot(e1, e1);
  const G f0 = v3dot(f, e0), f1 = v3dot(f, e1);
  const G den = d00 * d11 - d01 * d01;
  const G u = (d11 * f0 - d01 * f1) / den, v = (d00 * f1 - d01 * f0) / den;
  if (u >= G(0) && v >= G(0) && u + v <= G(1)) return h * h * nn;
  return dmin(seg_dist2(q, a, b), dmin(seg_dist2(q, b, c), seg_dist2(q, c, a)));
}

template <typename G>
__device__ inline G tri_solid_angle(V3<G> q, V3<G> a, V3<G> b, V3<G> c) {
  const V3<G> A = v3sub(a, q), B = v3sub(b, q), C = v3sub(c, q);
  const G la = dsqrt(v3dot(A, A)), lb = dsqrt(v3dot(B, B)), lc = dsqrt(v3dot(C, C));
  const G num = v3dot(A, v3cross(B, C));
  const G den = la * lb * lc + v3dot(A, B) * lc + v3dot(A, C) * lb + v3dot(B, C) * la;
  return G(2) * datan2(num, den);
}

// Signed distance of the body-frame point (x, y, z) to the mesh at `scale`.
template <typename G>
__device__ inline G mesh_sdf(const float4 *tri, int nt, G scale, G x, G y, G z) {
  const G is = G(1) / scale;
  const V3<G> q = {x * is, y * is, z * is};
  G d2 = G(1e30), omega = G(0);
  for (int t = 0; t < nt; ++t) {
    const V3<G> a = v3load<G>(tri[3 * t]), b = v3load<G>(tri[3 * t + 1]), c = v3load<G>(tri[3 * t + 2]);
    d2 = dmin(d2, tri_dist2(q, a, b, c));
    omega += tri_solid_angle(q, a, b, c);
  }
  const G d = scale * dsqrt(d2);
  return omega > G(6.283185307179586) ? -d : d;
}

// Inside test d_s <= 0 from the shape's implicit form (FP64).
__device__ inline bool inside_body(int shape, double p0, double p1, double b0, double b1, double b2) {
  if (shape == 0) return b0 * b0 + b1 * b1 + b2 * b2 <= p0 * p0;
  if (shape == 1) {
    const double core = p0 - p1;
    const double q0 = fabs(b0) - core, q1 = fabs(b1) - core, q2 = fabs(b2) - core;
    if (fmax(q0, fmax(q1, q2)) <= 0.0) return true;
    const double o0 = fmax(q0, 0.0), o1 = fmax(q1, 0.0), o2 = fmax(q2, 0.0);
    return o0 * o0 + o1 * o1 + o2 * o2 <= p1 * p1;
  }
  return (b0 * b0) / (p0 * p0) + (b1 * b1 + b2 * b2) / (p1 * p1) <= 1.0;
}

// Trigonometric indicator B(d) (Sec. 3.2 level-set equation), read as
// cos^2((pi/2)(d/eps + 1/2)) inside the band |d| < eps/2.
template <typename G>
__device__ inline G indicator(G d, G eps, G inv_eps) {
  if (d <= G(-0.5) * eps) return G(1);
  if (d >= G(0.5) * eps) return G(0);
  const G c = dcos(G(1.5707963267948966) * (d * inv_eps + G(0.5)));
  return c * c;
}

}  // namespace hlbm
