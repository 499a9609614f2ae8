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
constexpr int MAXC = 48;  // particles a tile can list

// Status bits raised by kernels.
constexpr int ST_UNSTABLE = 1;
constexpr int ST_WALL_EXIT = 2;
constexpr int ST_TILE_OVERFLOW = 4;

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
};

// Particle record on the device (FP64).  The first block mirrors the public
// record; the rest is derived each time the state changes.
struct DevParticle {
  double X[3], q[4], U[3], W[3];
  double m, V, I[3], prm[3];
  double R[9];     // body -> world rotation, row-major
  double rc;       // circumradius
  double reach;    // rc + max(eps/2, sqrt 2): cells farther away never couple
  double Fh[3];    // hydrodynamic force of the last momentum exchange
  double Th[3];    // hydrodynamic torque of the last momentum exchange
  int shape, flags;
  int lo[3], hi[3];  // cell range of the reach box (unwrapped coordinates)
};

// Candidate particle of a tile, staged in LDS.
struct Cand {
  double X[3], U[3], W[3];
  double R[9];
  double p0, p1;
  double reach2;
  int shape;
  int slot;
};

// ---------------------------------------------------------------------------
// Population storage.  All formats hold the deviation g_i = f_i - w_i.
// ---------------------------------------------------------------------------
struct StoreF64 {
  using S = double;
  using T = double;
  static constexpr int kind = 0;
  __device__ static inline T dec(S v, int) { return v; }
  __device__ static inline S enc(T g, int) { return g; }
};
struct StoreF32 {
  using S = float;
  using T = float;
  static constexpr int kind = 1;
  __device__ static inline T dec(S v, int) { return v; }
  __device__ static inline S enc(T g, int) { return g; }
};
// FP16 holding 256 (f_i - w_i) / w_i: every direction uses the same relative
// range, and deviations down to ~2e-7 of w_i stay normal numbers.
struct StoreF16S {
  using S = _Float16;
  using T = float;
  static constexpr int kind = 2;
  __device__ static inline T dec(S v, int i) {
    return (float)v * (i == 0 ? (1.0f / 768.0f) : (i <= 6 ? (1.0f / 4608.0f) : (1.0f / 9216.0f)));
  }
  __device__ static inline S enc(T g, int i) {
    return (_Float16)(g * (i == 0 ? 768.0f : (i <= 6 ? 4608.0f : 9216.0f)));
  }
};

// ---------------------------------------------------------------------------
// Geometry (FP64).  Signed distances are negative inside (Sec. 3.2).
// ---------------------------------------------------------------------------
__device__ inline double min_image(double d, int n, int periodic) {
  if (periodic) {
    double h = 0.5 * n;
    if (d > h) d -= n;
    else if (d < -h) d += n;
  }
  return d;
}

// Distance from (y0, y1) >= 0 to the ellipse (u/e0)^2 + (v/e1)^2 = 1, e0 >= e1.
// The nearest point is x_k = e_k^2 y_k / (t + e_k^2) where t is the root of
// G(t) = sum_k (e_k y_k / (t + e_k^2))^2 - 1.  G is convex and decreasing for
// t > -e1^2, so Newton's method started at t0 = e1 y1 - e1^2 (G >= 0 there)
// increases monotonically to the root.
__device__ inline double ellipse_distance(double e0, double e1, double y0, double y1) {
  const double e0s = e0 * e0, e1s = e1 * e1;
  if (y1 > 0.0) {
    if (y0 > 0.0) {
      const double a = e0 * y0, b = e1 * y1;
      double t = b - e1s;
      for (int it = 0; it < 100; ++it) {
        const double p0 = t + e0s, p1 = t + e1s;
        const double r0 = a / p0, r1 = b / p1;
        const double G = r0 * r0 + r1 * r1 - 1.0;
        const double dG = -2.0 * (r0 * r0 / p0 + r1 * r1 / p1);
        const double tn = t - G / dG;
        if (!(tn > t)) break;
        t = tn;
      }
      const double x0 = e0s * y0 / (t + e0s), x1 = e1s * y1 / (t + e1s);
      return sqrt((x0 - y0) * (x0 - y0) + (x1 - y1) * (x1 - y1));
    }
    return fabs(y1 - e1);
  }
  const double den = e0s - e1s;
  if (e0 * y0 < den) {
    const double x0 = e0s * y0 / den;
    const double s = x0 / e0;
    const double x1 = e1 * sqrt(fmax(0.0, 1.0 - s * s));
    return sqrt((x0 - y0) * (x0 - y0) + x1 * x1);
  }
  return fabs(y0 - e0);
}

// Body-frame signed distance.  Only called where |d| may be below eps/2 or the
// sign is needed; far-field cells are classified before calling.
__device__ inline double sdf_body(int shape, double p0, double p1, double b0, double b1, double b2) {
  if (shape == 0) return sqrt(b0 * b0 + b1 * b1 + b2 * b2) - p0;
  if (shape == 1) {
    const double core = p0 - p1;
    const double q0 = fabs(b0) - core, q1 = fabs(b1) - core, q2 = fabs(b2) - core;
    const double o0 = fmax(q0, 0.0), o1 = fmax(q1, 0.0), o2 = fmax(q2, 0.0);
    return sqrt(o0 * o0 + o1 * o1 + o2 * o2) + fmin(fmax(q0, fmax(q1, q2)), 0.0) - p1;
  }
  // spheroid: symmetry axis body x (semi-axis p0), equal semi-axes p1
  const double y0 = fabs(b0), y1 = sqrt(b1 * b1 + b2 * b2);
  const double d = (p0 >= p1) ? ellipse_distance(p0, p1, y0, y1) : ellipse_distance(p1, p0, y1, y0);
  const double k = (b0 * b0) / (p0 * p0) + (b1 * b1 + b2 * b2) / (p1 * p1);
  return k <= 1.0 ? -d : d;
}

// Inside test d_s <= 0 from the shape's implicit form.
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

// Signed distance for the indicator, with a cheap classification of cells that
// are certainly farther than eps/2 from the surface: returns +-BIG there.
__device__ inline double sdf_for_indicator(int shape, double p0, double p1, double b0, double b1,
                                           double b2, double half_eps) {
  if (shape == 2) {
    // s^2 = implicit value; |d| >= |s - 1| * min(p0, p1) (the scaled spheroids
    // s E and E are at least that far apart), so only a thin shell iterates.
    const double k = (b0 * b0) / (p0 * p0) + (b1 * b1 + b2 * b2) / (p1 * p1);
    const double s = sqrt(k);
    if (fabs(s - 1.0) * fmin(p0, p1) >= half_eps) return k <= 1.0 ? -1e30 : 1e30;
  }
  return sdf_body(shape, p0, p1, b0, b1, b2);
}

// Trigonometric indicator B(d) (Sec. 3.2 level-set equation), read as
// cos^2((pi/2)(d/eps + 1/2)) inside the band |d| < eps/2.
__device__ inline double indicator(double d, double eps) {
  if (d <= -0.5 * eps) return 1.0;
  if (d >= 0.5 * eps) return 0.0;
  const double c = cos(1.5707963267948966 * (d / eps + 0.5));
  return c * c;
}

}  // namespace hlbm
