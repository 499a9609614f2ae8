// hlbm_lattice.hip -- the gfx950 collide-and-stream kernel of the HLBM time
// step.
//
//   k_collide   one workgroup per tile of 64 x 4 x 4 cells: the tile's
//               particles staged in LDS, the indicator and solid velocity of
//               the tile's cells accumulated in LDS by a dense pre-pass over
//               each particle's part of the tile, then per cell: pull,
//               moments, exact-difference source, BGK, store; with MEA, the
//               next step's momentum exchange from the values just written.
#include "hlbm_internal.h"
#include "hlbm_tile.h"

namespace hlbm {

// ---------------------------------------------------------------------------
// Momentum exchange of the next step inside the collide kernel (Sec. 3.2 MEA,
// total-force and torque equations).  The values a step writes are the state
// the next step's exchange reads, and the particles the step couples are the
// ones that exchange uses (Sec. 4.2, Algorithm 1: the fluid -> particle
// coupling of step t + 1 follows the collision of step t).  In pull storage
// f_i(x_b + c_i) = A[i][x_b] and f_opp(i)(x_b) = A[opp i][x_b + c_i], so the
// value f = A[j][y] written by cell y enters
//   - the term of x_b = y, direction j, if y is inside and y + c_j is not past
//     a wall: (c_j - u_p(y)) f;
//   - the term of x_b = y + c_j, direction opp(j), if y + c_j is a cell inside
//     the particle: (-c_j + u_p(y + c_j)) f, with u_p(y + c_j) = u_p(y) + w x c_j.
// Summed over j, with rho, M, P the zeroth, first and second moments of f over
// the directions of each kind (_i: in-terms, _o: out-terms) and d = y - X:
//   F_h(y) = (M_i - u rho_i) - M_o + u rho_o + w x M_o,
//   T_h(y) = d x F_h + M_o x u + w tr(P_o) - P_o w,
// which regroups exactly the sum over inside cells x_b and directions i; the
// particle receives -F_h and -T_h.  FP64 throughout, on the stored values.
// ---------------------------------------------------------------------------
constexpr double kSqrt2 = 1.4142135623730951;

// Inside test d_s <= 0 of the cell centre at unwrapped coordinates u: the
// cell must lie in the particle's momentum-exchange box (centre within the
// circumradius along each axis, mlo..mhi), then the implicit form of the exact
// shape (the same arithmetic as k_mea) or, with a distance table tab (learned
// and mesh particles, over the coupling box), its entry.
__device__ inline bool mea_inside_point(const DevParticle &P, const float *tab, const int *mlo, const int *mhi,
                                        int u0, int u1, int u2) {
  if (u0 < mlo[0] || u0 > mhi[0] || u1 < mlo[1] || u1 > mhi[1] || u2 < mlo[2] || u2 > mhi[2]) return false;
  if (tab) {
    const int tsx = P.hi[0] - P.lo[0] + 1, tsy = P.hi[1] - P.lo[1] + 1;
    return tab[(u0 - P.lo[0]) + tsx * ((u1 - P.lo[1]) + tsy * (u2 - P.lo[2]))] <= 0.0f;
  }
  const double d0 = (u0 + 0.5) - P.X[0], d1 = (u1 + 0.5) - P.X[1], d2 = (u2 + 0.5) - P.X[2];
  double b0 = d0, b1 = d1, b2 = d2;
  if (P.shape != 0) {
    const double *R = P.R;
    b0 = R[0] * d0 + R[3] * d1 + R[6] * d2;
    b1 = R[1] * d0 + R[4] * d1 + R[7] * d2;
    b2 = R[2] * d0 + R[5] * d1 + R[8] * d2;
  }
  return inside_body(P.shape, P.prm[0], P.prm[1], b0, b1, b2);
}

// Geometry of one particle for the exchange, formed once per wavefront and
// candidate (all values uniform over the wavefront).
struct MeaGeom {
  int mlo[3], mhi[3];  // momentum-exchange box (unwrapped)
  double out2;         // |d| beyond sqrt(out2): the cell and its neighbours are outside
  double in2;          // |d| within sqrt(in2): the cell and its neighbours are inside (< 0: none)
  const float *tab;    // distance table (learned / mesh), else NULL
};

__device__ inline MeaGeom mea_geom(const Lattice &L, const DevParticle &P, int pid) {
  MeaGeom g;
  const int n[3] = {L.nx, L.ny, L.nz};
  for (int k = 0; k < 3; ++k) {
    // the box k_mea visits: centre within rc + 1e-9, clipped at walls
    int a = (int)ceil(P.X[k] - (P.rc + 1e-9) - 0.5), b = (int)floor(P.X[k] + (P.rc + 1e-9) - 0.5);
    if (L.bc[k]) {
      a = max(a, 0);
      b = min(b, n[k] - 1);
    }
    g.mlo[k] = a;
    g.mhi[k] = b;
  }
  g.tab = (P.learned && L.tables) ? L.tables + (size_t)pid * (size_t)L.table_cap : nullptr;
  // a table marks cells beyond rc + eps/2 outside and within r_in - eps/2
  // inside (r_in the inscribed radius); the exact shapes are outside beyond rc
  // and inside within r_in
  const double rin = P.shape == 2 ? fmin(P.prm[0], P.prm[1]) : (P.shape == 3 ? P.prm[2] : P.prm[0]);
  const double ro = (g.tab ? P.rc + 0.5 * L.eps : P.rc) + kSqrt2 + 1e-9;
  const double ri = (g.tab ? rin - 0.5 * L.eps : rin) - kSqrt2 - 1e-9;
  g.out2 = ro * ro;
  g.in2 = ri > 0.0 ? ri * ri : -1.0;
  return g;
}

// Masked sums over directions 1..18 of the lattice weights in units of 1/36
// (w_i = 2/36 along the axes, 1/36 along the diagonals): sum_i w_i, sum_i c_i
// w_i and the entries of sum_i w_i c_i c_i^T, from the set bits of m.
struct WeightMoments {
  int g, m[3], p[6];  // p: xx, yy, zz, xy, xz, yz
};
__device__ inline WeightMoments weight_moments(unsigned m) {
  WeightMoments r;
  r.g = 0;
  for (int k = 0; k < 3; ++k) r.m[k] = 0;
  for (int k = 0; k < 6; ++k) r.p[k] = 0;
#pragma unroll
  for (int j = 1; j < Q; ++j) {
    const int on = (m >> j) & 1u;
    const int w36 = j <= 6 ? 2 * on : on;
    r.g += w36;
    r.m[0] += kCX[j] * w36; r.m[1] += kCY[j] * w36; r.m[2] += kCZ[j] * w36;
    r.p[0] += kCX[j] * kCX[j] * w36; r.p[1] += kCY[j] * kCY[j] * w36; r.p[2] += kCZ[j] * kCZ[j] * w36;
    r.p[3] += kCX[j] * kCY[j] * w36; r.p[4] += kCX[j] * kCZ[j] * w36; r.p[5] += kCY[j] * kCZ[j] * w36;
  }
  return r;
}

// -F_h(y) and -T_h(y) of one particle from the values v[19] that cell y (at
// unwrapped coordinates u, offset d = y - X) writes; walls: bit j of wallmask
// is set where y + c_j lies past a wall.  Returns false (and leaves FT zero)
// when neither y nor any of its neighbours is inside.  With f = w (1 + v / K)
// the moments split into the lattice weights' (exact small integers over 36)
// and the stored deviations' (summed in the arithmetic precision TV: the
// deviations are small, so their rounding stays far below the storage's);
// from the moments on, everything is FP64.
template <typename TV>
__device__ inline bool mea_cell_terms(const DevParticle &P, const MeaGeom &g, int u0, int u1, int u2,
                                      unsigned wallmask, const TV *v, TV invK, double *FT) {
  const double d0 = (u0 + 0.5) - P.X[0], d1 = (u1 + 0.5) - P.X[1], d2 = (u2 + 0.5) - P.X[2];
  const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
  if (r2 > g.out2) return false;
  constexpr unsigned ALL = 0x7FFFEu;  // directions 1..18
  bool in_y;
  unsigned nb;
  bool uniform = r2 <= g.in2;  // the cell and all its neighbours inside
  bool side = true;
  if (!uniform && !g.tab && P.shape != 0) {
    // the exact signed distance (rounded cube) or a lower bound of its size
    // (spheroid: |s - 1| min(a, b), s^2 the implicit value) beyond sqrt 2
    // puts the cell and all its neighbours on one side
    const double *R = P.R;
    const double b0 = R[0] * d0 + R[3] * d1 + R[6] * d2;
    const double b1 = R[1] * d0 + R[4] * d1 + R[7] * d2;
    const double b2 = R[2] * d0 + R[5] * d1 + R[8] * d2;
    if (P.shape == 1) {
      const double ds = sdf_body<double>(1, P.prm[0], P.prm[1], b0, b1, b2);
      if (fabs(ds) > kSqrt2 + 1e-9) { uniform = true; side = ds < 0.0; }
    } else if (P.shape == 2) {
      const double k = b0 * b0 / (P.prm[0] * P.prm[0]) + (b1 * b1 + b2 * b2) / (P.prm[1] * P.prm[1]);
      if (fabs(sqrt(k) - 1.0) * fmin(P.prm[0], P.prm[1]) > kSqrt2 + 1e-9) { uniform = true; side = k <= 1.0; }
    }
  }
  if (uniform) {
    if (!side) return false;
    in_y = true;
    nb = ALL & ~wallmask;
  } else {
    in_y = mea_inside_point(P, g.tab, g.mlo, g.mhi, u0, u1, u2);
    nb = 0;
#pragma unroll
    for (int j = 1; j < Q; ++j)
      if (!((wallmask >> j) & 1u) && mea_inside_point(P, g.tab, g.mlo, g.mhi, u0 + kCX[j], u1 + kCY[j], u2 + kCZ[j]))
        nb |= 1u << j;
    if (!in_y && nb == 0) return false;
  }
  const unsigned inm = in_y ? (ALL & ~wallmask) : 0u;
  // deviation parts: sums of w_i v_i / K
  TV Gi = 0, Mi0 = 0, Mi1 = 0, Mi2 = 0;
  TV Go = 0, Mo0 = 0, Mo1 = 0, Mo2 = 0, Pxx = 0, Pyy = 0, Pzz = 0, Pxy = 0, Pxz = 0, Pyz = 0;
#pragma unroll
  for (int j = 1; j < Q; ++j) {
    const TV q = (TV)wgt(j) * invK * v[j];
    const TV fi = ((inm >> j) & 1u) ? q : (TV)0;
    const TV fo = ((nb >> j) & 1u) ? q : (TV)0;
    Gi += fi;
    Go += fo;
    if (kCX[j]) { Mi0 += kCX[j] > 0 ? fi : -fi; Mo0 += kCX[j] > 0 ? fo : -fo; Pxx += fo; }
    if (kCY[j]) { Mi1 += kCY[j] > 0 ? fi : -fi; Mo1 += kCY[j] > 0 ? fo : -fo; Pyy += fo; }
    if (kCZ[j]) { Mi2 += kCZ[j] > 0 ? fi : -fi; Mo2 += kCZ[j] > 0 ? fo : -fo; Pzz += fo; }
    if (kCX[j] && kCY[j]) Pxy += kCX[j] * kCY[j] > 0 ? fo : -fo;
    if (kCX[j] && kCZ[j]) Pxz += kCX[j] * kCZ[j] > 0 ? fo : -fo;
    if (kCY[j] && kCZ[j]) Pyz += kCY[j] * kCZ[j] > 0 ? fo : -fo;
  }
  // weight parts, exact
  const WeightMoments wi = weight_moments(inm), wo = weight_moments(nb);
  constexpr double i36 = 1.0 / 36.0;
  const double gi = wi.g * i36 + (double)Gi;
  const double mi0 = wi.m[0] * i36 + (double)Mi0, mi1 = wi.m[1] * i36 + (double)Mi1, mi2 = wi.m[2] * i36 + (double)Mi2;
  const double go = wo.g * i36 + (double)Go;
  const double mo0 = wo.m[0] * i36 + (double)Mo0, mo1 = wo.m[1] * i36 + (double)Mo1, mo2 = wo.m[2] * i36 + (double)Mo2;
  const double pxx = wo.p[0] * i36 + (double)Pxx, pyy = wo.p[1] * i36 + (double)Pyy, pzz = wo.p[2] * i36 + (double)Pzz;
  const double pxy = wo.p[3] * i36 + (double)Pxy, pxz = wo.p[4] * i36 + (double)Pxz, pyz = wo.p[5] * i36 + (double)Pyz;
  const double *W = P.W;
  const double u0v = P.U[0] + W[1] * d2 - W[2] * d1;
  const double u1v = P.U[1] + W[2] * d0 - W[0] * d2;
  const double u2v = P.U[2] + W[0] * d1 - W[1] * d0;
  const double F0 = (mi0 - u0v * gi) - mo0 + u0v * go + (W[1] * mo2 - W[2] * mo1);
  const double F1 = (mi1 - u1v * gi) - mo1 + u1v * go + (W[2] * mo0 - W[0] * mo2);
  const double F2 = (mi2 - u2v * gi) - mo2 + u2v * go + (W[0] * mo1 - W[1] * mo0);
  const double tr = pxx + pyy + pzz;
  const double T0 = (d1 * F2 - d2 * F1) + (mo1 * u2v - mo2 * u1v) + W[0] * tr - (pxx * W[0] + pxy * W[1] + pxz * W[2]);
  const double T1 = (d2 * F0 - d0 * F2) + (mo2 * u0v - mo0 * u2v) + W[1] * tr - (pxy * W[0] + pyy * W[1] + pyz * W[2]);
  const double T2 = (d0 * F1 - d1 * F0) + (mo0 * u1v - mo1 * u0v) + W[2] * tr - (pxz * W[0] + pyz * W[1] + pzz * W[2]);
  FT[0] = -F0; FT[1] = -F1; FT[2] = -F2;
  FT[3] = -T0; FT[4] = -T1; FT[5] = -T2;
  return true;
}

// Fused collide + stream with the exact-difference source (one workgroup per
// tile).  With stored values s_i = K (f_i - w_i) / w_i:
//   rho = 1 + sum_i w_i s_i / K,   rho u = sum_i w_i c_i s_i / K      (Sec. 3.1)
//   du = B (u_s - u) + (1 - B) a_f                                  (Sec. 3.2)
//   e_i(v) = K (rho - 1) + K rho (3 c_i.v + 4.5 (c_i.v)^2 - 1.5 v.v)
//   s*_i = (1 - 1/tau)(s_i - e_i(u)) + e_i(u + du)
// which is f_i - (f_i - feq_i(u))/tau + feq_i(u + du) - feq_i(u) in these
// units; without a source it is s_i - (s_i - e_i(u))/tau.  Opposite
// directions share the even part of e_i.
template <class ST>
__device__ inline void pull_fast(const typename ST::S *__restrict__ A, long long N, int x, int xm, int xp,
                                 const int *rowsrc, typename ST::T *s) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int sx = kCX[i] == 1 ? xm : (kCX[i] == -1 ? xp : x);
    const int r = rowsrc[(kCY[i] + 1) * 3 + (kCZ[i] + 1)];
    const typename ST::S *plane = A + (long long)i * N;
    s[i] = ST::dec(plane[(unsigned)(sx + r)]);
  }
}

template <class ST, bool MEA>
__global__ __launch_bounds__(256) void k_collide(Lattice L, const typename ST::S *__restrict__ A,
                                                 typename ST::S *__restrict__ Bo,
                                                 const DevParticle *__restrict__ parts,
                                                 const int *__restrict__ tcnt,
                                                 const int *__restrict__ tlist, int *tcnt_clear,
                                                 int *status, double *__restrict__ mea_out) {
  using T = typename ST::T;
  using G = typename ST::G;
  __shared__ TileCands<G> tc;
  // the coupling fields are dead after the cell loop: their space then holds
  // the wavefronts' momentum-exchange sums
  __shared__ union {
    TileFields<G> tf;
    double red[4][MAXC][6];
  } sh;
  TileFields<G> &tf = sh.tf;
  const T K = ST::K();
  const T invK = (T)1 / K;
  const T omega = (T)L.omega;
  const T one_m_omega = (T)1 - omega;
  const T afx = (T)L.af[0], afy = (T)L.af[1], afz = (T)L.af[2];
  const bool has_af = (L.af[0] != 0.0) || (L.af[1] != 0.0) || (L.af[2] != 0.0);
  const int nx = L.nx, ny = L.ny, nz = L.nz;

  const int tile = xcd_chunk(blockIdx.x, L.ntiles);
  const int tx = tile % L.ntx;
  const int ty = (tile / L.ntx) % L.nty;
  const int tz = tile / (L.ntx * L.nty);
  load_candidates<G>(L, parts, tcnt, tlist, tile, tc);
  const int nc = tc.n;
  // the other tile-list buffer is refilled by the next step's binning
  if (threadIdx.x == 0 && tcnt_clear) tcnt_clear[tile] = 0;
  tile_coupling<G>(L, tc, tx, ty, tz, tf);
  // momentum exchange: lane k holds this wavefront's sums for candidate k
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};

  for (int zz = 0; zz < TZ; ++zz) {
    CellPos cp;
    cp.x = tx * TX + lane_id();
    cp.y = ty * TY + wave_id();
    cp.z = tz * TZ + zz;
    if (cp.z >= nz || cp.y >= ny) break;
    cp.act = cp.x < nx;
    const int cell = cp.x + nx * (cp.y + ny * cp.z);

    T s[Q];
    if (cp.act) {
      // rows wholly away from walls take the direct pull: 32-bit offsets from
      // per-direction plane bases (the condition is uniform over the wave)
      const bool edge = L.bc[0] || (L.bc[1] && (cp.y == 0 || cp.y == ny - 1)) ||
                        (L.bc[2] && (cp.z == 0 || cp.z == nz - 1));
      if (!edge) {
        const int ys[3] = {cp.y == ny - 1 ? 0 : cp.y + 1, cp.y, cp.y == 0 ? ny - 1 : cp.y - 1};  // source y for c_y = -1, 0, +1
        const int zs[3] = {cp.z == nz - 1 ? 0 : cp.z + 1, cp.z, cp.z == 0 ? nz - 1 : cp.z - 1};
        int rowsrc[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) rowsrc[a * 3 + b] = nx * (ys[a] + ny * zs[b]);
        const int xm = cp.x == 0 ? nx - 1 : cp.x - 1, xp = cp.x == nx - 1 ? 0 : cp.x + 1;
        pull_fast<ST>(A, L.N, cp.x, xm, xp, rowsrc, s);
      } else {
        const PullIdx P = pull_index(L, cp);
        pull_all<ST>(L, A, cp, P, s);
      }
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) s[i] = (T)0;
    }
    // moments
    T rho1 = (T)0, jx = (T)0, jy = (T)0, jz = (T)0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T wk = (T)wgt(i) * invK;
      rho1 += wk * s[i];
      if (kCX[i]) jx += (T)kCX[i] * wk * s[i];
      if (kCY[i]) jy += (T)kCY[i] * wk * s[i];
      if (kCZ[i]) jz += (T)kCZ[i] * wk * s[i];
    }
    const T rho = (T)1 + rho1;
    const T inv = frcp(rho);
    const T ux = jx * inv, uy = jy * inv, uz = jz * inv;

    G S0 = G(0), S1[3] = {G(0), G(0), G(0)};
    if (nc > 0) {
      const int idx = lane_id() + TX * (wave_id() + TY * zz);
      S0 = tf.S0[idx];
      S1[0] = tf.S1[0][idx]; S1[1] = tf.S1[1][idx]; S1[2] = tf.S1[2][idx];
    }
    T du0 = afx, du1 = afy, du2 = afz;
    if (S0 > G(0)) {
      const T Bt = (T)(S0 < G(1) ? S0 : G(1));
      const G is0 = frcp(S0);
      const T usx = (T)(S1[0] * is0), usy = (T)(S1[1] * is0), usz = (T)(S1[2] * is0);
      du0 = Bt * (usx - ux) + ((T)1 - Bt) * afx;
      du1 = Bt * (usy - uy) + ((T)1 - Bt) * afy;
      du2 = Bt * (usz - uz) + ((T)1 - Bt) * afz;
    }
    const bool coupled = has_af || S0 > G(0);

    const T usq = ux * ux + uy * uy + uz * uz;
    // one flag per wavefront, raised by its first unstable lane
    const unsigned long long bad = __ballot(cp.act && !(rho > (T)0 && usq < (T)0.09));
    if (bad && lane_id() == __ffsll((long long)bad) - 1) atomicOr(status, ST_UNSTABLE);
    const T Kr1 = K * rho1, Krho = K * rho;
    const T o3 = (T)3 * Krho, e45 = (T)4.5 * Krho;  // e_i = base + e45 (c.u)^2 + o3 c.u
    const T base = Kr1 - (T)1.5 * Krho * usq;
    // plain BGK, then the exact-difference source e_i(u + du) - e_i(u) where
    // the cell is coupled
    T out[Q];
    out[0] = s[0] - omega * (s[0] - base);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      const T cu = (T)kCX[i] * ux + (T)kCY[i] * uy + (T)kCZ[i] * uz;
      const T E = base + e45 * cu * cu, O = o3 * cu;
      out[i] = s[i] - omega * (s[i] - (E + O));
      out[i + 1] = s[i + 1] - omega * (s[i + 1] - (E - O));
    }
    if (coupled) {
      const T vx = ux + du0, vy = uy + du1, vz = uz + du2;
      const T dE0 = (T)-1.5 * Krho * ((vx * vx + vy * vy + vz * vz) - usq);
      out[0] += dE0;
#pragma unroll
      for (int i = 1; i < Q; i += 2) {
        const T cu = (T)kCX[i] * ux + (T)kCY[i] * uy + (T)kCZ[i] * uz;
        const T cd = (T)kCX[i] * du0 + (T)kCY[i] * du1 + (T)kCZ[i] * du2;
        const T dE = dE0 + e45 * cd * (cd + (T)2 * cu), dO = o3 * cd;
        out[i] += dE + dO;
        out[i + 1] += dE - dO;
      }
    }
    if (cp.act) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        typename ST::S *plane = Bo + (long long)i * L.N;
        // streamed out: nothing in this step reads it back
        __builtin_nontemporal_store(ST::enc(out[i]), &plane[(unsigned)cell]);
      }
    }
    if constexpr (MEA) {
      if (nc > 0) {
        // the values as stored (what the next step reads)
        T v[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = ST::dec(ST::enc(out[i]));
        unsigned wallmask = 0;
#pragma unroll
        for (int j = 1; j < Q; ++j) {
          const bool past = (L.bc[0] && ((kCX[j] < 0 && cp.x == 0) || (kCX[j] > 0 && cp.x == nx - 1))) ||
                            (L.bc[1] && ((kCY[j] < 0 && cp.y == 0) || (kCY[j] > 0 && cp.y == ny - 1))) ||
                            (L.bc[2] && ((kCZ[j] < 0 && cp.z == 0) || (kCZ[j] > 0 && cp.z == nz - 1)));
          wallmask |= past ? (1u << j) : 0u;
        }
        for (int ci = 0; ci < nc; ++ci) {
          const Cand<G> &c = tc.c[ci];
          int u1, u2, u0 = 0;
          // rows outside the candidate's bin box add nothing (uniform)
          if (!unwrap_into(cp.y, c.blo[1], c.bhi[1], ny, !L.bc[1], u1)) continue;
          if (!unwrap_into(cp.z, c.blo[2], c.bhi[2], nz, !L.bc[2], u2)) continue;
          const bool lane_in = cp.act && unwrap_into(cp.x, c.blo[0], c.bhi[0], nx, !L.bc[0], u0);
          if (__ballot(lane_in) == 0) continue;
          const int pid = __builtin_amdgcn_readfirstlane(c.pid);
          const DevParticle &P = parts[pid];
          const MeaGeom g = mea_geom(L, P, pid);
          double ft[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
          const bool any = lane_in && mea_cell_terms<T>(P, g, u0, u1, u2, wallmask, v, invK, ft);
          if (__ballot(any) == 0) continue;
#pragma unroll
          for (int k = 0; k < 6; ++k) ft[k] = wave_sum(ft[k]);
          if (lane_id() == ci)
#pragma unroll
            for (int k = 0; k < 6; ++k) acc[k] += ft[k];
        }
      }
    }
  }
  if constexpr (MEA) {
    // one record per (particle, tile of its bin box): the four wavefronts'
    // sums added in order (zero where no row adds anything); the EoM kernel
    // sums the records in order
    if (nc > 0) {
      __syncthreads();  // every wavefront is done with the coupling fields
      const int k = lane_id();
      if (k < nc)
#pragma unroll
        for (int q = 0; q < 6; ++q) sh.red[wave_id()][k][q] = acc[q];
      __syncthreads();
      const int t = threadIdx.x;
      if (t < nc) {
        const Cand<G> &c = tc.c[t];
        if (c.rec >= 0 && c.rec < REC_TILES) {
          double *dst = mea_out + ((size_t)c.pid * REC_TILES + c.rec) * 6;
#pragma unroll
          for (int q = 0; q < 6; ++q) dst[q] = ((sh.red[0][t][q] + sh.red[1][t][q]) + sh.red[2][t][q]) + sh.red[3][t][q];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
static inline int blocks_for(long long n, int b) { return (int)((n + b - 1) / b); }

#define HLBM_DISPATCH(prec, CALL)                       \
  switch (prec) {                                       \
    case 0: { using ST = StoreF64; CALL; } break;       \
    case 1: { using ST = StoreF32; CALL; } break;       \
    default: { using ST = StoreF16S; CALL; } break;     \
  }

hipError_t launch_collide(int prec, const Lattice &L, const void *A, void *B, const DevParticle *parts,
                          const int *tcnt, const int *tlist, int *tcnt_clear, int *status, double *mea_out,
                          hipStream_t s) {
  if (mea_out) {
    HLBM_DISPATCH(prec, hipLaunchKernelGGL((k_collide<ST, true>), dim3(L.ntiles), dim3(256), 0, s, L,
                                           (const typename ST::S *)A, (typename ST::S *)B, parts, tcnt,
                                           tlist, tcnt_clear, status, mea_out));
  } else {
    HLBM_DISPATCH(prec, hipLaunchKernelGGL((k_collide<ST, false>), dim3(L.ntiles), dim3(256), 0, s, L,
                                           (const typename ST::S *)A, (typename ST::S *)B, parts, tcnt,
                                           tlist, tcnt_clear, status, mea_out));
  }
  return hipGetLastError();
}

}  // namespace hlbm
